// sur.hip -- HIP kernels (gfx950) and C ABI of the coarse-grid 3D U-Net
// surrogate: 3x3x3 convolutions as implicit GEMMs on BF16 matrix cores with
// FP32 accumulation (forward, data gradient, weight gradient), pooling,
// upsampling, channel concat, residual MSE, Adam, and the grid transfers and
// window checks that couple it to the LBM solver. See include/sur.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <type_traits>

#include "sur.h"

namespace {

// Discards an error that an earlier HIP call of another library left pending
// in this thread, so that the check after an entry point's launches
// (hipGetLastError) reports only that entry point's own failures.
inline void clear_stale_error() { (void)hipGetLastError(); }


typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float(uint32_t(v) << 16); }

// round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// f(integral_constant<int, i>) for i = B .. E - 1, unrolled at compile time.
template <int B, int E, class F>
__device__ __forceinline__ void unroll(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        unroll<B + 1, E>(f);
    }
}

// e / c and e % c for element indices below 2^31 (32-bit unsigned).
__device__ __forceinline__ long div32(long e, int c) { return (long)((uint32_t)e / (uint32_t)c); }
__device__ __forceinline__ int mod32(long e, int c) { return (int)((uint32_t)e % (uint32_t)c); }

// (x, y, z) of point p < 2^31 of an nx x ny x nz grid, x fastest (32-bit
// unsigned divisions: 64-bit ones cost several times more).
__device__ __forceinline__ void coords(long p, int nx, int ny, int &x, int &y, int &z) {
    const uint32_t u = (uint32_t)p, r = u / (uint32_t)nx;
    x = (int)(u - r * (uint32_t)nx);
    z = (int)(r / (uint32_t)ny);
    y = (int)(r - (uint32_t)z * (uint32_t)ny);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Signed distance of the equilibrium profile phi = (1 + tanh(2 psi / W)) / 2,
// psi = (W / 4) ln(phi / (1 - phi)), with phi clamped to [LS_EPS, 1 - LS_EPS].
constexpr double LS_EPS = 1e-4;
__device__ __forceinline__ float ls_psi_f(float f, float W) {
    f = fminf(fmaxf(f, (float)LS_EPS), 1.f - (float)LS_EPS);
    return 0.25f * W * logf(f / (1.f - f));
}
__device__ __forceinline__ double ls_psi(double f, double W) {
    f = fmin(fmax(f, LS_EPS), 1.0 - LS_EPS);
    return 0.25 * W * log(f / (1.0 - f));
}
__device__ __forceinline__ double ls_phi(double s, double W) { return 0.5 * (1.0 + tanh(2.0 * s / W)); }
__device__ __forceinline__ float ls_phi_f(float s, float W) { return 0.5f * (1.f + tanhf(2.f * s / W)); }

// ------------------------------------------------------------ convolution
// Implicit GEMM: Y[p][o] = sum_{t, i} X[p + s d_t][i] Wk[t][o][i].
// A wavefront owns 64 points (four 16-point M tiles) and a 64-channel block of
// outputs (up to four 16-channel N tiles); the K loop runs over the 27 taps and
// 16-channel slices of the input. MFMA 16x16x16 BF16 operand layout: lane l
// holds A[m = l % 16][k = 4 (l / 16) .. +3] (4 consecutive input channels of
// point m: one 8-byte load in channels-last storage) and B[k][n = l % 16]
// (4 consecutive input channels of output channel n: one 8-byte load of the
// [t][o][i] packing); the result D[m = 4 (l / 16) + j][n = l % 16] is in
// register j.
__global__ void __launch_bounds__(256) conv3d_kernel(const uint16_t *__restrict__ x, int cin,
                                                     const uint16_t *__restrict__ w,
                                                     const float *__restrict__ bias, int cout,
                                                     int nx, int ny, int nz, int flip, int relu,
                                                     const uint16_t *__restrict__ mask,
                                                     uint16_t *__restrict__ yb,
                                                     float *__restrict__ yf) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const long P = (long)nx * ny * nz;
    const long pbase = ((long)blockIdx.x * 4 + wave) * 64;
    const int cob = blockIdx.y * 64;
    const int ntiles = min(4, (cout - cob) >> 4);
    int px[4], py[4], pz[4];
    bool pv[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const long p = pbase + mt * 16 + r;
        pv[mt] = p < P;
        const long pp = pv[mt] ? p : 0;
        coords(pp, nx, ny, px[mt], py[mt], pz[mt]);
    }
    f4 acc[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
    const s4 zero = s4{0, 0, 0, 0};
    for (int t = 0; t < 27; ++t) {
        int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
        if (flip) {
            dx = -dx;
            dy = -dy;
            dz = -dz;
        }
        long nb[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            nb[mt] = (long)wrap(px[mt] + dx, nx) +
                     (long)nx * ((long)wrap(py[mt] + dy, ny) + (long)ny * wrap(pz[mt] + dz, nz));
        const uint16_t *wt = w + ((long)t * cout + cob) * cin;
        for (int cc = 0; cc < cin; cc += 16) {
            s4 a[4], b[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                a[mt] = pv[mt] ? *(const s4 *)(x + nb[mt] * cin + cc + 4 * q) : zero;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                b[nt] = nt < ntiles ? *(const s4 *)(wt + (long)(nt * 16 + r) * cin + cc + 4 * q)
                                    : zero;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                if (nt < ntiles) {
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mt], b[nt],
                                                                                 acc[mt][nt], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            if (nt >= ntiles) continue;
            const int co = cob + nt * 16 + r;
            const float bb = bias ? bias[co] : 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const long p = pbase + mt * 16 + 4 * q + j;
                if (p >= P) continue;
                float v = acc[mt][nt][j] + bb;
                if (relu) v = fmaxf(v, 0.f);
                if (mask && !(bf2f(mask[p * cout + co]) > 0.f)) v = 0.f;
                if (yb) yb[p * cout + co] = f2bf(v);
                if (yf) yf[p * cout + co] = v;
            }
        }
    }
}

// The same convolution for grids whose sizes are multiples of the 16 x 4 x 4
// point tile. Blocks are persistent: block b takes the tiles b, b + gridDim.x,
// ..., each over its 16-channel input chunks, and stages an item's 18 x 6 x 6
// halo (32 B per point, 20.7 KB) and the chunk's weights in LDS, so each
// input value is read from memory about 2.5 times instead of 27 times. While
// an item is computed from LDS, each thread's six 16-byte pieces of the next
// item's halo are already loading into registers. Wavefront w owns plane
// z0 + w of the tile: four rows of 16 points, the four M tiles; a block
// computes NT 16-channel N tiles (one for 16 output channels, run at four
// wavefronts per SIMD; two otherwise). The K steps use the
// 16x16x32 BF16 MFMA; one step covers two taps (lanes l / 16 = 0, 1: the
// step's first tap, 2, 3: its second) x 16 channels (8 per lane). A and B
// place the same (tap, channel) in the same lane group and element, so the
// product does not depend on how the hardware orders K within a step. The
// 14th step's second tap does not exist and enters as zeros.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
constexpr int kTX = 16, kTY = 4, kTZ = 4;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2, kHP = kHX * kHY * kHZ;
constexpr int kNT = 2;  // 16-channel output tiles per block at most (LDS <= 48.4 KB)

static_assert(kHP * 2 > 1280 && kHP * 2 <= 1536, "six 16-byte halo pieces per thread");

// The K steps' pairs of point offsets d = (dx, dy, dz): step s takes
// slots 2s (lanes l / 16 = 0, 1) and 2s + 1 (lanes 2, 3):
//   s = 3g + j, g = 0, 1, 2:  (g - 1, j - 1, -1) and (g - 1, j - 1, 0)
//   s = 9 + j:                (-1, j - 1, 1)    and (0, j - 1, 1)
//   s = 12:                   (1, -1, 1)        and (1, 0, 1)
//   s = 13:                   (1, 1, 1)         and none (zeros)
// In each of the first four groups of three steps the pair is the same but
// for dy, so row mt of step j reads halo row mt + j: six fragment reads
// serve the group's twelve products. The weight of slot sl is tap
// slot_tap(sl) (t = (dx + 1) + 3 (dy + 1) + 9 (dz + 1)); the flipped
// convolution, sum_t X[p - d_t] W[t], takes tap 26 - t for offset d_t.
__host__ __device__ constexpr int slot_tap(int sl, bool flip) {
    const int s = sl >> 1, h = sl & 1;
    int dx = 1, dy = 1, dz = 1;
    if (s < 9) {
        dx = s / 3 - 1;
        dy = s % 3 - 1;
        dz = h - 1;
    } else if (s < 12) {
        dx = h - 1;
        dy = s - 10;
    } else if (s == 12) {
        dy = h - 1;
    }
    const int t = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
    return flip ? 26 - t : t;
}
__host__ __device__ constexpr bool slots_cover_taps() {
    int seen = 0;
    for (int sl = 0; sl < 27; ++sl) seen |= 1 << slot_tap(sl, false);
    return seen == (1 << 27) - 1;
}
static_assert(slots_cover_taps(), "the 27 slots hold every tap once");

// Grid of the tiled convolution (host-computed): sizes, tile counts, and for
// power-of-two sizes the shifts that replace divisions and the periodic wrap.
struct ConvGeom {
    int nx, ny, nz;
    int ntx, nty, ntz;
    int lx, lxy;    // log2 nx, log2 (nx ny)
    int ltx, ltxy;  // log2 ntx, log2 (ntx nty)
    int wres;       // every input chunk's weights staged in LDS once per kernel
    int lys;        // log2 of the tile rows of an XCD's slab, or -1 (x-fastest order)
};

// Origin of work item tl's tile of TZ planes in z. Work items are dealt to
// the eight XCDs in turn (item tl on XCD tl % 8 when the grid's x size is a
// multiple of 8). With G.lys >= 0 (power-of-two sizes, at least 8 tile rows)
// XCD j takes the slab of tile rows j 2^lys .. (j + 1) 2^lys - 1 over all x
// and z, item tl / 8 of it x fastest, then y, then z, so that the tiles an
// XCD runs together are neighbours whose halos meet in its own L2; else the
// tiles go x fastest, then y, then z. Either way a bijection of 0 .. T - 1.
template <bool POW2, int TZ = kTZ>
__device__ __forceinline__ void tile_origin(const ConvGeom &G, int tl, int &x0, int &y0, int &z0) {
    int bx, by, bz;
    if constexpr (POW2) {
        if (G.lys >= 0) {
            const int u = tl >> 3, r = u >> G.ltx;
            bx = u & (G.ntx - 1);
            by = ((tl & 7) << G.lys) | (r & ((1 << G.lys) - 1));
            bz = r >> G.lys;
        } else {
            bx = tl & (G.ntx - 1);
            by = (tl >> G.ltx) & (G.nty - 1);
            bz = tl >> G.ltxy;
        }
    } else {
        bx = tl % G.ntx;
        const int rest = tl / G.ntx;
        by = rest % G.nty;
        bz = rest / G.nty;
    }
    x0 = bx * kTX;
    y0 = by * kTY;
    z0 = bz * TZ;
}

// Point index of (x, y, z), each at most one period outside the grid.
template <bool POW2>
__device__ __forceinline__ int grid_point(const ConvGeom &G, int x, int y, int z) {
    if constexpr (POW2)
        return (x & (G.nx - 1)) | ((y & (G.ny - 1)) << G.lx) | ((z & (G.nz - 1)) << G.lxy);
    else
        return wrap(x, G.nx) + G.nx * (wrap(y, G.ny) + G.ny * wrap(z, G.nz));
}

// One 16-byte piece of a work item's halo: halo point hp (packed hx | hy << 8
// | hz << 16, or -1 for no piece) of the tile at (x0, y0, z0), channels
// cc + 8 part .. + 7.
template <bool POW2>
__device__ __forceinline__ uint4 halo_piece(const uint16_t *__restrict__ x, int cin,
                                            const ConvGeom &G, int x0, int y0, int z0, int cc,
                                            int hp, int part) {
    if (hp < 0) return uint4{0u, 0u, 0u, 0u};
    const int gp = grid_point<POW2>(G, x0 - 1 + (hp & 255), y0 - 1 + ((hp >> 8) & 255),
                                    z0 - 1 + (hp >> 16));
    return *(const uint4 *)(x + (uint32_t)gp * (uint32_t)cin + cc + 8 * part);
}

// The same piece of the nearest 2x upsampling of the coarse tensor xc (cc
// channels, half the grid's sizes): fine point (x, y, z) reads coarse point
// (x / 2, y / 2, z / 2) after the periodic wrap on the fine grid.
template <bool POW2>
__device__ __forceinline__ uint4 halo_piece_up(const uint16_t *__restrict__ xc, int cc,
                                               const ConvGeom &G, int x0, int y0, int z0, int c0,
                                               int hp, int part) {
    if (hp < 0) return uint4{0u, 0u, 0u, 0u};
    const int fx = x0 - 1 + (hp & 255), fy = y0 - 1 + ((hp >> 8) & 255), fz = z0 - 1 + (hp >> 16);
    int gp;
    if constexpr (POW2)
        gp = ((fx & (G.nx - 1)) >> 1) | (((fy & (G.ny - 1)) >> 1) << (G.lx - 1)) |
             (((fz & (G.nz - 1)) >> 1) << (G.lxy - 2));
    else
        gp = (wrap(fx, G.nx) >> 1) + (G.nx >> 1) * ((wrap(fy, G.ny) >> 1) + (G.ny >> 1) * (wrap(fz, G.nz) >> 1));
    return *(const uint4 *)(xc + (uint32_t)gp * (uint32_t)cc + c0 + 8 * part);
}

// The 14 K steps of one work item from LDS into the accumulators of the
// first NTA of the block's NT output tiles (NTA is the number the block
// actually has, so the loop carries no per-step test of it). baseA0..3: the
// lane's point bases of the four pair forms (second offset equal to the
// first, one x, one y, one z further), baseB its weight base; every read
// adds an immediate. Fragment buffers alternate between groups (F) and
// steps (W). With PIPE (blocks of one output tile) the loop is
// software-pipelined: the reads of step s + 1 are issued before the MFMAs of
// step s (the scheduling barriers keep that order), so each wavefront has
// the next step's reads in flight while its MFMAs run. Two output tiles
// would need the registers of a third wavefront per SIMD for it.
template <int NTA, int NT, bool PIPE>
__device__ __forceinline__ void conv_kloop(const uint4 *tile, const uint4 *wl, int baseA0, int baseA1,
                                           int baseA2, int baseA3, int baseB, int second,
                                           f4 (&acc)[4][NT]) {
    constexpr int NCO = 16 * NT;
    constexpr int PL = kHX * kHY;
    const uint4 z4 = uint4{0u, 0u, 0u, 0u};
    bf8 F[2][6], W[2][NTA];
    // fragment k of group g (0..3: three steps sharing halo rows, k the
    // row; 4, 5: steps 12 and 13, k the output row)
    auto loadF = [&](auto G, auto K) __attribute__((always_inline)) {
        constexpr int g = decltype(G)::value, k = decltype(K)::value;
        uint4 v;
        if constexpr (g < 3) {
            v = tile[baseA3 + 2 * (g + kHX * k)];
        } else if constexpr (g == 3) {
            v = tile[baseA1 + 2 * (kHX * k + 2 * PL)];
        } else if constexpr (g == 4) {
            v = tile[baseA2 + 2 * (2 + kHX * k + 2 * PL)];
        } else {
            v = tile[baseA0 + 2 * (2 + kHX * (k + 2) + 2 * PL)];
            if (second) v = z4;
        }
        F[g & 1][k] = __builtin_bit_cast(bf8, v);
    };
    // the reads step st needs that no earlier step made
    auto loads = [&](auto Sx) __attribute__((always_inline)) {
        constexpr int st = decltype(Sx)::value;
        constexpr int g = st < 12 ? st / 3 : st - 8, j = st < 12 ? st % 3 : 0;
        if constexpr (j == 0)
            unroll<0, 4>([&](auto K) { loadF(std::integral_constant<int, g>{}, K); });
        else
            loadF(std::integral_constant<int, g>{}, std::integral_constant<int, j + 3>{});
#pragma unroll
        for (int nt = 0; nt < NTA; ++nt) {
            uint4 v = wl[baseB + 2 * (2 * st * NCO + nt * 16)];
            if (st == 13 && second) v = z4;
            W[st & 1][nt] = __builtin_bit_cast(bf8, v);
        }
    };
    auto mfmas = [&](auto Sx) __attribute__((always_inline)) {
        constexpr int st = decltype(Sx)::value;
        constexpr int g = st < 12 ? st / 3 : st - 8, j = st < 12 ? st % 3 : 0;
#pragma unroll
        for (int nt = 0; nt < NTA; ++nt)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[st & 1][nt], F[g & 1][mt + j],
                                                                       acc[mt][nt], 0, 0, 0);
    };
    if constexpr (PIPE) {
        loads(std::integral_constant<int, 0>{});
        unroll<0, 14>([&](auto K) {
            constexpr int k = decltype(K)::value;
            if constexpr (k + 1 < 14) loads(std::integral_constant<int, k + 1>{});
            __builtin_amdgcn_sched_barrier(0);
            mfmas(K);
            __builtin_amdgcn_sched_barrier(0);
        });
    } else {
        unroll<0, 14>([&](auto K) {
            loads(K);
            mfmas(K);
        });
    }
}

// The same convolution for grids whose sizes are multiples of the 16 x 4 x 4
// point tile. Blocks are persistent: block b takes the tiles b, b + gridDim.x,
// ..., each over its 16-channel input chunks, and stages an item's 18 x 6 x 6
// halo (32 B per point, 20.7 KB) and the chunk's weights in LDS, so each
// input value is read from memory about 2.5 times instead of 27 times. While
// an item is computed from LDS, each thread's six 16-byte pieces of the next
// item's halo are already loading into registers. Wavefront w owns plane
// z0 + w of the tile: four rows of 16 points, the four M tiles; a block
// computes NT 16-channel N tiles (one for 16 output channels, run at four
// wavefronts per SIMD; two otherwise). The K steps use the 16x16x32 BF16
// MFMA; one step covers two taps (lanes l / 16 = 0, 1: its first, 2, 3: its
// second, in the pairing of slot_tap) x 16 channels (8 per lane). A and B
// place the same (tap, channel) in the same lane group and element, so the
// product does not depend on how the hardware orders K within a step. The
// 14th step's second tap does not exist and enters as zeros.
// Addressing costs no vector instruction in the K loop: every LDS read is a
// per-lane base (one per pair form) plus an immediate, and the flipped
// convolution differs only in the taps its weight slots hold. The weights
// are the MFMA's first operand and the points its second, so the result
// tile is output
// channel x point: lane (px, q) holds channels 4q .. 4q + 3 of point px, and
// the lanes of one store instruction write 16 points x 16 channels of one
// row (512 contiguous bytes when cout = 16) straight from the accumulators,
// converted to BF16 by the hardware (round to nearest even). The forward's
// two kinds of layer and the data gradients take row code with their
// options fixed; any other combination of options the general code.
// With CAT the input is the decoder's concat [up2(xc), x] read in place: the
// first cc / 16 chunks come from the coarse tensor xc (cc channels) at the
// parent point, the others from x (cin - cc channels), so the concatenated
// tensor is never written; the products and their order are those of the
// convolution of the concatenated tensor.
// With WPF (grids of fewer blocks than two per CU) the next chunk's weights
// load into registers with its halo; those blocks run at two or three
// wavefronts per SIMD, which costs nothing where there are at most two
// blocks per CU. Otherwise each chunk stages its weights when it starts.
template <int NT, bool WPF>
constexpr int conv_min_waves() { return WPF ? 2 : (NT == 1 ? 4 : 1); }

// With POOL the block also writes yp, the 2 x 2 x 2 average pooling of the
// BF16 outputs it stores (a tile holds whole cells): the eight rounded
// values of a cell are summed in FP32 in the order x, then y, then z, scaled
// by 1/8 and rounded, as the pooling pass over the stored tensor does. The
// x pair is in the neighbouring lane, the y pair in the lane's next row and
// the z pair in the next wavefront, which hands its values over in LDS.
// With one output tile (no registers to spare) or eight wavefronts every
// stored value goes through LDS instead, and each thread sums one cell's
// channel pair of each output tile.
// WV = 8 (large grids): blocks of eight wavefronts on 16 x 4 x 8 point
// tiles, each wavefront as above on one plane; the halo (18 x 6 x 10, 34.6
// KB) is re-read 2.1 times instead of 2.5, and a block's staging and
// barriers serve twice the points. With a few input chunks their weights
// all stay in LDS (G.wres), staged once per kernel.
template <int NT, bool FLIP, bool POW2, bool CAT, bool WPF, bool POOL, int WV = 4>
__global__ void __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(conv_min_waves<NT, WPF>(), 8)))
conv3d_tiled_kernel(
    const uint16_t *__restrict__ x, int cin, const uint16_t *__restrict__ xc, int cc,
    const uint16_t *__restrict__ w,
    const float *__restrict__ bias, int cout, ConvGeom G, int relu,
    const uint16_t *__restrict__ mask, uint16_t *__restrict__ yb, float *__restrict__ yf,
    uint16_t *__restrict__ yp) {
    static_assert(WV == 4 || (WV == 8 && (NT == 1 || !WPF)), "eight wavefronts");
    constexpr int NTH = 64 * WV, TZ = WV, HP = kHX * kHY * (TZ + 2);
    constexpr int NPF = (2 * HP + NTH - 1) / NTH;  // halo pieces per thread
    constexpr bool POOL1 = POOL && (NT == 1 || WV == 8);  // pooling through LDS
    constexpr int PXQ = POOL1 ? 16 * 4 * TZ * 2 * NT : 0;  // its uint4: 2 NCO B per point
    // LDS: the input halo (HP points x 16 channels), the pooling's values
    // and the chunk's weights (27 taps x 16 NT output channels x 16
    // channels), 32 B per row
    extern __shared__ uint4 lds[];
    uint4 *tile = lds, *wl = lds + HP * 2 + PXQ;
    uint2 *pxl = (uint2 *)(lds + HP * 2);  // point (x, y, z) at x + 16 (y + 4 z)
    constexpr int NCO = 16 * NT;  // weight rows per tap in LDS
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int half = q & 1, second = q >> 1;
    const int ntile = G.ntx * G.nty * G.ntz;
    const int nchunk = cin >> 4;
    const int cob = blockIdx.y * NCO;
    const int ntiles = NT == 1 ? 1 : min(NT, (cout - cob) >> 4);
    const int nco = ntiles * 16;
    // point bases (uint4 units) of the K steps' pair forms: halo point
    // (r, 0, wave), part half, and the second tap one x, y or z further
    const int c0 = 2 * (r + kHX * kHY * wave) + half;
    int baseA0 = c0;
    int baseA1 = c0 + 2 * second;
    int baseA2 = c0 + 2 * second * kHX;
    int baseA3 = c0 + 2 * second * kHX * kHY;
    int baseB = 2 * (second * NCO + r) + half;
    // this thread's halo pieces c = threadIdx.x + NTH k: point (packed) or -1
    int hp[NPF];
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
        const int c = threadIdx.x + NTH * k, h = c >> 1;
        hp[k] = c < HP * 2 ? (h % kHX) | (((h / kHX) % kHY) << 8) | ((h / (kHX * kHY)) << 16) : -1;
    }
    const int part = threadIdx.x & 1;
    const int nmine = ntile > (int)blockIdx.x ? (ntile - 1 - (int)blockIdx.x) / (int)gridDim.x + 1 : 0;
    uint4 pf[NPF];
    auto load_halo = [&](int k, int chunk) {
        int ox, oy, oz;
        tile_origin<POW2, TZ>(G, (int)blockIdx.x + k * (int)gridDim.x, ox, oy, oz);
        if constexpr (CAT) {
            if (chunk * 16 < cc) {
#pragma unroll
                for (int j = 0; j < NPF; ++j)
                    pf[j] = halo_piece_up<POW2>(xc, cc, G, ox, oy, oz, chunk * 16, hp[j], part);
            } else {
#pragma unroll
                for (int j = 0; j < NPF; ++j)
                    pf[j] = halo_piece<POW2>(x, cin - cc, G, ox, oy, oz, chunk * 16 - cc, hp[j], part);
            }
        } else {
#pragma unroll
            for (int j = 0; j < NPF; ++j) pf[j] = halo_piece<POW2>(x, cin, G, ox, oy, oz, chunk * 16, hp[j], part);
        }
    };
    // weight rows (slot sl, o) of input chunk cc: w[slot_tap(sl)][cob + o][cc .. cc + 15]
    const int ls = ntiles == 2 ? 5 : 4;
    auto stage_weights = [&](int cc, int off) {
        for (int c = threadIdx.x; c < 27 * nco * 2; c += NTH) {
            const int row = c >> 1, sl = row >> ls, o = row & (nco - 1);
            wl[off + 2 * (sl * NCO + o) + (c & 1)] =
                *(const uint4 *)(w + (slot_tap(sl, FLIP) * cout + cob + o) * cin + cc + 8 * (c & 1));
        }
    };
    // weights of every chunk resident (chunk c at c 27 NCO 2): staged once
    const bool wres = nchunk > 1 && G.wres;
    constexpr int WCH = 27 * NCO * 2;  // uint4 per chunk's weights
    constexpr int NPW = WPF ? (27 * NCO * 2 + NTH - 1) / NTH : 1;
    u4v pw[NPW];
    auto load_weights = [&](int cc) __attribute__((always_inline)) {
        unroll<0, NPW>([&](auto J) {
            constexpr int j = decltype(J)::value;
            // a thread past the last piece loads the last piece again (an
            // unconditional load keeps pw in registers); it is not stored
            const int c = min((int)threadIdx.x + NTH * j, 27 * nco * 2 - 1);
            const int row = c >> 1, sl = row >> ls, o = row & (nco - 1);
            pw[j] = *(const u4v *)(w + (slot_tap(sl, FLIP) * cout + cob + o) * cin + cc + 8 * (c & 1));
        });
    };
    auto store_weights = [&]() __attribute__((always_inline)) {
        unroll<0, NPW>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const int c = threadIdx.x + NTH * j;
            if (c < 27 * nco * 2) {
                const int row = c >> 1, sl = row >> ls, o = row & (nco - 1);
                *(u4v *)&wl[2 * (sl * NCO + o) + (c & 1)] = pw[j];
            }
        });
    };
    if (nmine > 0) {
        load_halo(0, 0);
        if (WPF && nchunk > 1) load_weights(0);
    }
    if (nchunk == 1 || wres)  // the same for every item
        for (int c = 0; c < nchunk; ++c) stage_weights(c * 16, c * WCH);
    // Loads in the epilogue would wait for the next item's halo, issued
    // before them (loads complete in order): the bias is loaded once, and
    // the data gradient's mask words before that halo (PREMASK; not in the
    // four-wavefront one-tile form, whose 128 VGPRs have no room for them).
    constexpr bool PREMASK = FLIP && (WV == 8 || NT > 1 || WPF);
    float bvv[NT][4];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int j = 0; j < 4; ++j) bvv[nt][j] = bias && nt < ntiles ? bias[cob + nt * 16 + 4 * q + j] : 0.f;
    // output element of row mt of the lane's plane in the tile at (x0, y0, z0)
    auto out_off = [&](int x0, int y0, int z0, int mt, int nt) -> uint32_t {
        uint32_t p;
        if constexpr (POW2)
            p = (uint32_t)((x0 + r) | ((y0 + mt) << G.lx) | ((z0 + wave) << G.lxy));
        else
            p = (uint32_t)((x0 + r) + G.nx * ((y0 + mt) + G.ny * (z0 + wave)));
        return p * (uint32_t)cout + (uint32_t)(cob + nt * 16 + 4 * q);
    };
    uint2 mrow[PREMASK ? NT : 1][4];
    auto load_mask = [&](int k) {
        int x0, y0, z0;
        tile_origin<POW2, TZ>(G, (int)blockIdx.x + k * (int)gridDim.x, x0, y0, z0);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            if (nt >= ntiles) break;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) mrow[nt][mt] = *(const uint2 *)(mask + out_off(x0, y0, z0, mt, nt));
        }
    };
    f4 acc[4][NT];
    for (int k = 0; k < nmine; ++k) {
        for (int chunk = 0; chunk < nchunk; ++chunk) {
            __syncthreads();  // the previous item's reads are done
#pragma unroll
            for (int j = 0; j < NPF; ++j)
                if (NTH * (j + 1) <= HP * 2 || threadIdx.x + NTH * j < HP * 2) tile[threadIdx.x + NTH * j] = pf[j];
            if (nchunk > 1 && !wres) {
                if constexpr (WPF) store_weights();
                else stage_weights(chunk * 16, 0);
            }
            __syncthreads();
            if constexpr (PREMASK)
                if (mask && chunk + 1 == nchunk) load_mask(k);
            if (chunk + 1 < nchunk) {
                load_halo(k, chunk + 1);
                if (WPF) load_weights((chunk + 1) * 16);
            } else if (k + 1 < nmine) {
                load_halo(k + 1, 0);
                if (WPF && nchunk > 1) load_weights(0);
            }
            if (chunk == 0) {
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
            }
            // with the weights' registers in use, the lane bases are made
            // opaque here, so the compiler addresses the K loop's LDS reads
            // as base + immediate instead of keeping one register per (base,
            // offset) pair across the item loop
            if constexpr (WPF)
                asm volatile("" : "+v"(baseA0), "+v"(baseA1), "+v"(baseA2), "+v"(baseA3), "+v"(baseB));
            const int bB = wres ? baseB + chunk * WCH : baseB;
            // wavefronts in their K loop go first: the others are staging or
            // storing, which waits on memory anyway (about 1% on the forward)
            __builtin_amdgcn_s_setprio(1);
            if (NT == 1 || ntiles == NT)
                conv_kloop<NT, NT, NT == 1>(tile, wl, baseA0, baseA1, baseA2, baseA3, bB, second, acc);
            else
                conv_kloop<1, NT, false>(tile, wl, baseA0, baseA1, baseA2, baseA3, bB, second, acc);
            __builtin_amdgcn_s_setprio(0);
        }
        // epilogue: lane (px, q) holds output channels 4q .. 4q + 3 of point
        // x0 + px of row mt of its plane, in register j of acc[mt][nt]
        int x0, y0, z0;
        tile_origin<POW2, TZ>(G, (int)blockIdx.x + k * (int)gridDim.x, x0, y0, z0);
        float rv[POOL && !POOL1 ? NT : 1][4][4];  // the stored BF16 values, for the pooling
        // the rows; MODE 1: bias, ReLU and BF16 output only (the forward's
        // hidden layers), 2: bias and FP32 output only (its last layer), 3
        // and 4: mask and BF16 or FP32 output only (the data gradients), with
        // no test of the other options per row; 0: any options
        auto rows = [&](auto MODE) __attribute__((always_inline)) {
            constexpr int MD = decltype(MODE)::value;
            constexpr bool F = MD != 0;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                if (nt >= ntiles) break;
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    const uint32_t o = out_off(x0, y0, z0, mt, nt);
                    float v[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        v[j] = acc[mt][nt][j];
                        if (F ? MD <= 2 : bias != nullptr) v[j] += bvv[nt][j];
                        if (F ? MD == 1 : relu != 0) v[j] = fmaxf(v[j], 0.f);
                    }
                    if (F ? MD >= 3 : mask != nullptr) {
                        uint2 m;
                        if constexpr (PREMASK) m = mrow[nt][mt];
                        else m = *(const uint2 *)(mask + o);
                        const uint32_t mw[2] = {m.x, m.y};
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (!(bf2f((uint16_t)(mw[j >> 1] >> (16 * (j & 1)))) > 0.f)) v[j] = 0.f;
                    }
                    if (F ? (MD == 1 || MD == 3) : yb != nullptr) {
                        const uint32_t lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(fl2{v[0], v[1]}, bf2));
                        const uint32_t hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(fl2{v[2], v[3]}, bf2));
                        *(uint2 *)(yb + o) = uint2{lo, hi};
                        if constexpr (POOL1) {
                            pxl[((wave * 4 + mt) * 16 + r) * (NCO / 4) + nt * 4 + q] = uint2{lo, hi};
                        } else if constexpr (POOL) {
                            rv[nt][mt][0] = __uint_as_float(lo << 16);
                            rv[nt][mt][1] = __uint_as_float(lo & 0xffff0000u);
                            rv[nt][mt][2] = __uint_as_float(hi << 16);
                            rv[nt][mt][3] = __uint_as_float(hi & 0xffff0000u);
                        }
                    }
                    if (F ? (MD == 2 || MD == 4) : yf != nullptr) *(f4 *)(yf + o) = f4{v[0], v[1], v[2], v[3]};
                }
            }
        };
        if (bias && relu && !mask && yb && !yf)
            rows(std::integral_constant<int, 1>{});
        else if (bias && !relu && !mask && !yb && yf)
            rows(std::integral_constant<int, 2>{});
        else if (PREMASK && !bias && !relu && mask && yb && !yf)
            rows(std::integral_constant<int, 3>{});
        else if (PREMASK && !bias && !relu && mask && !yb && yf)
            rows(std::integral_constant<int, 4>{});
        else
            rows(std::integral_constant<int, 0>{});
        if constexpr (POOL1) {
            // thread: cell (cx, cy, cz) of the tile's 8 x 2 x (TZ / 2), channels
            // 2 sub, 2 sub + 1 of each output tile; the eight values in the
            // pooling pass's order
            __syncthreads();
            const int cl = threadIdx.x >> 3;
            const int cx = cl & 7, cy = (cl >> 3) & 1, cz = cl >> 4;
            const uint32_t *pw32 = (const uint32_t *)pxl;
            const int X = (x0 >> 1) + cx, Y = (y0 >> 1) + cy, Z = (z0 >> 1) + cz;
            const uint32_t cell = (uint32_t)(X + (G.nx >> 1) * (Y + (G.ny >> 1) * Z)) * (uint32_t)cout + cob;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                if (nt >= ntiles) break;
                const int sub = (threadIdx.x & 7) + 8 * nt;
                float s0 = 0.f, s1 = 0.f;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int pt = (2 * cx + (k & 1)) + 16 * ((2 * cy + ((k >> 1) & 1)) + 4 * (2 * cz + (k >> 2)));
                    const uint32_t v2 = pw32[pt * (NCO / 2) + sub];
                    s0 += __uint_as_float(v2 << 16);
                    s1 += __uint_as_float(v2 & 0xffff0000u);
                }
                *(uint32_t *)(yp + cell + 2 * sub) =
                    (uint32_t)f2bf(0.125f * s0) | ((uint32_t)f2bf(0.125f * s1) << 16);
            }
        } else if constexpr (POOL) {
            // cell (x0 + r, y0 + 2 pr, z0 + w) .. + 1 of the even lanes r and
            // wavefronts w; value i = dx + 2 dy of plane dz = w & 1, channel j
            float *ex = (float *)tile;  // free once every wavefront is here
            const int pair = wave >> 1;
            __syncthreads();
            // slot of an even lane's cell: 2 pairs x NT x 2 row pairs x 32
            // lanes x 4 values x 4 channels (at most 16 KB, inside the halo)
            auto slot = [&](int nt, int pr) {
                return (f4 *)(ex + ((((pair * NT + nt) * 2 + pr) * 32) + (q * 8 + (r >> 1))) * 16);
            };
            const int cx = G.nx >> 1, cy = G.ny >> 1;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                if (nt >= ntiles) break;
#pragma unroll
                for (int pr = 0; pr < 2; ++pr) {
                    // the x neighbours (lane r + 1), shuffled with every lane active
                    float n0[4], n1[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        n0[j] = __shfl_xor(rv[nt][2 * pr][j], 1, 64);
                        n1[j] = __shfl_xor(rv[nt][2 * pr + 1][j], 1, 64);
                    }
                    if ((wave & 1) && !(r & 1)) {
                        f4 *e = slot(nt, pr);
                        e[0] = f4{rv[nt][2 * pr][0], rv[nt][2 * pr][1], rv[nt][2 * pr][2], rv[nt][2 * pr][3]};
                        e[1] = f4{n0[0], n0[1], n0[2], n0[3]};
                        e[2] = f4{rv[nt][2 * pr + 1][0], rv[nt][2 * pr + 1][1], rv[nt][2 * pr + 1][2],
                                  rv[nt][2 * pr + 1][3]};
                        e[3] = f4{n1[0], n1[1], n1[2], n1[3]};
                    }
                    // the lower plane keeps its running sums over the barrier
                    if (!(wave & 1)) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            float sum = 0.f;
                            sum += rv[nt][2 * pr][j];
                            sum += n0[j];
                            sum += rv[nt][2 * pr + 1][j];
                            sum += n1[j];
                            rv[nt][2 * pr][j] = sum;
                        }
                    }
                }
            }
            __syncthreads();
            if (!(wave & 1) && !(r & 1)) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    if (nt >= ntiles) break;
                    const int co = cob + nt * 16 + 4 * q;
#pragma unroll
                    for (int pr = 0; pr < 2; ++pr) {
                        const f4 *e = slot(nt, pr);
                        float sum[4] = {rv[nt][2 * pr][0], rv[nt][2 * pr][1], rv[nt][2 * pr][2], rv[nt][2 * pr][3]};
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const f4 bv4 = e[i];
#pragma unroll
                            for (int j = 0; j < 4; ++j) sum[j] += bv4[j];
                        }
                        uint32_t h[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) h[j] = f2bf(0.125f * sum[j]);
                        const int X = (x0 + r) >> 1, Y = (y0 >> 1) + pr, Z = (z0 + wave) >> 1;
                        const uint32_t qo = (uint32_t)(X + cx * (Y + cy * Z)) * (uint32_t)cout + co;
                        *(uint2 *)(yp + qo) = uint2{h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
                    }
                }
            }
        }
    }
}

// LDS bytes of conv3d_tiled_kernel with NT output tiles per block, wv
// wavefronts, the weights of nw input chunks resident and (pool1) the
// pooling through LDS.
size_t conv_tiled_lds(int nt, int wv = 4, int nw = 1, bool pool1 = false) {
    return (size_t)(kHX * kHY * (wv + 2) * 2 + (pool1 ? 16 * 4 * wv * 2 * nt : 0) + 27 * 16 * nt * 2 * nw) *
           sizeof(uint4);
}

// Weight gradient of one tap over one chunk of points:
// dW[t][o][i] = sum_p dY[p][o] X[p + d_t][i], an M = cout, N = cin, K = points
// product. Lane l feeds A[m = l % 16][k = 4 (l / 16) + j] = dY[p_j][o] and
// B[k][n = l % 16] = X[p_j + d_t][i] for its four points p_j. The four
// wavefronts of a block take interleaved 16-point steps of the chunk and are
// summed in LDS (fixed order) into the chunk's partial.
template <int MT>
__global__ void __launch_bounds__(256) wgrad_kernel(const uint16_t *__restrict__ x, int cin,
                                                    const uint16_t *__restrict__ dy, int cout,
                                                    int nx, int ny, int nz, long chunk,
                                                    float *__restrict__ part) {
    __shared__ float red[4][MT * 16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int t = blockIdx.x;
    const long c = blockIdx.y;
    const int cib = blockIdx.z * 64;
    const int ntiles = min(4, (cin - cib) >> 4);
    const int dx = t % 3 - 1, dyy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    const long P = (long)nx * ny * nz;
    const long p0 = c * chunk, p1 = min(P, p0 + chunk);
    f4 acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
    for (long kb = p0 + wave * 16; kb < p1; kb += 64) {
        long pj[4], nbj[4];
        bool vj[4];
        // the lane's 4 points are consecutive: coordinates of the first, then
        // one point at a time (a step wraps at most one row)
        const long pb = kb + 4 * q;
        int X, Y, Z;
        coords(pb < p1 ? pb : p0, nx, ny, X, Y, Z);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long p = pb + j;
            vj[j] = p < p1;
            pj[j] = vj[j] ? p : p0;
            if (j > 0 && ++X >= nx) {
                X = 0;
                if (++Y >= ny) {
                    Y = 0;
                    ++Z;
                }
            }
            nbj[j] = vj[j] ? (long)wrap(X + dx, nx) +
                                 (long)nx * ((long)wrap(Y + dyy, ny) + (long)ny * wrap(Z + dz, nz))
                           : 0;
        }
        s4 a[MT], b[4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                a[mt][j] = vj[j] ? (short)dy[pj[j] * cout + mt * 16 + r] : (short)0;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[nt][j] = (vj[j] && nt < ntiles) ? (short)x[nbj[j] * cin + cib + nt * 16 + r]
                                                  : (short)0;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            if (nt < ntiles) {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[mt][nt] =
                        __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) red[wave][mt * 16 + 4 * q + j][nt * 16 + r] = acc[mt][nt][j];
    __syncthreads();
    const int nrow = MT * 16, ncol = ntiles * 16;
    for (int e = threadIdx.x; e < nrow * 64; e += 256) {
        const int o = e / 64, i = e % 64;
        if (i >= ncol) continue;
        const float s = ((red[0][o][i] + red[1][o][i]) + red[2][o][i]) + red[3][o][i];
        part[((c * 27 + t) * (long)cout + o) * cin + cib + i] = s;
    }
}

// Halves e of two 32-bit words as one word: the low halves (e = 0) or the
// high halves (e = 1) of w0 and w1, w0's in the low half (one byte permute).
__device__ __forceinline__ uint32_t pair_half(uint32_t w0, uint32_t w1, int e) {
    return __builtin_amdgcn_perm(w1, w0, e ? 0x07060302u : 0x05040100u);
}

// Staged tiles of the tiled weight gradient: transposed input halo rows of
// kWgRow elements, kWgCh elements per channel, and output-gradient rows of
// kWgDy elements per channel.
constexpr int kWgRow = 24;
constexpr int kWgCh = kHZ * kHY * kWgRow + 8;
constexpr int kWgDy = 256 + 8;

// The eight K steps of one tile for wavefront wave with NR tap rows (dy, dz)
// wave, wave + 4 (, wave + 8): arow and xlane are the lane's element offsets
// in the staged output gradient and halo at step 0; step st takes the
// tile's points 32 st .. 32 st + 31 (plane st / 2, rows 2 (st % 2) .. + 1),
// a constant further on. Accumulator 3 rr + d takes the tap dx = d - 1 of
// row rr. BIAS (a wavefront with two rows) also multiplies dY by ones into
// accumulator 6, the bias gradient (each column holds the channel sums).
template <int MT, int NR, bool BIAS>
__device__ __forceinline__ void wgrad_steps(const uint16_t *__restrict__ dyt,
                                            const uint16_t *__restrict__ xht, int arow, int xlane,
                                            int wave, f4 (&acc)[9][MT]) {
    static_assert(!BIAS || NR == 2, "the bias takes a free accumulator");
    int xrow[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
        const int rid = wave + 4 * rr, dyo = rid % 3 - 1, dz = rid / 3 - 1;
        xrow[rr] = xlane + ((dz + 1) * kHY + dyo + 1) * kWgRow;
    }
    const bf8 ones = __builtin_bit_cast(bf8, uint4{0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u});
#pragma unroll 1
    for (int st = 0; st < 8; ++st) {
        const int soff = ((st >> 1) * kHY + 2 * (st & 1)) * kWgRow;
        bf8 a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            a[mt] = __builtin_bit_cast(bf8, *(const uint4 *)(dyt + arow + mt * 16 * kWgDy + 32 * st));
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
            // the three dx taps of a row start dx + 1 elements into the same
            // two aligned 16-byte words
            const uint16_t *row = xht + xrow[rr] + soff;
            const uint4 w0 = *(const uint4 *)row;
            const uint32_t w1x = *(const uint32_t *)(row + 8);
            const uint4 bw[3] = {
                w0,  // dx = -1
                uint4{__builtin_amdgcn_alignbyte(w0.y, w0.x, 2),  // dx = 0: one element
                      __builtin_amdgcn_alignbyte(w0.z, w0.y, 2),
                      __builtin_amdgcn_alignbyte(w0.w, w0.z, 2),
                      __builtin_amdgcn_alignbyte(w1x, w0.w, 2)},
                uint4{w0.y, w0.z, w0.w, w1x}};  // dx = +1: two elements
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const bf8 b = __builtin_bit_cast(bf8, bw[d]);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[3 * rr + d][mt] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, acc[3 * rr + d][mt], 0, 0, 0);
            }
        }
        if constexpr (BIAS) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[6][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], ones, acc[6][mt], 0, 0, 0);
        }
    }
}

// Weight gradient on the 16 x 4 x 4 point tiles of the forward kernel:
// dW[t][o][i] = sum_p dY[p][o] X[p + d_t][i] as M = o, N = i, K = points
// products on the 16x16x32 BF16 MFMA. A persistent block takes work items
// blockIdx.x, + gridDim.x, ... (tiles in the forward's XCD slabs where the
// grid allows) for the 16 input channels blockIdx.y; the global reads of its
// next tile are issued into registers before the current tile's MFMAs. Per
// tile it stages in LDS the output gradient transposed, dYt[o][point], and the
// input halo transposed, XhT[i][hz][hy][hx] (rows of 24, 16-byte aligned;
// the planes of consecutive channels, and the rows dYt[o] of consecutive
// output channels, start an odd multiple of 16 bytes apart modulo 256, so the
// 16-byte fragment reads of eight consecutive lanes fall in distinct banks).
// K steps take 32 points (two 16-point rows); a lane's 8 consecutive k are
// 8 consecutive x, so its A fragment (dY of one output channel) is one
// aligned 16-byte read, shared by all the wavefront's taps, and its B
// fragment (X of one input channel, shifted by the tap) starts dx + 1
// elements into an aligned pair of 16-byte words (a byte shift that is the
// same for the whole wavefront). Wavefront w owns the tap rows (dy, dz)
// w, w + 4, w + 8 (9 or 6 taps: the three dx of a row share those two
// words) and keeps their sums over all its tiles in registers; the block's
// partial dW goes to part[block][t][o][i] and the partials are summed in
// fixed order. One M tile keeps four wavefronts per SIMD (the LDS allows
// four blocks per CU).
template <int MT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MT == 1 ? 4 : 1, 8)))
wgrad_tiled_kernel(const uint16_t *__restrict__ x, int cin,
                   const uint16_t *__restrict__ dy, int cout,
                   int nx, int ny, int nz,
                   float *__restrict__ part,
                   float *__restrict__ bpart) {
    constexpr int kRow = kWgRow;                // hx row length in XhT
    constexpr int kCh = kWgCh;                  // XhT channel stride (1744 B)
    constexpr int kXh = 16 * kCh;               // XhT elements
    constexpr int kDy = kWgDy;                  // dYt row stride (528 B)
    static_assert(kHX % 2 == 0 && kHP % 2 == 0 && kRow % 2 == 0 && kCh % 2 == 0 && kDy % 2 == 0,
                  "halo rows and strides hold whole pairs of points");
    constexpr int kNTap = 9;                    // taps per wavefront: 3 rows x 3 dx at most
    __shared__ __attribute__((aligned(16))) uint16_t xht[kXh];
    __shared__ __attribute__((aligned(16))) uint16_t dyt[MT * 16 * kDy];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int cc = blockIdx.y * 16;
    const int ntx = nx / kTX, nty = ny / kTY;
    const int ntile = ntx * nty * (nz / kTZ);
    f4 acc[kNTap][MT];
#pragma unroll
    for (int u = 0; u < kNTap; ++u)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[u][mt] = f4{0.f, 0.f, 0.f, 0.f};
    // bias gradient (blocks of the first input chunk): wavefront 3, which has
    // two tap rows to wavefront 0's three, adds dY times ones on the MFMA
    const bool do_bias = bpart != nullptr && blockIdx.y == 0;
    // the lane's offsets in the staged dY and halo at the first K step
    const int arow = r * kDy + 8 * q, xlane = r * kCh + (q >> 1) * kRow + 8 * (q & 1);
    // the forward's XCD slabs of tile rows where the rows and the grid allow
    // (tile % 8 is then the block's XCD for every input chunk, so the chunks
    // of a tile and its neighbours read their halos through one L2)
    const int nys = nty % 8 == 0 && gridDim.x % 8 == 0 ? nty / 8 : 0;
    auto origin = [&](int tile, int &x0, int &y0, int &z0) {
        int bx, by, bz;
        if (nys) {
            const int u = tile >> 3, rest = u / ntx;
            bx = u - rest * ntx;
            by = (tile & 7) * nys + rest % nys;
            bz = rest / nys;
        } else {
            const int rest = tile / ntx;
            bx = tile - rest * ntx;
            by = rest % nty;
            bz = rest / nty;
        }
        x0 = bx * kTX;
        y0 = by * kTY;
        z0 = bz * kTZ;
    };
    // a tile's global reads, held in registers from before the previous
    // tile's MFMAs to its staging: input halo, a thread taking two
    // neighbouring halo points (hx even) and 8 channels per piece; output
    // gradient, two neighbouring points (pl even) and 8 channels per piece
    // (lanes l and l + 32 of a wavefront take the two channel halves of one
    // pair of points, so a half-wavefront's LDS stores of a channel fall on
    // consecutive words within each halo row: a few bank conflicts where
    // the rows wrap, where lanes l and l + 1 used to meet in every bank)
    constexpr int kXPairs = kHP / 2, kXSlots = 2 * ((kXPairs + 31) / 32) * 32;
    constexpr int kXIt = (kXSlots + 255) / 256, kDIt = MT;
    auto xpiece = [](int c, int &h, int &e0) {
        h = 2 * (((c >> 6) << 5) | (c & 31));
        e0 = 8 * ((c >> 5) & 1);
        return h < kHP;
    };
    auto dpiece = [](int c, int &pl, int &oc) {
        pl = 2 * ((c / (64 * MT)) * 32 + (c & 31));
        oc = (c >> 5) % (2 * MT);
    };
    uint4 xv[kXIt][2], dv[kDIt][2];
    auto fetch = [&](int tile) {
        int x0, y0, z0;
        origin(tile, x0, y0, z0);
#pragma unroll
        for (int it = 0; it < kXIt; ++it) {
            const int c = threadIdx.x + 256 * it;
            int h, e0;
            if (xpiece(c, h, e0)) {
                const int hx = h % kHX, hy = (h / kHX) % kHY, hz = h / (kHX * kHY);
                const int gy = wrap(y0 - 1 + hy, ny), gz = wrap(z0 - 1 + hz, nz);
                const int g0 = wrap(x0 - 1 + hx, nx) + nx * (gy + ny * gz);
                const int g1 = wrap(x0 + hx, nx) + nx * (gy + ny * gz);
                xv[it][0] = *(const uint4 *)(x + g0 * cin + cc + e0);
                xv[it][1] = *(const uint4 *)(x + g1 * cin + cc + e0);
            }
        }
#pragma unroll
        for (int it = 0; it < kDIt; ++it) {
            const int c = threadIdx.x + 256 * it;
            int pl, oc;
            dpiece(c, pl, oc);
            const int gp = (x0 + (pl & 15)) + nx * ((y0 + ((pl >> 4) & 3)) + ny * (z0 + (pl >> 6)));
            dv[it][0] = *(const uint4 *)(dy + gp * cout + 8 * oc);
            dv[it][1] = *(const uint4 *)(dy + (gp + 1) * cout + 8 * oc);
        }
    };
    if ((int)blockIdx.x < ntile) fetch(blockIdx.x);
    for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        __syncthreads();  // the previous tile's reads are done
        // both staged transposed, each channel's pair of points as one
        // 4-byte word
#pragma unroll
        for (int it = 0; it < kXIt; ++it) {
            const int c = threadIdx.x + 256 * it;
            int h, e0;
            if (xpiece(c, h, e0)) {
                const int hx = h % kHX, hy = (h / kHX) % kHY, hz = h / (kHX * kHY);
                const uint32_t w0[4] = {xv[it][0].x, xv[it][0].y, xv[it][0].z, xv[it][0].w};
                const uint32_t w1[4] = {xv[it][1].x, xv[it][1].y, xv[it][1].z, xv[it][1].w};
                uint32_t *dst = (uint32_t *)(xht + e0 * kCh + (hz * kHY + hy) * kRow + hx);
#pragma unroll
                for (int e = 0; e < 8; ++e) dst[e * (kCh / 2)] = pair_half(w0[e >> 1], w1[e >> 1], e & 1);
            }
        }
#pragma unroll
        for (int it = 0; it < kDIt; ++it) {
            const int c = threadIdx.x + 256 * it;
            int pl, oc;
            dpiece(c, pl, oc);
            const uint32_t w0[4] = {dv[it][0].x, dv[it][0].y, dv[it][0].z, dv[it][0].w};
            const uint32_t w1[4] = {dv[it][1].x, dv[it][1].y, dv[it][1].z, dv[it][1].w};
            uint32_t *dst = (uint32_t *)(dyt + (8 * oc) * kDy + pl);
#pragma unroll
            for (int e = 0; e < 8; ++e) dst[e * (kDy / 2)] = pair_half(w0[e >> 1], w1[e >> 1], e & 1);
        }
        __syncthreads();
        // the next tile's reads go out before this tile's MFMAs
        if (tile + (int)gridDim.x < ntile) fetch(tile + (int)gridDim.x);
        // wavefronts at their MFMAs go first (about 1% on the training step)
        __builtin_amdgcn_s_setprio(1);
        if (wave == 0) wgrad_steps<MT, 3, false>(dyt, xht, arow, xlane, 0, acc);
        else if (wave < 3 || !do_bias) wgrad_steps<MT, 2, false>(dyt, xht, arow, xlane, wave, acc);
        else wgrad_steps<MT, 2, true>(dyt, xht, arow, xlane, 3, acc);
        __builtin_amdgcn_s_setprio(0);
    }
    // D[m = 4 q + j][n = r] of tap t, M tile mt: dW[t][mt 16 + 4 q + j][cc + r];
    // accumulator u = 3 rr + d holds tap t = d + 3 (dy + 1) + 9 (dz + 1) of row
    // rid = wave + 4 rr = (dy + 1) + 3 (dz + 1)
#pragma unroll
    for (int u = 0; u < kNTap; ++u) {
        const int rid = wave + 4 * (u / 3);
        if (rid >= 9) continue;
        const int t = u % 3 + 3 * rid;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                part[(((long)blockIdx.x * 27 + t) * cout + mt * 16 + 4 * q + j) * cin + cc + r] = acc[u][mt][j];
    }
    if (do_bias && wave == 3 && r == 0) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) bpart[(long)blockIdx.x * cout + mt * 16 + 4 * q + j] = acc[6][mt][j];
    }
}

// dw[e] = sum over chunks of part[chunk][e] (fixed order).
// A block sums 32 consecutive elements; its 8 thread groups take the chunks
// g, g + 8, g + 16, ... in order and are combined in group order (fixed
// order, so the result does not depend on scheduling).
__device__ __forceinline__ void sum_chunks_block(const float *__restrict__ part, long nchunks,
                                                 long n, float *__restrict__ out, long blk) {
    __shared__ float red[8][32];
    const int el = threadIdx.x & 31, g = threadIdx.x >> 5;
    const long e = blk * 32 + el;
    float s = 0.f;
    if (e < n)
        for (long c = g; c < nchunks; c += 8) s += part[c * n + e];
    red[g][el] = s;
    __syncthreads();
    if (g == 0 && e < n) {
        float t = red[0][el];
#pragma unroll
        for (int k = 1; k < 8; ++k) t += red[k][el];
        out[e] = t;
    }
}

__global__ void __launch_bounds__(256) sum_chunks_kernel(const float *__restrict__ part,
                                                         long nchunks, long n,
                                                         float *__restrict__ out) {
    sum_chunks_block(part, nchunks, n, out, blockIdx.x);
}

// Two independent sums of the same kind in one launch: blocks [0, nblk_a)
// reduce (part_a, rows_a, n_a) into out_a, the rest (part_b, ...) into out_b.
__global__ void __launch_bounds__(256) sum_chunks2_kernel(const float *__restrict__ part_a,
                                                          long rows_a, long n_a,
                                                          float *__restrict__ out_a, long nblk_a,
                                                          const float *__restrict__ part_b,
                                                          long rows_b, long n_b,
                                                          float *__restrict__ out_b) {
    const long b = blockIdx.x;
    if (b < nblk_a) sum_chunks_block(part_a, rows_a, n_a, out_a, b);
    else sum_chunks_block(part_b, rows_b, n_b, out_b, b - nblk_a);
}

// Per-block partial sums of dy over points for each channel: thread
// (tid % cout) owns a channel, (tid / cout) a strided slice of the block's points.
// First pass of the same fixed-order sum for wide rows (n a multiple of 4):
// block (x, k) sums rows [k L, min((k + 1) L, nrows)) of elements
// [128 x, 128 x + 128), four per thread with 16-byte loads, in 8 interleaved
// groups combined in order, into row k of mid; sum_chunks_kernel then adds
// the rows of mid in order. More blocks and wider loads keep more bytes in
// flight than one pass over all rows.
constexpr int kSumSeg = 8;
// Blocks with blockIdx.x >= nblk_a take a second array (part_b, n4_b, mid_b)
// with the same rows and segments (the bias partials beside the weights').
__global__ void __launch_bounds__(256) sum_rows4_kernel(const float4 *__restrict__ part,
                                                        long nrows, long n4, int L,
                                                        float4 *__restrict__ mid, long nblk_a,
                                                        const float4 *__restrict__ part_b,
                                                        long n4_b, float4 *__restrict__ mid_b) {
    __shared__ float4 red[8][32];
    const int l = threadIdx.x & 31, g = threadIdx.x >> 5;
    long bx = blockIdx.x;
    if (bx >= nblk_a) {
        bx -= nblk_a;
        part = part_b;
        n4 = n4_b;
        mid = mid_b;
    }
    const long e = bx * 32 + l;
    const long r0 = (long)blockIdx.y * L, r1 = r0 + L < nrows ? r0 + L : nrows;
    float4 acc = float4{0.f, 0.f, 0.f, 0.f};
    if (e < n4) {
#pragma unroll 4
        for (long r = r0 + g; r < r1; r += 8) {
            const float4 v = part[r * n4 + e];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
    }
    red[g][l] = acc;
    __syncthreads();
    if (g == 0 && e < n4) {
        float4 t = red[0][l];
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            t.x += red[k][l].x;
            t.y += red[k][l].y;
            t.z += red[k][l].z;
            t.w += red[k][l].w;
        }
        mid[(long)blockIdx.y * n4 + e] = t;
    }
}

__global__ void __launch_bounds__(256) bias_partial_kernel(const uint16_t *__restrict__ dy, int cout,
                                                           long P, long chunk,
                                                           float *__restrict__ part) {
    __shared__ float red[256];
    const int ch = threadIdx.x % cout, lanes = 256 / cout, sl = threadIdx.x / cout;
    const long p0 = (long)blockIdx.x * chunk, p1 = min(P, p0 + chunk);
    float s = 0.f;
    if (sl < lanes)
        for (long p = p0 + sl; p < p1; p += lanes) s += bf2f(dy[p * cout + ch]);
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < cout) {
        float t = 0.f;
        for (int k = 0; k < lanes; ++k) t += red[k * cout + threadIdx.x];
        part[(long)blockIdx.x * cout + threadIdx.x] = t;
    }
}

__global__ void pack_weights_kernel(const float *__restrict__ w, int cin, int cout,
                                    uint16_t *__restrict__ wf, uint16_t *__restrict__ wd) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long n = 27L * cin * cout;
    if (e >= n) return;
    const int t = (int)(e / ((long)cin * cout));
    const int rem = (int)(e % ((long)cin * cout));
    const int o = rem / cin, i = rem % cin;
    const uint16_t v = f2bf(w[e]);
    if (wf) wf[e] = v;
    if (wd) wd[((long)t * cin + i) * cout + o] = v;
}

// ------------------------------------------------------------ grid layers
// Every layer's packing in one launch. Layer l's FP32 weights start at
// woff[l] of w; its packings at poff[l] of wf and wd (poff[l + 1] - poff[l] =
// 27 cin cout).
constexpr int kMaxPackLayers = 32;
struct PackTable {
    int n;
    long woff[kMaxPackLayers];
    long poff[kMaxPackLayers + 1];
    int cin[kMaxPackLayers], cout[kMaxPackLayers];
};

__global__ void pack_all_kernel(const float *__restrict__ w, PackTable tb,
                                uint16_t *__restrict__ wf, uint16_t *__restrict__ wd) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= tb.poff[tb.n]) return;
    int l = 0;
    while (l + 1 < tb.n && e >= tb.poff[l + 1]) ++l;
    const long el = e - tb.poff[l];
    const int cin = tb.cin[l], cout = tb.cout[l];
    const int t = (int)(el / ((long)cin * cout));
    const int rem = (int)(el % ((long)cin * cout));
    const int o = rem / cin, i = rem % cin;
    const uint16_t v = f2bf(w[tb.woff[l] + el]);
    wf[e] = v;
    wd[tb.poff[l] + ((long)t * cin + i) * cout + o] = v;
}

__global__ void pool2_kernel(const uint16_t *__restrict__ x, int c, int nx, int ny, int nz,
                             uint16_t *__restrict__ y) {
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const long n = (long)cx * cy * cz * c;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int ch = mod32(e, c);
    const long qq = div32(e, c);
    int X, Y, Z;
    coords(qq, cx, cy, X, Y, Z);
    float s = 0.f;
    for (int k = 0; k < 8; ++k) {
        const long p = (2 * X + (k & 1)) + (long)nx * ((2 * Y + ((k >> 1) & 1)) + (long)ny * (2 * Z + (k >> 2)));
        s += bf2f(x[p * c + ch]);
    }
    y[e] = f2bf(0.125f * s);
}

__global__ void pool2_bwd_kernel(const float *__restrict__ dy, int c, int nx, int ny, int nz,
                                 float *__restrict__ dx) {
    const long n = (long)nx * ny * nz * c;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int ch = mod32(e, c);
    const long p = div32(e, c);
    int X, Y, Z;
    coords(p, nx, ny, X, Y, Z);
    const long qq = (X / 2) + (long)(nx / 2) * ((Y / 2) + (long)(ny / 2) * (Z / 2));
    dx[e] += 0.125f * dy[qq * c + ch];
}

__global__ void upsample2_kernel(const uint16_t *__restrict__ x, int c, int nx, int ny, int nz,
                                 uint16_t *__restrict__ y, int ystride, int yoff) {
    const int fx = 2 * nx, fy = 2 * ny, fz = 2 * nz;
    const long n = (long)fx * fy * fz * c;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int ch = mod32(e, c);
    const long p = div32(e, c);
    int X, Y, Z;
    coords(p, fx, fy, X, Y, Z);
    const long qq = (X / 2) + (long)nx * ((Y / 2) + (long)ny * (Z / 2));
    y[p * ystride + yoff + ch] = x[qq * c + ch];
}

__global__ void upsample2_bwd_kernel(const float *__restrict__ dy, int dystride, int dyoff, int c,
                                     int nx, int ny, int nz, float *__restrict__ dx) {
    const long n = (long)nx * ny * nz * c;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int ch = mod32(e, c);
    const long qq = div32(e, c);
    int X, Y, Z;
    coords(qq, nx, ny, X, Y, Z);
    const int fx = 2 * nx, fy = 2 * ny;
    float s = 0.f;
    for (int k = 0; k < 8; ++k) {
        const long p = (2 * X + (k & 1)) + (long)fx * ((2 * Y + ((k >> 1) & 1)) + (long)fy * (2 * Z + (k >> 2)));
        s += dy[p * dystride + dyoff + ch];
    }
    dx[e] = s;
}

__global__ void copy_channels_kernel(const uint16_t *__restrict__ x, int c, long P,
                                     uint16_t *__restrict__ y, int ystride, int yoff) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * c) return;
    const long p = div32(e, c);
    y[p * ystride + yoff + mod32(e, c)] = x[e];
}

// 16-byte variants (8 BF16 channels per thread) of pooling, upsampling and
// the channel copy, for channel counts, strides and offsets that are
// multiples of 8 and 16-byte aligned arrays; element e = point * (c / 8) + g.
__device__ __forceinline__ void unpack8(const uint4 v, float (&f)[8]) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f[2 * k] = __uint_as_float(w[k] << 16);
        f[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
    }
}

__global__ void pool2_v8_kernel(const uint16_t *__restrict__ x, int c, int nx, int ny, int nz,
                                uint16_t *__restrict__ y) {
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2, c8 = c / 8;
    const long n = (long)cx * cy * cz * c8;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int g = mod32(e, c8);
    const long qq = div32(e, c8);
    int X, Y, Z;
    coords(qq, cx, cy, X, Y, Z);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < 8; ++k) {
        const long p = (2 * X + (k & 1)) + (long)nx * ((2 * Y + ((k >> 1) & 1)) + (long)ny * (2 * Z + (k >> 2)));
        float f[8];
        unpack8(*(const uint4 *)(x + p * c + 8 * g), f);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] += f[j];
    }
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w[k] = uint32_t(f2bf(0.125f * s[2 * k])) | (uint32_t(f2bf(0.125f * s[2 * k + 1])) << 16);
    *(uint4 *)(y + qq * c + 8 * g) = uint4{w[0], w[1], w[2], w[3]};
}

__global__ void upsample2_v8_kernel(const uint16_t *__restrict__ x, int c, int nx, int ny, int nz,
                                    uint16_t *__restrict__ y, int ystride, int yoff) {
    const int fx = 2 * nx, fy = 2 * ny, fz = 2 * nz, c8 = c / 8;
    const long n = (long)fx * fy * fz * c8;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int g = mod32(e, c8);
    const long p = div32(e, c8);
    int X, Y, Z;
    coords(p, fx, fy, X, Y, Z);
    const long qq = (X / 2) + (long)nx * ((Y / 2) + (long)ny * (Z / 2));
    *(uint4 *)(y + p * ystride + yoff + 8 * g) = *(const uint4 *)(x + qq * c + 8 * g);
}

// The decoder's concat in one pass, 16 bytes per thread: row p of y is the
// upsampled coarse row (channels 0 .. hc) followed by row p of the skip
// tensor (channels hc .. hc + fc); every row is written whole, once.
__global__ void concat_up2_v8_kernel(const uint16_t *__restrict__ xc, int hc,
                                     const uint16_t *__restrict__ xf, int fc, int nx, int ny,
                                     int nz, uint16_t *__restrict__ y) {
    const int g8 = (hc + fc) / 8, h8 = hc / 8;
    const long n = (long)nx * ny * nz * g8;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int g = mod32(e, g8);
    const long p = div32(e, g8);
    uint4 v;
    if (g < h8) {
        int X, Y, Z;
        coords(p, nx, ny, X, Y, Z);
        const long qq = (X / 2) + (long)(nx / 2) * ((Y / 2) + (long)(ny / 2) * (Z / 2));
        v = *(const uint4 *)(xc + qq * hc + 8 * g);
    } else {
        v = *(const uint4 *)(xf + p * fc + 8 * (g - h8));
    }
    *(uint4 *)(y + 8 * e) = v;
}

__global__ void copy_channels_v8_kernel(const uint16_t *__restrict__ x, int c, long P,
                                        uint16_t *__restrict__ y, int ystride, int yoff) {
    const int c8 = c / 8;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * c8) return;
    const long p = div32(e, c8);
    const int g = mod32(e, c8);
    *(uint4 *)(y + p * ystride + yoff + 8 * g) = *(const uint4 *)(x + p * c + 8 * g);
}

// Gradient at an encoder output that feeds both the pooling and the skip
// connection, masked by its ReLU: dx[p][ch] = act > 0 ? dy[parent(p)][ch] / 8
// + skip[p][soff + ch] : 0, in one pass (the same two additions as zero,
// pool2_bwd, add_channels and relu_mask in turn), into FP32 dx and/or BF16
// dxb (the rounding to_bf16 would apply).
__global__ void pool2_bwd_skip_kernel(const float *__restrict__ dy, int c, int nx, int ny, int nz,
                                      const float *__restrict__ skip, int sstride, int soff,
                                      const uint16_t *__restrict__ act, float *__restrict__ dx,
                                      uint16_t *__restrict__ dxb) {
    const long n = (long)nx * ny * nz * c;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int ch = mod32(e, c);
    const long p = div32(e, c);
    float v = 0.f;
    if (bf2f(act[e]) > 0.f) {
        int X, Y, Z;
        coords(p, nx, ny, X, Y, Z);
        const long qq = (X / 2) + (long)(nx / 2) * ((Y / 2) + (long)(ny / 2) * (Z / 2));
        v = 0.125f * dy[qq * c + ch] + skip[p * sstride + soff + ch];
    }
    if (dx) dx[e] = v;
    if (dxb) dxb[e] = f2bf(v);
}

// The same four channels per thread (c, sstride, soff multiples of 4, 16-byte
// aligned FP32 rows): 16-byte loads of dy and skip, 8-byte act loads and
// BF16 stores; the same arithmetic per element.
__global__ void pool2_bwd_skip4_kernel(const float4 *__restrict__ dy, int c, int nx, int ny, int nz,
                                       const float4 *__restrict__ skip, int sstride, int soff,
                                       const uint2 *__restrict__ act, float4 *__restrict__ dx,
                                       uint2 *__restrict__ dxb) {
    const int c4 = c / 4;
    const long n4 = (long)nx * ny * nz * c4;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n4) return;
    const int ch4 = mod32(e, c4);
    const long p = div32(e, c4);
    int X, Y, Z;
    coords(p, nx, ny, X, Y, Z);
    const long qq = (X / 2) + (long)(nx / 2) * ((Y / 2) + (long)(ny / 2) * (Z / 2));
    const float4 d = dy[qq * c4 + ch4];
    const float4 k = skip[(p * sstride + soff) / 4 + ch4];
    const uint2 a = act[e];
    const float dd[4] = {d.x, d.y, d.z, d.w}, kk[4] = {k.x, k.y, k.z, k.w};
    const uint16_t aa[4] = {uint16_t(a.x), uint16_t(a.x >> 16), uint16_t(a.y), uint16_t(a.y >> 16)};
    float v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = bf2f(aa[j]) > 0.f ? 0.125f * dd[j] + kk[j] : 0.f;
    if (dx) dx[e] = float4{v[0], v[1], v[2], v[3]};
    if (dxb)
        dxb[e] = uint2{uint32_t(f2bf(v[0])) | (uint32_t(f2bf(v[1])) << 16),
                       uint32_t(f2bf(v[2])) | (uint32_t(f2bf(v[3])) << 16)};
}

// Upsampling backward through the ReLU of the coarse activation, into BF16:
// dxb[q][ch] = bf16(act[q][ch] > 0 ? sum of the 8 children : 0) (the same sum
// as upsample2_bwd, then relu_mask and to_bf16).
__global__ void upsample2_bwd_mask_kernel(const float *__restrict__ dy, int dystride, int dyoff,
                                          int c, int nx, int ny, int nz,
                                          const uint16_t *__restrict__ act,
                                          uint16_t *__restrict__ dxb) {
    const long n = (long)nx * ny * nz * c;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float s = 0.f;
    if (bf2f(act[e]) > 0.f) {
        const int ch = mod32(e, c);
        const long qq = div32(e, c);
        int X, Y, Z;
        coords(qq, nx, ny, X, Y, Z);
        const int fx = 2 * nx, fy = 2 * ny;
        for (int k = 0; k < 8; ++k) {
            const long p = (2 * X + (k & 1)) +
                           (long)fx * ((2 * Y + ((k >> 1) & 1)) + (long)fy * (2 * Z + (k >> 2)));
            s += dy[p * dystride + dyoff + ch];
        }
    }
    dxb[e] = f2bf(s);
}

// The same four channels per thread (c, dystride, dyoff multiples of 4,
// 16-byte aligned FP32 rows); the children are added in the same order.
__global__ void upsample2_bwd_mask4_kernel(const float4 *__restrict__ dy, int dystride, int dyoff,
                                           int c, int nx, int ny, int nz,
                                           const uint2 *__restrict__ act,
                                           uint2 *__restrict__ dxb) {
    const int c4 = c / 4;
    const long n4 = (long)nx * ny * nz * c4;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n4) return;
    const uint2 a = act[e];
    const uint16_t aa[4] = {uint16_t(a.x), uint16_t(a.x >> 16), uint16_t(a.y), uint16_t(a.y >> 16)};
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    if (bf2f(aa[0]) > 0.f || bf2f(aa[1]) > 0.f || bf2f(aa[2]) > 0.f || bf2f(aa[3]) > 0.f) {
        const int ch4 = mod32(e, c4);
        const long qq = div32(e, c4);
        int X, Y, Z;
        coords(qq, nx, ny, X, Y, Z);
        const int fx = 2 * nx, fy = 2 * ny;
        for (int k = 0; k < 8; ++k) {
            const long p = (2 * X + (k & 1)) +
                           (long)fx * ((2 * Y + ((k >> 1) & 1)) + (long)fy * (2 * Z + (k >> 2)));
            const float4 v = dy[(p * dystride + dyoff) / 4 + ch4];
            s[0] += v.x;
            s[1] += v.y;
            s[2] += v.z;
            s[3] += v.w;
        }
    }
    float o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = bf2f(aa[j]) > 0.f ? s[j] : 0.f;
    dxb[e] = uint2{uint32_t(f2bf(o[0])) | (uint32_t(f2bf(o[1])) << 16),
                   uint32_t(f2bf(o[2])) | (uint32_t(f2bf(o[3])) << 16)};
}

__global__ void add_channels_kernel(const float *__restrict__ dy, int dystride, int dyoff, int c,
                                    long P, float *__restrict__ dx) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * c) return;
    const long p = div32(e, c);
    dx[e] += dy[p * dystride + dyoff + mod32(e, c)];
}

__global__ void to_bf16_kernel(const float *__restrict__ x, long n, uint16_t *__restrict__ y) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] = f2bf(x[e]);
}

__global__ void relu_mask_kernel(float *__restrict__ dx, const uint16_t *__restrict__ act, long n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n && !(bf2f(act[e]) > 0.f)) dx[e] = 0.f;
}

// ------------------------------------------------------------ loss, Adam
__global__ void __launch_bounds__(256) mse_kernel(const float *__restrict__ pred,
                                                  const float *__restrict__ tgt, int cu, int cs,
                                                  long P, const float *__restrict__ wch,
                                                  float *__restrict__ grad,
                                                  uint16_t *__restrict__ gradb,
                                                  double *__restrict__ part, int vec4) {
    __shared__ double red[4];
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (vec4 == 2) {
        // 16 stored channels: four lanes per point, lane j of a quad taking
        // channels 4j .. 4j + 3, so a wavefront's 16-byte accesses cover 16
        // consecutive points' rows; the block's 256 points in four passes
        // (the same arithmetic per channel as below)
        const float inv = 1.0f / (float)((double)P * cu);
        const int j = threadIdx.x & 3;
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const long pp = (long)blockIdx.x * blockDim.x + it * 64 + (threadIdx.x >> 2);
            if (pp < P) {
                float gg[4] = {0.f, 0.f, 0.f, 0.f};
                if (4 * j < cu) {
                    const float4 a = ((const float4 *)(pred + pp * 16))[j];
                    const float4 b = ((const float4 *)(tgt + pp * 16))[j];
                    const float pa[4] = {a.x, a.y, a.z, a.w}, tb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int ch = 4 * j + k;
                        if (ch < cu) {
                            const float d = pa[k] - tb[k];
                            l += (double)wch[ch] * d * d;
                            gg[k] = 2.f * wch[ch] * d * inv;
                        }
                    }
                }
                if (grad) ((float4 *)(grad + pp * 16))[j] = float4{gg[0], gg[1], gg[2], gg[3]};
                if (gradb)
                    ((uint2 *)(gradb + pp * 16))[j] =
                        uint2{uint32_t(f2bf(gg[0])) | (uint32_t(f2bf(gg[1])) << 16),
                              uint32_t(f2bf(gg[2])) | (uint32_t(f2bf(gg[3])) << 16)};
            }
        }
    } else if (p < P) {
        const float inv = 1.0f / (float)((double)P * cu);
        if (vec4) {
            // 16-byte accesses, four channels at a time (same arithmetic)
            const float4 *p4 = (const float4 *)(pred + p * cs), *t4 = (const float4 *)(tgt + p * cs);
            float4 *g4 = grad ? (float4 *)(grad + p * cs) : nullptr;
            uint2 *b4 = gradb ? (uint2 *)(gradb + p * cs) : nullptr;
            for (int c4 = 0; c4 < cs / 4; ++c4) {
                if (4 * c4 >= cu) {  // padding channels: no loss, zero gradient
                    if (g4) g4[c4] = float4{0.f, 0.f, 0.f, 0.f};
                    if (b4) b4[c4] = uint2{0u, 0u};
                    continue;
                }
                const float4 a = p4[c4], b = t4[c4];
                const float pa[4] = {a.x, a.y, a.z, a.w}, tb[4] = {b.x, b.y, b.z, b.w};
                float gg[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int ch = 4 * c4 + k;
                    gg[k] = 0.f;
                    if (ch < cu) {
                        const float d = pa[k] - tb[k];
                        l += (double)wch[ch] * d * d;
                        gg[k] = 2.f * wch[ch] * d * inv;
                    }
                }
                if (g4) g4[c4] = float4{gg[0], gg[1], gg[2], gg[3]};
                if (b4)
                    b4[c4] = uint2{uint32_t(f2bf(gg[0])) | (uint32_t(f2bf(gg[1])) << 16),
                                   uint32_t(f2bf(gg[2])) | (uint32_t(f2bf(gg[3])) << 16)};
            }
        } else {
            for (int ch = 0; ch < cs; ++ch) {
                float g = 0.f;
                if (ch < cu) {
                    const float d = pred[p * cs + ch] - tgt[p * cs + ch];
                    l += (double)wch[ch] * d * d;
                    g = 2.f * wch[ch] * d * inv;
                }
                if (grad) grad[p * cs + ch] = g;
                if (gradb) gradb[p * cs + ch] = f2bf(g);
            }
        }
    }
    l = wsum(l);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void __launch_bounds__(1024) final_sum_kernel(const double *__restrict__ part, long n,
                                                         double scale, double *__restrict__ out) {
    __shared__ double red[16];
    double s = 0.0;
    for (long k = threadIdx.x; k < n; k += 1024) s += part[k];
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += red[k];
        *out = t * scale;
    }
}

__global__ void adam_kernel(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, long n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    w[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

// ------------------------------------------------------ grid transfer
__global__ void coarsen_kernel(const float *__restrict__ phi, const float *__restrict__ u,
                               const float *__restrict__ p, int nx, int ny, int nz,
                               const float *__restrict__ scale, float *__restrict__ cf,
                               uint16_t *__restrict__ cb) {
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const long Pc = (long)cx * cy * cz;
    const long qq = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (qq >= Pc) return;
    const long N = (long)nx * ny * nz;
    int X, Y, Z;
    coords(qq, cx, cy, X, Y, Z);
    float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < 8; ++k) {
        const long f = (2 * X + (k & 1)) + (long)nx * ((2 * Y + ((k >> 1) & 1)) + (long)ny * (2 * Z + (k >> 2)));
        s[0] += phi[f];
        s[1] += u[f];
        s[2] += u[N + f];
        s[3] += u[2 * N + f];
        s[4] += p[f];
    }
    for (int ch = 0; ch < 16; ++ch) {
        const float v = ch < 5 ? 0.125f * s[ch] / scale[ch] : 0.f;
        if (cf) cf[qq * 16 + ch] = v;
        if (cb) cb[qq * 16 + ch] = f2bf(v);
    }
}

__global__ void prolong_add_kernel(const float *__restrict__ d, int cx, int cy, int cz,
                                   const float *__restrict__ scale, double *__restrict__ phi,
                                   double *__restrict__ u, double *__restrict__ p) {
    const int nx = 2 * cx, ny = 2 * cy, nz = 2 * cz;
    const long N = (long)nx * ny * nz;
    const long f = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= N) return;
    int X, Y, Z;
    coords(f, nx, ny, X, Y, Z);
    // fine node X sits at coarse coordinate (X + 1/2)/2 - 1/2
    auto lo = [](int X) { return (X - 1) >> 1; };  // floor((X - 1)/2)
    const int x0 = lo(X), y0 = lo(Y), z0 = lo(Z);
    const float wx = (X & 1) ? 0.25f : 0.75f, wy = (Y & 1) ? 0.25f : 0.75f, wz = (Z & 1) ? 0.25f : 0.75f;
    float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < 8; ++k) {
        const int ix = wrap(x0 + (k & 1), cx), iy = wrap(y0 + ((k >> 1) & 1), cy), iz = wrap(z0 + (k >> 2), cz);
        const float w = ((k & 1) ? wx : 1.f - wx) * (((k >> 1) & 1) ? wy : 1.f - wy) * ((k >> 2) ? wz : 1.f - wz);
        const long qq = ix + (long)cx * (iy + (long)cy * iz);
        for (int ch = 0; ch < 5; ++ch) acc[ch] += w * d[qq * 16 + ch];
    }
    phi[f] += (double)(scale[0] * acc[0]);
    u[f] += (double)(scale[1] * acc[1]);
    u[N + f] += (double)(scale[2] * acc[2]);
    u[2 * N + f] += (double)(scale[3] * acc[3]);
    p[f] += (double)(scale[4] * acc[4]);
}

constexpr int NCHK = 7;

__global__ void __launch_bounds__(256) checks_kernel(const float *__restrict__ s, int nx, int ny,
                                                     int nz, double *__restrict__ part) {
    __shared__ double red[NCHK][4];
    const long P = (long)nx * ny * nz;
    const long qq = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[NCHK] = {0.0, 1e300, -1e300, 0.0, 0.0, 0.0, 0.0};
    if (qq < P) {
        int X, Y, Z;
    coords(qq, nx, ny, X, Y, Z);
        auto at = [&](int x, int y, int z) {
            return (long)wrap(x, nx) + (long)nx * ((long)wrap(y, ny) + (long)ny * wrap(z, nz));
        };
        const double phi = s[qq * 16];
        const double div = 0.5 * ((double)s[at(X + 1, Y, Z) * 16 + 1] - s[at(X - 1, Y, Z) * 16 + 1] +
                                  (double)s[at(X, Y + 1, Z) * 16 + 2] - s[at(X, Y - 1, Z) * 16 + 2] +
                                  (double)s[at(X, Y, Z + 1) * 16 + 3] - s[at(X, Y, Z - 1) * 16 + 3]);
        const double ux = s[qq * 16 + 1], uy = s[qq * 16 + 2], uz = s[qq * 16 + 3];
        v[0] = phi;
        v[1] = phi;
        v[2] = phi;
        v[3] = div * div;
        v[4] = ux * ux + uy * uy + uz * uz;
        v[5] = 1.0;
        v[6] = fmax(phi * (1.0 - phi), 0.0);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < NCHK; ++k) {
        const double r = k == 1 ? wmin(v[k]) : (k == 2 ? wmax(v[k]) : wsum(v[k]));
        if (lane == 0) red[k][wv] = r;
    }
    __syncthreads();
    if (threadIdx.x < NCHK) {
        const int k = threadIdx.x;
        double r = red[k][0];
        for (int w = 1; w < 4; ++w) r = k == 1 ? fmin(r, red[k][w]) : (k == 2 ? fmax(r, red[k][w]) : r + red[k][w]);
        part[(long)blockIdx.x * NCHK + k] = r;
    }
}

__global__ void __launch_bounds__(1024) checks_final_kernel(const double *__restrict__ part, long nb,
                                                            double *__restrict__ out) {
    __shared__ double red[NCHK][16];
    double v[NCHK] = {0.0, 1e300, -1e300, 0.0, 0.0, 0.0, 0.0};
    for (long b = threadIdx.x; b < nb; b += 1024)
        for (int k = 0; k < NCHK; ++k) {
            const double x = part[b * NCHK + k];
            v[k] = k == 1 ? fmin(v[k], x) : (k == 2 ? fmax(v[k], x) : v[k] + x);
        }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < NCHK; ++k) {
        const double r = k == 1 ? wmin(v[k]) : (k == 2 ? wmax(v[k]) : wsum(v[k]));
        if (lane == 0) red[k][wv] = r;
    }
    __syncthreads();
    if (threadIdx.x < NCHK) {
        const int k = threadIdx.x;
        double r = red[k][0];
        for (int w = 1; w < 16; ++w) r = k == 1 ? fmin(r, red[k][w]) : (k == 2 ? fmax(r, red[k][w]) : r + red[k][w]);
        out[k] = r;
    }
}

// s[p][c] += rscale[c] * out[p][c] for the used channels c < cu.
// s[p][c] += rscale[c] out[p][c] for c < cu; with width > 0 channel 0 (phi)
// moves in level-set coordinates: phi <- phi + Phi(Psi(phi) + r o) - Phi(Psi(phi)).
__global__ void apply_residual_kernel(float *__restrict__ s, const float *__restrict__ out,
                                      const float *__restrict__ rscale, int cu, long P,
                                      float width) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * cu) return;
    const long p = div32(e, cu);
    const int c = mod32(e, cu);
    const float d = rscale[c] * out[p * 16 + c];
    if (c == 0 && width > 0.f) {
        const float f = s[p * 16];
        const float so = ls_psi_f(f, width);
        s[p * 16] = f + (ls_phi_f(so + d, width) - ls_phi_f(so, width));
    } else {
        s[p * 16 + c] += d;
    }
}

// t[p][c] = (s1[p][c] - s0[p][c]) / rscale[c] for c < cu, 0 otherwise.
// t = (s1 - s0)/rscale on the first cu channels (channel 0 as the change of
// Psi(phi) when width > 0), 0 beyond.
__global__ void residual_target_kernel(const float *__restrict__ s0, const float *__restrict__ s1,
                                       const float *__restrict__ rscale, int cu, long P,
                                       float width, float *__restrict__ t) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * 16) return;
    const int c = (int)(e & 15);
    float d = 0.f;
    if (c < cu)
        d = (c == 0 && width > 0.f) ? ls_psi_f(s1[e], width) - ls_psi_f(s0[e], width) : s1[e] - s0[e];
    t[e] = c < cu ? d / rscale[c] : 0.f;
}

// s[p][0] += c w(phi), c = (target - sum phi)/sum w from a checks result.
__global__ void fix_mass_kernel(float *__restrict__ s, long P, const double *__restrict__ chk,
                                const double *__restrict__ target) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double sw = chk[6];
    const double c = sw > 0.0 ? (*target - chk[0]) / sw : 0.0;
    const float phi = s[p * 16];
    s[p * 16] = phi + (float)(c * fmax((double)phi * (1.0 - (double)phi), 0.0));
}

// Input features of the network, written into channels 5..11 of the coarse
// state from channels 0..4 of the node and its six neighbours (periodic):
// central differences of phi (5, 6, 7), u . grad phi (8), div u (9),
// phi (1 - phi) (10), |grad phi| (11). Channels 12..15 are left as they are.
__global__ void features_kernel(float *__restrict__ s, int nx, int ny, int nz) {
    const long P = (long)nx * ny * nz;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    int x, y, z;
    coords(q, nx, ny, x, y, z);
    auto at = [&](int X, int Y, int Z) {
        return (wrap(X, nx) + (long)nx * (wrap(Y, ny) + (long)ny * wrap(Z, nz))) * 16;
    };
    const long xp = at(x + 1, y, z), xm = at(x - 1, y, z), yp = at(x, y + 1, z), ym = at(x, y - 1, z),
               zp = at(x, y, z + 1), zm = at(x, y, z - 1);
    const float gx = 0.5f * (s[xp] - s[xm]), gy = 0.5f * (s[yp] - s[ym]), gz = 0.5f * (s[zp] - s[zm]);
    const float div = 0.5f * (s[xp + 1] - s[xm + 1] + s[yp + 2] - s[ym + 2] + s[zp + 3] - s[zm + 3]);
    float *o = s + q * 16;
    const float phi = o[0];
    o[5] = gx;
    o[6] = gy;
    o[7] = gz;
    o[8] = o[1] * gx + o[2] * gy + o[3] * gz;
    o[9] = div;
    o[10] = phi * (1.f - phi);
    o[11] = sqrtf(gx * gx + gy * gy + gz * gz);
}

// Fine update from two coarse states s0 -> s1: u and p get the trilinear
// prolongation of the change; phi moves its level set: the coarse change of
// psi is prolonged and phi <- phi + Phi(Psi(phi) + dpsi) - Phi(Psi(phi))
// (no change where dpsi = 0).
__global__ void prolong_update_kernel(const float *__restrict__ s0, const float *__restrict__ s1,
                                      int cx, int cy, int cz, const float *__restrict__ scale,
                                      float width, double *__restrict__ phi,
                                      double *__restrict__ u, double *__restrict__ p) {
    const int nx = 2 * cx, ny = 2 * cy, nz = 2 * cz;
    const long N = (long)nx * ny * nz;
    const long f = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= N) return;
    int X, Y, Z;
    coords(f, nx, ny, X, Y, Z);
    auto lo = [](int X) { return (X - 1) >> 1; };
    const int x0 = lo(X), y0 = lo(Y), z0 = lo(Z);
    const float wx = (X & 1) ? 0.25f : 0.75f, wy = (Y & 1) ? 0.25f : 0.75f, wz = (Z & 1) ? 0.25f : 0.75f;
    float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < 8; ++k) {
        const int ix = wrap(x0 + (k & 1), cx), iy = wrap(y0 + ((k >> 1) & 1), cy), iz = wrap(z0 + (k >> 2), cz);
        const float w = ((k & 1) ? wx : 1.f - wx) * (((k >> 1) & 1) ? wy : 1.f - wy) * ((k >> 2) ? wz : 1.f - wz);
        const long qq = (ix + (long)cx * (iy + (long)cy * iz)) * 16;
        acc[0] += w * (ls_psi_f(scale[0] * s1[qq], width) - ls_psi_f(scale[0] * s0[qq], width));
        for (int ch = 1; ch < 5; ++ch) acc[ch] += w * (s1[qq + ch] - s0[qq + ch]);
    }
    const double f0 = phi[f];
    const double so = ls_psi(f0, width);
    phi[f] = f0 + (ls_phi(so + (double)acc[0], width) - ls_phi(so, width));
    u[f] += (double)(scale[1] * acc[1]);
    u[N + f] += (double)(scale[2] * acc[2]);
    u[2 * N + f] += (double)(scale[3] * acc[3]);
    p[f] += (double)(scale[4] * acc[4]);
}

// Per-block FP64 sums {sum phi, sum max(phi (1 - phi), 0)} of a fine field.
__global__ void __launch_bounds__(256) field_sums_kernel(const double *__restrict__ phi, long N,
                                                         double *__restrict__ part) {
    __shared__ double red[2][4];
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (i < N) {
        a = phi[i];
        b = fmax(a * (1.0 - a), 0.0);
    }
    a = wsum(a);
    b = wsum(b);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = a;
        red[1][wv] = b;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int k = threadIdx.x;
        part[(long)blockIdx.x * 2 + k] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
    }
}

__global__ void __launch_bounds__(1024) sums2_final_kernel(const double *__restrict__ part, long nb,
                                                           double *__restrict__ out) {
    __shared__ double red[2][16];
    double a = 0.0, b = 0.0;
    for (long k = threadIdx.x; k < nb; k += 1024) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    a = wsum(a);
    b = wsum(b);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = a;
        red[1][wv] = b;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double r = 0.0;
        for (int w = 0; w < 16; ++w) r += red[threadIdx.x][w];
        out[threadIdx.x] = r;
    }
}

// phi += c max(phi (1 - phi), 0), c = (*target - sums[0]) / sums[1].
__global__ void fix_mass_field_kernel(double *__restrict__ phi, long N, const double *__restrict__ sums,
                                      const double *__restrict__ target) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double c = sums[1] > 0.0 ? (*target - sums[0]) / sums[1] : 0.0;
    const double f = phi[i];
    phi[i] = f + c * fmax(f * (1.0 - f), 0.0);
}

// ------------------------------------------------------------ host helpers
int launched() { return hipGetLastError() == hipSuccess ? SUR_OK : SUR_EDEVICE; }

dim3 grid1(long n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

bool dims_ok(int nx, int ny, int nz) {
    return nx > 0 && ny > 0 && nz > 0 && (long)nx * ny * nz < 2147483647L;
}

// element counts of channel arrays stay below 2^31 (32-bit index math)
bool elems_ok(long points, long channels) {
    return points > 0 && channels > 0 && points * channels < 2147483647L;
}

constexpr long kWgradChunk = 8192;

long wgrad_chunks(long P) { return (P + kWgradChunk - 1) / kWgradChunk; }

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

bool pow2_ok(int n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// Persistent blocks of the tiled convolution (over all output-channel
// blocks): eight per CU for one output tile and one input chunk (two rounds
// of four resident blocks, so a block's next item overlaps another's
// epilogue), otherwise as many as are resident at once (four per CU with
// one output tile, register bound; three with two, LDS bound), which keeps
// the last round of a grid from running a third full.
// Blocks of eight wavefronts: as many as are resident at once (register
// bound: two per CU with one output tile, one with two); a second round of
// one-tile blocks measured slower at every chunk count.
// SUR_CONV_BLOCKS overrides it (tuning only; results do not depend on it).
int conv_blocks(int nt, int nchunk, int cus, int wv) {
    const char *v = std::getenv("SUR_CONV_BLOCKS");
    if (v && *v) return std::max(1, std::atoi(v));
    if (cus <= 0) return 2048;
    if (wv == 8) return (nt == 1 ? 2 : 1) * cus;
    return (nt == 1 ? (nchunk == 1 ? 8 : 4) : 3) * cus;
}

// The tiled weight gradient: lattice sizes multiples of the 16 x 4 x 4 tile,
// 32-bit element indices, aligned operands, at most 64 output channels.
bool wgrad_tiled_ok(const void *x, int cin, const void *dy, int cout, int nx, int ny, int nz) {
    const long P = (long)nx * ny * nz;
    return nx % kTX == 0 && ny % kTY == 0 && nz % kTZ == 0 && cout <= 64 && elems_ok(P, cin) &&
           elems_ok(P, cout) && ((uintptr_t)x & 15) == 0 && ((uintptr_t)dy & 15) == 0;
}

// Persistent blocks of the tiled weight gradient per 16-channel input chunk:
// about 768 blocks in all for one chunk and 512 for several (the chunk
// blocks of a tile fetch the same halo lines; with fewer tiles in flight
// per XCD those lines stay in its L2 across the blocks' drift), at most one
// per tile, a multiple of 8 where there are 8 or more (one run per XCD).
long wgrad_tiled_blocks(int cin, long P) {
    const long tiles = P / (kTX * kTY * kTZ);
    const long nb = std::max(1L, std::min(tiles, (cin > 16 ? 512L : 768L) / (cin / 16)));
    return nb >= 8 ? nb / 8 * 8 : nb;
}


}  // namespace

// Partial sums of sur_checks_noalloc: one per 256-point block and check, for
// up to SUR_CHECKS_NOALLOC_MAX_POINTS points (917,504 bytes). Every GPU the
// library runs on holds its own copy until the process ends. In host code the
// array's name is no device address: the kernels are given the address that
// hipGetSymbolAddress returns on each device (checks_scratch_here).
constexpr long kChecksScratchDoubles = NCHK * (SUR_CHECKS_NOALLOC_MAX_POINTS / 256);
static __device__ __align__(256) double checks_scratch[kChecksScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex checks_scratch_mu;
double *checks_scratch_dev[kMaxDevices];

// Device address of checks_scratch on the current device, looked up once per
// device (with that device current) and kept; NULL if the lookup fails.
double *checks_scratch_here() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(checks_scratch_mu);
    if (!checks_scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(checks_scratch)) != hipSuccess || !p) return nullptr;
        checks_scratch_dev[dev] = (double *)p;
    }
    return checks_scratch_dev[dev];
}

// The tiled convolution applies: sizes multiples of its tile, 32-bit element
// indices, 16-byte aligned x and w (its 16-byte loads).
bool conv_tiled_ok(const void *x, int cin, const void *w, int cout, int nx, int ny, int nz) {
    const long P = (long)nx * ny * nz;
    return nx % kTX == 0 && ny % kTY == 0 && nz % kTZ == 0 && elems_ok(P, cin) && elems_ok(P, cout) &&
           ((uintptr_t)x & 15) == 0 && ((uintptr_t)w & 15) == 0;
}

// Compute units of the current device (0 if the runtime cannot say).
int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return cus;
}

// Wavefronts per block of conv3d_tiled_kernel: eight on 16 x 4 x 8 tiles
// for one output tile and at least four such tiles per CU; for two output
// tiles (one block per CU) where the tiles make whole rounds of the CUs
// and at most eight input chunks (up to four keep their weights in LDS);
// else four (SUR_CONV_WV=4 keeps four; for comparisons only, both give the
// same bits).
int conv_waves(int cin, int cout, int nx, int ny, int nz, int cus) {
    const char *v = std::getenv("SUR_CONV_WV");
    const long P = (long)nx * ny * nz, tiles = P / (kTX * kTY * 8);
    if ((v && *v == '4') || nz % 8 || cus <= 0) return 4;
    if (cout <= 16) return tiles >= 4L * cus ? 8 : 4;
    return cin <= 128 && tiles >= cus && tiles % cus == 0 ? 8 : 4;
}

// Launches conv3d_tiled_kernel; xc != NULL selects the concat form (cc
// channels of the upsampled coarse tensor first, then cin - cc of x);
// y_pool != NULL the pooled output as well (forward form, BF16 output; with
// one output tile only on eight wavefronts or in the small-grid form).
void conv_tiled_launch(const void *x, int cin, const void *xc, int cc, const void *w,
                       const float *bias, int cout, int nx, int ny, int nz, bool flip, int relu,
                       const void *mask, void *y_bf16, float *y_f32, void *y_pool, hipStream_t st) {
    const long P = (long)nx * ny * nz;
    // one N tile per block for 16 output channels (fewer registers), two otherwise
    int nt = cout <= 16 ? 1 : kNT;
    long ncb = (cout + 16 * nt - 1) / (16 * nt);
    const int cus = device_cus();
    const int nwv = conv_waves(cin, cout, nx, ny, nz, cus);
    const long tiles = P / (kTX * kTY * nwv);
    long nblk = std::max(1L, std::min(tiles, (long)conv_blocks(nt, cin / 16, cus, nwv) / ncb));
    // grids of fewer two-tile blocks than two per CU (the 32^3 and 16^3
    // levels, a block's one item sets the time): one output tile per block
    // instead, with the next chunk's weights prefetched, so each block's
    // chain of chunks runs half the MFMAs; as many blocks per output tile
    // as the two-tile form (SUR_CONV_SPLITN=0 keeps two tiles; for
    // comparisons only, both give the same bits)
    const char *sn = std::getenv("SUR_CONV_SPLITN");
    const bool splitn = nt == kNT && nwv == 4 && cin > 16 && cus > 0 && nblk * ncb < 2L * cus &&
                        !(sn && *sn == '0');
    if (splitn) {
        nt = 1;
        ncb = cout / 16;
        nblk = std::max(1L, std::min(tiles, (long)conv_blocks(kNT, cin / 16, cus, nwv) / ncb));
    }
    const dim3 grid((unsigned)nblk, (unsigned)ncb);
    // eight-wavefront blocks with a few input chunks keep every chunk's
    // weights in LDS (at most 80 KB a block keeps two blocks per CU), so no
    // item stages them again (SUR_CONV_WRES=0 turns it off; for comparisons
    // only, both give the same bits)
    const char *wrv = std::getenv("SUR_CONV_WRES");
    const int nchunk = cin / 16;
    const bool pool1 = y_pool && (nt == 1 || nwv == 8);
    const bool wres = nwv == 8 && nchunk > 1 && conv_tiled_lds(nt, nwv, nchunk, pool1) <= (nt == 1 ? 80 : 160) * 1024 &&
                      !(wrv && *wrv == '0');
    const size_t lds = conv_tiled_lds(nt, nwv, wres ? nchunk : 1, pool1);
    ConvGeom G{nx, ny, nz, nx / kTX, ny / kTY, nz / nwv, 0, 0, 0, 0, wres ? 1 : 0, -1};
    const bool pow2 = pow2_ok(nx) && pow2_ok(ny) && pow2_ok(nz);
    if (pow2) {
        G.lx = ilog2(nx);
        G.lxy = ilog2(nx) + ilog2(ny);
        G.ltx = ilog2(G.ntx);
        G.ltxy = ilog2(G.ntx) + ilog2(G.nty);
        // XCD slabs of tile rows (SUR_CONV_XCD=0 keeps the x-fastest order;
        // for comparisons only, both give the same bits)
        const char *xv = std::getenv("SUR_CONV_XCD");
        if (G.nty >= 8 && nblk % 8 == 0 && !(xv && *xv == '0')) G.lys = ilog2(G.nty / 8);
    }
    const uint16_t *xb = (const uint16_t *)x, *xcb = (const uint16_t *)xc;
    const uint16_t *wb = (const uint16_t *)w, *mb = (const uint16_t *)mask;
    uint16_t *yb = (uint16_t *)y_bf16, *yp = (uint16_t *)y_pool;
    // weights prefetched with the halo: two output tiles, several input
    // chunks, fewer blocks than two per CU (SUR_CONV_WPF=0 turns it off; for
    // comparisons only, both give the same bits)
    const char *wv = std::getenv("SUR_CONV_WPF");
    const bool wpf = nt == kNT && cin > 16 && cus > 0 && nblk * ncb < 2L * cus && !(wv && *wv == '0');
#define SUR_CONV_LAUNCH(NTV, FL, P2, CT, WP, PL)                                                     \
    hipLaunchKernelGGL((conv3d_tiled_kernel<NTV, FL, P2, CT, WP, PL>), grid, dim3(256), lds, st, xb, \
                       cin, xcb, cc, wb, bias, cout, G, relu, mb, yb, y_f32, yp)
#define SUR_CONV_POW2(NTV, FL, CT, WP, PL)                               \
    do {                                                                 \
        if (pow2) SUR_CONV_LAUNCH(NTV, FL, true, CT, WP, PL);            \
        else SUR_CONV_LAUNCH(NTV, FL, false, CT, WP, PL);                \
    } while (0)
#define SUR_CONV_NT2(FL, CT, PL)                                         \
    do {                                                                 \
        if (wpf) SUR_CONV_POW2(kNT, FL, CT, true, PL);                   \
        else SUR_CONV_POW2(kNT, FL, CT, false, PL);                      \
    } while (0)
#define SUR_CONV_WV8(FL, P2, CT, PL)                                                           \
    hipLaunchKernelGGL((conv3d_tiled_kernel<1, FL, P2, CT, false, PL, 8>), grid, dim3(512), lds, st, \
                       xb, cin, xcb, cc, wb, bias, cout, G, relu, mb, yb, y_f32, yp)
#define SUR_CONV_WV8N2(FL, P2, CT, PL)                                                         \
    hipLaunchKernelGGL((conv3d_tiled_kernel<kNT, FL, P2, CT, false, PL, 8>), grid, dim3(512), lds, st, \
                       xb, cin, xcb, cc, wb, bias, cout, G, relu, mb, yb, y_f32, yp)
    if (nwv == 8 && nt == kNT) {
        if (pool1) {
            if (pow2) SUR_CONV_WV8N2(false, true, false, true); else SUR_CONV_WV8N2(false, false, false, true);
        } else if (xc) {
            if (pow2) SUR_CONV_WV8N2(false, true, true, false); else SUR_CONV_WV8N2(false, false, true, false);
        } else if (flip) {
            if (pow2) SUR_CONV_WV8N2(true, true, false, false); else SUR_CONV_WV8N2(true, false, false, false);
        } else {
            if (pow2) SUR_CONV_WV8N2(false, true, false, false); else SUR_CONV_WV8N2(false, false, false, false);
        }
    } else if (nwv == 8) {
        if (pool1) {
            if (pow2) SUR_CONV_WV8(false, true, false, true); else SUR_CONV_WV8(false, false, false, true);
        } else if (xc) {
            if (pow2) SUR_CONV_WV8(false, true, true, false); else SUR_CONV_WV8(false, false, true, false);
        } else if (flip) {
            if (pow2) SUR_CONV_WV8(true, true, false, false); else SUR_CONV_WV8(true, false, false, false);
        } else {
            if (pow2) SUR_CONV_WV8(false, true, false, false); else SUR_CONV_WV8(false, false, false, false);
        }
    } else if (splitn) {
        if (pool1) SUR_CONV_POW2(1, false, false, true, true);
        else if (xc) SUR_CONV_POW2(1, false, true, true, false);
        else if (flip) SUR_CONV_POW2(1, true, false, true, false);
        else SUR_CONV_POW2(1, false, false, true, false);
    } else if (xc) {
        if (nt == 1) SUR_CONV_POW2(1, false, true, false, false);
        else SUR_CONV_NT2(false, true, false);
    } else if (y_pool && nt == kNT) {
        SUR_CONV_NT2(false, false, true);
    } else if (nt == 1) {
        if (flip) SUR_CONV_POW2(1, true, false, false, false);
        else SUR_CONV_POW2(1, false, false, false, false);
    } else {
        if (flip) SUR_CONV_NT2(true, false, false);
        else SUR_CONV_NT2(false, false, false);
    }
#undef SUR_CONV_WV8
#undef SUR_CONV_WV8N2
#undef SUR_CONV_NT2
#undef SUR_CONV_POW2
#undef SUR_CONV_LAUNCH
}

}  // namespace

extern "C" {

int sur_conv3d(const void *x, int32_t cin, const void *w, const float *bias, int32_t cout,
               int32_t nx, int32_t ny, int32_t nz, int32_t flip, int32_t relu, const void *mask,
               void *y_bf16, float *y_f32, void *stream) {
    clear_stale_error();
    if (!x || !w || (!y_bf16 && !y_f32) || cin <= 0 || cout <= 0 || cin % 16 || cout % 16 ||
        !dims_ok(nx, ny, nz))
        return SUR_EINVAL;
    const long P = (long)nx * ny * nz;
    if (conv_tiled_ok(x, cin, w, cout, nx, ny, nz)) {
        conv_tiled_launch(x, cin, nullptr, 0, w, bias, cout, nx, ny, nz, flip != 0, relu, mask,
                          y_bf16, y_f32, nullptr, (hipStream_t)stream);
        return launched();
    }
    const dim3 grid((unsigned)((P + 255) / 256), (unsigned)((cout + 63) / 64));
    hipLaunchKernelGGL(conv3d_kernel, grid, dim3(256), 0, (hipStream_t)stream, (const uint16_t *)x,
                       cin, (const uint16_t *)w, bias, cout, nx, ny, nz, flip, relu,
                       (const uint16_t *)mask, (uint16_t *)y_bf16, y_f32);
    return launched();
}

int sur_conv3d_cat(const void *xc, int32_t cc, const void *xf, int32_t fc, const void *w,
                   const float *bias, int32_t cout, int32_t nx, int32_t ny, int32_t nz,
                   int32_t relu, void *y_bf16, float *y_f32, void *stream) {
    clear_stale_error();
    if (!xc || !xf || !w || (!y_bf16 && !y_f32) || cc <= 0 || fc <= 0 || cout <= 0 || cc % 16 ||
        fc % 16 || cout % 16 || !dims_ok(nx, ny, nz) || !conv_tiled_ok(xf, cc + fc, w, cout, nx, ny, nz) ||
        ((uintptr_t)xc & 15) != 0 || !elems_ok((long)nx * ny * nz, cc))
        return SUR_EINVAL;
    conv_tiled_launch(xf, cc + fc, xc, cc, w, bias, cout, nx, ny, nz, false, relu, nullptr, y_bf16,
                      y_f32, nullptr, (hipStream_t)stream);
    return launched();
}

int sur_conv3d_pool(const void *x, int32_t cin, const void *w, const float *bias, int32_t cout,
                    int32_t nx, int32_t ny, int32_t nz, int32_t relu, void *y_bf16, void *y_pool,
                    void *stream) {
    clear_stale_error();
    if (!x || !w || !y_bf16 || !y_pool || cin <= 0 || cout <= 0 || cin % 16 || cout % 16 ||
        !dims_ok(nx, ny, nz) || !conv_tiled_ok(x, cin, w, cout, nx, ny, nz) ||
        ((uintptr_t)y_bf16 & 7) != 0 || ((uintptr_t)y_pool & 7) != 0)
        return SUR_EINVAL;
    if (cout <= 16 && conv_waves(cin, cout, nx, ny, nz, device_cus()) == 4) {
        // one output tile on four wavefronts: pooling in the epilogue would
        // take LDS that a fourth block per CU needs, so pool after
        conv_tiled_launch(x, cin, nullptr, 0, w, bias, cout, nx, ny, nz, false, relu, nullptr,
                          y_bf16, nullptr, nullptr, (hipStream_t)stream);
        if (launched() != SUR_OK) return SUR_EDEVICE;
        return sur_pool2(y_bf16, cout, nx, ny, nz, y_pool, stream);
    }
    conv_tiled_launch(x, cin, nullptr, 0, w, bias, cout, nx, ny, nz, false, relu, nullptr, y_bf16,
                      nullptr, y_pool, (hipStream_t)stream);
    return launched();
}

size_t sur_wgrad_scratch_floats(int32_t cin, int32_t cout, int32_t nx, int32_t ny, int32_t nz) {
    const long P = (long)nx * ny * nz;
    const long parts = std::max(wgrad_chunks(P), wgrad_tiled_blocks(cin, P));
    // bias partials: one per 1024 points, or one per tiled block
    const long bparts = std::max((long)grid1(P, 1024).x, wgrad_tiled_blocks(cin, P));
    // the rows of the first reduction pass (weights, then bias)
    return (size_t)(parts * 27L * cin * cout + bparts * (long)cout + kSumSeg * 27L * cin * cout +
                    kSumSeg * (long)cout);
}

int sur_conv3d_wgrad(const void *x, int32_t cin, const void *dy, int32_t cout, int32_t nx,
                     int32_t ny, int32_t nz, float *scratch, size_t scratch_floats, float *dw,
                     float *dbias, void *stream) {
    clear_stale_error();
    if (!x || !dy || !scratch || !dw || cin <= 0 || cout <= 0 || cin % 16 || cout % 16 ||
        cout > 64 || !dims_ok(nx, ny, nz))
        return SUR_EINVAL;
    if (scratch_floats < sur_wgrad_scratch_floats(cin, cout, nx, ny, nz)) return SUR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const long P = (long)nx * ny * nz;
    const uint16_t *xb = (const uint16_t *)x, *db = (const uint16_t *)dy;
    long nch;  // partial sums in scratch
    const long n = 27L * cin * cout;
    bool bias_done = false;
    float *tiled_bp = nullptr;  // bias partials of the tiled kernel, summed with dw's last pass
    if (wgrad_tiled_ok(x, cin, dy, cout, nx, ny, nz)) {
        nch = wgrad_tiled_blocks(cin, P);
        const dim3 grid((unsigned)nch, (unsigned)(cin / 16));
        // the bias partials follow the weight partials: one per block
        float *bp = dbias ? scratch + nch * n : nullptr;
        switch (cout / 16) {
            case 1: hipLaunchKernelGGL(wgrad_tiled_kernel<1>, grid, dim3(256), 0, s, xb, cin, db, cout, nx, ny, nz, scratch, bp); break;
            case 2: hipLaunchKernelGGL(wgrad_tiled_kernel<2>, grid, dim3(256), 0, s, xb, cin, db, cout, nx, ny, nz, scratch, bp); break;
            case 3: hipLaunchKernelGGL(wgrad_tiled_kernel<3>, grid, dim3(256), 0, s, xb, cin, db, cout, nx, ny, nz, scratch, bp); break;
            default: hipLaunchKernelGGL(wgrad_tiled_kernel<4>, grid, dim3(256), 0, s, xb, cin, db, cout, nx, ny, nz, scratch, bp); break;
        }
        tiled_bp = bp;
        bias_done = true;
    } else {
        nch = wgrad_chunks(P);
        const dim3 grid(27, (unsigned)nch, (unsigned)((cin + 63) / 64));
        switch (cout / 16) {
            case 1: hipLaunchKernelGGL(wgrad_kernel<1>, grid, dim3(256), 0, s, xb, cin, db, cout, nx, ny, nz, kWgradChunk, scratch); break;
            case 2: hipLaunchKernelGGL(wgrad_kernel<2>, grid, dim3(256), 0, s, xb, cin, db, cout, nx, ny, nz, kWgradChunk, scratch); break;
            case 3: hipLaunchKernelGGL(wgrad_kernel<3>, grid, dim3(256), 0, s, xb, cin, db, cout, nx, ny, nz, kWgradChunk, scratch); break;
            default: hipLaunchKernelGGL(wgrad_kernel<4>, grid, dim3(256), 0, s, xb, cin, db, cout, nx, ny, nz, kWgradChunk, scratch); break;
        }
    }
    {
        // two passes: kSumSeg row segments into mid, then mid's rows in order
        // (n = 27 cin cout is a multiple of 4; the partial rows are 16-byte
        // aligned when the scratch is)
        const long bparts = std::max((long)grid1(P, 1024).x, wgrad_tiled_blocks(cin, P));
        float *mid = scratch + nch * n + bparts * (long)cout;
        if (aligned16(scratch) && aligned16(mid) && n % 4 == 0 && nch >= 2 * kSumSeg) {
            const long n4 = n / 4;
            const int L = (int)((nch + kSumSeg - 1) / kSumSeg);
            const long na4 = (n4 + 31) / 32;
            // the bias partials (rows of cout, 16-byte aligned: cout % 16 == 0)
            // take the same two passes, in the same launches
            float *mid_b = mid + kSumSeg * n;
            const bool with_b = tiled_bp && aligned16(tiled_bp);
            const long nb4 = with_b ? ((long)cout / 4 + 31) / 32 : 0;
            const dim3 g1((unsigned)(na4 + nb4), (unsigned)kSumSeg);
            hipLaunchKernelGGL(sum_rows4_kernel, g1, dim3(256), 0, s, (const float4 *)scratch, nch,
                               n4, L, (float4 *)mid, na4, (const float4 *)tiled_bp,
                               (long)cout / 4, (float4 *)mid_b);
            if (with_b) {  // dw's and dbias's last passes in one launch
                const long na = grid1(n, 32).x;
                hipLaunchKernelGGL(sum_chunks2_kernel, dim3((unsigned)(na + grid1(cout, 32).x)),
                                   dim3(256), 0, s, (const float *)mid, (long)kSumSeg, n, dw, na,
                                   (const float *)mid_b, (long)kSumSeg, (long)cout, dbias);
                tiled_bp = nullptr;
            } else {
                hipLaunchKernelGGL(sum_chunks_kernel, grid1(n, 32), dim3(256), 0, s,
                                   (const float *)mid, (long)kSumSeg, n, dw);
            }
        } else {
            hipLaunchKernelGGL(sum_chunks_kernel, grid1(n, 32), dim3(256), 0, s,
                               (const float *)scratch, nch, n, dw);
        }
    }
    if (tiled_bp)
        hipLaunchKernelGGL(sum_chunks_kernel, grid1(cout, 32), dim3(256), 0, s,
                           (const float *)tiled_bp, nch, (long)cout, dbias);
    if (dbias && !bias_done) {
        const long nb = grid1(P, 1024).x;
        float *bp = scratch + nch * n;
        hipLaunchKernelGGL(bias_partial_kernel, dim3((unsigned)nb), dim3(256), 0, s, db, cout, P, 1024L, bp);
        hipLaunchKernelGGL(sum_chunks_kernel, grid1(cout, 32), dim3(256), 0, s, (const float *)bp, nb, (long)cout, dbias);
    }
    return launched();
}

int sur_pack_weights_all(const float *w, int32_t nlayers, const int64_t *w_off, const int32_t *cin,
                         const int32_t *cout, void *wf, void *wd, void *stream) {
    clear_stale_error();
    if (!w || !w_off || !cin || !cout || !wf || !wd || nlayers <= 0 || nlayers > kMaxPackLayers)
        return SUR_EINVAL;
    PackTable tb;
    tb.n = nlayers;
    tb.poff[0] = 0;
    for (int l = 0; l < nlayers; ++l) {
        if (cin[l] <= 0 || cout[l] <= 0 || w_off[l] < 0) return SUR_EINVAL;
        tb.woff[l] = (long)w_off[l];
        tb.cin[l] = cin[l];
        tb.cout[l] = cout[l];
        tb.poff[l + 1] = tb.poff[l] + 27L * cin[l] * cout[l];
    }
    hipLaunchKernelGGL(pack_all_kernel, grid1(tb.poff[nlayers]), dim3(256), 0, (hipStream_t)stream,
                       w, tb, (uint16_t *)wf, (uint16_t *)wd);
    return launched();
}

int sur_pack_weights(const float *w, int32_t cin, int32_t cout, void *wf, void *wd, void *stream) {
    clear_stale_error();
    if (!w || (!wf && !wd) || cin <= 0 || cout <= 0) return SUR_EINVAL;
    const long n = 27L * cin * cout;
    hipLaunchKernelGGL(pack_weights_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream, w, cin,
                       cout, (uint16_t *)wf, (uint16_t *)wd);
    return launched();
}

int sur_pool2(const void *x, int32_t c, int32_t nx, int32_t ny, int32_t nz, void *y, void *stream) {
    clear_stale_error();
    if (!x || !y || c <= 0 || !dims_ok(nx, ny, nz) || nx % 2 || ny % 2 || nz % 2 ||
        !elems_ok((long)nx * ny * nz, c))
        return SUR_EINVAL;
    const long n = (long)(nx / 2) * (ny / 2) * (nz / 2) * c;
    if (c % 8 == 0 && aligned16(x) && aligned16(y)) {
        hipLaunchKernelGGL(pool2_v8_kernel, grid1(n / 8), dim3(256), 0, (hipStream_t)stream,
                           (const uint16_t *)x, c, nx, ny, nz, (uint16_t *)y);
        return launched();
    }
    hipLaunchKernelGGL(pool2_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream,
                       (const uint16_t *)x, c, nx, ny, nz, (uint16_t *)y);
    return launched();
}

int sur_pool2_bwd(const float *dy, int32_t c, int32_t nx, int32_t ny, int32_t nz, float *dx,
                  void *stream) {
    clear_stale_error();
    if (!dy || !dx || c <= 0 || !dims_ok(nx, ny, nz) || nx % 2 || ny % 2 || nz % 2 ||
        !elems_ok((long)nx * ny * nz, c))
        return SUR_EINVAL;
    const long n = (long)nx * ny * nz * c;
    hipLaunchKernelGGL(pool2_bwd_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream, dy, c, nx,
                       ny, nz, dx);
    return launched();
}

int sur_pool2_bwd_skip(const float *dy, int32_t c, int32_t nx, int32_t ny, int32_t nz,
                       const float *skip, int32_t skip_stride, int32_t skip_off, const void *act,
                       float *dx, void *dx_bf16, void *stream) {
    clear_stale_error();
    if (!dy || !skip || !act || (!dx && !dx_bf16) || c <= 0 || !dims_ok(nx, ny, nz) || nx % 2 || ny % 2 ||
        nz % 2 || skip_off < 0 || skip_off + c > skip_stride ||
        !elems_ok((long)nx * ny * nz, skip_stride))
        return SUR_EINVAL;
    const long n = (long)nx * ny * nz * c;
    const bool v4 = c % 4 == 0 && skip_stride % 4 == 0 && skip_off % 4 == 0 && aligned16(dy) &&
                    aligned16(skip) && ((uintptr_t)act & 7) == 0 && (!dx || aligned16(dx)) &&
                    ((uintptr_t)dx_bf16 & 7) == 0;
    if (v4)
        hipLaunchKernelGGL(pool2_bwd_skip4_kernel, grid1(n / 4), dim3(256), 0, (hipStream_t)stream,
                           (const float4 *)dy, c, nx, ny, nz, (const float4 *)skip, skip_stride,
                           skip_off, (const uint2 *)act, (float4 *)dx, (uint2 *)dx_bf16);
    else
        hipLaunchKernelGGL(pool2_bwd_skip_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream, dy,
                           c, nx, ny, nz, skip, skip_stride, skip_off, (const uint16_t *)act, dx,
                           (uint16_t *)dx_bf16);
    return launched();
}

int sur_upsample2_bwd_mask(const float *dy, int32_t dystride, int32_t dyoff, int32_t c,
                           int32_t nx, int32_t ny, int32_t nz, const void *act, void *dx_bf16,
                           void *stream) {
    clear_stale_error();
    if (!dy || !act || !dx_bf16 || c <= 0 || !dims_ok(nx, ny, nz) || dyoff < 0 ||
        dyoff + c > dystride || !elems_ok(8L * nx * ny * nz, dystride))
        return SUR_EINVAL;
    const long n = (long)nx * ny * nz * c;
    const bool v4 = c % 4 == 0 && dystride % 4 == 0 && dyoff % 4 == 0 && aligned16(dy) &&
                    ((uintptr_t)act & 7) == 0 && ((uintptr_t)dx_bf16 & 7) == 0;
    if (v4)
        hipLaunchKernelGGL(upsample2_bwd_mask4_kernel, grid1(n / 4), dim3(256), 0,
                           (hipStream_t)stream, (const float4 *)dy, dystride, dyoff, c, nx, ny, nz,
                           (const uint2 *)act, (uint2 *)dx_bf16);
    else
        hipLaunchKernelGGL(upsample2_bwd_mask_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream,
                           dy, dystride, dyoff, c, nx, ny, nz, (const uint16_t *)act,
                           (uint16_t *)dx_bf16);
    return launched();
}

int sur_upsample2(const void *x, int32_t c, int32_t nx, int32_t ny, int32_t nz, void *y,
                  int32_t ystride, int32_t yoff, void *stream) {
    clear_stale_error();
    if (!x || !y || c <= 0 || !dims_ok(nx, ny, nz) || yoff < 0 || yoff + c > ystride ||
        !elems_ok(8L * nx * ny * nz, ystride))
        return SUR_EINVAL;
    const long n = 8L * nx * ny * nz * c;
    if (c % 8 == 0 && ystride % 8 == 0 && yoff % 8 == 0 && aligned16(x) && aligned16(y)) {
        hipLaunchKernelGGL(upsample2_v8_kernel, grid1(n / 8), dim3(256), 0, (hipStream_t)stream,
                           (const uint16_t *)x, c, nx, ny, nz, (uint16_t *)y, ystride, yoff);
        return launched();
    }
    hipLaunchKernelGGL(upsample2_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream,
                       (const uint16_t *)x, c, nx, ny, nz, (uint16_t *)y, ystride, yoff);
    return launched();
}

int sur_upsample2_bwd(const float *dy, int32_t dystride, int32_t dyoff, int32_t c, int32_t nx,
                      int32_t ny, int32_t nz, float *dx, void *stream) {
    clear_stale_error();
    if (!dy || !dx || c <= 0 || !dims_ok(nx, ny, nz) || dyoff < 0 || dyoff + c > dystride ||
        !elems_ok(8L * nx * ny * nz, dystride))
        return SUR_EINVAL;
    const long n = (long)nx * ny * nz * c;
    hipLaunchKernelGGL(upsample2_bwd_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream, dy,
                       dystride, dyoff, c, nx, ny, nz, dx);
    return launched();
}

int sur_concat_up2(const void *xc, int32_t hc, const void *xf, int32_t fc, int32_t nx, int32_t ny,
                   int32_t nz, void *y, void *stream) {
    clear_stale_error();
    if (!xc || !xf || !y || hc <= 0 || fc <= 0 || !dims_ok(nx, ny, nz) || nx % 2 || ny % 2 ||
        nz % 2 || !elems_ok((long)nx * ny * nz, hc + fc))
        return SUR_EINVAL;
    if (hc % 8 == 0 && fc % 8 == 0 && aligned16(xc) && aligned16(xf) && aligned16(y)) {
        const long n = (long)nx * ny * nz * ((hc + fc) / 8);
        hipLaunchKernelGGL(concat_up2_v8_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream,
                           (const uint16_t *)xc, hc, (const uint16_t *)xf, fc, nx, ny, nz,
                           (uint16_t *)y);
        return launched();
    }
    // otherwise the two separate passes
    const int rc = sur_upsample2(xc, hc, nx / 2, ny / 2, nz / 2, y, hc + fc, 0, stream);
    if (rc != SUR_OK) return rc;
    return sur_copy_channels(xf, fc, (long)nx * ny * nz, y, hc + fc, hc, stream);
}

int sur_copy_channels(const void *x, int32_t c, int64_t P, void *y, int32_t ystride, int32_t yoff,
                      void *stream) {
    clear_stale_error();
    if (!x || !y || c <= 0 || P <= 0 || yoff < 0 || yoff + c > ystride || !elems_ok(P, ystride))
        return SUR_EINVAL;
    if (c % 8 == 0 && ystride % 8 == 0 && yoff % 8 == 0 && aligned16(x) && aligned16(y)) {
        hipLaunchKernelGGL(copy_channels_v8_kernel, grid1(P * c / 8), dim3(256), 0,
                           (hipStream_t)stream, (const uint16_t *)x, c, (long)P, (uint16_t *)y,
                           ystride, yoff);
        return launched();
    }
    hipLaunchKernelGGL(copy_channels_kernel, grid1(P * c), dim3(256), 0, (hipStream_t)stream,
                       (const uint16_t *)x, c, (long)P, (uint16_t *)y, ystride, yoff);
    return launched();
}

int sur_add_channels(const float *dy, int32_t dystride, int32_t dyoff, int32_t c, int64_t P,
                     float *dx, void *stream) {
    clear_stale_error();
    if (!dy || !dx || c <= 0 || P <= 0 || dyoff < 0 || dyoff + c > dystride ||
        !elems_ok(P, dystride))
        return SUR_EINVAL;
    hipLaunchKernelGGL(add_channels_kernel, grid1(P * c), dim3(256), 0, (hipStream_t)stream, dy,
                       dystride, dyoff, c, (long)P, dx);
    return launched();
}

int sur_to_bf16(const float *x, int64_t n, void *y, void *stream) {
    clear_stale_error();
    if (!x || !y || n < 0) return SUR_EINVAL;
    if (n == 0) return SUR_OK;
    hipLaunchKernelGGL(to_bf16_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream, x, (long)n,
                       (uint16_t *)y);
    return launched();
}

int sur_relu_mask(float *dx, const void *act, int64_t n, void *stream) {
    clear_stale_error();
    if (!dx || !act || n < 0) return SUR_EINVAL;
    if (n == 0) return SUR_OK;
    hipLaunchKernelGGL(relu_mask_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream, dx,
                       (const uint16_t *)act, (long)n);
    return launched();
}

int sur_mse(const float *pred, const float *target, int32_t cu, int32_t cs, int64_t P,
            const float *wch, float *grad, void *grad_bf16, double *scratch, double *loss_out,
            void *stream) {
    clear_stale_error();
    if (!pred || !target || !wch || (!grad && !grad_bf16) || !scratch || !loss_out || cu <= 0 ||
        cs < cu || P <= 0)
        return SUR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const long nb = grid1(P).x;
    // 1: 16-byte accesses per point; 2: the same for 16 stored channels,
    // four lanes per point
    int vec4 = cs % 4 == 0 && ((uintptr_t)pred & 15) == 0 && ((uintptr_t)target & 15) == 0 &&
               ((uintptr_t)grad & 15) == 0 && ((uintptr_t)grad_bf16 & 7) == 0;
    if (vec4 && cs == 16) vec4 = 2;
    hipLaunchKernelGGL(mse_kernel, dim3((unsigned)nb), dim3(256), 0, s, pred, target, cu, cs,
                       (long)P, wch, grad, (uint16_t *)grad_bf16, scratch, vec4);
    hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(1024), 0, s, (const double *)scratch, nb,
                       1.0 / ((double)P * cu), loss_out);
    return launched();
}

int sur_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float beta1,
             float beta2, float eps, int32_t t, void *stream) {
    clear_stale_error();
    if (!w || !m || !v || !g || n <= 0 || t < 1) return SUR_EINVAL;
    const float bc1 = 1.f - (float)pow((double)beta1, (double)t);
    const float bc2 = 1.f - (float)pow((double)beta2, (double)t);
    hipLaunchKernelGGL(adam_kernel, grid1(n), dim3(256), 0, (hipStream_t)stream, w, m, v, g,
                       (long)n, lr, beta1, beta2, eps, bc1, bc2);
    return launched();
}

int sur_coarsen(const float *phi, const float *u, const float *p, int32_t nx, int32_t ny, int32_t nz,
                const float *scale, float *coarse_f32, void *coarse_bf16, void *stream) {
    clear_stale_error();
    if (!phi || !u || !p || !scale || (!coarse_f32 && !coarse_bf16) || !dims_ok(nx, ny, nz) ||
        nx % 2 || ny % 2 || nz % 2)
        return SUR_EINVAL;
    const long Pc = (long)(nx / 2) * (ny / 2) * (nz / 2);
    hipLaunchKernelGGL(coarsen_kernel, grid1(Pc), dim3(256), 0, (hipStream_t)stream, phi, u, p, nx,
                       ny, nz, scale, coarse_f32, (uint16_t *)coarse_bf16);
    return launched();
}

int sur_prolong_add(const float *delta, int32_t cnx, int32_t cny, int32_t cnz, const float *scale,
                    double *phi, double *u, double *p, void *stream) {
    clear_stale_error();
    if (!delta || !scale || !phi || !u || !p || !dims_ok(cnx, cny, cnz)) return SUR_EINVAL;
    const long N = 8L * cnx * cny * cnz;
    hipLaunchKernelGGL(prolong_add_kernel, grid1(N), dim3(256), 0, (hipStream_t)stream, delta, cnx,
                       cny, cnz, scale, phi, u, p);
    return launched();
}

int sur_apply_residual(float *state, const float *out, const float *rscale, int32_t cu, int64_t P,
                       double width, void *stream) {
    clear_stale_error();
    if (!state || !out || !rscale || cu <= 0 || cu > 16 || !elems_ok(P, 16)) return SUR_EINVAL;
    if (!(width >= 0.0)) return SUR_EINVAL;
    hipLaunchKernelGGL(apply_residual_kernel, grid1(P * cu), dim3(256), 0, (hipStream_t)stream,
                       state, out, rscale, cu, (long)P, (float)width);
    return launched();
}

int sur_residual_target(const float *s0, const float *s1, const float *rscale, int32_t cu, int64_t P,
                        double width, float *target, void *stream) {
    clear_stale_error();
    if (!s0 || !s1 || !rscale || !target || cu <= 0 || cu > 16 || !elems_ok(P, 16)) return SUR_EINVAL;
    if (!(width >= 0.0)) return SUR_EINVAL;
    hipLaunchKernelGGL(residual_target_kernel, grid1(P * 16), dim3(256), 0, (hipStream_t)stream,
                       s0, s1, rscale, cu, (long)P, (float)width, target);
    return launched();
}

int sur_fix_mass(float *state, int64_t P, const double *checks_out, const double *target_mass,
                 void *stream) {
    clear_stale_error();
    if (!state || !checks_out || !target_mass || P <= 0) return SUR_EINVAL;
    hipLaunchKernelGGL(fix_mass_kernel, grid1(P), dim3(256), 0, (hipStream_t)stream, state, (long)P,
                       checks_out, target_mass);
    return launched();
}

int sur_features(float *state, int32_t nx, int32_t ny, int32_t nz, void *stream) {
    clear_stale_error();
    if (!state || !dims_ok(nx, ny, nz)) return SUR_EINVAL;
    const long P = (long)nx * ny * nz;
    hipLaunchKernelGGL(features_kernel, grid1(P), dim3(256), 0, (hipStream_t)stream, state, nx, ny, nz);
    return launched();
}

size_t sur_prolong_update_scratch_doubles(int32_t cnx, int32_t cny, int32_t cnz) {
    const long N = 8L * cnx * cny * cnz;
    return (size_t)(2 * grid1(N).x);
}

int sur_prolong_update(const float *s0, const float *s1, int32_t cnx, int32_t cny, int32_t cnz,
                       const float *scale, double width, double *phi, double *u, double *p,
                       double *scratch, double *sums, void *stream) {
    clear_stale_error();
    if (!s0 || !s1 || !scale || !phi || !u || !p || !scratch || !sums ||
        !dims_ok(2 * cnx, 2 * cny, 2 * cnz) || !(width > 0.0))
        return SUR_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const long N = 8L * cnx * cny * cnz;
    const long nb = grid1(N).x;
    hipLaunchKernelGGL(field_sums_kernel, dim3((unsigned)nb), dim3(256), 0, st, (const double *)phi, N, scratch);
    hipLaunchKernelGGL(sums2_final_kernel, dim3(1), dim3(1024), 0, st, (const double *)scratch, nb, sums);
    hipLaunchKernelGGL(prolong_update_kernel, dim3((unsigned)nb), dim3(256), 0, st, s0, s1, cnx, cny, cnz,
                       scale, (float)width, phi, u, p);
    hipLaunchKernelGGL(field_sums_kernel, dim3((unsigned)nb), dim3(256), 0, st, (const double *)phi, N, scratch);
    hipLaunchKernelGGL(sums2_final_kernel, dim3(1), dim3(1024), 0, st, (const double *)scratch, nb, sums + 2);
    hipLaunchKernelGGL(fix_mass_field_kernel, dim3((unsigned)nb), dim3(256), 0, st, phi, N,
                       (const double *)(sums + 2), (const double *)sums);
    return launched();
}

int sur_checks(const float *state, int32_t nx, int32_t ny, int32_t nz, double *scratch, double *out,
               void *stream) {
    clear_stale_error();
    if (!state || !scratch || !out || !dims_ok(nx, ny, nz)) return SUR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const long P = (long)nx * ny * nz;
    const long nb = grid1(P).x;
    hipLaunchKernelGGL(checks_kernel, dim3((unsigned)nb), dim3(256), 0, s, state, nx, ny, nz, scratch);
    hipLaunchKernelGGL(checks_final_kernel, dim3(1), dim3(1024), 0, s, (const double *)scratch, nb, out);
    return launched();
}

int sur_checks_noalloc(const float *state, int32_t nx, int32_t ny, int32_t nz, double *out,
                       void *stream) {
    clear_stale_error();
    if (!state || !out || !dims_ok(nx, ny, nz)) return SUR_EINVAL;
    const long P = (long)nx * ny * nz;
    if (P > SUR_CHECKS_NOALLOC_MAX_POINTS) return SUR_EINVAL;
    double *part = checks_scratch_here();
    if (!part) return SUR_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const long nb = grid1(P).x;
    hipLaunchKernelGGL(checks_kernel, dim3((unsigned)nb), dim3(256), 0, s, state, nx, ny, nz, part);
    hipLaunchKernelGGL(checks_final_kernel, dim3(1), dim3(1024), 0, s, (const double *)part, nb, out);
    return launched();
}

}  // extern "C"
