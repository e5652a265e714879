// lbm_kernels.hpp -- HIP kernels (gfx950) of the fused difference-free
// conservative phase-field LBM step (Zhao, Patel & Lee, arXiv 2407.12263).
//
// One thread per lattice node, one pass per step: each thread pulls the
// Lax-Wendroff taps of its 2 x Q populations (D3Q19, or D3Q27) from the
// post-collision buffer, recovers phi, u, K1, n, grad(phi), p in registers,
// collides both populations and writes 2 x Q post-collision values. The only non-local
// operation is the propagation; the interface normal and grad(phi) come from
// the node's own K1 (Sec. 2.3), so no neighbour field is ever differenced.
//
// Memory access: structure-of-arrays planes (population i of all nodes is
// contiguous, x fastest), read and written with buffer instructions whose
// plane offset i*N*size is a scalar register and whose per-lane offset is
// one of the Q stencil-node offsets computed once per thread, so no vector
// instruction is spent on addresses. A block is a tile of whole x-rows of one
// z-plane (a wavefront covers 64 contiguous nodes of a row: every load is a
// coalesced row segment); the block-to-tile order is selectable (plain, XCD
// runs, z-banded XCD runs) for tuning the L2 reuse of the y/z taps.
//
// Precision policies: FP64; FP32; FP32 compute with 16-bit storage of the
// deviations f_i - t_i rho0 and g_i - t_i phi_s scaled by 2^k (FP16 or
// BF16, round-to-nearest-even) plus the FP32 per-node phi_s chosen so that the
// stored g of a node sums exactly (to FP32 rounding) to the collided phi.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace cpf {

// ---------------------------------------------------------------- lattice
// D3Q19: rest, 6 axis vectors, 12 edge vectors; weights 1/3, 1/18, 1/36.
// D3Q27: the same 19 followed by the 8 corner vectors; weights 8/27, 2/27,
// 1/54, 1/216 (products of the 1D weights 2/3, 1/6, 1/6). In both, the
// directions after the rest come in opposite pairs (i, i + 1) for odd i.
template <int NQ>
struct LatQ;

template <>
struct LatQ<19> {
    static constexpr int Q = 19;
    static constexpr int EX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int EY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int EZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr int cls(int i) { return EX[i] * EX[i] + EY[i] * EY[i] + EZ[i] * EZ[i]; }
};

template <>
struct LatQ<27> {
    static constexpr int Q = 27;
    static constexpr int EX[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                   1, -1, 1, -1, 1, -1, -1, 1};
    static constexpr int EY[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                                   1, -1, 1, -1, -1, 1, 1, -1};
    static constexpr int EZ[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                                   1, -1, -1, 1, 1, -1, 1, -1};
    static constexpr int OPP[27] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17,
                                    20, 19, 22, 21, 24, 23, 26, 25};
    static constexpr int cls(int i) { return EX[i] * EX[i] + EY[i] * EY[i] + EZ[i] * EZ[i]; }
};

// Weights by speed class. In FP32 the rounded 1/3, 1/18, 1/36 sum to
// 1 + 1.5e-8, which would make every collision create that fraction of phi
// (a 1e-4 relative drift of the phase mass over 1e4 steps); the FP32 sets
// below are exactly representable, sum to exactly 1 (t0 + 6 t1 + 12 t2
// [+ 8 t3]) and are within 2.1 ulp of the true weights.
template <class R, int NQ = 19>
__device__ __forceinline__ constexpr R wgt(int cls) {
    constexpr float s = 1.0f / 268435456.0f;  // 2^-28
    if constexpr (NQ == 27) {
        if constexpr (std::is_same_v<R, float>) {
            return cls == 0 ? 79536440.0f * s
                            : (cls == 1 ? 19884104.0f * s
                                        : (cls == 2 ? 4971028.0f * s : 1242757.0f * s));
        } else {
            return cls == 0 ? R(8) / R(27)
                            : (cls == 1 ? R(2) / R(27) : (cls == 2 ? R(1) / R(54) : R(1) / R(216)));
        }
    } else {
        if constexpr (std::is_same_v<R, float>) {
            return cls == 0 ? 89478496.0f * s : (cls == 1 ? 14913080.0f * s : 7456540.0f * s);
        } else {
            return cls == 0 ? R(1) / R(3) : (cls == 1 ? R(1) / R(18) : R(1) / R(36));
        }
    }
}

template <int B, int E, class F>
__device__ __forceinline__ void unroll(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        unroll<B + 1, E>(f);
    }
}

// sum_i v_i * e^_ia with compile-time integer components
template <int A, class R, int NQ>
__device__ __forceinline__ R first_moment(const R (&v)[NQ]) {
    using L = LatQ<NQ>;
    R s = R(0);
    unroll<1, NQ>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int e = A == 0 ? L::EX[i] : (A == 1 ? L::EY[i] : L::EZ[i]);
        if constexpr (e > 0) s += v[i];
        if constexpr (e < 0) s -= v[i];
    });
    return s;
}

// e^_i . v for a compile-time direction
template <int i, int NQ, class R>
__device__ __forceinline__ R edot(const R (&v)[3]) {
    using L = LatQ<NQ>;
    constexpr int ex = L::EX[i], ey = L::EY[i], ez = L::EZ[i];
    R s = R(0);
    bool first = true;
    auto add = [&](int e, R x) {
        if (e == 0) return;
        R t = e > 0 ? x : -x;
        s = first ? t : s + t;
        first = false;
    };
    add(ex, v[0]);
    add(ey, v[1]);
    add(ez, v[2]);
    return s;
}

// ------------------------------------------------------------ parameters
// A block is 256 threads covering a tile of 2^tx_log2 x (256 >> tx_log2) nodes
// of one z-plane.
constexpr int BLOCK = 256;

// Division by a launch constant d for dividends below 2^31 (Granlund and
// Montgomery, 1994): q = floor(n m / 2^(31 + l)) with 2^(l-1) < d <= 2^l and
// m = ceil(2^(31 + l)/d) < 2^32; d = 1 is passed through.
struct FastDiv {
    uint32_t m, s, d;
};

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f) {
    return f.d == 1u ? n : (__umulhi(n, f.m) >> f.s);
}

template <class R>
struct DevParams {
    int nx, ny, nz, N;
    int wall[3];
    int tx_log2;             // tile width 2^tx_log2, tile height 256 >> tx_log2
    int ntx, nty, ntiles;    // tiles per row, per column, in total
    int order;               // 0: tile = block id; 1: XCD runs; 2: XCD runs of z-banded order
    int band;                // tile-rows per band (order 2)
    int xq, xr;              // ntiles = 8 xq + xr (XCD runs)
    int bty0, bnty, btz0, bnz;  // tile rows bty0 + k bty_step (k < bnty) x planes
    int bty_step, btz_step;     // btz0 + k btz_step (k < bnz) covered by one launch
                                // (ntiles = ntx bnty bnz)
    int nfull;                  // full bands of the z-banded order: bnty / band
    FastDiv d_ntx, d_nty, d_band, d_perband, d_rem;  // divisors of the tile decomposition
    R c, h;                  // Courant number, c(1-c)/2
    R lwA, lwD;              // Lax-Wendroff weights of x-e and x+e: c(1+c)/2, -c(1-c)/2
    R cs2, inv_cs2, half_inv_cs4;
    R rho2, drho;            // rho = rho2 + drho*phi
    R eta2, deta;            // eta = eta2 + deta*phi
    R omega_g, tau_phi_c;    // 1/(tau_phi+1/2), tau_phi*c
    R tau_phi_cs2, inv_tp;   // tau_phi*cs2, 1/((tau_phi+1/2) cs2)
    R sigma, four_over_delta;
    R G[3];
    R k1_eps;
    R rho0;                  // p_ref/cs2: gauge of the 16-bit f storage
    R scale_f, iscale_f, scale_g, iscale_g;
    R wA_f, wB_f, wD_f;      // 2^-k (A, 1 - c^2, D): the three-tap weights of the stored
    R wA_g, wB_g, wD_g;      // 16-bit deviations with their scale folded in (exact)
    R *phi_fd;               // phi field of the finite-difference variant (or NULL)
    uint32_t plane_bytes;    // bytes from one population plane to the next
};

// Wetting walls: contact angle theta at every wall (on = 0: neutral walls).
// A kernel argument of the wall-aware launches only.
template <class R>
struct Wet {
    int on;
    R cos_theta, sin_theta;
};

// Linear index of this block in its launch grid (x fastest).
__device__ __forceinline__ uint32_t linear_block() {
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

// ---------------------------------------------------------- storage types
// Q: populations per field (the lattice); BF: BF16 storage.
struct SF64 { using R = double; using T = double; static constexpr bool DEV = false, BF = false; static constexpr int Q = 19; };
struct SF32 { using R = float;  using T = float;  static constexpr bool DEV = false, BF = false; static constexpr int Q = 19; };
struct SH16 { using R = float;  using T = _Float16; static constexpr bool DEV = true, BF = false; static constexpr int Q = 19; };
struct SB16 { using R = float;  using T = uint16_t; static constexpr bool DEV = true, BF = true; static constexpr int Q = 19; };
// The same storage on D3Q27.
template <class S>
struct Q27 : S { static constexpr int Q = 27; };

template <class St>
__device__ __forceinline__ typename St::R decode(typename St::T v) {
    if constexpr (St::BF) {
        return __uint_as_float(uint32_t(v) << 16);
    } else {
        return typename St::R(v);
    }
}

template <class St>
__device__ __forceinline__ typename St::T encode(typename St::R x) {
    if constexpr (St::BF) {
        // round to nearest even (finite inputs)
        uint32_t u = __float_as_uint(x);
        u += 0x7fffu + ((u >> 16) & 1u);
        return uint16_t(u >> 16);
    } else {
        return typename St::T(x);
    }
}

template <class St>
struct Buf {
    typename St::T *f;   // Q planes of N
    typename St::T *g;   // Q planes of N
    float *phis;         // N (16-bit storage only)
};

template <class St>
struct CBuf {
    const typename St::T *f;
    const typename St::T *g;
    const float *phis;
};

// ------------------------------------------------------- buffer access
using rsrc_t = __amdgpu_buffer_rsrc_t;

// Raw buffer over [p, p + bytes); accesses beyond it read 0 and write nothing.
// Word 3 is the gfx9-family raw-buffer configuration.
__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

template <class T>
__device__ __forceinline__ T bload(rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    } else if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
    }
}

// Stores of the post-collision state are nontemporal (cache policy nt): no
// kernel re-reads them before the next step, which reads them from HBM, and
// streaming them past L2 leaves it to the neighbour taps of the current band
// (RT 128x512x128: FP16 27.9 -> 28.8 GLUPS, FP32 16.2 -> 16.8; 256^3 FP16
// 26.2 -> 27.5).
constexpr int kStoreNT = 2;

template <class T>
__device__ __forceinline__ void bstore(T v, rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 8) {
        using V2 = unsigned int __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, voff, soff, kStoreNT);
    } else if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, kStoreNT);
    } else {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, voff, soff, kStoreNT);
    }
}

// ------------------------------------------------------- node geometry
template <int NQ>
struct Site {
    int x, y, z;
    bool valid;
    uint32_t n;          // node index
    uint32_t nb[NQ];     // index of node x + e^_j (wrapped), nb[0] = n
    bool lo[3], hi[3];   // node on the first / last layer of a wall axis
    bool wall;           // lo or hi on some axis
};

// Block -> tile. Workgroups are dispatched round-robin to the 8 XCDs; with
// order >= 1, XCD k takes the contiguous run of logical tiles
// [start_k, start_k + count_k), so neighbouring tiles share its L2. Logical
// tiles run x fastest, then (order 1) y, then z, or (order 2) y within a band
// of `band` tile-rows, then z, then the band: the z-neighbour planes a tile
// re-reads are then only a band's width of tiles away.
template <int NQ, class R>
__device__ __forceinline__ Site<NQ> make_site(const DevParams<R> &P) {
    using L = LatQ<NQ>;
    Site<NQ> s;
    const uint32_t b = blockIdx.x;
    uint32_t t = b;
    if (P.order == 0) {
        // the launch grid is (ntx, bnty, bnz)
        t = 0;
    } else {
        // XCD runs: block b runs on XCD b mod 8; the XCD's blocks take one
        // contiguous run of tiles
        const uint32_t xcd = b & 7u, slot = b >> 3;
        const uint32_t q = (uint32_t)P.xq, r = (uint32_t)P.xr;
        t = (xcd < r ? xcd * (q + 1u) : r * (q + 1u) + (xcd - r) * q) + slot;
    }
    const uint32_t ntx = (uint32_t)P.ntx, nty = (uint32_t)P.bnty, nz = (uint32_t)P.bnz;
    uint32_t tx, rr, ty, tz;
    if (P.order == 0) {
        tx = blockIdx.x;
        rr = 0;
        ty = blockIdx.y;
        tz = blockIdx.z;
    } else {
        rr = fdiv(t, P.d_ntx);
        tx = t - rr * ntx;
    }
    if (P.order == 0) {
    } else if (P.order == 2) {
        const uint32_t bw = (uint32_t)P.band, full = (uint32_t)P.nfull, per_band = bw * nz;
        if (rr < full * per_band) {
            const uint32_t k = fdiv(rr, P.d_perband), w = rr - k * per_band;
            tz = fdiv(w, P.d_band);
            ty = k * bw + (w - tz * bw);
        } else {
            const uint32_t rem = nty - full * bw, w = rr - full * per_band;
            tz = fdiv(w, P.d_rem);
            ty = full * bw + (w - tz * rem);
        }
    } else {
        tz = fdiv(rr, P.d_nty);
        ty = rr - tz * nty;
    }
    ty = (uint32_t)P.bty0 + ty * (uint32_t)P.bty_step;
    tz = (uint32_t)P.btz0 + tz * (uint32_t)P.btz_step;
    const uint32_t lx = threadIdx.x & ((1u << P.tx_log2) - 1u), ly = threadIdx.x >> P.tx_log2;
    s.x = (int)((tx << P.tx_log2) + lx);
    s.y = (int)(ty * (uint32_t)(BLOCK >> P.tx_log2) + ly);
    s.z = (int)tz;
    s.valid = s.x < P.nx && s.y < P.ny && s.z < P.nz;
    const int x = s.valid ? s.x : 0, y = s.valid ? s.y : 0, z = s.valid ? s.z : 0;
    const uint32_t nx = P.nx, nxy = (uint32_t)P.nx * P.ny;
    const uint32_t X[3] = {uint32_t(x == 0 ? P.nx - 1 : x - 1), uint32_t(x),
                           uint32_t(x == P.nx - 1 ? 0 : x + 1)};
    const uint32_t Y[3] = {uint32_t(y == 0 ? P.ny - 1 : y - 1) * nx, uint32_t(y) * nx,
                           uint32_t(y == P.ny - 1 ? 0 : y + 1) * nx};
    const uint32_t Z[3] = {uint32_t(z == 0 ? P.nz - 1 : z - 1) * nxy, uint32_t(z) * nxy,
                           uint32_t(z == P.nz - 1 ? 0 : z + 1) * nxy};
    unroll<0, NQ>([&](auto J) {
        constexpr int j = decltype(J)::value;
        s.nb[j] = X[L::EX[j] + 1] + Y[L::EY[j] + 1] + Z[L::EZ[j] + 1];
    });
    s.n = s.nb[0];
    const int c[3] = {x, y, z};
    const int nn[3] = {P.nx, P.ny, P.nz};
    s.wall = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s.lo[a] = P.wall[a] && c[a] == 0;
        s.hi[a] = P.wall[a] && c[a] == nn[a] - 1;
        s.wall = s.wall || s.lo[a] || s.hi[a];
    }
    s.wall = s.wall && s.valid;
    return s;
}

// x - s*e^_i lies beyond a wall (s = +1: upstream, s = -1: downstream)
template <int i, int sgn, int NQ>
__device__ __forceinline__ bool beyond_wall(const Site<NQ> &s) {
    using L = LatQ<NQ>;
    constexpr int e[3] = {sgn * L::EX[i], sgn * L::EY[i], sgn * L::EZ[i]};
    bool b = false;
    if constexpr (e[0] > 0) b = b || s.lo[0];
    if constexpr (e[0] < 0) b = b || s.hi[0];
    if constexpr (e[1] > 0) b = b || s.lo[1];
    if constexpr (e[1] < 0) b = b || s.hi[1];
    if constexpr (e[2] > 0) b = b || s.lo[2];
    if constexpr (e[2] < 0) b = b || s.hi[2];
    return b;
}

// Inward unit normal of the walls a wall node touches (the normalised sum of
// its faces' at an edge or corner); 0 on other nodes (then l2 = 0).
template <class R, int NQ>
__device__ __forceinline__ R wall_normal(const Site<NQ> &s, R (&nw)[3]) {
    R l2 = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        nw[a] = (s.lo[a] ? R(1) : R(0)) - (s.hi[a] ? R(1) : R(0));
        l2 += nw[a] * nw[a];
    }
    const R r = l2 > R(0) ? R(1) / sqrt(l2) : R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) nw[a] *= r;
    return l2;
}

// ------------------------------------------------------------ propagation
enum Mode { LOCAL = 0, SHIFT = 1, LW = 2 };

template <class St>
struct Src {
    rsrc_t f, g, phis;
    uint32_t plane;      // bytes from one population plane to the next (padded)
};

template <class St>
__device__ __forceinline__ Src<St> make_src(const CBuf<St> &b, const DevParams<typename St::R> &P) {
    Src<St> s;
    // 16-bit storage keeps f_i and g_i of a node together in one 32-bit word
    // (f in the low half): one load per tap serves both fields
    const uint32_t plane = P.plane_bytes;
    s.plane = plane;
    s.f = make_rsrc(b.f, (uint32_t)St::Q * plane);
    s.g = St::DEV ? s.f : make_rsrc(b.g, (uint32_t)St::Q * plane);
    s.phis = make_rsrc(b.phis, St::DEV ? (uint32_t)P.N * 4u : 0u);
    return s;
}

// Stored values of population i of f and g at stencil node j (16-bit
// storage: the decoded deviations).
template <class St, int i>
__device__ __forceinline__ void rawfg(const Src<St> &src, const Site<St::Q> &s, int j,
                                      typename St::R &f, typename St::R &g) {
    using T = typename St::T;
    using R = typename St::R;
    if constexpr (St::DEV) {
        const uint32_t w = bload<uint32_t>(src.f, s.nb[j] * 4u, (uint32_t)i * src.plane);
        if constexpr (St::BF) {
            f = __uint_as_float(w << 16);
            g = __uint_as_float(w & 0xffff0000u);
        } else {
            f = R(__builtin_bit_cast(_Float16, uint16_t(w)));
            g = R(__builtin_bit_cast(_Float16, uint16_t(w >> 16)));
        }
    } else {
        f = R(bload<T>(src.f, s.nb[j] * (uint32_t)sizeof(T), (uint32_t)i * src.plane));
        g = R(bload<T>(src.g, s.nb[j] * (uint32_t)sizeof(T), (uint32_t)i * src.plane));
    }
}

// Lax-Wendroff step of one population from its three taps (Sec. 2.2):
// a0 - c[a0 - am] - c(1-c)/2 [ap - 2 a0 + am] = a0 + A (am - a0) + D (ap - a0).
template <class R>
__device__ __forceinline__ R lw3(const DevParams<R> &P, R am, R a0, R ap) {
    return fma(P.lwA, am - a0, fma(P.lwD, ap - a0, a0));
}

// The same step in flux form, out = a0 + [flux in through x - e/2] - [flux
// out through x + e/2]: each face flux is computed bit-identically by both of
// its nodes, so in FP32 storage the transfers between nodes cancel exactly and
// only the final addition rounds (the three-tap form loses the sub-ulp part of
// the net transfer at every node, which drifts the phase mass by ~1e-5 over
// 1e4 steps on a static droplet).
template <class R>
__device__ __forceinline__ R lw_flux(const DevParams<R> &P, R am, R a0, R ap) {
    const R fout = fma(P.h, ap - a0, P.c * a0);
    const R fin = fma(P.h, a0 - am, P.c * am);
    return a0 + (fin - fout);
}

// Same step in flux form next to a wall: out = a0 + [in flux] - [out flux],
// flux(x + e/2) = c a(x) + h (a(x+e) - a(x)), h = c(1-c)/2; a face beyond a
// wall takes the node itself as its far value and returns its outgoing flux
// into the opposite population (halfway bounce-back at c = 1).
template <class R>
__device__ __forceinline__ R lw_wall(const DevParams<R> &P, R am, R a0, R ap, R aopp,
                                     bool up_solid, bool dn_solid) {
    const R fout = dn_solid ? P.c * a0 : fma(P.h, ap - a0, P.c * a0);
    const R fin = up_solid ? P.c * aopp : fma(P.h, a0 - am, P.c * am);
    return a0 + (fin - fout);
}

// Gathers the post-propagation f and g of one node. WALLS adds the
// wall-aware recomputation (used only by wavefronts that contain a wall node).
template <Mode M, bool WALLS, class St>
__device__ __forceinline__ void gather(const Src<St> &src, const Site<St::Q> &s,
                                       const DevParams<typename St::R> &P,
                                       typename St::R (&fb)[St::Q], typename St::R (&gb)[St::Q]) {
    using R = typename St::R;
    using L = LatQ<St::Q>;
    constexpr int NQ = St::Q;
    R ph[NQ];  // phi_s at the stencil nodes x + e^_j (16-bit storage only)
    if constexpr (St::DEV) {
        unroll<0, NQ>([&](auto J) {
            constexpr int j = decltype(J)::value;
            if constexpr (M == LOCAL && j > 0) {
                ph[j] = R(0);
            } else {
                ph[j] = bload<float>(src.phis, s.nb[j] * 4u, 0u);
            }
        });
    }
    unroll<0, NQ>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int o = L::OPP[i];
        constexpr R t = wgt<R, NQ>(L::cls(i));
        if constexpr (M == LOCAL || i == 0) {
            R hf, hg;
            rawfg<St, i>(src, s, 0, hf, hg);
            if constexpr (St::DEV) {
                fb[i] = fma(P.iscale_f, hf, t * P.rho0);
                gb[i] = fma(P.iscale_g, hg, t * ph[0]);
            } else {
                fb[i] = hf;
                gb[i] = hg;
            }
        } else {
            R fm, gm;
            rawfg<St, i>(src, s, o, fm, gm);
            if constexpr (M == SHIFT) {
                if constexpr (St::DEV) {
                    fb[i] = fma(P.iscale_f, fm, t * P.rho0);
                    gb[i] = fma(P.iscale_g, gm, t * ph[o]);
                } else {
                    fb[i] = fm;
                    gb[i] = gm;
                }
            } else {
                R f0, fp, g0, gp;
                rawfg<St, i>(src, s, 0, f0, g0);
                rawfg<St, i>(src, s, i, fp, gp);
                if constexpr (St::DEV) {
                    // propagate the stored deviations and the phi_s bases apart;
                    // the deviations in the weighted form B h0 + A hm + D hp with
                    // the storage scale in the weights (FP16 values enter the
                    // FP32 fmas without a separate conversion)
                    const R tb = fma(t * P.lwA, ph[o] - ph[0], fma(t * P.lwD, ph[i] - ph[0], t * ph[0]));
                    fb[i] = fma(P.wA_f, fm, fma(P.wD_f, fp, fma(P.wB_f, f0, t * P.rho0)));
                    gb[i] = fma(P.wA_g, gm, fma(P.wD_g, gp, fma(P.wB_g, g0, tb)));
                } else {
                    fb[i] = lw_flux(P, fm, f0, fp);
                    gb[i] = lw_flux(P, gm, g0, gp);
                }
            }
        }
    });
    if constexpr (WALLS && M != LOCAL) {
        // wall-aware: the populations whose taps cross a wall face are
        // recomputed, on the lanes where they do, in flux form with
        // bounce-back from the full values of the taps and of the opposite
        // population at the node (the wall-free values above stand elsewhere)
        unroll<1, NQ>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int o = L::OPP[i];
            constexpr R t = wgt<R, NQ>(L::cls(i));
            const bool up = beyond_wall<i, 1>(s), dn = beyond_wall<i, -1>(s);
            if (up || dn) {
                auto full_f = [&](R h) -> R {
                    if constexpr (St::DEV) return fma(P.iscale_f, h, t * P.rho0);
                    else return h;
                };
                auto full_g = [&](R h, R phs) -> R {
                    if constexpr (St::DEV) return fma(P.iscale_g, h, t * phs);
                    else return h;
                };
                R hfm, hgm, hfo, hgo;
                rawfg<St, i>(src, s, o, hfm, hgm);
                rawfg<St, o>(src, s, 0, hfo, hgo);
                if constexpr (M == SHIFT) {
                    fb[i] = up ? full_f(hfo) : full_f(hfm);
                    gb[i] = up ? full_g(hgo, ph[0]) : full_g(hgm, ph[o]);
                } else {
                    R hf0, hfp, hg0, hgp;
                    rawfg<St, i>(src, s, 0, hf0, hg0);
                    rawfg<St, i>(src, s, i, hfp, hgp);
                    fb[i] = lw_wall(P, full_f(hfm), full_f(hf0), full_f(hfp), full_f(hfo), up, dn);
                    gb[i] = lw_wall(P, full_g(hgm, ph[o]), full_g(hg0, ph[0]), full_g(hgp, ph[i]),
                                    full_g(hgo, ph[0]), up, dn);
                }
            }
        });
    }
}

// --------------------------------------------------------------- moments
template <class R>
struct Macro {
    R phi, rho, omega_f;
    R u[3];
    R p;
    R n[3];
    R gnorm;      // |grad phi|
    R gradrho[3];
    R S[3];
};

// Moments of the post-propagation PDFs (Sec. 2.2 Eqs. 11-12, Sec. 2.3
// Eqs. 15, 17-19): phi = sum g, rho(phi), u = (sum f e + rho G/2)/rho,
// K1 = sum g e - phi u, n = -K1/|K1| times floor_weight(|K1|),
// S = 4 phi (1 - phi)/delta n, grad(phi) = (tau cs2 S - K1)/((tau + 1/2) cs2),
// grad(rho) = (rho1 - rho2) grad(phi), p = cs2 sum f + cs2/2 u.grad(rho).
// 1/x: the hardware reciprocal (1 ulp) in FP32, the division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Weight of the normal at a central moment (or a given gradient) of size k:
// 0 up to k1_eps, 1 from 2 k1_eps, linear between; with k1_eps = 0 it is 1
// for any k > 0 ((k - 0)/0 = inf). The normal is continuous in K1, so a
// perturbation of K1 near the floor moves it a little, never by a whole
// unit vector.
template <class R>
__device__ __forceinline__ R floor_weight(const DevParams<R> &P, R k) {
    return k > P.k1_eps ? fmin((k - P.k1_eps) / P.k1_eps, R(1)) : R(0);
}

// FD: grad(phi) is given (the finite-difference variant) instead of recovered
// from K1: n = grad/|grad| times floor_weight(|grad|), as for K1, S = s n,
// |grad phi| = |grad|.
// nw (wetting walls): the inward unit normal of the walls the node touches.
// The normal from K1 is turned, keeping its direction along the wall, until
// n . nw = -cos(theta); S and grad(phi) then follow from that normal. With
// the wall passing no phase flux, the wall-normal part of M (grad phi - s n)
// then vanishes at grad(phi) . nw = -s cos(theta), the contact-angle
// condition of the equilibrium profile. A normal with no part along the wall
// (|n_t| <= 1e-6) is kept.
// A wall node's inward normal for the wetting walls (on: the node touches a
// wetting wall).
template <class R>
struct WallNormal {
    R v[3];
    bool on;
};

template <bool FD = false, bool WET = false, class R, int NQ>
__device__ __forceinline__ Macro<R> moments(const DevParams<R> &P, const R (&fb)[NQ],
                                            const R (&gb)[NQ], const R *gfd = nullptr,
                                            const WallNormal<R> &nw = WallNormal<R>{},
                                            const Wet<R> &wp = Wet<R>{}) {
    Macro<R> m;
    R phi = gb[0], sf = fb[0];
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
        phi += gb[i];
        sf += fb[i];
    }
    m.phi = phi;
    m.rho = fma(P.drho, phi, P.rho2);
    const R eta = fma(P.deta, phi, P.eta2);
    const R irho = recip(m.rho);
    // omega_f = 1/(tau_rho + 1/2), tau_rho = eta/(rho cs2)
    m.omega_f = recip(fma(eta * irho, P.inv_cs2, R(0.5)));
    const R jx = first_moment<0>(fb), jy = first_moment<1>(fb), jz = first_moment<2>(fb);
    m.u[0] = fma(P.c, jx, R(0.5) * m.rho * P.G[0]) * irho;
    m.u[1] = fma(P.c, jy, R(0.5) * m.rho * P.G[1]) * irho;
    m.u[2] = fma(P.c, jz, R(0.5) * m.rho * P.G[2]) * irho;
    const R s = P.four_over_delta * phi * (R(1) - phi);
    if constexpr (FD) {
        const R gn = sqrt(fma(gfd[0], gfd[0], fma(gfd[1], gfd[1], gfd[2] * gfd[2])));
        const R wg = floor_weight(P, gn);
        const R rg = wg > R(0) ? wg * recip(gn) : R(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            m.n[a] = gfd[a] * rg;
            m.S[a] = s * m.n[a];
            m.gradrho[a] = P.drho * gfd[a];
        }
        m.gnorm = gn;
        const R ug = fma(m.u[0], m.gradrho[0], fma(m.u[1], m.gradrho[1], m.u[2] * m.gradrho[2]));
        m.p = P.cs2 * fma(R(0.5), ug, sf);
        return m;
    }
    const R K[3] = {fma(P.c, first_moment<0>(gb), -phi * m.u[0]),
                    fma(P.c, first_moment<1>(gb), -phi * m.u[1]),
                    fma(P.c, first_moment<2>(gb), -phi * m.u[2])};
    const R k = sqrt(fma(K[0], K[0], fma(K[1], K[1], K[2] * K[2])));
    const R wn = floor_weight(P, k);
    const bool has_n = wn > R(0);
    const R rk = has_n ? recip(k) : R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) m.n[a] = -K[a] * rk;  // the unit normal (or 0)
    bool turned = false;
    if constexpr (WET) {
        if (nw.on && has_n) {
            const R dn = fma(m.n[0], nw.v[0], fma(m.n[1], nw.v[1], m.n[2] * nw.v[2]));
            R t[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) t[a] = fma(-dn, nw.v[a], m.n[a]);
            const R tt = sqrt(fma(t[0], t[0], fma(t[1], t[1], t[2] * t[2])));
            if (tt > R(1e-6)) {
                const R st = wp.sin_theta / tt;
#pragma unroll
                for (int a = 0; a < 3; ++a) m.n[a] = fma(st, t[a], -wp.cos_theta * nw.v[a]);
                turned = true;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        m.n[a] *= wn;
        m.S[a] = s * m.n[a];
    }
    // |grad phi|: with n = -wn K1/|K1|, grad phi = n^ (tau cs2 s wn + |K1|)/((tau+1/2)cs2)
    m.gnorm = fabs(fma(P.tau_phi_cs2, s * wn, k)) * P.inv_tp;
    if (turned) {
        R gp[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) gp[a] = fma(P.tau_phi_cs2, m.S[a], -K[a]) * P.inv_tp;
        m.gnorm = sqrt(fma(gp[0], gp[0], fma(gp[1], gp[1], gp[2] * gp[2])));
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
        m.gradrho[a] = P.drho * fma(P.tau_phi_cs2, m.S[a], -K[a]) * P.inv_tp;
    const R ug = fma(m.u[0], m.gradrho[0], fma(m.u[1], m.gradrho[1], m.u[2] * m.gradrho[2]));
    m.p = P.cs2 * fma(R(0.5), ug, sf);
    return m;
}

// ------------------------------------------------------------- collision
// Equilibria and forcing of direction i, each divided by t_i:
//   feq/t  = p/cs2 + rho poly - Pi_s:(e e - cs2 I)/(2 cs4)      (Eq. 8, minus)
//   F/t    = poly (e - u).grad(rho)                             (App. A, S_i)
//          + [(e - u)/cs2 + (e.u) e/cs4].(rho G)                (Eq. 7, R_i)
//   geq/t  = phi (1 + poly) + tau_phi e.S                       (Eq. 14)
// with poly = e.u/cs2 + (e.u)^2/(2 cs4) - u^2/(2 cs2), so Gamma_i = t_i (1 + poly).
template <class R>
struct NodeCoef {
    R cu[3];          // c u
    R cgr[3];         // c grad(rho)
    R crG[3];         // c rho G
    R tS[3];          // tau_phi c S
    R a3;             // u^2/(2 cs2)
    R ug, uG;         // u.grad(rho), u.(rho G)
    R A0[4];          // p/cs2 - Pi_s:(e e - cs2 I)/(2cs4) minus the (e.n)^2 part, per speed class
    R kpsi;           // sigma |grad phi| c^2/(2 cs4): coefficient of (e^.n)^2
};

template <class R>
__device__ __forceinline__ NodeCoef<R> node_coef(const DevParams<R> &P, const Macro<R> &m) {
    NodeCoef<R> q;
    R rG[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        rG[a] = m.rho * P.G[a];
        q.cu[a] = P.c * m.u[a];
        q.cgr[a] = P.c * m.gradrho[a];
        q.crG[a] = P.c * rG[a];
        q.tS[a] = P.tau_phi_c * m.S[a];
    }
    const R uu = fma(m.u[0], m.u[0], fma(m.u[1], m.u[1], m.u[2] * m.u[2]));
    q.a3 = R(0.5) * uu * P.inv_cs2;
    q.ug = fma(m.u[0], m.gradrho[0], fma(m.u[1], m.gradrho[1], m.u[2] * m.gradrho[2]));
    q.uG = fma(m.u[0], rG[0], fma(m.u[1], rG[1], m.u[2] * rG[2]));
    const R nn = fma(m.n[0], m.n[0], fma(m.n[1], m.n[1], m.n[2] * m.n[2]));
    // Pi_s:(e e - cs2 I)/(2cs4) = ps [c^2 |e^|^2 - c^2 (e^.n)^2 - cs2 (3 - |n|^2)]
    const R ps = P.sigma * m.gnorm * P.half_inv_cs4;
    const R c2 = P.c * P.c;
    q.kpsi = ps * c2;
    const R base = fma(m.p, P.inv_cs2, ps * P.cs2 * (R(3) - nn));
    q.A0[0] = base;
    q.A0[1] = base - q.kpsi;
    q.A0[2] = base - R(2) * q.kpsi;
    q.A0[3] = base - R(3) * q.kpsi;   // corner vectors (D3Q27)
    return q;
}

// f* = f - omega_f (f - feq + F/2) + F ;  g* = g - omega_g (g - geq)   (Eqs. 10, 16)
// evaluated as the population plus its increment, f + [omega_f (feq - f) +
// (1 - omega_f/2) F], so that a node at equilibrium is an exact fixed point in
// floating point: the over-relaxed form (1 - omega) f + omega feq rounds the
// same way at every node of a uniform region and makes the phase mass drift
// coherently (about 3e-4 over 1e4 FP32 steps).
template <class R, int NQ>
__device__ __forceinline__ void collide(const DevParams<R> &P, const Macro<R> &m,
                                        const NodeCoef<R> &q, R (&fb)[NQ], R (&gb)[NQ]) {
    using L = LatQ<NQ>;
    const R of = m.omega_f, cf = R(1) - R(0.5) * of;
    const R og = P.omega_g;
    auto update = [&](auto I, R A, R B, R Gq) {
        constexpr int i = decltype(I)::value;
        constexpr R t = wgt<R, NQ>(L::cls(i));
        fb[i] = fma(of, fma(t, A, -fb[i]), fma(t * cf, B, fb[i]));
        gb[i] = fma(og, fma(t, Gq, -gb[i]), gb[i]);
    };
    {
        const R poly = -q.a3;
        update(std::integral_constant<int, 0>{}, fma(m.rho, poly, q.A0[0]),
               -poly * q.ug - q.uG * P.inv_cs2, fma(m.phi, poly, m.phi));
    }
    // the directions come in opposite pairs (i, i + 1) for odd i: every e.v
    // changes sign across a pair, so poly splits into an even part E and an
    // odd part O and the pair shares one evaluation of each projection
    const R uGs = q.uG * P.inv_cs2;
    unroll<0, (NQ - 1) / 2>([&](auto K) {
        constexpr int i = 2 * decltype(K)::value + 1;
        constexpr int cl = L::cls(i);
        const R eu = edot<i, NQ>(q.cu);
        const R en = edot<i, NQ>(m.n);
        const R eg = edot<i, NQ>(q.cgr);
        const R eG = edot<i, NQ>(q.crG);
        const R es = edot<i, NQ>(q.tS);
        const R E = fma(eu * eu, P.half_inv_cs4, -q.a3);
        const R O = eu * P.inv_cs2;
        const R pp = E + O, pm = E - O;
        const R kn = fma(q.kpsi * en, en, q.A0[cl]);
        const R t1 = fma(R(2) * P.half_inv_cs4 * eu, eG, -uGs);
        const R eGs = eG * P.inv_cs2;
        update(std::integral_constant<int, i>{}, fma(m.rho, pp, kn), fma(pp, eg - q.ug, t1 + eGs),
               fma(m.phi, pp, m.phi + es));
        update(std::integral_constant<int, i + 1>{}, fma(m.rho, pm, kn),
               fma(pm, -eg - q.ug, t1 - eGs), fma(m.phi, pm, m.phi - es));
    });
}


// ---------------------------------------------------------------- store
template <class St>
struct Dst {
    rsrc_t f, g, phis;
    uint32_t plane;
};

template <class St>
__device__ __forceinline__ Dst<St> make_dst(const Buf<St> &b, const DevParams<typename St::R> &P) {
    Dst<St> d;
    const uint32_t plane = P.plane_bytes;
    d.plane = plane;
    d.f = make_rsrc(b.f, (uint32_t)St::Q * plane);
    d.g = St::DEV ? d.f : make_rsrc(b.g, (uint32_t)St::Q * plane);
    d.phis = make_rsrc(b.phis, St::DEV ? (uint32_t)P.N * 4u : 0u);
    return d;
}

template <class St>
__device__ __forceinline__ void store(const Dst<St> &dst, uint32_t n,
                                      const DevParams<typename St::R> &P,
                                      const typename St::R (&fs)[St::Q],
                                      const typename St::R (&gs)[St::Q]) {
    using R = typename St::R;
    using T = typename St::T;
    using L = LatQ<St::Q>;
    constexpr int NQ = St::Q;
    const uint32_t voff = n * (uint32_t)(St::DEV ? 4 : sizeof(T));
    if constexpr (!St::DEV) {
        unroll<0, NQ>([&](auto I) {
            constexpr int i = decltype(I)::value;
            bstore<T>(T(fs[i]), dst.f, voff, (uint32_t)i * dst.plane);
            bstore<T>(T(gs[i]), dst.g, voff, (uint32_t)i * dst.plane);
        });
    } else {
        R phi_a = gs[0];
#pragma unroll
        for (int i = 1; i < NQ; ++i) phi_a += gs[i];
        R resid = R(0);
        unroll<0, NQ>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr R t = wgt<R, NQ>(L::cls(i));
            const T hf = encode<St>(P.scale_f * (fs[i] - t * P.rho0));
            const R dg = fma(-t, phi_a, gs[i]);
            const T hg = encode<St>(P.scale_g * dg);
            resid += fma(-P.iscale_g, decode<St>(hg), dg);
            const uint32_t w = uint32_t(__builtin_bit_cast(uint16_t, hf)) |
                               (uint32_t(__builtin_bit_cast(uint16_t, hg)) << 16);
            bstore<uint32_t>(w, dst.f, voff, (uint32_t)i * dst.plane);
        });
        // sum_i (t_i phi_s + 2^-k h_i) = sum_i g*_i: the storage rounding of g
        // is absorbed by phi_s, so the node keeps its phase mass
        bstore<float>(phi_a + resid, dst.phis, n * 4u, 0u);
    }
}

// ---------------------------------------------------------------- kernels
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Deterministic FP64 block sums of two values; thread 0 writes them.
__device__ __forceinline__ void block_sum2(double a, double b, double *out) {
    __shared__ double red[BLOCK / 64][2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
        red[wv][0] = a;
        red[wv][1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = red[0][0], sb = red[0][1];
        for (int w = 1; w < BLOCK / 64; ++w) {
            sa += red[w][0];
            sb += red[w][1];
        }
        out[0] = sa;
        out[1] = sb;
    }
}

// Phase-mass bookkeeping in FP64. Every few steps a step reports per-block
// sums of phi and of the interface weight w = max(phi (1 - phi), 0);
// massfix_kernel turns them into c = (M0 - M)/sum(w), and the next step adds
// c w t_i to the g of each node before its collision, which puts back, on the
// interface and isotropically, the phase mass that FP32 / 16-bit rounding
// has added or removed since the start (M0 = sum phi0 in FP64).
struct MassFix {
    int mode;               // bit 0: report partial sums; bit 1: apply coef
    double *partials;       // 2 per block
    const double *coef;     // c
    int block_off;          // index of this launch's first block among the step's blocks
};

template <class R>
__device__ __forceinline__ R mass_weight(R phi) {
    return fmax(phi * (R(1) - phi), R(0));
}

// Fused step: propagate (mode M) from src, moments, collide, store to dst.
// The wall-aware instance recomputes only the populations that cross a wall,
// on the lanes where they do. The host
// launches the wall-free instance (WALLS = false) over the tiles that touch
// no wall and the wall-aware one over the wall slabs: the wall path's code
// and registers then cost nothing in the interior.
// The pending phase-mass correction: g_i += t_i c w(phi) before the moments.
template <class R, int NQ>
__device__ __forceinline__ void apply_massfix(const MassFix &mf, R (&gb)[NQ]) {
    if (mf.mode & 2) {
        R phi = gb[0];
#pragma unroll
        for (int i = 1; i < NQ; ++i) phi += gb[i];
        const R cw = R(*mf.coef) * mass_weight(phi);
        unroll<0, NQ>([&](auto I) {
            constexpr int i = decltype(I)::value;
            gb[i] = fma(wgt<R, NQ>(LatQ<NQ>::cls(i)), cw, gb[i]);
        });
    }
}

// Isotropic central difference of the stored phi field,
// grad = 3 sum_i t_i e^_i [phi(x + e^_i) - phi(x - e^_i)]/2, summed over
// opposite pairs; a neighbour beyond a wall takes the node's own value (the
// finite-difference scheme the paper compares with, Sec. 3.4).
template <bool WALLS, class R, int NQ>
__device__ __forceinline__ void fd_grad(const DevParams<R> &P, const Site<NQ> &s, R (&g)[3]) {
    using L = LatQ<NQ>;
    const R *phi = P.phi_fd;
    const R p0 = phi[s.n];
    g[0] = g[1] = g[2] = R(0);
    unroll<0, (NQ - 1) / 2>([&](auto K) {
        constexpr int i = 2 * decltype(K)::value + 1;
        constexpr int o = L::OPP[i];
        R pp = phi[s.nb[i]], pm = phi[s.nb[o]];
        if constexpr (WALLS) {
            if (beyond_wall<i, -1>(s)) pp = p0;
            if (beyond_wall<i, 1>(s)) pm = p0;
        }
        const R d = R(3) * wgt<R, NQ>(L::cls(i)) * (pp - pm);
        if constexpr (L::EX[i] != 0) g[0] += R(L::EX[i]) * d;
        if constexpr (L::EY[i] != 0) g[1] += R(L::EY[i]) * d;
        if constexpr (L::EZ[i] != 0) g[2] += R(L::EZ[i]) * d;
    });
}

// Moments of one node; the wall-aware instances apply the wetting walls.
template <bool WALLS, bool FD, class R, int NQ>
__device__ __forceinline__ Macro<R> site_moments(const DevParams<R> &P, const Site<NQ> &s,
                                                 const R (&fb)[NQ], const R (&gb)[NQ],
                                                 const R (&gfd)[3], const Wet<R> &wp) {
    if constexpr (WALLS && !FD) {
        WallNormal<R> nw;
        const R l2 = wall_normal(s, nw.v);
        nw.on = wp.on && s.wall && l2 > R(0);
        return moments<FD, true>(P, fb, gb, gfd, nw, wp);
    } else {
        return moments<FD>(P, fb, gb, gfd);
    }
}

template <class St, Mode M, bool WALLS, bool FD>
__device__ __forceinline__ void step_body(const CBuf<St> &src, const Buf<St> &dst,
                                          const DevParams<typename St::R> &P, const MassFix &mf,
                                          const Wet<typename St::R> &wp) {
    using R = typename St::R;
    const Site<St::Q> s = make_site<St::Q>(P);
    double rep_phi = 0.0, rep_w = 0.0;
    if (s.valid) {
        const Src<St> in = make_src(src, P);
        R fb[St::Q], gb[St::Q];
        // Wavefronts still issuing their propagation loads go first, so the
        // loads of every wavefront are in flight sooner: 2-3% on the
        // wall-free D3Q19 steps in FP32 arithmetic (16-bit and FP32
        // storage); slower with walls, D3Q27 or FP64, which keep the
        // default. The arithmetic is unchanged.
        constexpr bool PRIO = !WALLS && !FD && St::Q == 19 && std::is_same<R, float>::value;
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
        gather<M, WALLS, St>(in, s, P, fb, gb);
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
        apply_massfix(mf, gb);
        R gfd[3];
        if constexpr (FD) fd_grad<WALLS>(P, s, gfd);
        const Macro<R> m = site_moments<WALLS, FD>(P, s, fb, gb, gfd, wp);
        if (mf.mode & 1) {
            rep_phi = m.phi;
            rep_w = mass_weight(m.phi);
        }
        const NodeCoef<R> q = node_coef(P, m);
        collide(P, m, q, fb, gb);
        store<St>(make_dst(dst, P), s.n, P, fb, gb);
    }
    if (mf.mode & 1)
        block_sum2(rep_phi, rep_w, mf.partials + 2 * ((size_t)mf.block_off + linear_block()));
}

template <class St, Mode M, bool WALLS, bool FD>
__global__ void __launch_bounds__(BLOCK) step_kernel(CBuf<St> src, Buf<St> dst,
                                                     DevParams<typename St::R> P, MassFix mf,
                                                     Wet<typename St::R> wp) {
    step_body<St, M, WALLS, FD>(src, dst, P, mf, wp);
}

// The same step held to 96 VGPRs (5 wavefronts per SIMD) for the wall-free
// 16-bit storage step, whose registers fit without spilling; at the
// compiler's own choice (97) it would run 4 per SIMD.
template <class St, Mode M, bool WALLS, bool FD>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(5, 8)))
step_kernel_o5(CBuf<St> src, Buf<St> dst, DevParams<typename St::R> P, MassFix mf) {
    step_body<St, M, WALLS, FD>(src, dst, P, mf, Wet<typename St::R>{0, 0, 1});
}

// First pass of the finite-difference variant: phi = sum of the propagated g
// (with the pending phase-mass correction, as the step applies it) into
// P.phi_fd, which the step then differences.
template <class St, Mode M, bool WALLS>
__global__ void __launch_bounds__(BLOCK) phi_kernel(CBuf<St> src, DevParams<typename St::R> P,
                                                    MassFix mf) {
    using R = typename St::R;
    const Site<St::Q> s = make_site<St::Q>(P);
    if (!s.valid) return;
    const Src<St> in = make_src(src, P);
    R fb[St::Q], gb[St::Q];
    gather<M, WALLS, St>(in, s, P, fb, gb);
    apply_massfix(mf, gb);
    R phi = gb[0];
#pragma unroll
    for (int i = 1; i < St::Q; ++i) phi += gb[i];
    P.phi_fd[s.n] = phi;
}

// Sums the per-block pairs in a fixed order (1024 threads, each a strided
// run of blocks, then the waves in order). init: *M0 = sum phi; otherwise
// *coef = (M0 - sum phi)/sum w (0 when there is no interface).
constexpr int RBLOCK = 1024;

__global__ void __launch_bounds__(RBLOCK) massfix_kernel(const double *partials, int nblocks,
                                                         double *M0, double *coef, int init) {
    __shared__ double red[RBLOCK / 64][2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += RBLOCK) {
        a += partials[2 * (size_t)k];
        b += partials[2 * (size_t)k + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
        red[wv][0] = a;
        red[wv][1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int w = 0; w < RBLOCK / 64; ++w) {
            sa += red[w][0];
            sb += red[w][1];
        }
        if (init) {
            *M0 = sa;
            *coef = 0.0;
        } else {
            *coef = sb > 0.0 ? (*M0 - sa) / sb : 0.0;
        }
    }
}

// Number of FP64 partial sums per block in the diagnostics reduction.
constexpr int NSUM = 17;
// layout: 0 sum_phi 1 mass 2-4 mom 5 ekin 6 umax(max) 7 phi_min(min)
//         8 phi_max(max) 9-11 com 12-14 phiu 15 l2_num 16 l2_den

struct FieldOut {
    void *phi, *u, *p;
    int dtype;                 // 0 double, 1 float
    double *pdf_f, *pdf_g;     // FP64 post-propagation PDFs (or NULL)
    const double *phi_ref;     // for the L2 entries (or NULL)
    double *partials;          // NSUM per block (or NULL)
};

// Moments of the state at t (propagation mode M from the previous buffer):
// fields, FP64 PDFs and/or per-block FP64 partial sums of the diagnostics.
template <class St, Mode M, bool WALLS, bool FD>
__global__ void __launch_bounds__(BLOCK) moments_kernel(CBuf<St> src, DevParams<typename St::R> P,
                                                        FieldOut out, Wet<typename St::R> wp) {
    using R = typename St::R;
    const Site<St::Q> s = make_site<St::Q>(P);
    double acc[NSUM];
#pragma unroll
    for (int k = 0; k < NSUM; ++k) acc[k] = 0.0;
    acc[7] = 1e300;
    acc[8] = -1e300;
    if (s.valid) {
        const Src<St> in = make_src(src, P);
        R fb[St::Q], gb[St::Q];
        gather<M, WALLS, St>(in, s, P, fb, gb);
        R gfd[3];
        if constexpr (FD) fd_grad<WALLS>(P, s, gfd);
        const Macro<R> m = site_moments<WALLS, FD>(P, s, fb, gb, gfd, wp);
        const size_t N = (size_t)P.N, n = s.n;
        if (out.phi) {
            if (out.dtype == 0) ((double *)out.phi)[n] = m.phi;
            else ((float *)out.phi)[n] = (float)m.phi;
        }
        if (out.u) {
            for (int a = 0; a < 3; ++a) {
                if (out.dtype == 0) ((double *)out.u)[a * N + n] = m.u[a];
                else ((float *)out.u)[a * N + n] = (float)m.u[a];
            }
        }
        if (out.p) {
            if (out.dtype == 0) ((double *)out.p)[n] = m.p;
            else ((float *)out.p)[n] = (float)m.p;
        }
        if (out.pdf_f) {
#pragma unroll
            for (int i = 0; i < St::Q; ++i) {
                out.pdf_f[i * N + n] = fb[i];
                out.pdf_g[i * N + n] = gb[i];
            }
        }
        if (out.partials) {
            const double phi = m.phi, rho = m.rho;
            const double ux = m.u[0], uy = m.u[1], uz = m.u[2];
            const double uu = ux * ux + uy * uy + uz * uz;
            acc[0] = phi;
            acc[1] = rho * phi;
            acc[2] = rho * ux;
            acc[3] = rho * uy;
            acc[4] = rho * uz;
            acc[5] = 0.5 * rho * uu;
            acc[6] = sqrt(uu);
            acc[7] = phi;
            acc[8] = phi;
            acc[9] = phi * s.x;
            acc[10] = phi * s.y;
            acc[11] = phi * s.z;
            acc[12] = phi * ux;
            acc[13] = phi * uy;
            acc[14] = phi * uz;
            if (out.phi_ref) {
                const double r = out.phi_ref[n];
                acc[15] = (phi - r) * (phi - r);
                acc[16] = r * r;
            }
        }
    }
    if (out.partials) {
        // deterministic block reduction: wave shuffles, then waves in order
        __shared__ double red[BLOCK / 64][NSUM];
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int k = 0; k < NSUM; ++k) {
            double v = acc[k];
            v = (k == 6 || k == 8) ? wave_max(v) : (k == 7 ? wave_min(v) : wave_sum(v));
            if (lane == 0) red[wv][k] = v;
        }
        __syncthreads();
        if (threadIdx.x < NSUM) {
            const int k = threadIdx.x;
            double v = red[0][k];
            for (int w = 1; w < BLOCK / 64; ++w) {
                const double x = red[w][k];
                v = (k == 6 || k == 8) ? fmax(v, x) : (k == 7 ? fmin(v, x) : v + x);
            }
            out.partials[(size_t)linear_block() * NSUM + k] = v;
        }
    }
}

// Final reduction of the per-block partials (one block of RBLOCK threads:
// each thread folds a strided run of blocks for all NSUM entries, then the
// waves are combined in order, so the result does not depend on timing).
__global__ void __launch_bounds__(RBLOCK) reduce_partials_kernel(const double *partials, int nblocks,
                                                                 double *result) {
    __shared__ double red[RBLOCK / 64][NSUM];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double acc[NSUM];
#pragma unroll
    for (int k = 0; k < NSUM; ++k) acc[k] = (k == 6 || k == 8) ? -1e300 : (k == 7 ? 1e300 : 0.0);
    for (int b = threadIdx.x; b < nblocks; b += RBLOCK) {
#pragma unroll
        for (int k = 0; k < NSUM; ++k) {
            const double x = partials[(size_t)b * NSUM + k];
            acc[k] = (k == 6 || k == 8) ? fmax(acc[k], x) : (k == 7 ? fmin(acc[k], x) : acc[k] + x);
        }
    }
#pragma unroll
    for (int k = 0; k < NSUM; ++k) {
        const double v = (k == 6 || k == 8) ? wave_max(acc[k]) : (k == 7 ? wave_min(acc[k]) : wave_sum(acc[k]));
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NSUM) {
        const int k = threadIdx.x;
        const bool mx = (k == 6 || k == 8), mn = (k == 7);
        double v = red[0][k];
        for (int w = 1; w < RBLOCK / 64; ++w) {
            const double x = red[w][k];
            v = mx ? fmax(v, x) : (mn ? fmin(v, x) : v + x);
        }
        result[k] = v;
    }
}

// Initial state (at t = 0, post-propagation) from phi0, u0, p0 (FP64):
// f = f_eq - F/2, g = g_eq - (tau_phi + 1/2) t_i e_i.grad(phi0), with
// grad(phi0) = 3 sum_i t_i e^_i [phi0(x + e^_i) - phi0(x - e^_i)]/2 (a
// neighbour beyond a wall takes the node's own value). Computed in FP64 and
// rounded once to the storage precision. Sets *bad if an input is
// non-finite or phi0 lies outside [-0.5, 1.5].
template <class St, bool WALLS>
__device__ __forceinline__ void init_node(const double *phi0, const double *u0, const double *p0,
                                          const DevParams<double> &P,
                                          const DevParams<typename St::R> &PR, const Buf<St> &dst,
                                          int *bad, const Site<St::Q> &s) {
    using R = typename St::R;
    using L = LatQ<St::Q>;
    constexpr int NQ = St::Q;
    const size_t N = (size_t)P.N, n = s.n;
    const double ph0 = phi0[n];
    double g[3] = {0.0, 0.0, 0.0};
    unroll<1, NQ>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = L::EX[i], ey = L::EY[i], ez = L::EZ[i];
        constexpr double t = wgt<double, NQ>(L::cls(i));
        double vp = phi0[s.nb[i]];
        double vm = phi0[s.nb[L::OPP[i]]];
        if constexpr (WALLS) {
            if (beyond_wall<i, -1>(s)) vp = ph0;
            if (beyond_wall<i, 1>(s)) vm = ph0;
        }
        const double d = 0.5 * (vp - vm) * t;
        g[0] += ex * d;
        g[1] += ey * d;
        g[2] += ez * d;
    });
#pragma unroll
    for (int a = 0; a < 3; ++a) g[a] *= 3.0;

    Macro<double> m;
    m.phi = ph0;
    m.rho = fma(P.drho, ph0, P.rho2);
    m.omega_f = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) m.u[a] = u0 ? u0[a * N + n] : 0.0;
    m.p = p0 ? p0[n] : 0.0;
    const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    const double s4 = P.four_over_delta * ph0 * (1.0 - ph0);
    const double wg = floor_weight(P, gn);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        m.n[a] = wg > 0.0 ? wg * g[a] / gn : 0.0;
        m.S[a] = s4 * m.n[a];
        m.gradrho[a] = P.drho * g[a];
    }
    m.gnorm = gn;
    if (!(isfinite(ph0) && isfinite(m.p) && isfinite(m.u[0]) && isfinite(m.u[1]) &&
          isfinite(m.u[2]) && ph0 >= -0.5 && ph0 <= 1.5))
        atomicOr(bad, 1);

    const NodeCoef<double> q = node_coef(P, m);
    R fo[NQ], go[NQ];
    unroll<0, NQ>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cl = L::cls(i);
        constexpr double t = wgt<double, NQ>(cl);
        double poly, A, B, Gq, eg0;
        if constexpr (i == 0) {
            poly = -q.a3;
            A = fma(m.rho, poly, q.A0[0]);
            B = -poly * q.ug - q.uG * P.inv_cs2;
            Gq = fma(m.phi, poly, m.phi);
            eg0 = 0.0;
        } else {
            const double eu = edot<i, NQ>(q.cu);
            const double en = edot<i, NQ>(m.n);
            const double eg = edot<i, NQ>(q.cgr);
            const double eG = edot<i, NQ>(q.crG);
            const double es = edot<i, NQ>(q.tS);
            poly = fma(eu, fma(eu, P.half_inv_cs4, P.inv_cs2), -q.a3);
            A = fma(m.rho, poly, fma(q.kpsi * en, en, q.A0[cl]));
            B = fma(poly, eg - q.ug, fma(eG - q.uG, P.inv_cs2, 2.0 * P.half_inv_cs4 * eu * eG));
            Gq = fma(m.phi, poly, m.phi + es);
            eg0 = P.c * edot<i, NQ>(g);
        }
        fo[i] = R(t * (A - 0.5 * B));
        go[i] = R(t * (Gq - (1.0 / P.omega_g) * eg0));
    });
    store<St>(make_dst(dst, PR), s.n, PR, fo, go);
}

template <class St, bool WALLS>
__global__ void __launch_bounds__(BLOCK) init_kernel(const double *phi0, const double *u0,
                                                     const double *p0, DevParams<double> P,
                                                     DevParams<typename St::R> PR, Buf<St> dst,
                                                     int *bad, double *partials) {
    const Site<St::Q> s = make_site<St::Q>(P);
    if (s.valid) init_node<St, WALLS>(phi0, u0, p0, P, PR, dst, bad, s);
    block_sum2(s.valid ? phi0[s.n] : 0.0, 0.0, partials + 2 * (size_t)linear_block());
}


// Loads FP64 post-propagation PDFs into the storage format (restart).
template <class St>
__global__ void __launch_bounds__(BLOCK) load_kernel(const double *f, const double *g,
                                                     DevParams<typename St::R> P, Buf<St> dst) {
    using R = typename St::R;
    const Site<St::Q> s = make_site<St::Q>(P);
    if (!s.valid) return;
    const size_t N = (size_t)P.N, n = s.n;
    R fo[St::Q], go[St::Q];
#pragma unroll
    for (int i = 0; i < St::Q; ++i) {
        fo[i] = R(f[i * N + n]);
        go[i] = R(g[i * N + n]);
    }
    store<St>(make_dst(dst, P), s.n, P, fo, go);
}

__global__ void clear_int_kernel(int *p) { *p = 0; }

}  // namespace cpf
