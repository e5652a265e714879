// lbm.hip -- host side of the C ABI declared in include/lbm.h.
//
// The context holds two ping-pong population buffers A, B carved from the
// caller's workspace. The state "at time t" is the post-collision buffer
// cur, whose propagation gives the post-propagation PDFs at t + 1; the other
// buffer still holds what the last step read, so the moments at t are
// obtained by propagating it again (or, right after lbm_init / lbm_set_pdfs,
// by reading it in place, since it then holds the post-propagation PDFs at t).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "lbm.h"
#include "lbm_kernels.hpp"

using namespace cpf;

namespace {

// Discards an error that an earlier HIP call of another library left pending
// in this thread, so that the check after an entry point's launches
// (hipGetLastError) reports only that entry point's own failures.
inline void clear_stale_error() { (void)hipGetLastError(); }


constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Launch shape: one 256-thread block per tile of 2^tx_log2 x (256 >> tx_log2)
// nodes of one z-plane. The tile spans whole x-rows up to 128 nodes (a
// wavefront reads 64 contiguous nodes of a row, and a row's periodic wrap
// stays inside the tile): on the 128 x 512 x 128 Rayleigh-Taylor lattice this
// measured best among 32/64/128-wide tiles. LBM_TILE_X_LOG2, LBM_TILE_ORDER and
// LBM_TILE_BAND override the choice (tuning only; results do not depend on it).
struct TileCfg {
    int tx_log2, order, band;
};

int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

TileCfg tile_cfg(const lbm_params *P) {
    TileCfg t;
    int l = 0;
    while ((1 << l) < P->nx && l < 7) ++l;
    t.tx_log2 = env_int("LBM_TILE_X_LOG2", l);
    if (t.tx_log2 < 0 || t.tx_log2 > 8) t.tx_log2 = l;
    // default: XCD runs of the z-banded order with bands of 32 tile rows (the
    // y/z taps of a band stay in L2; on RT: FP32 14.6 against 13.9 GLUPS and
    // FP16 25.6 against 24.3 in the plain order)
    const int dflt_order = 2;
    t.order = env_int("LBM_TILE_ORDER", dflt_order);
    if (t.order < 0 || t.order > 2) t.order = dflt_order;
    t.band = env_int("LBM_TILE_BAND", 32);
    if (t.band < 1) t.band = 32;
    return t;
}

size_t num_tiles(const lbm_params *P, const TileCfg &t) {
    const size_t tw = (size_t)1 << t.tx_log2, th = (size_t)BLOCK >> t.tx_log2;
    const size_t ntx = (P->nx + tw - 1) / tw, nty = (P->ny + th - 1) / th;
    return ntx * nty * (size_t)P->nz;
}

size_t elem_bytes(int precision) {
    switch (precision) {
        case LBM_FP64: return 8;
        case LBM_FP32: return 4;
        default: return 2;
    }
}

bool is16(int precision) {
    return precision == LBM_FP32_FP16STORE || precision == LBM_FP32_BF16STORE;
}

// Populations per field: 19 (D3Q19; lattice = 0 means the same) or 27.
int num_pop(const lbm_params *P) { return P->lattice == 27 ? 27 : 19; }

// Bytes from one population plane to the next: N elements (16-bit storage:
// the 32-bit f/g words) rounded up to 256 B, plus a pad of 64 KiB + 256 B.
// With power-of-two strides (the usual lattice sizes) the 19 planes of a
// node fall on the same L2 sets and channels and evict each other's tap
// lines: unpadded, 256^3 FP16 steps fetch 1.6x the algorithmic bytes. The
// pad was measured best over 256 B .. 128 KiB on the Rayleigh-Taylor,
// rising-bubble and 256^3 lattices. LBM_PLANE_PAD (bytes) overrides it
// (tuning only; results do not depend on it).
size_t plane_pitch(const lbm_params *P) {
    const size_t N = (size_t)P->nx * P->ny * P->nz;
    const size_t pe = is16(P->precision) ? 4 : (size_t)elem_bytes(P->precision);
    const int pad = env_int("LBM_PLANE_PAD", 65536 + 256);
    return align_up(N * pe) + align_up((size_t)(pad > 0 ? pad : 0));
}

struct Layout {
    size_t pdf_bytes;      // f (16-bit storage: f and g words), Q planes
    size_t g_bytes;        // g, Q planes (0 for 16-bit storage)
    size_t phis_bytes;     // N floats (16-bit storage) or 0
    size_t buf_bytes;      // f + g + phis of one ping-pong buffer
    size_t partial_bytes;  // NSUM doubles per reduction block
    size_t result_bytes;
    size_t flag_bytes;
    size_t mf_bytes;
    size_t phifd_bytes;    // phi field of the finite-difference variant (or 0)
    size_t total;
};

Layout layout_of(const lbm_params *P) {
    Layout L;
    const size_t N = (size_t)P->nx * P->ny * P->nz;
    // the reduction partials are sized for the largest tile count any launch
    // shape can give (tile width 1)
    TileCfg narrow{0, 0, 1};
    const size_t nblocks = num_tiles(P, narrow);
    L.pdf_bytes = align_up((size_t)num_pop(P) * plane_pitch(P));
    L.g_bytes = is16(P->precision) ? 0 : L.pdf_bytes;
    L.phis_bytes = is16(P->precision) ? align_up(N * sizeof(float)) : 0;
    L.buf_bytes = L.pdf_bytes + L.g_bytes + L.phis_bytes;
    L.partial_bytes = align_up(nblocks * NSUM * sizeof(double));
    L.result_bytes = align_up(NSUM * sizeof(double));
    L.flag_bytes = kAlign;
    L.mf_bytes = kAlign;  // M0, coef
    L.phifd_bytes = P->normal_fd ? align_up(N * sizeof(double)) : 0;
    L.total = 2 * L.buf_bytes + L.partial_bytes + L.result_bytes + L.flag_bytes + L.mf_bytes +
              L.phifd_bytes;
    return L;
}

int validate(const lbm_params *P) {
    if (!P) return LBM_EINVAL;
    if (P->nx < 1 || P->ny < 1 || P->nz < 1) return LBM_EINVAL;
    if (P->lattice != 0 && P->lattice != 19 && P->lattice != 27) return LBM_EINVAL;
    // the finite-difference comparison scheme is built for D3Q19 only
    if (P->lattice == 27 && P->normal_fd) return LBM_EINVAL;
    // wetting walls act on the K1 normal; not combined with the FD scheme
    if (P->wetting != 0 && P->wetting != 1) return LBM_EINVAL;
    if (P->wetting && P->normal_fd) return LBM_EINVAL;
    if (P->wetting && !(std::isfinite(P->cos_theta) && P->cos_theta >= -1.0 && P->cos_theta <= 1.0))
        return LBM_EINVAL;
    const double N = (double)P->nx * P->ny * P->nz;
    const double Q = num_pop(P);
    if (Q * N >= 2147483647.0) return LBM_EINVAL;
    if (P->precision < LBM_FP64 || P->precision > LBM_FP32_BF16STORE) return LBM_EINVAL;
    // every population field is addressed through one 32-bit buffer range
    // (16-bit storage keeps f and g of a population in one 32-bit plane)
    if (Q * (double)plane_pitch(P) >= 4294967295.0) return LBM_EINVAL;
    const int nn[3] = {P->nx, P->ny, P->nz};
    for (int a = 0; a < 3; ++a) {
        if (P->wall[a] != 0 && P->wall[a] != 1) return LBM_EINVAL;
        if (P->wall[a] && nn[a] < 2) return LBM_EINVAL;
    }
    for (int k = 0; k < 2; ++k)
        if (P->store_log2[k] < -24 || P->store_log2[k] > 24) return LBM_EINVAL;
    if (P->check_every < 0 || P->mass_fix_every < 0) return LBM_EINVAL;
    if (P->normal_fd != 0 && P->normal_fd != 1) return LBM_EINVAL;
    auto fin = [](double x) { return std::isfinite(x); };
    if (!(fin(P->courant) && P->courant > 0.0 && P->courant <= 1.0)) return LBM_EINVAL;
    if (!(fin(P->rho1) && fin(P->rho2) && P->rho1 > 0.0 && P->rho2 > 0.0)) return LBM_EINVAL;
    if (!(fin(P->tau_rho1) && fin(P->tau_rho2) && P->tau_rho1 > 0.0 && P->tau_rho2 > 0.0))
        return LBM_EINVAL;
    if (!(fin(P->tau_phi) && P->tau_phi > 0.0)) return LBM_EINVAL;
    if (!(fin(P->sigma) && P->sigma >= 0.0)) return LBM_EINVAL;
    if (!(fin(P->delta) && P->delta > 0.0)) return LBM_EINVAL;
    if (!(fin(P->G[0]) && fin(P->G[1]) && fin(P->G[2]))) return LBM_EINVAL;
    if (!(fin(P->k1_eps) && P->k1_eps >= 0.0)) return LBM_EINVAL;
    if (!fin(P->p_ref)) return LBM_EINVAL;
    return LBM_OK;
}

FastDiv make_fastdiv(uint32_t d) {
    FastDiv f{0u, 0u, d < 1u ? 1u : d};
    if (f.d == 1u) return f;
    uint32_t l = 0;
    while ((1ull << l) < f.d) ++l;  // 2^(l-1) < d <= 2^l
    const unsigned __int128 num = (unsigned __int128)1 << (31 + l);
    f.m = (uint32_t)((num + f.d - 1) / f.d);
    f.s = l - 1;
    return f;
}

// Divisors of the tile decomposition of a launch box.
template <class R>
void set_divisors(DevParams<R> &d) {
    d.nfull = d.bnty / d.band;
    const int rem = d.bnty - d.nfull * d.band;
    d.d_ntx = make_fastdiv((uint32_t)d.ntx);
    d.d_nty = make_fastdiv((uint32_t)d.bnty);
    d.d_band = make_fastdiv((uint32_t)d.band);
    d.d_perband = make_fastdiv((uint32_t)(d.band * d.bnz));
    d.d_rem = make_fastdiv((uint32_t)(rem > 0 ? rem : 1));
}

template <class R>
DevParams<R> make_params(const lbm_params *P, const TileCfg &tc) {
    DevParams<R> d;
    d.nx = P->nx;
    d.ny = P->ny;
    d.nz = P->nz;
    d.N = P->nx * P->ny * P->nz;
    d.plane_bytes = (uint32_t)plane_pitch(P);
    for (int a = 0; a < 3; ++a) d.wall[a] = P->wall[a];
    d.tx_log2 = tc.tx_log2;
    d.ntx = (P->nx + (1 << tc.tx_log2) - 1) >> tc.tx_log2;
    d.nty = (P->ny + (BLOCK >> tc.tx_log2) - 1) / (BLOCK >> tc.tx_log2);
    d.ntiles = d.ntx * d.nty * P->nz;
    d.order = tc.order;
    d.band = tc.band < d.nty ? tc.band : d.nty;
    d.xq = d.ntiles / 8;
    d.xr = d.ntiles % 8;
    d.bty0 = 0;
    d.bnty = d.nty;
    d.btz0 = 0;
    d.bnz = P->nz;
    d.bty_step = 1;
    d.btz_step = 1;
    set_divisors(d);
    const double c = P->courant, cs2 = c * c / 3.0;
    const double eta1 = P->rho1 * cs2 * P->tau_rho1, eta2 = P->rho2 * cs2 * P->tau_rho2;
    d.c = R(c);
    d.h = R(0.5 * c * (1.0 - c));
    d.lwA = R(0.5 * c * (1.0 + c));
    d.lwD = R(-0.5 * c * (1.0 - c));
    d.cs2 = R(cs2);
    d.inv_cs2 = R(1.0 / cs2);
    d.half_inv_cs4 = R(0.5 / (cs2 * cs2));
    d.rho2 = R(P->rho2);
    d.drho = R(P->rho1 - P->rho2);
    d.eta2 = R(eta2);
    d.deta = R(eta1 - eta2);
    d.omega_g = R(1.0 / (P->tau_phi + 0.5));
    d.tau_phi_c = R(P->tau_phi * c);
    d.tau_phi_cs2 = R(P->tau_phi * cs2);
    d.inv_tp = R(1.0 / ((P->tau_phi + 0.5) * cs2));
    d.sigma = R(P->sigma);
    d.four_over_delta = R(4.0 / P->delta);
    for (int a = 0; a < 3; ++a) d.G[a] = R(P->G[a]);
    d.k1_eps = R(P->k1_eps);
    d.rho0 = R(P->p_ref / cs2);
    d.scale_f = R(std::ldexp(1.0, P->store_log2[0]));
    d.iscale_f = R(std::ldexp(1.0, -P->store_log2[0]));
    d.scale_g = R(std::ldexp(1.0, P->store_log2[1]));
    d.iscale_g = R(std::ldexp(1.0, -P->store_log2[1]));
    const double lwA = 0.5 * c * (1.0 + c), lwD = -0.5 * c * (1.0 - c), lwB = 1.0 - c * c;
    d.wA_f = R(std::ldexp(lwA, -P->store_log2[0]));
    d.wB_f = R(std::ldexp(lwB, -P->store_log2[0]));
    d.wD_f = R(std::ldexp(lwD, -P->store_log2[0]));
    d.wA_g = R(std::ldexp(lwA, -P->store_log2[1]));
    d.wB_g = R(std::ldexp(lwB, -P->store_log2[1]));
    d.wD_g = R(std::ldexp(lwD, -P->store_log2[1]));
    d.phi_fd = nullptr;
    return d;
}

template <class R>
Wet<R> make_wet(const lbm_params *P) {
    Wet<R> w;
    w.on = P->wetting;
    w.cos_theta = R(P->wetting ? P->cos_theta : 0.0);
    w.sin_theta = R(P->wetting ? std::sqrt(1.0 - P->cos_theta * P->cos_theta) : 1.0);
    return w;
}

}  // namespace

struct lbm_ctx {
    lbm_params P;
    Layout L;
    hipStream_t stream;
    char *ws;
    char *buf[2];
    double *partials;
    double *result;
    int *flag;
    double *mf;         // M0, coef of the phase-mass bookkeeping
    void *phifd;        // phi field of the finite-difference variant (or NULL)
    bool mf_pending;    // the next step applies coef
    TileCfg tc;
    int cur;            // buffer holding the post-collision state
    bool prev_local;    // the other buffer holds post-propagation PDFs at t
    int64_t t;
    int status;
    int nblocks;
};

namespace {

template <class St>
Buf<St> buf_of(lbm_ctx *c, int k) {
    Buf<St> b;
    b.f = (typename St::T *)c->buf[k];
    b.g = (typename St::T *)(c->buf[k] + c->L.pdf_bytes);
    b.phis = c->L.phis_bytes ? (float *)(c->buf[k] + c->L.pdf_bytes + c->L.g_bytes) : nullptr;
    return b;
}

template <class St>
CBuf<St> cbuf_of(lbm_ctx *c, int k) {
    Buf<St> b = buf_of<St>(c, k);
    return CBuf<St>{b.f, b.g, b.phis};
}

int check_launch(lbm_ctx *c) {
    if (hipGetLastError() != hipSuccess) {
        if (c) c->status = LBM_EDEVICE;
        return LBM_EDEVICE;
    }
    return LBM_OK;
}

// Launch grid of a tile box: (ntx, rows, planes) in the plain order, a 1-D
// run of tiles for the XCD-aware orders.
template <class R>
dim3 tile_grid(const DevParams<R> &P) {
    return P.order == 0 ? dim3((unsigned)P.ntx, (unsigned)P.bnty, (unsigned)P.bnz)
                        : dim3((unsigned)P.ntiles);
}

// Restricts a launch to tile rows ty0 + k ystep (k < nty) and planes
// tz0 + k zstep (k < nz).
template <class R>
DevParams<R> with_box(DevParams<R> d, int ty0, int nty, int tz0, int nz, int band, int ystep = 1,
                      int zstep = 1) {
    d.bty0 = ty0;
    d.bnty = nty;
    d.btz0 = tz0;
    d.bnz = nz;
    d.bty_step = ystep;
    d.btz_step = zstep;
    d.ntiles = d.ntx * nty * nz;
    d.band = band < nty ? band : nty;
    d.xq = d.ntiles / 8;
    d.xr = d.ntiles % 8;
    set_divisors(d);
    return d;
}

template <class St, Mode M, bool W, bool FD>
void launch_step(lbm_ctx *c, int src, int dst, const DevParams<typename St::R> &P, MassFix mf,
                 int &block_off) {
    mf.block_off = block_off;
    if constexpr (St::DEV && !W && !FD && St::Q == 19)
        hipLaunchKernelGGL((step_kernel_o5<St, M, W, FD>), tile_grid(P), dim3(BLOCK), 0,
                           c->stream, cbuf_of<St>(c, src), buf_of<St>(c, dst), P, mf);
    else
        hipLaunchKernelGGL((step_kernel<St, M, W, FD>), tile_grid(P), dim3(BLOCK), 0, c->stream,
                           cbuf_of<St>(c, src), buf_of<St>(c, dst), P, mf,
                           make_wet<typename St::R>(&c->P));
    block_off += P.ntiles;
}

// Parameters of a launch, with the phi field of the finite-difference variant.
template <class R>
DevParams<R> launch_params(lbm_ctx *c) {
    DevParams<R> P = make_params<R>(&c->P, c->tc);
    P.phi_fd = (R *)c->phifd;
    return P;
}

// First pass of the finite-difference variant: phi of the state the next
// launch reads from buffer src, split into interior and wall slabs as the
// step is.
template <class St, Mode M, bool W>
void launch_phi_box(lbm_ctx *c, int src, const DevParams<typename St::R> &P, const MassFix &mf) {
    hipLaunchKernelGGL((phi_kernel<St, M, W>), tile_grid(P), dim3(BLOCK), 0, c->stream,
                       cbuf_of<St>(c, src), P, mf);
}

template <class St, Mode M>
void launch_phi(lbm_ctx *c, int src, const MassFix &mf) {
    using R = typename St::R;
    const DevParams<R> P = launch_params<R>(c);
    const int *w = c->P.wall;
    if (!w[0] && !w[1] && !w[2]) {
        launch_phi_box<St, M, false>(c, src, P, mf);
        return;
    }
    const int ylo = w[1] ? 1 : 0, yhi = w[1] ? P.nty - 1 : P.nty;
    const int zlo = w[2] ? 1 : 0, zhi = w[2] ? P.nz - 1 : P.nz;
    if (w[0] || yhi <= ylo || zhi <= zlo) {
        launch_phi_box<St, M, true>(c, src, P, mf);
        return;
    }
    const int band = c->tc.band;
    launch_phi_box<St, M, false>(c, src, with_box(P, ylo, yhi - ylo, zlo, zhi - zlo, band), mf);
    if (w[1]) launch_phi_box<St, M, true>(c, src, with_box(P, 0, 2, 0, P.nz, band, P.nty - 1), mf);
    if (w[2])
        launch_phi_box<St, M, true>(c, src, with_box(P, ylo, yhi - ylo, 0, 2, band, 1, P.nz - 1), mf);
}

// Periodic lattices: one wall-free launch. Walls in y and/or z: the interior
// box of tiles runs the wall-free instance, the wall slabs (first and last
// tile row; first and last plane) one wall-aware launch each. Walls in x
// touch every tile row: one wall-aware launch.
template <class St, Mode M, bool FD>
void launch_step_w(lbm_ctx *c, int src, int dst, const MassFix &mf) {
    using R = typename St::R;
    const DevParams<R> P = launch_params<R>(c);
    const int *w = c->P.wall;
    int off = 0;
    if (!w[0] && !w[1] && !w[2]) {
        launch_step<St, M, false, FD>(c, src, dst, P, mf, off);
        return;
    }
    const int ylo = w[1] ? 1 : 0, yhi = w[1] ? P.nty - 1 : P.nty;
    const int zlo = w[2] ? 1 : 0, zhi = w[2] ? P.nz - 1 : P.nz;
    if (w[0] || yhi <= ylo || zhi <= zlo) {
        launch_step<St, M, true, FD>(c, src, dst, P, mf, off);
        return;
    }
    const int band = c->tc.band;
    launch_step<St, M, false, FD>(c, src, dst, with_box(P, ylo, yhi - ylo, zlo, zhi - zlo, band),
                                  mf, off);
    if (w[1])  // first and last tile row, all planes
        launch_step<St, M, true, FD>(c, src, dst, with_box(P, 0, 2, 0, P.nz, band, P.nty - 1), mf,
                                     off);
    if (w[2])  // first and last plane, the interior tile rows
        launch_step<St, M, true, FD>(c, src, dst,
                                     with_box(P, ylo, yhi - ylo, 0, 2, band, 1, P.nz - 1), mf, off);
}

template <class St, Mode M>
void launch_step_fd(lbm_ctx *c, int src, int dst, const MassFix &mf) {
    if constexpr (St::Q == 19) {
        if (c->P.normal_fd) {
            MassFix apply = mf;
            apply.mode &= 2;
            launch_phi<St, M>(c, src, apply);
            launch_step_w<St, M, true>(c, src, dst, mf);
            return;
        }
    }
    launch_step_w<St, M, false>(c, src, dst, mf);
}

template <class St>
void step_dispatch(lbm_ctx *c, Mode m, int src, int dst, const MassFix &mf) {
    switch (m) {
        case LOCAL: launch_step_fd<St, LOCAL>(c, src, dst, mf); break;
        case SHIFT: launch_step_fd<St, SHIFT>(c, src, dst, mf); break;
        default: launch_step_fd<St, LW>(c, src, dst, mf); break;
    }
}

// Calls F::template run<St>(args...) with the storage type of the context's
// precision and lattice.
template <class F, class... A>
void with_storage(const lbm_ctx *c, A &&...args) {
    const bool q27 = num_pop(&c->P) == 27;
    switch (c->P.precision) {
        case LBM_FP64:
            q27 ? F::template run<Q27<SF64>>(args...) : F::template run<SF64>(args...);
            break;
        case LBM_FP32:
            q27 ? F::template run<Q27<SF32>>(args...) : F::template run<SF32>(args...);
            break;
        case LBM_FP32_FP16STORE:
            q27 ? F::template run<Q27<SH16>>(args...) : F::template run<SH16>(args...);
            break;
        default:
            q27 ? F::template run<Q27<SB16>>(args...) : F::template run<SB16>(args...);
            break;
    }
}

struct StepOp {
    template <class St>
    static void run(lbm_ctx *c, Mode m, int src, int dst, const MassFix &mf) {
        step_dispatch<St>(c, m, src, dst, mf);
    }
};

void step_any(lbm_ctx *c, Mode m, int src, int dst, int mf_mode = 0) {
    const MassFix mf{mf_mode, c->partials, c->mf + 1, 0};
    with_storage<StepOp>(c, c, m, src, dst, mf);
}

Mode prop_mode(const lbm_ctx *c) { return c->P.courant == 1.0 ? SHIFT : LW; }

template <class St, Mode M, bool W>
void launch_moments(lbm_ctx *c, const FieldOut &o) {
    using R = typename St::R;
    const DevParams<R> P = launch_params<R>(c);
    if constexpr (St::Q == 19) {
        if (c->P.normal_fd) {
            launch_phi<St, M>(c, c->cur ^ 1, MassFix{0, nullptr, nullptr, 0});
            hipLaunchKernelGGL((moments_kernel<St, M, W, true>), tile_grid(P), dim3(BLOCK), 0,
                               c->stream, cbuf_of<St>(c, c->cur ^ 1), P, o, make_wet<R>(&c->P));
            return;
        }
    }
    hipLaunchKernelGGL((moments_kernel<St, M, W, false>), tile_grid(P), dim3(BLOCK), 0,
                       c->stream, cbuf_of<St>(c, c->cur ^ 1), P, o, make_wet<R>(&c->P));
}

template <class St, Mode M>
void moments_w(lbm_ctx *c, const FieldOut &o) {
    const bool walls = c->P.wall[0] || c->P.wall[1] || c->P.wall[2];
    if (walls) launch_moments<St, M, true>(c, o);
    else launch_moments<St, M, false>(c, o);
}

template <class St>
void moments_dispatch(lbm_ctx *c, const FieldOut &o) {
    if (c->prev_local) moments_w<St, LOCAL>(c, o);
    else if (prop_mode(c) == SHIFT) moments_w<St, SHIFT>(c, o);
    else moments_w<St, LW>(c, o);
}

struct MomentsOp {
    template <class St>
    static void run(lbm_ctx *c, const FieldOut &o) {
        moments_dispatch<St>(c, o);
    }
};

void moments_any(lbm_ctx *c, const FieldOut &o) { with_storage<MomentsOp>(c, c, o); }

template <class St>
void launch_init(lbm_ctx *c, const double *phi0, const double *u0, const double *p0, int dst) {
    using R = typename St::R;
    const DevParams<double> PD = make_params<double>(&c->P, c->tc);
    const DevParams<R> PR = make_params<R>(&c->P, c->tc);
    const bool walls = c->P.wall[0] || c->P.wall[1] || c->P.wall[2];
    if (walls)
        hipLaunchKernelGGL((init_kernel<St, true>), tile_grid(PR), dim3(BLOCK), 0, c->stream,
                           phi0, u0, p0, PD, PR, buf_of<St>(c, dst), c->flag, c->partials);
    else
        hipLaunchKernelGGL((init_kernel<St, false>), tile_grid(PR), dim3(BLOCK), 0, c->stream,
                           phi0, u0, p0, PD, PR, buf_of<St>(c, dst), c->flag, c->partials);
}

struct InitOp {
    template <class St>
    static void run(lbm_ctx *c, const double *phi0, const double *u0, const double *p0, int dst) {
        launch_init<St>(c, phi0, u0, p0, dst);
    }
};

void init_any(lbm_ctx *c, const double *phi0, const double *u0, const double *p0, int dst) {
    with_storage<InitOp>(c, c, phi0, u0, p0, dst);
}

template <class St>
void launch_load(lbm_ctx *c, const double *f, const double *g, int dst) {
    using R = typename St::R;
    const DevParams<R> P = make_params<R>(&c->P, c->tc);
    hipLaunchKernelGGL((load_kernel<St>), tile_grid(P), dim3(BLOCK), 0, c->stream, f, g, P,
                       buf_of<St>(c, dst));
}

struct LoadOp {
    template <class St>
    static void run(lbm_ctx *c, const double *f, const double *g, int dst) {
        launch_load<St>(c, f, g, dst);
    }
};

void load_any(lbm_ctx *c, const double *f, const double *g, int dst) {
    with_storage<LoadOp>(c, c, f, g, dst);
}

// Runs the diagnostics reduction of the state at t into c->result (device).
int reduce_diag(lbm_ctx *c, const double *phi_ref) {
    FieldOut o{};
    o.phi_ref = phi_ref;
    o.partials = c->partials;
    moments_any(c, o);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(RBLOCK), 0, c->stream,
                       (const double *)c->partials, c->nblocks, c->result);
    return check_launch(c);
}

// State at the current time from fields (device FP64): post-propagation
// PDFs into buffer 1, M0 = sum phi (FP64) for the phase-mass bookkeeping, one
// collision into buffer 0; checks the inputs (synchronises the stream).
int build_state(lbm_ctx *c, const double *d_phi, const double *d_u, const double *d_p) {
    hipLaunchKernelGGL(clear_int_kernel, dim3(1), dim3(1), 0, c->stream, c->flag);
    init_any(c, d_phi, d_u, d_p, 1);
    hipLaunchKernelGGL(massfix_kernel, dim3(1), dim3(RBLOCK), 0, c->stream,
                       (const double *)c->partials, c->nblocks, c->mf, c->mf + 1, 1);
    step_any(c, LOCAL, 1, 0);
    c->cur = 0;
    c->prev_local = true;
    c->mf_pending = false;
    int bad = 0;
    if (check_launch(c) != LBM_OK ||
        hipMemcpyAsync(&bad, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return LBM_EDEVICE;
    return bad ? LBM_EINVAL : LBM_OK;
}

}  // namespace

extern "C" {

void lbm_lattice(int32_t e[57], double t[19]) { lbm_lattice_q(19, e, t); }

int lbm_lattice_q(int32_t q, int32_t *e, double *t) {
    if ((q != 19 && q != 27) || !e || !t) return LBM_EINVAL;
    for (int i = 0; i < q; ++i) {
        const int ex = q == 27 ? LatQ<27>::EX[i] : LatQ<19>::EX[i];
        const int ey = q == 27 ? LatQ<27>::EY[i] : LatQ<19>::EY[i];
        const int ez = q == 27 ? LatQ<27>::EZ[i] : LatQ<19>::EZ[i];
        e[3 * i + 0] = ex;
        e[3 * i + 1] = ey;
        e[3 * i + 2] = ez;
        const int cl = ex * ex + ey * ey + ez * ez;
        if (q == 27)
            t[i] = cl == 0 ? 8.0 / 27.0 : (cl == 1 ? 2.0 / 27.0 : (cl == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
        else
            t[i] = cl == 0 ? 1.0 / 3.0 : (cl == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    return LBM_OK;
}

int lbm_workspace_bytes(const lbm_params *P, size_t *bytes) {
    if (!bytes) return LBM_EINVAL;
    const int rc = validate(P);
    if (rc != LBM_OK) return rc;
    *bytes = layout_of(P).total;
    return LBM_OK;
}

int lbm_init(const lbm_params *P, void *d_workspace, size_t bytes, void *stream,
             const double *d_phi0, const double *d_u0, const double *d_p0, lbm_ctx **out) {
    clear_stale_error();
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    int rc = validate(P);
    if (rc != LBM_OK) return rc;
    if (!d_workspace || !d_phi0) return LBM_EINVAL;
    if (((uintptr_t)d_workspace) % kAlign != 0) return LBM_EINVAL;
    const Layout L = layout_of(P);
    if (bytes < L.total) return LBM_ENOMEM;

    lbm_ctx *c = new (std::nothrow) lbm_ctx;
    if (!c) return LBM_ENOMEM;
    std::memset(c, 0, sizeof(*c));
    c->P = *P;
    c->L = L;
    c->stream = (hipStream_t)stream;
    c->ws = (char *)d_workspace;
    c->buf[0] = c->ws;
    c->buf[1] = c->ws + L.buf_bytes;
    c->partials = (double *)(c->ws + 2 * L.buf_bytes);
    c->result = (double *)(c->ws + 2 * L.buf_bytes + L.partial_bytes);
    c->flag = (int *)(c->ws + 2 * L.buf_bytes + L.partial_bytes + L.result_bytes);
    c->mf = (double *)(c->ws + 2 * L.buf_bytes + L.partial_bytes + L.result_bytes + L.flag_bytes);
    c->phifd = L.phifd_bytes ? (void *)(c->ws + 2 * L.buf_bytes + L.partial_bytes + L.result_bytes +
                                        L.flag_bytes + L.mf_bytes)
                             : nullptr;
    c->tc = tile_cfg(P);
    c->nblocks = (int)num_tiles(P, c->tc);
    c->mf_pending = false;
    c->status = LBM_OK;

    c->t = 0;
    const int rc2 = build_state(c, d_phi0, d_u0, d_p0);
    if (rc2 != LBM_OK) {
        delete c;
        return rc2;
    }
    *out = c;
    return LBM_OK;
}

int lbm_reset(lbm_ctx *c, const double *d_phi, const double *d_u, const double *d_p, int64_t t) {
    clear_stale_error();
    if (!c || !d_phi || t < 0) return LBM_EINVAL;
    if (c->status == LBM_EDEVICE) return LBM_ESTATE;
    const int rc = build_state(c, d_phi, d_u, d_p);
    if (rc == LBM_OK) {
        c->t = t;
        c->status = LBM_OK;
    } else {
        // the buffers now hold the rejected fields' state: refuse lbm_step
        // until a reset succeeds
        c->status = rc == LBM_EDEVICE ? LBM_EDEVICE : LBM_ESTATE;
    }
    return rc;
}

int lbm_step(lbm_ctx *c, int64_t n) {
    clear_stale_error();
    if (!c || n < 0) return LBM_EINVAL;
    if (c->status != LBM_OK) return LBM_ESTATE;
    const Mode m = prop_mode(c);
    const int mfe = c->P.mass_fix_every;
    for (int64_t k = 0; k < n; ++k) {
        int mf_mode = c->mf_pending ? 2 : 0;
        if (mfe > 0 && (c->t + 1) % mfe == 0) mf_mode |= 1;
        step_any(c, m, c->cur, c->cur ^ 1, mf_mode);
        c->mf_pending = false;
        if (mf_mode & 1) {
            hipLaunchKernelGGL(massfix_kernel, dim3(1), dim3(RBLOCK), 0, c->stream,
                               (const double *)c->partials, c->nblocks, c->mf, c->mf + 1, 0);
            c->mf_pending = true;
        }
        c->cur ^= 1;
        c->prev_local = false;
        c->t += 1;
        if (c->P.check_every > 0 && c->t % c->P.check_every == 0) {
            if (reduce_diag(c, nullptr) != LBM_OK) return LBM_EDEVICE;
            double r[NSUM];
            if (hipMemcpyAsync(r, c->result, sizeof(r), hipMemcpyDeviceToHost, c->stream) !=
                    hipSuccess ||
                hipStreamSynchronize(c->stream) != hipSuccess) {
                c->status = LBM_EDEVICE;
                return LBM_EDEVICE;
            }
            const double cs = c->P.courant / std::sqrt(3.0);
            bool ok = true;
            for (int k2 = 0; k2 < NSUM; ++k2) ok = ok && std::isfinite(r[k2]);
            if (!ok || r[6] >= cs) {
                c->status = LBM_EUNSTABLE;
                return LBM_EUNSTABLE;
            }
        }
    }
    return check_launch(c);
}

int lbm_fields(lbm_ctx *c, void *d_phi, void *d_u, void *d_p, int32_t dtype) {
    clear_stale_error();
    if (!c || (dtype != 0 && dtype != 1)) return LBM_EINVAL;
    if (c->status == LBM_EDEVICE) return LBM_ESTATE;
    FieldOut o{};
    o.phi = d_phi;
    o.u = d_u;
    o.p = d_p;
    o.dtype = dtype;
    moments_any(c, o);
    return check_launch(c);
}

int lbm_diagnostics(lbm_ctx *c, const double *d_phi_ref, lbm_diag *out) {
    clear_stale_error();
    if (!c || !out) return LBM_EINVAL;
    if (c->status == LBM_EDEVICE) return LBM_ESTATE;
    if (reduce_diag(c, d_phi_ref) != LBM_OK) return LBM_EDEVICE;
    double r[NSUM];
    if (hipMemcpyAsync(r, c->result, sizeof(r), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        c->status = LBM_EDEVICE;
        return LBM_EDEVICE;
    }
    out->step = c->t;
    out->sum_phi = r[0];
    out->mass = r[1];
    out->mom[0] = r[2];
    out->mom[1] = r[3];
    out->mom[2] = r[4];
    out->ekin = r[5];
    out->umax = r[6];
    out->phi_min = r[7];
    out->phi_max = r[8];
    for (int a = 0; a < 3; ++a) {
        out->com[a] = r[9 + a];
        out->phiu[a] = r[12 + a];
    }
    out->l2_num = r[15];
    out->l2_den = r[16];
    return LBM_OK;
}

int lbm_get_pdfs(lbm_ctx *c, double *d_f, double *d_g) {
    clear_stale_error();
    if (!c || !d_f || !d_g) return LBM_EINVAL;
    if (c->status == LBM_EDEVICE) return LBM_ESTATE;
    FieldOut o{};
    o.pdf_f = d_f;
    o.pdf_g = d_g;
    moments_any(c, o);
    return check_launch(c);
}

int lbm_set_pdfs(lbm_ctx *c, const double *d_f, const double *d_g) {
    clear_stale_error();
    if (!c || !d_f || !d_g) return LBM_EINVAL;
    if (c->status == LBM_EDEVICE) return LBM_ESTATE;
    const int prev = c->cur ^ 1;
    load_any(c, d_f, d_g, prev);
    // collide in place of a step; the loaded state's sum of phi becomes the
    // target of the phase-mass bookkeeping
    step_any(c, LOCAL, prev, c->cur, 1);
    hipLaunchKernelGGL(massfix_kernel, dim3(1), dim3(RBLOCK), 0, c->stream,
                       (const double *)c->partials, c->nblocks, c->mf, c->mf + 1, 1);
    c->mf_pending = false;
    c->prev_local = true;
    c->status = LBM_OK;
    return check_launch(c);
}

int64_t lbm_time(const lbm_ctx *c) { return c ? c->t : -1; }

void lbm_destroy(lbm_ctx *c) { delete c; }

const char *lbm_strerror(int status) {
    switch (status) {
        case LBM_OK: return "ok";
        case LBM_EINVAL: return "invalid argument";
        case LBM_ENOMEM: return "workspace too small";
        case LBM_EDEVICE: return "HIP device error";
        case LBM_EUNSTABLE: return "simulation became unstable";
        case LBM_ESTATE: return "context is in an error state";
        default: return "unknown status";
    }
}

}  // extern "C"
