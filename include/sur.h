/*
 * sur.h -- C ABI of the learned surrogate that accompanies the
 * difference-free CPF-LBM solver: a 3D convolutional U-Net on a 2x-coarsened
 * grid that advances (phi, u, p) by a window of LBM steps, trained and run
 * with hand-written HIP kernels (BF16 matrix-core products with FP32
 * accumulation; FP32 master weights and Adam).
 *
 * The paper has no learned component; this ABI serves a surrogate
 * acceleration scheme around the solver: it generates training snapshots, the network
 * predicts windows on the coarse grid, per-window checks (phase mass, phi
 * range, velocity divergence) send a window back to the plain solver when
 * they fail, and the plain solver runs every re-synchronisation window.
 *
 * Tensors: activations are channels-last, [P][C] with P = nx*ny*nz points
 * (x fastest) and C a multiple of 16, stored as BF16 (uint16_t bit pattern,
 * round-to-nearest-even) unless the argument says float. Convolutions are
 * 3x3x3 with periodic wrap. Weights: FP32 master [27][cout][cin] with tap
 * t = (dx+1) + 3 (dy+1) + 9 (dz+1) reading the input at x + (dx, dy, dz);
 * packed BF16 copies are [27][cout][cin] (forward) and [27][cin][cout]
 * (data gradient).
 *
 * All pointers are device pointers owned by the caller; every call is
 * queued on `stream` (a hipStream_t, NULL = null stream) and returns
 * SUR_OK or SUR_EINVAL (bad sizes / NULL) or SUR_EDEVICE (launch failed).
 * Nothing is allocated by the library; sur_checks_noalloc alone keeps one
 * static device buffer per GPU (see there).
 */
#ifndef SUR_H
#define SUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SUR_OK = 0, SUR_EINVAL = -1, SUR_EDEVICE = -3 };

/* y[p][co] = act( bias[co] + sum_t sum_ci x[p + s d_t][ci] w[t][co][ci] ),
 * s = +1 (flip = 0) or -1 (flip = 1, the data-gradient form, with w the
 * [27][cin][cout] packing of the forward weights). bias may be NULL.
 * act: relu if relu != 0. If mask != NULL (BF16 [P][cout]) the result is
 * multiplied by (mask > 0) (the ReLU derivative of the layer below). Writes
 * y_bf16 and/or y_f32 (either may be NULL). cin, cout multiples of 16. */
int sur_conv3d(const void *x, int32_t cin, const void *w, const float *bias, int32_t cout,
               int32_t nx, int32_t ny, int32_t nz, int32_t flip, int32_t relu,
               const void *mask, void *y_bf16, float *y_f32, void *stream);

/* The decoder's first convolution of a level, reading its input concat in
 * place: sur_conv3d (flip = 0, no mask) of x = [xc[parent(p)][0 .. cc),
 * xf[p][0 .. fc)] with cin = cc + fc, bitwise the result of sur_concat_up2
 * followed by sur_conv3d, without writing the concat. xc is BF16 at half the
 * fine sizes (nx/2, ny/2, nz/2), parent(p) = (x/2, y/2, z/2); xf, y and the
 * sizes are fine-grid. w: the [27][cout][cc + fc] packing. Needs the tiled
 * kernel: nx a multiple of 16, ny and nz of 4, 16-byte aligned xc, xf and w;
 * otherwise SUR_EINVAL (concat first, then sur_conv3d). */
int sur_conv3d_cat(const void *xc, int32_t cc, const void *xf, int32_t fc, const void *w,
                   const float *bias, int32_t cout, int32_t nx, int32_t ny, int32_t nz,
                   int32_t relu, void *y_bf16, float *y_f32, void *stream);

/* The encoder's second convolution of a level with its pooling: sur_conv3d
 * (flip = 0, no mask) into BF16 y_bf16 [P][cout], and y_pool
 * [P/8][cout] = sur_pool2 of y_bf16 (the mean of each 2 x 2 x 2 cell of
 * the stored BF16 values, summed in FP32 in x, y, z order, rounded to BF16),
 * bitwise, in one pass (for cout = 16 only where nz is a multiple of 8 and
 * the grid holds at least four 16 x 4 x 8 point tiles per compute unit;
 * two passes otherwise). Needs the tiled kernel (nx a multiple of 16, ny
 * and nz of 4, 16-byte aligned x and w) and 8-byte aligned outputs;
 * otherwise SUR_EINVAL (call sur_conv3d, then sur_pool2). */
int sur_conv3d_pool(const void *x, int32_t cin, const void *w, const float *bias, int32_t cout,
                    int32_t nx, int32_t ny, int32_t nz, int32_t relu, void *y_bf16, void *y_pool,
                    void *stream);

/* Floats of scratch that sur_conv3d_wgrad needs for these sizes. */
size_t sur_wgrad_scratch_floats(int32_t cin, int32_t cout, int32_t nx, int32_t ny, int32_t nz);

/* dw[t][co][ci] = sum_p dy[p][co] x[p + d_t][ci], dbias[co] = sum_p dy[p][co]
 * (overwritten; FP32), from BF16 x [P][cin] and dy [P][cout]. Fixed
 * summation order (deterministic). scratch: >= sur_wgrad_scratch_floats. */
int sur_conv3d_wgrad(const void *x, int32_t cin, const void *dy, int32_t cout, int32_t nx,
                     int32_t ny, int32_t nz, float *scratch, size_t scratch_floats, float *dw,
                     float *dbias, void *stream);

/* BF16 packings of FP32 master weights w[27][cout][cin]: wf (same layout)
 * and wd[27][cin][cout] (per-tap transpose, for the data gradient). */
int sur_pack_weights(const float *w, int32_t cin, int32_t cout, void *wf, void *wd, void *stream);
/* The same for nlayers (<= 32) layers in one launch: layer l's FP32 weights
 * [27][cout[l]][cin[l]] start at float offset w_off[l] of w (host array); its
 * packings are written back to back into wf and wd, layer l at offset
 * sum_{k<l} 27 cin[k] cout[k] (BF16 elements). cin, cout: host arrays. */
int sur_pack_weights_all(const float *w, int32_t nlayers, const int64_t *w_off, const int32_t *cin,
                         const int32_t *cout, void *wf, void *wd, void *stream);

/* 2x2x2 average pooling of BF16 x (fine grid nx, ny, nz even) into BF16 y. */
int sur_pool2(const void *x, int32_t c, int32_t nx, int32_t ny, int32_t nz, void *y, void *stream);
/* dx[p][c] += dy[parent(p)][c] / 8 (FP32; fine grid sizes). */
int sur_pool2_bwd(const float *dy, int32_t c, int32_t nx, int32_t ny, int32_t nz, float *dx,
                  void *stream);
/* The gradient at an encoder output that feeds both the 2x2x2 pooling and
 * the skip connection, through its ReLU, in one pass (fine grid sizes):
 * dx[p][c'] = act[p][c'] > 0 ? dy[parent(p)][c'] / 8 + skip[p][skip_off + c']
 * : 0, dy FP32 on the coarse grid, skip FP32 [P][skip_stride], act BF16
 * [P][c]; written to FP32 dx and/or BF16 dx_bf16 [P][c] (either may be NULL,
 * not both). */
int sur_pool2_bwd_skip(const float *dy, int32_t c, int32_t nx, int32_t ny, int32_t nz,
                       const float *skip, int32_t skip_stride, int32_t skip_off, const void *act,
                       float *dx, void *dx_bf16, void *stream);
/* sur_upsample2_bwd through the ReLU of the coarse activation act (BF16
 * [P_coarse][c]), rounded to BF16: dx_bf16[q][c'] = bf16(act[q][c'] > 0 ?
 * sum over the 8 fine children p of dy[p][dyoff + c'] : 0) (coarse sizes). */
int sur_upsample2_bwd_mask(const float *dy, int32_t dystride, int32_t dyoff, int32_t c,
                           int32_t nx, int32_t ny, int32_t nz, const void *act, void *dx_bf16,
                           void *stream);
/* Nearest 2x upsampling of BF16 x [P_coarse][c] (coarse sizes) into channels
 * [yoff, yoff + c) of BF16 y [P_fine][ystride]. */
int sur_upsample2(const void *x, int32_t c, int32_t nx, int32_t ny, int32_t nz, void *y,
                  int32_t ystride, int32_t yoff, void *stream);
/* dx[q][c] = sum over the 8 fine children p of dy[p][dyoff + c] (FP32;
 * coarse sizes; dx overwritten). */
int sur_upsample2_bwd(const float *dy, int32_t dystride, int32_t dyoff, int32_t c, int32_t nx,
                      int32_t ny, int32_t nz, float *dx, void *stream);
/* The decoder's concat (fine grid sizes): y[p] = [xc[parent(p)][0 .. hc),
 * xf[p][0 .. fc)], BF16, y [P][hc + fc]: sur_upsample2 and sur_copy_channels
 * in one pass. */
int sur_concat_up2(const void *xc, int32_t hc, const void *xf, int32_t fc, int32_t nx, int32_t ny,
                   int32_t nz, void *y, void *stream);
/* y[p][yoff + c'] = x[p][c'] for c' < c (BF16 channel copy, for concat). */
int sur_copy_channels(const void *x, int32_t c, int64_t P, void *y, int32_t ystride,
                      int32_t yoff, void *stream);
/* dx[p][c'] += dy[p][dyoff + c'] (FP32). */
int sur_add_channels(const float *dy, int32_t dystride, int32_t dyoff, int32_t c, int64_t P,
                     float *dx, void *stream);
/* y = bf16(x), n values. */
int sur_to_bf16(const float *x, int64_t n, void *y, void *stream);
/* dx[i] *= (act[i] > 0) (FP32 gradient, BF16 activation), n values. */
int sur_relu_mask(float *dx, const void *act, int64_t n, void *stream);

/* Residual MSE on the first cu channels of FP32 pred/target [P][cs]:
 * L = sum_p sum_c wch[c] (pred - target)^2 / (P cu); grad = dL/dpred
 * ([P][cs], channels >= cu zero) in FP32 grad and/or BF16 grad_bf16 (either
 * may be NULL, not both). loss_out: one double (device), written after an
 * FP64 reduction in fixed order; scratch >= (P/256 + 1) doubles. */
int sur_mse(const float *pred, const float *target, int32_t cu, int32_t cs, int64_t P,
            const float *wch, float *grad, void *grad_bf16, double *scratch, double *loss_out,
            void *stream);

/* Adam step t >= 1 (Kingma & Ba, bias-corrected) on n FP32 weights. */
int sur_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float beta1,
             float beta2, float eps, int32_t t, void *stream);

/* Grid transfer between the solver's fine fields and the network's coarse
 * channels-last state (5 used channels of 16: phi, ux, uy, uz, p).
 *   coarsen: coarse[q][c] = mean over the 2x2x2 children of the fine field c
 *            (fine FP32 SoA phi[N], u[3N], p[N]; fine sizes even), scaled by
 *            1/scale[c]; written FP32 (and BF16 if coarse_bf16 != NULL).
 *   prolong_add: fine[c] += scale[c] * trilinear(delta)[c] (periodic;
 *            delta FP32 [Pc][16]; fine FP64 SoA phi, u, p). */
int sur_coarsen(const float *phi, const float *u, const float *p, int32_t nx, int32_t ny,
                int32_t nz, const float *scale, float *coarse_f32, void *coarse_bf16,
                void *stream);
int sur_prolong_add(const float *delta, int32_t cnx, int32_t cny, int32_t cnz,
                    const float *scale, double *phi, double *u, double *p, void *stream);

/* Level-set prolongation of a coarse change s0 -> s1 (FP32 [Pc][16], scaled
 * as coarsen writes them) onto fine FP64 fields (sizes 2 cnx, 2 cny, 2 cnz):
 *   u, p    += scale[c] * trilinear(s1 - s0)[c];
 *   phi     += Phi(Psi(phi) + dpsi) - Phi(Psi(phi)), dpsi = trilinear of
 *              Psi(s1[0]) - Psi(s0[0]) over the coarse nodes, with
 *              Psi(f) = (width/4) ln(f/(1-f)) (f clamped to [1e-4, 1-1e-4])
 *              and Phi(psi) = (1 + tanh(2 psi / width))/2 the equilibrium
 *              interface profile: the interface moves, its fine profile is
 *              kept;
 *   then phi += c max(phi(1-phi), 0) with c restoring the sum of phi before
 *   the update (FP64, fixed order).
 * sums (device, 4 doubles) receives {sum phi, sum w} before and after the
 * update, before the mass fix. scratch >= sur_prolong_update_scratch_doubles. */
size_t sur_prolong_update_scratch_doubles(int32_t cnx, int32_t cny, int32_t cnz);
int sur_prolong_update(const float *s0, const float *s1, int32_t cnx, int32_t cny, int32_t cnz,
                       const float *scale, double width, double *phi, double *u, double *p,
                       double *scratch, double *sums, void *stream);

/* Network input features from channels 0..4 of a coarse state [P][16]
 * (periodic central differences in coarse-grid units): channels 5..7 grad
 * phi, 8 u . grad phi, 9 div u, 10 phi (1 - phi), 11 |grad phi| (in place;
 * channels 12..15 untouched). */
int sur_features(float *state, int32_t nx, int32_t ny, int32_t nz, void *stream);

/* Per-window checks on a coarse FP32 state [P][16] (channel c is the
 * physical field / scale[c] as coarsen wrote it): FP64 results written to
 * out[7] = {sum phi, min phi, max phi, sum (div u)^2, sum |u|^2, P,
 * sum max(phi (1 - phi), 0)} (div by central differences on the coarse grid,
 * in coarse-grid units, of the scaled velocity). scratch >= 7 * (P/256 + 1)
 * doubles. */
int sur_checks(const float *state, int32_t nx, int32_t ny, int32_t nz, double *scratch,
               double *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * sur_checks with its per-block partial sums in a buffer the library keeps
 * in device memory instead of a caller's scratch. Same kernels and
 * summation order, so the same out[7] bit for bit. P = nx*ny*nz must not
 * exceed SUR_CHECKS_NOALLOC_MAX_POINTS (2^22, e.g. 256 x 128 x 128;
 * SUR_EINVAL otherwise). Each GPU holds one such buffer (917,504 bytes) from
 * the first call on it until the process ends; every call on that GPU
 * shares it, so calls that may overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller. Nothing needs to start
 * at zero: each call writes every partial it reads. The buffer's address is
 * looked up on the first call on each device, with the caller's current
 * device (the stream's device); SUR_EDEVICE if that lookup fails. Allocates
 * nothing. */
#define SUR_CHECKS_NOALLOC_MAX_POINTS (1L << 22)
int sur_checks_noalloc(const float *state, int32_t nx, int32_t ny, int32_t nz, double *out,
                       void *stream);

/* state[p][c] += rscale[c] * out[p][c] for c < cu (the network's residual,
 * in residual units, applied to the scaled state). With width > 0 channel 0
 * (phi) moves in level-set coordinates instead:
 * phi += Phi(Psi(phi) + rscale[0] out[p][0]) - Phi(Psi(phi)), with Psi and Phi
 * of sur_prolong_update (phi stays inside (0, 1) whatever the output). */
int sur_apply_residual(float *state, const float *out, const float *rscale, int32_t cu,
                       int64_t P, double width, void *stream);

/* target[p][c] = (s1[p][c] - s0[p][c]) / rscale[c] for c < cu, 0 beyond;
 * with width > 0 channel 0 is (Psi(s1) - Psi(s0)) / rscale[0]. */
int sur_residual_target(const float *s0, const float *s1, const float *rscale, int32_t cu,
                        int64_t P, double width, float *target, void *stream);

/* Puts the phase mass back to *target_mass: phi += c phi (1 - phi) with
 * c = (target - sum phi) / sum phi (1 - phi) from a sur_checks result (all on
 * the device: no host round trip). */
int sur_fix_mass(float *state, int64_t P, const double *checks_out, const double *target_mass,
                 void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SUR_H */
