/*
 * lbm.h -- C ABI of the MI355X difference-free conservative phase-field
 * lattice Boltzmann solver (Zhao, Patel & Lee, arXiv 2407.12263).
 *
 * One time step advances two populations per lattice node (D3Q19, or D3Q27
 * with lbm_params.lattice = 27):
 *   f  -- the one-fluid hydrodynamic PDF: sum f = p/c_s^2, surface tension as
 *         a continuous surface stress inside its equilibrium (Sec. 2.2,
 *         Eqs. 6-12; the surface-stress term enters f_eq with a minus sign so
 *         that the second moment is rho u u + p I - Pi_s, App. A);
 *   g  -- the conservative phase-field PDF: sum g = phi, its first central
 *         moment K1 gives the interface normal and grad(phi) locally (Sec. 2.3,
 *         Eqs. 13-19), so no finite difference between nodes is taken.
 * Each step is one fused pass: Lax-Wendroff propagation (Sec. 2.2, Courant
 * number c) of the stored post-collision PDFs, moment recovery, and the
 * Crank-Nicolson collision of both populations (Eqs. 10, 16).
 *
 * Units: grid units, dx = dt = 1, discrete velocities c*e^_i (e^_i integer
 * lattice vectors), c_s^2 = c^2/3, nu = tau_rho c_s^2, M = tau_phi c_s^2.
 * Scalar fields are structure-of-arrays with index n = x + nx*(y + ny*z);
 * a vector field stores component a at a*N + n; a PDF field stores
 * population i at i*N + n, in the library's own lattice order (see
 * lbm_lattice_q); Q = 19 or 27 populations per field.
 *
 * Ownership: the caller owns every device buffer (workspace, inputs,
 * outputs) and the stream; the library only borrows them. The library owns
 * the host-side context, freed by lbm_destroy, and never allocates device
 * memory. All work is queued on the caller's stream; only lbm_diagnostics
 * and lbm_init block (they synchronise that stream). Calls on one context must not run
 * concurrently.
 *
 * Errors: every call returns an lbm_status. A failed lbm_init leaves *out
 * NULL. After LBM_EDEVICE or LBM_EUNSTABLE, and after an lbm_reset that
 * rejected its fields, the context refuses lbm_step with LBM_ESTATE until an
 * lbm_reset succeeds (after LBM_EDEVICE it refuses every call).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid parameter, size, pointer or input value  */
    LBM_ENOMEM = -2,     /* workspace smaller than lbm_workspace_bytes       */
    LBM_EDEVICE = -3,    /* a HIP call or kernel launch failed               */
    LBM_EUNSTABLE = -4,  /* a periodic check found non-finite or |u| >= c_s  */
    LBM_ESTATE = -5      /* the context is in an error state                 */
} lbm_status;

/* Arithmetic and storage of the populations between steps. */
typedef enum {
    LBM_FP64 = 0,            /* FP64 compute, FP64 storage (608 B/node/step)  */
    LBM_FP32 = 1,            /* FP32 compute, FP32 storage (304 B/node/step)  */
    LBM_FP32_FP16STORE = 2,  /* FP32 compute; f_i - t_i p_ref/c_s^2 and       */
                             /* g_i - t_i phi_s stored as FP16 times 2^k, plus */
                             /* the FP32 per-node phi_s (160 B/node/step)      */
    LBM_FP32_BF16STORE = 3   /* as FP16STORE with BF16                         */
} lbm_precision;

typedef struct {
    int32_t nx, ny, nz;        /* lattice size; N = nx*ny*nz, Q*N < 2^31 and  */
                               /* Q*N*bytes per value < 2^32                  */
    int32_t precision;         /* lbm_precision                               */
    int32_t wall[3];           /* per axis: 0 periodic, 1 no-slip walls on    */
                               /* both faces (halfway between nodes; neutral  */
                               /* wetting); a wall axis needs n >= 2          */
    int32_t store_log2[2];     /* k of the 2^k scale of the FP16/BF16 f and g */
                               /* deviations (ignored otherwise); |k| <= 24   */
    int32_t check_every;       /* lbm_step checks finiteness and |u| < c_s    */
                               /* every this many steps (0: never)            */
    int32_t mass_fix_every;    /* FP64 phase-mass bookkeeping: every this     */
                               /* many steps the total of phi is measured in  */
                               /* FP64 and the drift from sum(phi0) is put    */
                               /* back on the interface, weighted by          */
                               /* phi(1 - phi), at the next step (0: never)   */
    int32_t normal_fd;         /* 0: the difference-free method (n and        */
                               /* |grad phi| from K1, Eqs. 17-19); 1: the     */
                               /* comparison scheme of Sec. 3.4: grad phi by  */
                               /* isotropic central differences of phi, which */
                               /* takes a second pass over the lattice per    */
                               /* step (phi of the propagated g, stored; a    */
                               /* neighbour beyond a wall takes the node's    */
                               /* own value)                                  */
    double courant;            /* c in (0, 1]; the paper uses 0.997; 1 gives  */
                               /* exact streaming                             */
    double rho1, rho2;         /* density of the phi = 1 and phi = 0 phases   */
    double tau_rho1, tau_rho2; /* relaxation time of each phase (> 0); the    */
                               /* dynamic viscosity is linear in phi          */
    double tau_phi;            /* phase-field relaxation time (> 0)           */
    double sigma;              /* surface tension (>= 0)                      */
    double delta;              /* interface thickness (> 0)                   */
    double G[3];               /* body acceleration                           */
    double k1_eps;             /* floor of the normal (>= 0; 1e-4 recommended):*/
                               /* n = -w K1/|K1| with w = 0 for |K1| <=       */
                               /* k1_eps, 1 for |K1| >= 2 k1_eps, linear      */
                               /* between (0: w = 1 wherever K1 != 0); the    */
                               /* same for |grad phi| with normal_fd = 1      */
    double p_ref;              /* pressure gauge of the 16-bit f storage      */
    int32_t lattice;           /* 19 or 0: D3Q19; 27: D3Q27 (the same method  */
                               /* on the 27-vector lattice, weights 8/27,     */
                               /* 2/27, 1/54, 1/216; no normal_fd = 1 on it)  */
    int32_t wetting;           /* 0: neutral walls; 1: contact angle theta at */
                               /* every wall (the paper has neutral walls):   */
                               /* on the first node layer next to a wall the  */
                               /* K1 normal is turned along the wall until    */
                               /* n . n_wall = -cos(theta); not with          */
                               /* normal_fd = 1                               */
    double cos_theta;          /* cos(theta) in [-1, 1], theta measured       */
                               /* through the phi = 1 phase                   */
} lbm_params;

/* Diagnostics of the state at the current time t (moments of the
 * post-propagation PDFs), accumulated in FP64. Sums run over all nodes with
 * node coordinates x, y, z as integers 0..n-1. */
typedef struct {
    int64_t step;              /* t                                           */
    double sum_phi;            /* sum phi                                     */
    double mass;               /* sum rho*phi (Sec. 3.3)                      */
    double mom[3];             /* sum rho*u                                   */
    double ekin;               /* sum rho*|u|^2/2 (Sec. 3.4)                  */
    double umax;               /* max |u| (Sec. 3.1)                          */
    double phi_min, phi_max;
    double com[3];             /* sum phi*x_a; centroid = com/sum_phi         */
    double phiu[3];            /* sum phi*u_a; phase velocity = phiu/sum_phi  */
    double l2_num;             /* sum (phi - phi_ref)^2  (Sec. 3.1)           */
    double l2_den;             /* sum phi_ref^2                               */
} lbm_diag;

/* The library's D3Q19 order: e (19x3 integers, row-major) and weights t. */
void lbm_lattice(int32_t e[57], double t[19]);

/* The library's order of lattice q (19 or 27): e (q x 3 integers, row-major)
 * and weights t (q); the PDFs of lbm_get_pdfs / lbm_set_pdfs follow it. The
 * D3Q27 order is the D3Q19 order followed by the 8 corner vectors, opposite
 * directions adjacent. Returns LBM_EINVAL for another q or a NULL pointer. */
int lbm_lattice_q(int32_t q, int32_t *e, double *t);

/* Bytes of device workspace a context with these parameters needs. */
int lbm_workspace_bytes(const lbm_params *P, size_t *bytes);

/* Creates a context and builds the state at t = 0 from the initial fields
 * (device FP64): phi0 (N), u0 (3N, NULL = 0), p0 (N, NULL = 0).
 * f(0) = f_eq - F/2 and g(0) = g_eq - (tau_phi + 1/2) t_i e_i.grad(phi0),
 * grad(phi0) by isotropic central differences, so the moments of the state
 * return phi0, u0, p0 and K1 returns grad(phi0); then one collision.
 * d_workspace: >= lbm_workspace_bytes, 256-byte aligned, owned by the caller
 * until lbm_destroy. stream: a hipStream_t (NULL = the null stream).
 * lbm_init synchronises the stream before it returns, so the inputs may be
 * freed afterwards. Invalid parameters give LBM_EINVAL before any device
 * work; inputs outside range (non-finite, phi0 outside [-0.5, 1.5]) give
 * LBM_EINVAL after the check on the device. */
int lbm_init(const lbm_params *P, void *d_workspace, size_t bytes, void *stream,
             const double *d_phi0, const double *d_u0, const double *d_p0, lbm_ctx **out);

/* Advances the state by n >= 0 time steps (asynchronous). */
int lbm_step(lbm_ctx *ctx, int64_t n);

/* Writes phi (N), u (3N) and p (N) of the state at t into device buffers
 * (any may be NULL); dtype 0 = double, 1 = float. Asynchronous. */
int lbm_fields(lbm_ctx *ctx, void *d_phi, void *d_u, void *d_p, int32_t dtype);

/* Computes the diagnostics at t; d_phi_ref (device FP64, N) may be NULL.
 * Blocks until the result is on the host. */
int lbm_diagnostics(lbm_ctx *ctx, const double *d_phi_ref, lbm_diag *out);

/* Writes the post-propagation PDFs at t as FP64 (Q*N each, device).
 * Together with lbm_set_pdfs this is checkpoint and restart. */
int lbm_get_pdfs(lbm_ctx *ctx, double *d_f, double *d_g);

/* Replaces the state at the current t by the given post-propagation PDFs
 * (device FP64, Q*N each), rounded to the storage precision. */
int lbm_set_pdfs(lbm_ctx *ctx, const double *d_f, const double *d_g);

/* Rebuilds the state in place from fields (device FP64, as lbm_init) and
 * sets the time to t; the phase-mass bookkeeping then targets sum(d_phi).
 * Used to hand a state back to the solver (restart from fields, or after a
 * window advanced by another model). Synchronises the stream. Fields outside
 * the range lbm_init accepts give LBM_EINVAL after the device check; the
 * state buffers are overwritten by then, so the context refuses lbm_step
 * (LBM_ESTATE) until a later lbm_reset succeeds. */
int lbm_reset(lbm_ctx *ctx, const double *d_phi, const double *d_u, const double *d_p, int64_t t);

/* Current time t (number of steps since lbm_init). */
int64_t lbm_time(const lbm_ctx *ctx);

/* Frees the host context; the workspace is the caller's again once the
 * stream has drained. NULL is allowed. */
void lbm_destroy(lbm_ctx *ctx);

const char *lbm_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
