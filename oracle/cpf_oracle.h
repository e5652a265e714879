/*
 * cpf_oracle.h -- plain FP64 CPU oracle of the difference-free conservative
 * phase-field lattice Boltzmann step (Zhao, Patel & Lee, arXiv 2407.12263).
 *
 * TEST INFRASTRUCTURE. This library exists to check the GPU library, not to
 * be used by it: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it. It shares no header, table or helper with
 * the GPU path; the two agree only through the paper.
 *
 * Units: grid units, dx = dt = 1. The discrete velocities are e_i = c*e^_i
 * with e^_i the integer vectors of the lattice and c the Courant number of
 * the Lax-Wendroff propagation (Sec. 2.2), so c_s^2 = c^2/3.
 *
 * The lattice is fixed at compile time by ORC_Q: 19 (D3Q19, the default) or
 * 27 (D3Q27, built as a second library with -DORC_Q=27). Both carry the same
 * sound speed and the fourth-order isotropy the equilibria need.
 *
 * Arrays are host arrays, structure-of-arrays, index  n = x + nx*(y + ny*z),
 * a population i at  i*N + n,  a vector component a at  a*N + n.
 */
#ifndef CPF_ORACLE_H
#define CPF_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#ifndef ORC_Q
#define ORC_Q 19
#endif
#if ORC_Q != 19 && ORC_Q != 27
#error "ORC_Q must be 19 or 27"
#endif

typedef struct {
    int nx, ny, nz;
    int wall[3];        /* per axis: 0 periodic, 1 no-slip walls on both faces   */
    double courant;     /* c in (0,1]; the paper fixes 0.997                     */
    double rho1, rho2;  /* density of the phi=1 phase and of the phi=0 phase     */
    double tau_rho1, tau_rho2; /* relaxation time of each phase, nu = tau*cs^2   */
    double tau_phi;     /* phase-field relaxation time, M = tau_phi*cs^2         */
    double sigma;       /* surface tension                                       */
    double delta;       /* interface thickness                                   */
    double G[3];        /* body acceleration                                     */
    int normal_fd;      /* 0: normal and grad(phi) from K1 (the paper's scheme)  */
                        /* 1: isotropic central differences of phi (comparison)  */
    double k1_eps;      /* floor of the normal: weight 0 up to k1_eps, 1 from    */
                        /* 2 k1_eps, linear between (0: no floor)               */
    int wetting;        /* 0: neutral walls; 1: contact angle theta at the walls  */
    double cos_theta;   /* cos(theta), theta measured through the phi = 1 phase   */
} orc_params;

/* diagnostics of the state at the current time, see orc_diag */
enum {
    ORC_D_SUM_PHI = 0, ORC_D_MASS, ORC_D_MOMX, ORC_D_MOMY, ORC_D_MOMZ,
    ORC_D_EKIN, ORC_D_UMAX, ORC_D_PHIMIN, ORC_D_PHIMAX,
    ORC_D_COMX, ORC_D_COMY, ORC_D_COMZ, ORC_D_PHIUX, ORC_D_PHIUY, ORC_D_PHIUZ,
    ORC_D_L2NUM, ORC_D_L2DEN, ORC_NDIAG
};

typedef struct orc_state orc_state;

/* Lattice table of this oracle: e^_i (integers) and weights t_i. */
void orc_lattice(int e[ORC_Q][3], double t[ORC_Q]);

/* Builds the state at t = 0 from phi0 (N), u0 (3N or NULL = 0), p0 (N or
 * NULL = 0). Returns 0, or -1 on invalid input. */
int  orc_create(const orc_params *P, const double *phi0, const double *u0,
                const double *p0, orc_state **out);
void orc_destroy(orc_state *S);
void orc_step(orc_state *S, long nsteps);
long orc_time(const orc_state *S);
/* phi (N), u (3N), p (N) of the post-propagation PDFs at the current time */
void orc_fields(const orc_state *S, double *phi, double *u, double *p);
/* phi_ref may be NULL (then the L2 entries are 0) */
void orc_diag(const orc_state *S, const double *phi_ref, double out[ORC_NDIAG]);
/* copy out / in the post-propagation PDFs f-bar and g (ORC_Q*N each) */
void orc_get_pdfs(const orc_state *S, double *f, double *g);
void orc_set_pdfs(orc_state *S, const double *f, const double *g);

/* ---- single pieces, exposed for the moment-identity pins ---- */

/* Equilibria and forcings at one node for given macroscopic values and a given
 * order-parameter gradient (normal and |grad phi| follow from it):
 * feq, geq, S_i (compensation), R_i (body force), all of length ORC_Q. */
void orc_node_equilibria(const orc_params *P, double phi, const double u[3],
                         double p, const double gradphi[3],
                         double feq[ORC_Q], double geq[ORC_Q],
                         double Sf[ORC_Q], double Rf[ORC_Q]);

/* Macroscopic recovery at one node from its post-propagation PDFs (K1 mode):
 * out = {phi, rho, tau_rho, ux, uy, uz, p, gx, gy, gz} with g = grad(phi). */
void orc_node_macro(const orc_params *P, const double fb[ORC_Q],
                    const double g[ORC_Q], double out[10]);

/* Lax-Wendroff propagation of one ORC_Q-population field (with the walls of P). */
void orc_propagate(const orc_params *P, const double *in, double *out);

/* Isotropic central-difference gradient of a scalar field (3N out). */
void orc_fd_gradient(const orc_params *P, const double *phi, double *grad);

/* OpenMP threads the grid passes use; set them (n > 0). */
int orc_num_threads(void);
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
