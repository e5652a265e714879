/*
 * cpf_oracle.c -- plain FP64 CPU oracle of the difference-free conservative
 * phase-field lattice Boltzmann method (Zhao, Patel & Lee, arXiv 2407.12263).
 *
 * TEST INFRASTRUCTURE: it checks the GPU library and is never called by it.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.
 *
 * It follows the paper's algorithm step by step, in the paper's order, one
 * node at a time, with no blocking, fusion or reordering:
 *   1. phi = sum g_i, rho(phi)                         (Sec. 2.3)
 *   2. u from the first moment of f-bar and rho*G      (Sec. 2.2, Eq. 12)
 *   3. K1 = sum g_i (e_i - u), n = -K1/|K1|            (Sec. 2.3, Eqs. 17-18)
 *   4. S, grad(phi) from K1 and S, grad(rho)           (Sec. 2.3, Eqs. 15, 19)
 *   5. p from the zeroth moment of f-bar and u.grad(rho) (Sec. 2.2, Eq. 11)
 *   6. f* and g* by the Crank-Nicolson collision       (Sec. 2.2 Eq. 10, Sec. 2.3 Eq. 16)
 *   7. Lax-Wendroff propagation of f* and g*           (Sec. 2.2)
 *
 * Readings of the paper taken where it is silent or inconsistent (each is
 * listed with its justification in the design notes of the repository):
 *   - 3D lattice: D3Q19 for both f and g (the paper prints only D2Q9); the
 *     same steps on D3Q27 when built with -DORC_Q=27 (a variant the method
 *     admits: only the lattice table changes).
 *   - velocities e_i = c*e^_i with the Courant number c, c_s^2 = c^2/3.
 *   - surface-stress term of f_eq enters with a minus sign (App. A requires
 *     Pi_eq = rho u u + p I - Pi_s; the printed "+" gives the opposite).
 *   - rho*u = sum f-bar_i e_i + rho*G/2 (the sign consistent with the
 *     Crank-Nicolson transform and with the pressure recovery, Eq. 11).
 *   - the sharpening term of g_eq carries tau_phi: g_eq has t_i*tau_phi*e_i.S,
 *     so that K1_eq = tau_phi c_s^2 S as used by Eq. 19 and App. B (Eq. B.13).
 *   - Gamma_i(u) = t_i[1 + e.u/cs2 + (e.u)^2/(2cs4) - u^2/(2cs2)], w_i = t_i.
 *   - dynamic viscosity linear in phi; tau_rho = eta/(rho cs2).
 *   - a floor on the normal: n = -w K1/|K1| with w = 0 where |K1| <= k1_eps,
 *     w = 1 where |K1| >= 2 k1_eps and linear between. Where grad(phi)
 *     vanishes inside the interface (droplet centres, where two tails meet)
 *     K1 is rounding noise, and next to accelerated walls it carries a part
 *     of order 1e-5 that is no gradient; the sharpening term S = s*n then
 *     injects a flux of size s in a direction set by that noise, which the
 *     scheme amplifies. A floor above those values and far below interface
 *     values of |K1| (about c_s^2/(2W)) removes this without touching
 *     resolved interfaces; the linear rise keeps the normal continuous in
 *     K1, so a small change of K1 near the floor (a rounding) cannot switch
 *     a whole unit normal on or off. The same floor applies to a given
 *     gradient (the finite-difference variant and the initial state).
 *   - initial state: equilibrium plus the first-order non-equilibrium part of
 *     g that makes the K1 recovery return the initial gradient.
 *   - planar no-slip walls halfway between nodes: flux-form Lax-Wendroff
 *     with the solid-side neighbour replaced by the node itself and the
 *     outgoing flux returned into the opposite population.
 *   - wetting walls (the paper has neutral walls only): on the first node
 *     layer next to a wall, the normal recovered from K1 is turned, keeping
 *     its direction along the wall, until n . n_w = -cos(theta) (n_w the
 *     inward wall normal); S and grad(phi) of Eq. 19 then use that normal.
 *     Since the wall passes no phase flux, the wall-normal part of
 *     M (grad phi - s n) vanishes there at grad(phi) . n_w = -s cos(theta),
 *     the contact-angle condition of the equilibrium profile. Nodes whose
 *     normal has no component along the wall (|n_t| <= 1e-6) keep it.
 */
#include "cpf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q ORC_Q

/* ------------------------------------------------------------------ lattice */

static int    EH[Q][3];  /* integer directions e^_i */
static double TW[Q];     /* weights t_i            */
static int    OPP[Q];    /* index of -e^_i         */
static int    lattice_done = 0;

/* The lattice built from its definition, ordered by speed class |e^|^2:
 * D3Q19 = every vector of {-1,0,1}^3 with |e^|^2 <= 2, weights 1/3, 1/18,
 * 1/36; D3Q27 = all of {-1,0,1}^3, weights 8/27, 2/27, 1/54, 1/216 (the
 * tensor product of the one-dimensional weights 2/3, 1/6, 1/6). */
static void lattice_build(void)
{
    if (lattice_done) return;
    const double w19[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
    const double w27[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
    const int smax = Q == 27 ? 3 : 2;
    int i = 0;
    for (int s = 0; s <= smax; ++s)
        for (int z = -1; z <= 1; ++z)
            for (int y = -1; y <= 1; ++y)
                for (int x = -1; x <= 1; ++x) {
                    if (x * x + y * y + z * z != s) continue;
                    EH[i][0] = x; EH[i][1] = y; EH[i][2] = z;
                    TW[i] = Q == 27 ? w27[s] : w19[s];
                    ++i;
                }
    for (int a = 0; a < Q; ++a)
        for (int b = 0; b < Q; ++b)
            if (EH[a][0] == -EH[b][0] && EH[a][1] == -EH[b][1] && EH[a][2] == -EH[b][2])
                OPP[a] = b;
    lattice_done = 1;
}

void orc_lattice(int e[ORC_Q][3], double t[ORC_Q])
{
    lattice_build();
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) e[i][a] = EH[i][a];
        t[i] = TW[i];
    }
}

/* ------------------------------------------------------------------- state */

struct orc_state {
    orc_params P;
    long N, t;
    double *fb, *g;    /* post-propagation PDFs at time t */
    double *fs, *gs;   /* post-collision PDFs (work)       */
    double *phi, *grad;/* work for the finite-difference variant */
};

typedef struct {
    double phi, rho, tau_rho;
    double u[3];
    double p;
    double n[3];
    double gnorm;      /* |grad phi| */
    double S[3];
    double gradphi[3];
    double gradrho[3];
} macro_t;

static double cs2_of(const orc_params *P) { return P->courant * P->courant / 3.0; }

static long node_index(const orc_params *P, int x, int y, int z)
{
    return (long)x + (long)P->nx * ((long)y + (long)P->ny * (long)z);
}

/* ---------------------------------------------------------- node physics */

/* tau_rho from a dynamic viscosity linear in phi (each phase has its own
 * tau_rho_k, eta_k = rho_k cs2 tau_rho_k; nu = tau_rho cs2, Sec. 2.2). */
static double tau_rho_of(const orc_params *P, double phi, double rho)
{
    const double cs2 = cs2_of(P);
    const double eta1 = P->rho1 * cs2 * P->tau_rho1;
    const double eta2 = P->rho2 * cs2 * P->tau_rho2;
    const double eta = eta2 + (eta1 - eta2) * phi;
    return eta / (rho * cs2);
}

/* Inward unit normal of the walls node n touches (the first layer next to a
 * wall face; at an edge or corner the normalised sum of its faces'), or NULL
 * when wetting is off or the node touches no wall. */
static const double *wall_normal(const orc_params *P, long n, double nw[3])
{
    if (!P->wetting) return NULL;
    const int nn[3] = {P->nx, P->ny, P->nz};
    const long c[3] = {n % P->nx, (n / P->nx) % P->ny, n / ((long)P->nx * P->ny)};
    double len2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        nw[a] = 0.0;
        if (P->wall[a] && c[a] == 0) nw[a] += 1.0;
        if (P->wall[a] && c[a] == nn[a] - 1) nw[a] -= 1.0;
        len2 += nw[a] * nw[a];
    }
    if (len2 == 0.0) return NULL;
    for (int a = 0; a < 3; ++a) nw[a] /= sqrt(len2);
    return nw;
}

/* Turns a unit normal n so that n . n_w = -cos(theta), keeping its part along
 * the wall (the wetting reading in the header); n = 0 stays 0. */
static void wet_normal(const orc_params *P, const double nw[3], double n[3])
{
    const double dn = n[0] * nw[0] + n[1] * nw[1] + n[2] * nw[2];
    double t[3], tt = 0.0;
    for (int a = 0; a < 3; ++a) {
        t[a] = n[a] - dn * nw[a];
        tt += t[a] * t[a];
    }
    tt = sqrt(tt);
    if (tt <= 1e-6) return;
    const double ct = P->cos_theta, st = sqrt(1.0 - ct * ct);
    for (int a = 0; a < 3; ++a) n[a] = -ct * nw[a] + st * t[a] / tt;
}

/* Weight of the normal at a central moment or gradient of size k: 0 up to
 * k1_eps, 1 from 2 k1_eps, linear between (k1_eps = 0: 1 for any k > 0). */
static double floor_weight(const orc_params *P, double k)
{
    if (P->k1_eps <= 0.0) return k > 0.0 ? 1.0 : 0.0;
    if (k <= P->k1_eps) return 0.0;
    if (k >= 2.0 * P->k1_eps) return 1.0;
    return (k - P->k1_eps) / P->k1_eps;
}

/* Normal, S and grad(phi) from the central moment K1 (Sec. 2.3, Eqs. 15,
 * 18, 19); nw: inward wall normal of a wetting wall node, or NULL. */
static void gradient_from_K1(const orc_params *P, double phi, const double K1[3],
                             const double *nw, macro_t *m)
{
    const double cs2 = cs2_of(P);
    const double k = sqrt(K1[0] * K1[0] + K1[1] * K1[1] + K1[2] * K1[2]);
    /* Eq. 18; the direction of a vanishing K1 is undefined: n = 0 where
     * |K1| <= k1_eps, the unit normal where |K1| >= 2 k1_eps, and between
     * the two the unit normal scaled linearly from 0 to 1 (reading of the
     * degenerate case, see header) */
    const double w = floor_weight(P, k);
    for (int a = 0; a < 3; ++a) m->n[a] = w > 0.0 ? -K1[a] / k : 0.0;
    if (nw && w > 0.0) wet_normal(P, nw, m->n);
    for (int a = 0; a < 3; ++a) m->n[a] *= w;
    const double s = 4.0 * phi * (1.0 - phi) / P->delta;
    for (int a = 0; a < 3; ++a) m->S[a] = s * m->n[a];                       /* Eq. 15 */
    for (int a = 0; a < 3; ++a)                                              /* Eq. 19 */
        m->gradphi[a] = (P->tau_phi * cs2 * m->S[a] - K1[a]) / ((P->tau_phi + 0.5) * cs2);
    m->gnorm = sqrt(m->gradphi[0] * m->gradphi[0] + m->gradphi[1] * m->gradphi[1] +
                    m->gradphi[2] * m->gradphi[2]);
}

/* Normal, S and |grad phi| from a given gradient (finite-difference variant,
 * n = grad(phi)/|grad(phi)|, and the initial state). As for K1, the direction
 * of a vanishing gradient is undefined: n = 0 where |grad phi| <= k1_eps. */
static void gradient_given(const orc_params *P, double phi, const double gp[3], macro_t *m)
{
    const double gn = sqrt(gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2]);
    const double s = 4.0 * phi * (1.0 - phi) / P->delta;
    const double w = floor_weight(P, gn);
    for (int a = 0; a < 3; ++a) {
        m->gradphi[a] = gp[a];
        m->n[a] = w > 0.0 ? w * gp[a] / gn : 0.0;
        m->S[a] = s * m->n[a];
    }
    m->gnorm = gn;
}

/* Macroscopic recovery at one node from its post-propagation PDFs. With
 * gradphi_fd != NULL the gradient is that one (comparison scheme); nw: the
 * inward normal of a wetting wall the node touches, or NULL. */
static void node_macro(const orc_params *P, const double fb[Q], const double g[Q],
                       const double *gradphi_fd, const double *nw, macro_t *m)
{
    const double c = P->courant, cs2 = cs2_of(P);
    double phi = 0.0;
    for (int i = 0; i < Q; ++i) phi += g[i];                       /* Sec. 2.3 */
    m->phi = phi;
    m->rho = P->rho1 * phi + P->rho2 * (1.0 - phi);                 /* Sec. 2.3 */
    m->tau_rho = tau_rho_of(P, phi, m->rho);

    double j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i)
        for (int a = 0; a < 3; ++a) j[a] += fb[i] * c * EH[i][a];
    for (int a = 0; a < 3; ++a)                                     /* Eq. 12 (A4) */
        m->u[a] = (j[a] + 0.5 * m->rho * P->G[a]) / m->rho;

    if (gradphi_fd) {
        gradient_given(P, phi, gradphi_fd, m);
    } else {
        double K1[3] = {0.0, 0.0, 0.0};                              /* Eq. 17 */
        for (int i = 0; i < Q; ++i)
            for (int a = 0; a < 3; ++a) K1[a] += g[i] * (c * EH[i][a] - m->u[a]);
        gradient_from_K1(P, phi, K1, nw, m);
    }
    for (int a = 0; a < 3; ++a) m->gradrho[a] = (P->rho1 - P->rho2) * m->gradphi[a];

    double sf = 0.0;
    for (int i = 0; i < Q; ++i) sf += fb[i];
    double ugr = 0.0;
    for (int a = 0; a < 3; ++a) ugr += m->u[a] * m->gradrho[a];
    m->p = cs2 * sf + 0.5 * cs2 * ugr;                             /* Eq. 11 */
}

/* Equilibria and forcings (Sec. 2.2 Eqs. 7-8, App. A; Sec. 2.3 Eq. 14). */
static void node_equilibria(const orc_params *P, const macro_t *m, double feq[Q],
                            double geq[Q], double Sf[Q], double Rf[Q])
{
    const double c = P->courant, cs2 = cs2_of(P), cs4 = cs2 * cs2;
    double Pis[3][3];                                               /* Eq. 5 */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            Pis[a][b] = P->sigma * m->gnorm * ((a == b ? 1.0 : 0.0) - m->n[a] * m->n[b]);
    const double uu = m->u[0] * m->u[0] + m->u[1] * m->u[1] + m->u[2] * m->u[2];

    for (int i = 0; i < Q; ++i) {
        double e[3];
        for (int a = 0; a < 3; ++a) e[a] = c * EH[i][a];
        const double eu = e[0] * m->u[0] + e[1] * m->u[1] + e[2] * m->u[2];

        double PiE = 0.0;  /* Pi_s : (e e - cs2 I) */
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                PiE += Pis[a][b] * (e[a] * e[b] - (a == b ? cs2 : 0.0));

        /* Eq. 8 with the surface-stress term taken with a minus sign */
        feq[i] = TW[i] * (m->p / cs2 + m->rho * (eu / cs2 + eu * eu / (2.0 * cs4) - uu / (2.0 * cs2)))
                 - TW[i] * PiE / (2.0 * cs4);

        const double Gam = TW[i] * (1.0 + eu / cs2 + eu * eu / (2.0 * cs4) - uu / (2.0 * cs2));
        double emu_gr = 0.0, rG = 0.0;
        for (int a = 0; a < 3; ++a) {
            emu_gr += (e[a] - m->u[a]) * m->gradrho[a];
            rG += ((e[a] - m->u[a]) / cs2 + eu * e[a] / cs4) * (m->rho * P->G[a]);
        }
        Sf[i] = (Gam - TW[i]) * emu_gr;                             /* App. A, S_i */
        Rf[i] = TW[i] * rG;                                         /* Eq. 7, R_i */

        double eS = e[0] * m->S[0] + e[1] * m->S[1] + e[2] * m->S[2];
        /* Eq. 14 with the sharpening term scaled by tau_phi */
        geq[i] = TW[i] * m->phi * (1.0 + eu / cs2 + eu * eu / (2.0 * cs4) - uu / (2.0 * cs2))
                 + P->tau_phi * TW[i] * eS;
    }
}

/* Crank-Nicolson collision of one node (Sec. 2.2 Eq. 10 with
 * f-bar_eq = f_eq - F/2; Sec. 2.3 Eq. 16). */
static void node_collide(const orc_params *P, const double fb[Q], const double g[Q],
                         const double *gradphi_fd, const double *nw, double fs[Q], double gs[Q])
{
    macro_t m;
    node_macro(P, fb, g, gradphi_fd, nw, &m);
    double feq[Q], geq[Q], Sf[Q], Rf[Q];
    node_equilibria(P, &m, feq, geq, Sf, Rf);
    for (int i = 0; i < Q; ++i) {
        const double F = Sf[i] + Rf[i];
        const double fbeq = feq[i] - 0.5 * F;
        fs[i] = fb[i] - (fb[i] - fbeq) / (m.tau_rho + 0.5) + F;
        gs[i] = g[i] - (g[i] - geq[i]) / (P->tau_phi + 0.5);
    }
}

/* ------------------------------------------------------------ grid passes */

static void gather(const double *A, long N, long n, double v[Q])
{
    for (int i = 0; i < Q; ++i) v[i] = A[(long)i * N + n];
}

/* Neighbour at offset s*e^_i of (x,y,z): returns 0 and the index, or 1 if it
 * lies beyond a wall. Periodic axes wrap. */
static int neighbour(const orc_params *P, int x, int y, int z, int i, int s, long *idx)
{
    int q[3] = {x + s * EH[i][0], y + s * EH[i][1], z + s * EH[i][2]};
    const int nn[3] = {P->nx, P->ny, P->nz};
    for (int a = 0; a < 3; ++a) {
        if (q[a] < 0 || q[a] >= nn[a]) {
            if (P->wall[a]) return 1;
            q[a] = (q[a] % nn[a] + nn[a]) % nn[a];
        }
    }
    *idx = node_index(P, q[0], q[1], q[2]);
    return 0;
}

/* Lax-Wendroff propagation (Sec. 2.2):
 *   f(x,t+1) = f*(x) - c[f*(x) - f*(x-e)] - c(1-c)/2 [f*(x+e) - 2f*(x) + f*(x-e)].
 * At c = 1 this is the exact shift f*(x-e). Next to a wall the same scheme is
 * written in flux form, with the solid-side neighbour replaced by the node
 * itself and the flux that leaves through the wall face returned into the
 * opposite population (halfway bounce-back at c = 1). */
void orc_propagate(const orc_params *P, const double *in, double *out)
{
    lattice_build();
    const long N = (long)P->nx * P->ny * P->nz;
    const double c = P->courant, h = 0.5 * c * (1.0 - c);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                const long n = node_index(P, x, y, z);
                for (int i = 0; i < Q; ++i) {
                    long im = 0, ip = 0;
                    const int up_solid = neighbour(P, x, y, z, i, -1, &im);
                    const int dn_solid = neighbour(P, x, y, z, i, +1, &ip);
                    const double a0 = in[(long)i * N + n];
                    const double am = up_solid ? 0.0 : in[(long)i * N + im];
                    const double ap = dn_solid ? 0.0 : in[(long)i * N + ip];
                    double r;
                    if (!up_solid && !dn_solid) {
                        if (c == 1.0) r = am;
                        else r = a0 - c * (a0 - am) - 0.5 * c * (1.0 - c) * (ap - 2.0 * a0 + am);
                    } else {
                        const double flux_out = dn_solid ? c * a0 : c * a0 + h * (ap - a0);
                        const double flux_in = up_solid ? c * in[(long)OPP[i] * N + n]
                                                        : c * am + h * (a0 - am);
                        r = a0 - flux_out + flux_in;
                    }
                    out[(long)i * N + n] = r;
                }
            }
}

/* Isotropic central difference, grad phi = 3 sum_i t_i e^_i [phi(x+e^_i) -
 * phi(x-e^_i)]/2 (the finite-difference scheme the paper compares with,
 * Sec. 3.4). A neighbour beyond a wall takes the node's own value. */
void orc_fd_gradient(const orc_params *P, const double *phi, double *grad)
{
    lattice_build();
    const long N = (long)P->nx * P->ny * P->nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                const long n = node_index(P, x, y, z);
                double gsum[3] = {0.0, 0.0, 0.0};
                for (int i = 1; i < Q; ++i) {
                    long ip = 0, im = 0;
                    const double vp = neighbour(P, x, y, z, i, +1, &ip) ? phi[n] : phi[ip];
                    const double vm = neighbour(P, x, y, z, i, -1, &im) ? phi[n] : phi[im];
                    for (int a = 0; a < 3; ++a) gsum[a] += TW[i] * EH[i][a] * (vp - vm) * 0.5;
                }
                for (int a = 0; a < 3; ++a) grad[(long)a * N + n] = 3.0 * gsum[a];
            }
}

/* phi field and, in the finite-difference variant, its gradient */
static void phase_field(orc_state *S)
{
    const long N = S->N;
    for (long n = 0; n < N; ++n) {
        double phi = 0.0;
        for (int i = 0; i < Q; ++i) phi += S->g[(long)i * N + n];
        S->phi[n] = phi;
    }
    orc_fd_gradient(&S->P, S->phi, S->grad);
}

static const double *fd_at(const orc_state *S, long n, double buf[3])
{
    if (!S->P.normal_fd) return NULL;
    for (int a = 0; a < 3; ++a) buf[a] = S->grad[(long)a * S->N + n];
    return buf;
}

void orc_step(orc_state *S, long nsteps)
{
    const orc_params *P = &S->P;
    const long N = S->N;
    for (long t = 0; t < nsteps; ++t) {
        if (P->normal_fd) phase_field(S);
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; ++n) {
            double fb[Q], g[Q], fs[Q], gs[Q], gbuf[3], wbuf[3];
            gather(S->fb, N, n, fb);
            gather(S->g, N, n, g);
            node_collide(P, fb, g, fd_at(S, n, gbuf), wall_normal(P, n, wbuf), fs, gs);
            for (int i = 0; i < Q; ++i) {
                S->fs[(long)i * N + n] = fs[i];
                S->gs[(long)i * N + n] = gs[i];
            }
        }
        orc_propagate(P, S->fs, S->fb);
        orc_propagate(P, S->gs, S->g);
        S->t += 1;
    }
}

/* ----------------------------------------------------------------- set-up */

int orc_create(const orc_params *Pin, const double *phi0, const double *u0,
               const double *p0, orc_state **out)
{
    lattice_build();
    *out = NULL;
    const orc_params *P = Pin;
    if (P->nx < 1 || P->ny < 1 || P->nz < 1) return -1;
    if (!(P->courant > 0.0 && P->courant <= 1.0)) return -1;
    if (!(P->rho1 > 0.0 && P->rho2 > 0.0 && P->delta > 0.0)) return -1;
    if (!(P->tau_phi > -0.5 && P->tau_rho1 > -0.5 && P->tau_rho2 > -0.5)) return -1;
    const int nn[3] = {P->nx, P->ny, P->nz};
    for (int a = 0; a < 3; ++a)
        if (P->wall[a] && nn[a] < 2) return -1;
    if (P->wetting != 0 && P->wetting != 1) return -1;
    if (P->wetting && !(P->cos_theta >= -1.0 && P->cos_theta <= 1.0)) return -1;
    const long N = (long)P->nx * P->ny * P->nz;
    for (long n = 0; n < N; ++n) {
        if (!isfinite(phi0[n])) return -1;
        if (u0) for (int a = 0; a < 3; ++a) if (!isfinite(u0[(long)a * N + n])) return -1;
        if (p0 && !isfinite(p0[n])) return -1;
    }

    orc_state *S = (orc_state *)calloc(1, sizeof(orc_state));
    if (!S) return -2;
    S->P = *P;
    S->N = N;
    S->t = 0;
    S->fb = (double *)malloc(sizeof(double) * Q * N);
    S->g = (double *)malloc(sizeof(double) * Q * N);
    S->fs = (double *)malloc(sizeof(double) * Q * N);
    S->gs = (double *)malloc(sizeof(double) * Q * N);
    S->phi = (double *)malloc(sizeof(double) * N);
    S->grad = (double *)malloc(sizeof(double) * 3 * N);
    if (!S->fb || !S->g || !S->fs || !S->gs || !S->phi || !S->grad) {
        orc_destroy(S);
        return -2;
    }

    /* Initial state: f-bar(0) = f_eq - F/2 and g(0) = g_eq - (tau_phi+1/2)
     * t_i e_i.grad(phi0), with grad(phi0) from isotropic central differences,
     * so that the moments of the state return phi0, u0, p0 and the K1
     * recovery returns grad(phi0). */
    memcpy(S->phi, phi0, sizeof(double) * N);
    orc_fd_gradient(P, S->phi, S->grad);
    const double c = P->courant;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        macro_t m;
        memset(&m, 0, sizeof(m));
        m.phi = phi0[n];
        m.rho = P->rho1 * m.phi + P->rho2 * (1.0 - m.phi);
        for (int a = 0; a < 3; ++a) m.u[a] = u0 ? u0[(long)a * N + n] : 0.0;
        m.p = p0 ? p0[n] : 0.0;
        double gp[3];
        for (int a = 0; a < 3; ++a) gp[a] = S->grad[(long)a * N + n];
        gradient_given(P, m.phi, gp, &m);
        for (int a = 0; a < 3; ++a) m.gradrho[a] = (P->rho1 - P->rho2) * m.gradphi[a];
        double feq[Q], geq[Q], Sf[Q], Rf[Q];
        node_equilibria(P, &m, feq, geq, Sf, Rf);
        for (int i = 0; i < Q; ++i) {
            double egp = 0.0;
            for (int a = 0; a < 3; ++a) egp += c * EH[i][a] * gp[a];
            S->fb[(long)i * N + n] = feq[i] - 0.5 * (Sf[i] + Rf[i]);
            S->g[(long)i * N + n] = geq[i] - (P->tau_phi + 0.5) * TW[i] * egp;
        }
    }
    *out = S;
    return 0;
}

void orc_destroy(orc_state *S)
{
    if (!S) return;
    free(S->fb); free(S->g); free(S->fs); free(S->gs); free(S->phi); free(S->grad);
    free(S);
}

long orc_time(const orc_state *S) { return S->t; }

void orc_get_pdfs(const orc_state *S, double *f, double *g)
{
    memcpy(f, S->fb, sizeof(double) * Q * S->N);
    memcpy(g, S->g, sizeof(double) * Q * S->N);
}

void orc_set_pdfs(orc_state *S, const double *f, const double *g)
{
    memcpy(S->fb, f, sizeof(double) * Q * S->N);
    memcpy(S->g, g, sizeof(double) * Q * S->N);
}

/* --------------------------------------------------------------- outputs */

void orc_fields(const orc_state *Sc, double *phi, double *u, double *p)
{
    orc_state *S = (orc_state *)Sc;
    const long N = S->N;
    if (S->P.normal_fd) phase_field(S);
    for (long n = 0; n < N; ++n) {
        double fb[Q], g[Q], gbuf[3], wbuf[3];
        gather(S->fb, N, n, fb);
        gather(S->g, N, n, g);
        macro_t m;
        node_macro(&S->P, fb, g, fd_at(S, n, gbuf), wall_normal(&S->P, n, wbuf), &m);
        if (phi) phi[n] = m.phi;
        if (u) for (int a = 0; a < 3; ++a) u[(long)a * N + n] = m.u[a];
        if (p) p[n] = m.p;
    }
}

/* Diagnostics of the paper: sum phi, mass m = sum rho phi (Sec. 3.3), net
 * momentum, kinetic energy E_k = sum rho u^2/2 (Sec. 3.4), max |u| (Sec. 3.1),
 * phi range, centroid and phase velocity numerators (Sec. 3.3), and the
 * numerator and denominator of ||delta phi||_2 (Sec. 3.1). */
void orc_diag(const orc_state *Sc, const double *phi_ref, double out[ORC_NDIAG])
{
    orc_state *S = (orc_state *)Sc;
    const orc_params *P = &S->P;
    const long N = S->N;
    for (int k = 0; k < ORC_NDIAG; ++k) out[k] = 0.0;
    out[ORC_D_PHIMIN] = INFINITY;
    out[ORC_D_PHIMAX] = -INFINITY;
    if (P->normal_fd) phase_field(S);
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                const long n = node_index(P, x, y, z);
                double fb[Q], g[Q], gbuf[3], wbuf[3];
                gather(S->fb, N, n, fb);
                gather(S->g, N, n, g);
                macro_t m;
                node_macro(P, fb, g, fd_at(S, n, gbuf), wall_normal(P, n, wbuf), &m);
                const double uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
                out[ORC_D_SUM_PHI] += m.phi;
                out[ORC_D_MASS] += m.rho * m.phi;
                out[ORC_D_MOMX] += m.rho * m.u[0];
                out[ORC_D_MOMY] += m.rho * m.u[1];
                out[ORC_D_MOMZ] += m.rho * m.u[2];
                out[ORC_D_EKIN] += 0.5 * m.rho * uu;
                if (sqrt(uu) > out[ORC_D_UMAX]) out[ORC_D_UMAX] = sqrt(uu);
                if (m.phi < out[ORC_D_PHIMIN]) out[ORC_D_PHIMIN] = m.phi;
                if (m.phi > out[ORC_D_PHIMAX]) out[ORC_D_PHIMAX] = m.phi;
                out[ORC_D_COMX] += m.phi * x;
                out[ORC_D_COMY] += m.phi * y;
                out[ORC_D_COMZ] += m.phi * z;
                out[ORC_D_PHIUX] += m.phi * m.u[0];
                out[ORC_D_PHIUY] += m.phi * m.u[1];
                out[ORC_D_PHIUZ] += m.phi * m.u[2];
                if (phi_ref) {
                    const double d = m.phi - phi_ref[n];
                    out[ORC_D_L2NUM] += d * d;
                    out[ORC_D_L2DEN] += phi_ref[n] * phi_ref[n];
                }
            }
}

/* ---------------------------------------------------- exposed node pieces */

void orc_node_equilibria(const orc_params *P, double phi, const double u[3], double p,
                         const double gradphi[3], double feq[ORC_Q], double geq[ORC_Q],
                         double Sf[ORC_Q], double Rf[ORC_Q])
{
    lattice_build();
    macro_t m;
    memset(&m, 0, sizeof(m));
    m.phi = phi;
    m.rho = P->rho1 * phi + P->rho2 * (1.0 - phi);
    m.tau_rho = tau_rho_of(P, phi, m.rho);
    for (int a = 0; a < 3; ++a) m.u[a] = u[a];
    m.p = p;
    gradient_given(P, phi, gradphi, &m);
    for (int a = 0; a < 3; ++a) m.gradrho[a] = (P->rho1 - P->rho2) * m.gradphi[a];
    node_equilibria(P, &m, feq, geq, Sf, Rf);
}

void orc_node_macro(const orc_params *P, const double fb[ORC_Q], const double g[ORC_Q],
                    double out[10])
{
    lattice_build();
    macro_t m;
    node_macro(P, fb, g, NULL, NULL, &m);
    out[0] = m.phi; out[1] = m.rho; out[2] = m.tau_rho;
    out[3] = m.u[0]; out[4] = m.u[1]; out[5] = m.u[2];
    out[6] = m.p;
    out[7] = m.gradphi[0]; out[8] = m.gradphi[1]; out[9] = m.gradphi[2];
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
