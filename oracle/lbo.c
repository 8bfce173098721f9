/*
 * lbo.c -- plain FP64 CPU oracle of the regularized colour-gradient lattice
 * Boltzmann model for direct-writing printing (arXiv:2102.02655).
 *
 * TEST INFRASTRUCTURE ONLY: the reference that the GPU library is checked
 * against.  It is deliberately slow and literal: every population of every
 * colour is stored, every moment is a plain sum over the velocity set, every
 * equilibrium is evaluated from its formula, streaming is a push over links.
 * It shares no code with the GPU library.  Built with -ffp-contract=off so
 * that the head geometry (decided in FP64) rounds exactly as written.
 *
 * Section / equation references are to the paper:
 *   Sec. II.A  Eq. (lbm), (cgoperator), (modbgk), the modified equilibrium,
 *              the phi_i table, (cgoef), (pertopform), the colour-gradient
 *              force, (lattgrad), the B_i table, sigma = 2 tau A / 9, the
 *              recolouring operator, (tauinter), (wet), (reg)
 *   Sec. II.B  (notnewvisc), (stressvsstrain), (tauofgammadot), the moving
 *              template, (movwall), node creation/deletion, (movnozzle),
 *              anti-bounce-back, the drag force with the exact-difference
 *              method
 * Readings of silent or garbled passages are listed with each function.
 */
#include "lbo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 19

/* ------------------------------------------------------------------------ */
/* Lattice                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int D, Q;
    int c[QMAX][3];
    double w[QMAX];
    int opp[QMAX];
    double cs2;
} lattice_t;

/* Sec. II.A: D2Q9, i = 0 at rest, i = 1..8 at angle (i-1) pi/4, |c| = 1 for
 * odd i and sqrt(2) for even i, w = 4/9, 1/9, 1/36.  The paper's 2-D plane is
 * (x, vertical); here the vertical axis is z, so c_y = 0.
 * D3Q19 (the 3-D generalisation): rest, the 6 axis links and the 12 face
 * diagonals, w = 1/3, 1/18, 1/36, enumerated shell by shell.  c_s^2 = 1/3. */
static int lattice_build(int lattice, lattice_t *L)
{
    memset(L, 0, sizeof(*L));
    L->cs2 = 1.0 / 3.0;
    if (lattice == LBO_D2Q9) {
        static const int cx[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
        static const int cz[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
        L->D = 2;
        L->Q = 9;
        for (int i = 0; i < 9; ++i) {
            L->c[i][0] = cx[i];
            L->c[i][1] = 0;
            L->c[i][2] = cz[i];
            int c2 = cx[i] * cx[i] + cz[i] * cz[i];
            L->w[i] = c2 == 0 ? 4.0 / 9.0 : (c2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
    } else if (lattice == LBO_D3Q19) {
        L->D = 3;
        L->Q = 0;
        for (int shell = 0; shell <= 2; ++shell)
            for (int a = -1; a <= 1; ++a)
                for (int b = -1; b <= 1; ++b)
                    for (int d = -1; d <= 1; ++d) {
                        if (a * a + b * b + d * d != shell) continue;
                        int i = L->Q++;
                        L->c[i][0] = a;
                        L->c[i][1] = b;
                        L->c[i][2] = d;
                        L->w[i] = shell == 0 ? 1.0 / 3.0 : (shell == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
                    }
    } else {
        return LBO_EINVAL;
    }
    for (int i = 0; i < L->Q; ++i)
        for (int j = 0; j < L->Q; ++j)
            if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] && L->c[j][2] == -L->c[i][2])
                L->opp[i] = j;
    return LBO_OK;
}

static int csq(const lattice_t *L, int i)
{
    return L->c[i][0] * L->c[i][0] + L->c[i][1] * L->c[i][1] + L->c[i][2] * L->c[i][2];
}

/* phi_i^k of the modified equilibrium (Sec. II.A).  The paper prints the
 * D2Q9 table: alpha, (1-alpha)/5 on the axes, (1-alpha)/20 on the diagonals.
 * Generating rule, which reproduces that table exactly and is used for every
 * lattice: phi_0 = alpha, phi_i = (1 - alpha) w_i / (1 - w_0). */
static void phi_build(const lattice_t *L, double alpha, double *phi)
{
    phi[0] = alpha;
    for (int i = 1; i < L->Q; ++i) phi[i] = (1.0 - alpha) * L->w[i] / (1.0 - L->w[0]);
}

/* B_i of the perturbation operator, Eq. (pertopform).  The paper prints the
 * D2Q9 values -4/27, 2/27, 5/108.  Generating rule, reproducing them exactly:
 * B_i = w_i (|c_i|^2 - (D-1)/3).  It gives sum_i B_i = c_s^2 and
 * sum_i B_i c_ia c_ib = c_s^2 delta_ab on D2Q9 and D3Q19. */
static void B_build(const lattice_t *L, double *B)
{
    for (int i = 0; i < L->Q; ++i) B[i] = L->w[i] * ((double)csq(L, i) - (L->D - 1) / 3.0);
}

int lbo_lattice(int lattice, int *D, int *Q, int *c, double *w, double *cs2)
{
    lattice_t L;
    if (lattice_build(lattice, &L)) return LBO_EINVAL;
    if (D) *D = L.D;
    if (Q) *Q = L.Q;
    for (int i = 0; i < L.Q; ++i) {
        if (c)
            for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
        if (w) w[i] = L.w[i];
    }
    if (cs2) *cs2 = L.cs2;
    return LBO_OK;
}

int lbo_phi(int lattice, double alpha, double *phi)
{
    lattice_t L;
    if (lattice_build(lattice, &L)) return LBO_EINVAL;
    phi_build(&L, alpha, phi);
    return LBO_OK;
}

int lbo_B(int lattice, double *B)
{
    lattice_t L;
    if (lattice_build(lattice, &L)) return LBO_EINVAL;
    B_build(&L, B);
    return LBO_OK;
}

/* Partial pressure of one colour, Eq. (cgoef): the isotropic second moment of
 * the rest-frame equilibrium, p^k = rho^k sum_i phi_i c_ix^2 (the paper's
 * (3/5) rho^k (1 - phi_0) on D2Q9). */
double lbo_partial_pressure(int lattice, double alpha, double rho)
{
    lattice_t L;
    double phi[QMAX], s = 0.0;
    if (lattice_build(lattice, &L)) return NAN;
    phi_build(&L, alpha, phi);
    for (int i = 0; i < L.Q; ++i) s += phi[i] * L.c[i][0] * L.c[i][0];
    return rho * s;
}

/* ------------------------------------------------------------------------ */
/* Single-site operators                                                     */
/* ------------------------------------------------------------------------ */

/* Modified equilibrium of one colour (Sec. II.A), with the quadratic term
 * read as (c.u)^2 / (2 c_s^4) (the printed 2 c_s^2 is a typo; the
 * anti-bounce-back formula of Sec. II.B prints c_s^4 and the second moment
 * requires it). */
static void feq_site(const lattice_t *L, const double *phi, double rho, const double *u, double *feq)
{
    double cs2 = L->cs2;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < L->Q; ++i) {
        double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
        feq[i] = rho * (phi[i] + L->w[i] * (cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2)));
    }
}

/* Second moment sum_i g_i c_ia c_ib. */
static void second_moment(const lattice_t *L, const double *g, double P[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) {
            double s = 0.0;
            for (int i = 0; i < L->Q; ++i) s += g[i] * L->c[i][a] * L->c[i][b];
            P[a][b] = s;
            P[b][a] = s;
        }
}

/* Pi^neq = sum_i f_i c c - sum_i f_i^eq c c (Eq. (reg)). */
static void pi_neq(const lattice_t *L, const double *f, const double *feq, double Pi[3][3])
{
    double Pf[3][3], Pe[3][3];
    second_moment(L, f, Pf);
    second_moment(L, feq, Pe);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Pi[a][b] = Pf[a][b] - Pe[a][b];
}

/* Regularised population, Eq. (reg):
 * f^reg_i = f^eq_i + w_i / (2 c_s^4) Q_iab Pi^neq_ab, Q_iab = c_ia c_ib - c_s^2 delta_ab. */
static void regularize_site(const lattice_t *L, const double *feq, double Pi[3][3], double *freg)
{
    double cs2 = L->cs2;
    for (int i = 0; i < L->Q; ++i) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double Qab = L->c[i][a] * L->c[i][b] - (a == b ? cs2 : 0.0);
                s += Qab * Pi[a][b];
            }
        freg[i] = feq[i] + L->w[i] / (2.0 * cs2 * cs2) * s;
    }
}

int lbo_feq(int lattice, double alpha, double rho, const double *u, double *feq)
{
    lattice_t L;
    double phi[QMAX];
    if (lattice_build(lattice, &L)) return LBO_EINVAL;
    phi_build(&L, alpha, phi);
    feq_site(&L, phi, rho, u, feq);
    return LBO_OK;
}

int lbo_regularize(int lattice, double alpha, double rho, const double *u, const double *f, double *freg)
{
    lattice_t L;
    double phi[QMAX], feq[QMAX], Pi[3][3];
    if (lattice_build(lattice, &L)) return LBO_EINVAL;
    phi_build(&L, alpha, phi);
    feq_site(&L, phi, rho, u, feq);
    pi_neq(&L, f, feq, Pi);
    regularize_site(&L, feq, Pi, freg);
    return LBO_OK;
}

/* Perturbation operator, Eq. (pertopform):
 * Omega2_i = (A/2) |grad rho^N| [ w_i (F.c_i)^2 / |F|^2 - B_i ].
 * Where F_cg vanishes exactly the direction is undefined; the operator is
 * taken as zero there (it is multiplied by a vanishing gradient anyway). */
static void perturb_site(const lattice_t *L, const double *B, double A, const double *gN, const double *F,
                         double *om)
{
    double gn = sqrt(gN[0] * gN[0] + gN[1] * gN[1] + gN[2] * gN[2]);
    double FF = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
    for (int i = 0; i < L->Q; ++i) {
        if (FF == 0.0) {
            om[i] = 0.0;
            continue;
        }
        double Fc = F[0] * L->c[i][0] + F[1] * L->c[i][1] + F[2] * L->c[i][2];
        om[i] = 0.5 * A * gn * (L->w[i] * Fc * Fc / FF - B[i]);
    }
}

int lbo_perturbation(int lattice, double A, const double *gradN, const double *Fcg, double *omega2)
{
    lattice_t L;
    double B[QMAX];
    if (lattice_build(lattice, &L)) return LBO_EINVAL;
    B_build(&L, B);
    perturb_site(&L, B, A, gradN, Fcg, omega2);
    return LBO_OK;
}

/* Recolouring operator (Sec. II.A).  Reading: both colours use the
 * rest-frame equilibrium sum_k f^eq(rho_k, u = 0) = sum_k rho_k phi_i^k (the
 * printed u for the blue colour is a typo: only u = 0 conserves each colour),
 * so f^B = f* - f^Y.  cos(phi_i) = c_i . grad rho^N / (|c_i| |grad rho^N|_eps)
 * with |g|_eps = sqrt(|g|^2 + eps^2), continuous where the gradient vanishes;
 * cos(phi_0) = 0. */
static void recolour_site(const lattice_t *L, const double *phiY, const double *phiB, double beta, double eps,
                          double rhoY, double rhoB, const double *gN, const double *fstar, double *fY, double *fB)
{
    double rho = rhoY + rhoB;
    double gmag = sqrt(gN[0] * gN[0] + gN[1] * gN[1] + gN[2] * gN[2] + eps * eps);
    for (int i = 0; i < L->Q; ++i) {
        double cosphi = 0.0;
        if (csq(L, i) > 0 && gmag > 0.0) {
            double cg = L->c[i][0] * gN[0] + L->c[i][1] * gN[1] + L->c[i][2] * gN[2];
            cosphi = cg / (sqrt((double)csq(L, i)) * gmag);
        }
        double eqsum = rhoY * phiY[i] + rhoB * phiB[i];
        fY[i] = rhoY / rho * fstar[i] + beta * rhoY * rhoB / (rho * rho) * cosphi * eqsum;
        fB[i] = fstar[i] - fY[i];
    }
}

int lbo_recolour(int lattice, const double *alpha, double beta, double eps_g, double rhoY, double rhoB,
                 const double *gradN, const double *fstar, double *fY, double *fB)
{
    lattice_t L;
    double phiY[QMAX], phiB[QMAX];
    if (lattice_build(lattice, &L)) return LBO_EINVAL;
    phi_build(&L, alpha[0], phiY);
    phi_build(&L, alpha[1], phiB);
    recolour_site(&L, phiY, phiB, beta, eps_g, rhoY, rhoB, gradN, fstar, fY, fB);
    return LBO_OK;
}

/* ------------------------------------------------------------------------ */
/* Ink rheology: Eqs. (notnewvisc), (stressvsstrain), (tauofgammadot)        */
/* ------------------------------------------------------------------------ */

/* Unclamped tau_Y(gdot) = 1/2 + nu(gdot) / c_s^2 for the selected law. */
static double tau_law(const lbo_params *p, double gdot)
{
    const double cs2 = 1.0 / 3.0;
    double nu;
    if (p->rheology == LBO_POWER_LAW) {
        if (gdot > 0.0)
            nu = p->K * pow(gdot, p->n - 1.0);
        else
            nu = p->n < 1.0 ? INFINITY : (p->n == 1.0 ? p->K : 0.0);
    } else { /* Cross, Eq. (notnewvisc) divided by the density */
        nu = p->nu_inf + (p->nu0 - p->nu_inf) / (1.0 + pow(p->lambda * gdot, p->m));
    }
    return 0.5 + nu / cs2;
}

static double tau_clamped(const lbo_params *p, double gdot)
{
    double t = tau_law(p, gdot);
    if (t < p->tau_min) t = p->tau_min;
    if (t > p->tau_max) t = p->tau_max;
    return t;
}

/* Implicit strain rate, Eq. (stressvsstrain) with Eq. (tauofgammadot):
 *   gdot = |Pi^Y| / (rho_Y tau_Y(gdot) c_s^2).
 * Reading: tau_Y is clamped to [tau_min, tau_max]; rho_Y in the denominator
 * is floored at rho_eps (continuous; only trace-ink cells are affected, and
 * there the ink carries a harmonic weight below rho_eps).  The left side
 * gdot * tau_Y(gdot) is strictly increasing, so the root is unique and lies
 * in [s / tau_max, s / tau_min], s = |Pi^Y| / (c_s^2 rho_Y).  The ends are
 * tested first (root on a clamp); otherwise plain geometric bisection to a
 * relative width of 1e-14.  A Newtonian ink has tau_Y = tau_y. */
int lbo_tau_ink(const lbo_params *p, double S, double rhoY, double *gdot_out, double *tau_out)
{
    const double cs2 = 1.0 / 3.0;
    if (p->rheology == LBO_NEWTONIAN) {
        double r = rhoY > p->rho_eps ? rhoY : p->rho_eps;
        if (tau_out) *tau_out = p->tau_y;
        if (gdot_out) *gdot_out = S / (r * p->tau_y * cs2);
        return LBO_OK;
    }
    double r = rhoY > p->rho_eps ? rhoY : p->rho_eps;
    double s = S / (cs2 * r);
    double gdot, tau;
    if (!(s > 0.0)) {
        gdot = 0.0;
        tau = tau_clamped(p, 0.0);
    } else {
        double lo = s / p->tau_max, hi = s / p->tau_min;
        if (tau_law(p, lo) >= p->tau_max) {
            gdot = lo;
            tau = p->tau_max;
        } else if (tau_law(p, hi) <= p->tau_min) {
            gdot = hi;
            tau = p->tau_min;
        } else {
            for (int it = 0; it < 200 && hi > lo * (1.0 + 1e-14); ++it) {
                double mid = sqrt(lo * hi);
                if (mid * tau_clamped(p, mid) - s > 0.0)
                    hi = mid;
                else
                    lo = mid;
            }
            gdot = sqrt(lo * hi);
            tau = tau_clamped(p, gdot);
        }
    }
    if (gdot_out) *gdot_out = gdot;
    if (tau_out) *tau_out = tau;
    return LBO_OK;
}

/* ------------------------------------------------------------------------ */
/* Wall density on a bounce-back link, Sec. II.B ("third-order               */
/* interpolation in the direction -c_i")                                     */
/* ------------------------------------------------------------------------ */

/* Reading: quadratic Lagrange extrapolation to the link midpoint from the
 * boundary node (r0), one node inward (r1) and two nodes inward (r2):
 * rho_w = (15 r0 - 10 r1 + 3 r2) / 8; with only r0, r1 available the linear
 * (3 r0 - r1) / 2; with only r0, r0.  Clamped at zero. */
double lbo_wall_density(double r0, double r1, double r2, int has1, int has2)
{
    double v;
    if (has1 && has2)
        v = (15.0 * r0 - 10.0 * r1 + 3.0 * r2) / 8.0;
    else if (has1)
        v = (3.0 * r0 - r1) / 2.0;
    else
        v = r0;
    return v > 0.0 ? v : 0.0;
}

/* Isotropic central gradient, Eq. (lattgrad), evaluated at the interior nodes
 * of a box (borders left at zero). */
int lbo_gradient(int lattice, int nx, int ny, int nz, const double *chi, double *grad)
{
    lattice_t L;
    if (lattice_build(lattice, &L)) return LBO_EINVAL;
    long N = (long)nx * ny * nz;
    memset(grad, 0, sizeof(double) * 3 * N);
    int ylo = ny > 2 ? 1 : 0, yhi = ny > 2 ? ny - 1 : ny;
    for (int z = 1; z < nz - 1; ++z)
        for (int y = ylo; y < yhi; ++y)
            for (int x = 1; x < nx - 1; ++x) {
                long cell = ((long)z * ny + y) * nx + x;
                for (int a = 0; a < 3; ++a) {
                    double s = 0.0;
                    for (int i = 0; i < L.Q; ++i) {
                        long nb = ((long)(z + L.c[i][2]) * ny + (y + L.c[i][1])) * nx + (x + L.c[i][0]);
                        s += L.w[i] * chi[nb] * L.c[i][a];
                    }
                    grad[3 * cell + a] = s / L.cs2;
                }
            }
    return LBO_OK;
}

/* ------------------------------------------------------------------------ */
/* Simulation                                                                */
/* ------------------------------------------------------------------------ */

enum { S_FLUID = 0, S_NOZ, S_WALL_LO, S_WALL_HI, S_OPEN_LO, S_OPEN_HI, S_LID };

struct lbo_sim {
    lbo_params p;
    lattice_t L;
    double phi[2][QMAX], B[QMAX];
    int nx, ny, nz;
    long N;
    long t;
    double *f[2], *fnew[2], *fc[2];
    unsigned char *solid;
    double *rho[2], *j[3], *u[3], *F[3];
    double *plane_acc; /* per-z-plane partial flux sums (4 per colour) */
    double mass_wall[2], mass_open[2], mass_created[2], mass_deleted[2];
};

typedef struct {
    int type;
    long cell; /* in-box index, -1 for ghosts */
    int x, y, z;
} site_t;

static long cell_index(const lbo_sim *s, int x, int y, int z) { return ((long)z * s->ny + y) * s->nx + x; }

static int wrapi(int a, int n) { return ((a % n) + n) % n; }

/* Head axis at step t, wrapped into [0, n) (Sec. II.B: a constant velocity
 * is an input; the template is translated rigidly). */
static void head_position(const lbo_params *p, int nx, int ny, long t, double *hx, double *hy)
{
    double x = p->noz_x0[0] + p->noz_v[0] * (double)t;
    double y = p->noz_x0[1] + p->noz_v[1] * (double)t;
    *hx = x - (double)nx * floor(x / (double)nx);
    *hy = y - (double)ny * floor(y / (double)ny);
}

/* Squared horizontal distance of column (x, y) from the head axis, with the
 * periodic minimum image. */
static double column_r2(int nx, int ny, int x, int y, double hx, double hy)
{
    double dx = (double)x - hx, dy = (double)y - hy;
    if (dx >= 0.5 * nx) dx -= nx;
    if (dx < -0.5 * nx) dx += nx;
    if (dy >= 0.5 * ny) dy -= ny;
    if (dy < -0.5 * ny) dy += ny;
    return dx * dx + dy * dy;
}

/* Column class: 0 = outside the head, 1 = bore, 2 = shell.  Reading of the 3-D
 * template: a cylindrical shell of inner radius r_in and thickness noz_wall,
 * from z = tip up through the top face; its bore is fluid fed by the lid. */
static int column_class(const lbo_sim *s, int x, int y, double hx, double hy)
{
    const lbo_params *p = &s->p;
    if (!p->has_nozzle) return 0;
    double r2 = column_r2(s->nx, s->ny, x, y, hx, hy);
    double ri2 = p->noz_r_in * p->noz_r_in;
    double ro = p->noz_r_in + p->noz_wall;
    double ro2 = ro * ro;
    if (r2 < ri2) return 1;
    if (r2 < ro2) return 2;
    return 0;
}

static int nozzle_solid(const lbo_sim *s, int x, int y, int z, double hx, double hy)
{
    if (!s->p.has_nozzle) return 0;
    if ((double)z < s->p.noz_tip_z) return 0;
    return column_class(s, x, y, hx, hy) == 2;
}

static void geometry(const lbo_sim *s, long t, unsigned char *solid)
{
    double hx, hy;
    head_position(&s->p, s->nx, s->ny, t, &hx, &hy);
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) solid[cell_index(s, x, y, z)] = (unsigned char)nozzle_solid(s, x, y, z, hx, hy);
}

/* Classify the lattice site (x, y, z) (possibly outside the box) with the
 * geometry of step t.  x, y are periodic; z is periodic or bounded by the z
 * faces; above the top face the head's columns override the face. */
static site_t classify(const lbo_sim *s, const unsigned char *solid, double hx, double hy, int x, int y, int z)
{
    site_t st;
    st.x = wrapi(x, s->nx);
    st.y = wrapi(y, s->ny);
    st.z = z;
    st.cell = -1;
    if (z < 0 || z >= s->nz) {
        int lo = z < 0;
        int face = lo ? s->p.face_zlo : s->p.face_zhi;
        if (face == LBO_PERIODIC) {
            st.z = wrapi(z, s->nz);
        } else {
            if (!lo && s->p.has_nozzle) {
                int cc = column_class(s, st.x, st.y, hx, hy);
                if (cc == 1) {
                    st.type = S_LID;
                    return st;
                }
                if (cc == 2) {
                    st.type = S_NOZ;
                    return st;
                }
            }
            if (face == LBO_WALL)
                st.type = lo ? S_WALL_LO : S_WALL_HI;
            else
                st.type = lo ? S_OPEN_LO : S_OPEN_HI;
            return st;
        }
    }
    st.cell = cell_index(s, st.x, st.y, st.z);
    st.type = solid[st.cell] ? S_NOZ : S_FLUID;
    return st;
}

/* Densities seen at a site by the colour-gradient stencil.
 * Fluid: its own rho^k.  Walls (nozzle, z walls): the fictitious density of
 * Eq. (wet), read as rho_s^k = zeta^k sum_i w_i s_i rho^k(x+c_i) / sum_i w_i s_i
 * over the fluid neighbours (s_i = 1 for a fluid neighbour), zero if the site
 * has no fluid neighbour.  Pressure faces: the imposed densities.  Inlet lid:
 * pure ink at the lid density. */
static void site_rho(const lbo_sim *s, const unsigned char *solid, double hx, double hy, site_t st, double out[2])
{
    const lbo_params *p = &s->p;
    switch (st.type) {
    case S_FLUID:
        out[0] = s->rho[0][st.cell];
        out[1] = s->rho[1][st.cell];
        return;
    case S_OPEN_LO:
        out[0] = p->rho_zlo[0];
        out[1] = p->rho_zlo[1];
        return;
    case S_OPEN_HI:
        out[0] = p->rho_zhi[0];
        out[1] = p->rho_zhi[1];
        return;
    case S_LID:
        out[0] = p->lid_rho_y;
        out[1] = 0.0;
        return;
    default: {
        const double *zeta = st.type == S_NOZ ? p->zeta_noz : p->zeta_wall;
        double num[2] = {0.0, 0.0}, den = 0.0;
        for (int i = 1; i < s->L.Q; ++i) {
            site_t nb = classify(s, solid, hx, hy, st.x + s->L.c[i][0], st.y + s->L.c[i][1], st.z + s->L.c[i][2]);
            if (nb.type != S_FLUID) continue;
            den += s->L.w[i];
            num[0] += s->L.w[i] * s->rho[0][nb.cell];
            num[1] += s->L.w[i] * s->rho[1][nb.cell];
        }
        out[0] = den > 0.0 ? zeta[0] * num[0] / den : 0.0;
        out[1] = den > 0.0 ? zeta[1] * num[1] / den : 0.0;
        return;
    }
    }
}

/* Colour fields at a site: rho^N (reading: the standard phase field
 * (rho_Y/rho_Y^0 - rho_B/rho_B^0) / (rho_Y/rho_Y^0 + rho_B/rho_B^0), zero where
 * both vanish) and the fractions rho_Y/rho, rho_B/rho. */
static void site_colour(const lbo_sim *s, const double r[2], double *chiN, double *chiY, double *chiB)
{
    double a = r[0] / s->p.rho0[0], b = r[1] / s->p.rho0[1];
    double tot = r[0] + r[1];
    *chiN = a + b != 0.0 ? (a - b) / (a + b) : 0.0;
    *chiY = tot != 0.0 ? r[0] / tot : 0.0;
    *chiB = tot != 0.0 ? r[1] / tot : 0.0;
}

/* Moments of the post-stream populations at fluid cells (Sec. II.A):
 * rho^k = sum_i f_i^k, rho u = sum_k sum_i f_i^k c_i, and the force of the
 * drag (Sec. II.B) plus the test body force.  Reading of the drag: it acts on
 * cells with z + 1/2 < drag_range above a z-low wall, as
 * -gamma rho_Y (u - u_wall). */
static void compute_moments(lbo_sim *s)
{
    const lattice_t *L = &s->L;
    const lbo_params *p = &s->p;
    long N = s->N;
#pragma omp parallel for schedule(static) if (N > 8192)
    for (long cell = 0; cell < N; ++cell) {
        if (s->solid[cell]) {
            s->rho[0][cell] = s->rho[1][cell] = 0.0;
            for (int a = 0; a < 3; ++a) s->j[a][cell] = s->u[a][cell] = s->F[a][cell] = 0.0;
            continue;
        }
        double r[2] = {0.0, 0.0}, jj[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 2; ++k)
            for (int i = 0; i < L->Q; ++i) {
                double v = s->f[k][(long)i * N + cell];
                r[k] += v;
                for (int a = 0; a < 3; ++a) jj[a] += v * L->c[i][a];
            }
        double rho = r[0] + r[1];
        int z = (int)(cell / ((long)s->nx * s->ny));
        int drag = p->face_zlo == LBO_WALL && (double)z + 0.5 < p->drag_range;
        s->rho[0][cell] = r[0];
        s->rho[1][cell] = r[1];
        for (int a = 0; a < 3; ++a) {
            s->j[a][cell] = jj[a];
            s->u[a][cell] = jj[a] / rho;
        }
        for (int a = 0; a < 3; ++a) {
            double Fa = rho * p->body_g[a];
            if (drag) Fa += -p->drag_gamma * r[0] * (s->u[a][cell] - p->u_zlo[a]);
            s->F[a][cell] = Fa;
        }
    }
}

/* The collision of one fluid cell, Eq. (cgoperator):
 * Omega = Omega3 [ Omega1 + Omega2 ], with every population regularised
 * (Eq. (reg)) before the BGK step (Eq. (modbgk)); the force enters Omega1 by
 * the exact-difference method; Omega2 (Eq. (pertopform)) is applied once to
 * the colour-blind total; Omega3 recolours. */
static void collide_cell(lbo_sim *s, long cell, int x, int y, int z, double hx, double hy, double *outY, double *outB)
{
    const lattice_t *L = &s->L;
    const lbo_params *p = &s->p;
    const int Q = L->Q;
    const long N = s->N;
    const double cs2 = L->cs2;
    double rk[2] = {s->rho[0][cell], s->rho[1][cell]};
    double rho = rk[0] + rk[1];
    double u[3] = {s->u[0][cell], s->u[1][cell], s->u[2][cell]};
    double du[3], u2[3];
    for (int a = 0; a < 3; ++a) {
        du[a] = s->F[a][cell] / rho;
        u2[a] = u[a] + du[a];
    }

    /* per-colour equilibria, non-equilibrium stresses */
    double fk[2][QMAX], feq[2][QMAX], feq2[2][QMAX], Pi[2][3][3];
    for (int k = 0; k < 2; ++k) {
        for (int i = 0; i < Q; ++i) fk[k][i] = s->f[k][(long)i * N + cell];
        feq_site(L, s->phi[k], rk[k], u, feq[k]);
        feq_site(L, s->phi[k], rk[k], u2, feq2[k]);
        pi_neq(L, fk[k], feq[k], Pi[k]);
    }

    /* ink relaxation time from the strain rate, mixture viscosity Eq. (tauinter) */
    double S2 = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S2 += Pi[0][a][b] * Pi[0][a][b];
    double tauY;
    lbo_tau_ink(p, sqrt(S2), rk[0], NULL, &tauY);
    double nuY = cs2 * (tauY - 0.5), nuB = cs2 * (p->tau_b - 0.5);
    double inv_nu = (rk[0] / rho) / nuY + (rk[1] / rho) / nuB;
    double tau = 0.5 + (1.0 / inv_nu) / cs2;

    /* regularised BGK per colour plus exact-difference forcing, summed */
    double fstar[QMAX];
    for (int i = 0; i < Q; ++i) fstar[i] = 0.0;
    for (int k = 0; k < 2; ++k) {
        double freg[QMAX];
        regularize_site(L, feq[k], Pi[k], freg);
        for (int i = 0; i < Q; ++i) {
            double om1 = -(freg[i] - feq[k][i]) / tau;
            double edm = feq2[k][i] - feq[k][i];
            fstar[i] += freg[i] + om1 + edm;
        }
    }

    /* colour gradients from the neighbours, Eq. (lattgrad) */
    double gN[3] = {0, 0, 0}, gY[3] = {0, 0, 0}, gB[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        site_t nb = classify(s, s->solid, hx, hy, x + L->c[i][0], y + L->c[i][1], z + L->c[i][2]);
        double r[2], cN, cY, cB;
        site_rho(s, s->solid, hx, hy, nb, r);
        site_colour(s, r, &cN, &cY, &cB);
        for (int a = 0; a < 3; ++a) {
            gN[a] += L->w[i] * cN * L->c[i][a] / cs2;
            gY[a] += L->w[i] * cY * L->c[i][a] / cs2;
            gB[a] += L->w[i] * cB * L->c[i][a] / cs2;
        }
    }
    /* colour-gradient force (Sec. II.A) */
    double Fcg[3];
    for (int a = 0; a < 3; ++a) Fcg[a] = rk[1] / rho * gY[a] - rk[0] / rho * gB[a];

    double om2[QMAX];
    perturb_site(L, s->B, p->A, gN, Fcg, om2);
    for (int i = 0; i < Q; ++i) fstar[i] += om2[i];

    recolour_site(L, s->phi[0], s->phi[1], p->beta, p->eps_g, rk[0], rk[1], gN, fstar, outY, outB);
}

static void collide_all(lbo_sim *s)
{
    double hx, hy;
    head_position(&s->p, s->nx, s->ny, s->t, &hx, &hy);
    const int Q = s->L.Q;
    const long N = s->N;
#pragma omp parallel for schedule(dynamic, 1) if (s->N > 8192)
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long cell = cell_index(s, x, y, z);
                if (s->solid[cell]) continue;
                double oY[QMAX], oB[QMAX];
                if (s->p.collide) {
                    collide_cell(s, cell, x, y, z, hx, hy, oY, oB);
                } else {
                    for (int i = 0; i < Q; ++i) {
                        oY[i] = s->f[0][(long)i * N + cell];
                        oB[i] = s->f[1][(long)i * N + cell];
                    }
                }
                for (int i = 0; i < Q; ++i) {
                    s->fc[0][(long)i * N + cell] = oY[i];
                    s->fc[1][(long)i * N + cell] = oB[i];
                }
            }
}

/* Push streaming, Eq. (lbm), with the boundary rules of Sec. II.B applied on
 * links whose far end is not fluid:
 *  - nozzle shell / z walls: moving-wall halfway bounce-back, Eq. (movwall),
 *    f_ibar(x_b, t+1) = f*_i(x_b) - 2 w_i rho_w^k (U . c_i) / c_s^2, with U
 *    the head velocity (nozzle) or the face velocity (z walls) and rho_w^k
 *    extrapolated along -c_i (lbo_wall_density);
 *  - inlet lid: the same rule with U = u_ink + v_nozzle, Eq. (movnozzle), and
 *    imposed rho_w = (lid_rho_y, 0);
 *  - pressure faces: anti-bounce-back,
 *    f_ibar = -f*_i + 2 rho_w^k { phi_i^k + w_i [ (c_i.u_w)^2/(2 c_s^4) - u_w^2/(2 c_s^2) ] },
 *    with the imposed rho_w^k and u_w = (3 u(x_b) - u(x_b - c_i)) / 2.
 * The mass each rule adds is accumulated per colour. */
static void stream_all(lbo_sim *s)
{
    const lattice_t *L = &s->L;
    const lbo_params *p = &s->p;
    const int Q = L->Q;
    const long N = s->N;
    const double cs2 = L->cs2;
    double hx, hy;
    head_position(p, s->nx, s->ny, s->t, &hx, &hy);
    const double vnoz[3] = {p->has_nozzle ? p->noz_v[0] : 0.0, p->has_nozzle ? p->noz_v[1] : 0.0, 0.0};
    for (long q = 0; q < (long)s->nz * 4; ++q) s->plane_acc[q] = 0.0;

#pragma omp parallel for schedule(dynamic, 1) if (s->N > 8192)
    for (int z = 0; z < s->nz; ++z) {
        double acc[4] = {0, 0, 0, 0}; /* wall Y, wall B, open Y, open B */
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long cell = cell_index(s, x, y, z);
                if (s->solid[cell]) continue;
                for (int i = 0; i < Q; ++i) {
                    const int *c = L->c[i];
                    site_t d = classify(s, s->solid, hx, hy, x + c[0], y + c[1], z + c[2]);
                    int ib = L->opp[i];
                    if (d.type == S_FLUID) {
                        for (int k = 0; k < 2; ++k) s->fnew[k][(long)i * N + d.cell] = s->fc[k][(long)i * N + cell];
                        continue;
                    }
                    if (d.type == S_OPEN_LO || d.type == S_OPEN_HI) {
                        const double *rw = d.type == S_OPEN_LO ? p->rho_zlo : p->rho_zhi;
                        double uw[3];
                        site_t in = classify(s, s->solid, hx, hy, x - c[0], y - c[1], z - c[2]);
                        for (int a = 0; a < 3; ++a)
                            uw[a] = in.type == S_FLUID ? (3.0 * s->u[a][cell] - s->u[a][in.cell]) / 2.0 : s->u[a][cell];
                        double cu = c[0] * uw[0] + c[1] * uw[1] + c[2] * uw[2];
                        double uu = uw[0] * uw[0] + uw[1] * uw[1] + uw[2] * uw[2];
                        for (int k = 0; k < 2; ++k) {
                            double out = s->fc[k][(long)i * N + cell];
                            double val = -out + 2.0 * rw[k] * (s->phi[k][i] + L->w[i] * (cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2)));
                            s->fnew[k][(long)ib * N + cell] = val;
                            acc[2 + k] += val - out;
                        }
                        continue;
                    }
                    /* bounce-back family */
                    double U[3];
                    double rw[2];
                    if (d.type == S_LID) {
                        for (int a = 0; a < 3; ++a) U[a] = p->u_ink[a] + vnoz[a];
                        rw[0] = p->lid_rho_y;
                        rw[1] = 0.0;
                    } else {
                        const double *Uw = d.type == S_NOZ ? vnoz : (d.type == S_WALL_LO ? p->u_zlo : p->u_zhi);
                        for (int a = 0; a < 3; ++a) U[a] = Uw[a];
                        site_t s1 = classify(s, s->solid, hx, hy, x - c[0], y - c[1], z - c[2]);
                        site_t s2 = classify(s, s->solid, hx, hy, x - 2 * c[0], y - 2 * c[1], z - 2 * c[2]);
                        int h1 = s1.type == S_FLUID, h2 = h1 && s2.type == S_FLUID;
                        for (int k = 0; k < 2; ++k)
                            rw[k] = lbo_wall_density(s->rho[k][cell], h1 ? s->rho[k][s1.cell] : 0.0,
                                                     h2 ? s->rho[k][s2.cell] : 0.0, h1, h2);
                    }
                    double Uc = U[0] * c[0] + U[1] * c[1] + U[2] * c[2];
                    for (int k = 0; k < 2; ++k) {
                        double out = s->fc[k][(long)i * N + cell];
                        double val = out - 2.0 * L->w[i] * rw[k] * Uc / cs2;
                        s->fnew[k][(long)ib * N + cell] = val;
                        acc[k] += val - out;
                    }
                }
            }
        for (int q = 0; q < 4; ++q) s->plane_acc[4 * z + q] = acc[q];
    }
    for (int z = 0; z < s->nz; ++z) {
        s->mass_wall[0] += s->plane_acc[4 * z + 0];
        s->mass_wall[1] += s->plane_acc[4 * z + 1];
        s->mass_open[0] += s->plane_acc[4 * z + 2];
        s->mass_open[1] += s->plane_acc[4 * z + 3];
    }
}

/* Moving template, Sec. II.B: after the head has moved to its position at
 * step t, fluid nodes now covered by the shell are deleted (their mass is
 * recorded; the infinite-mass head takes no momentum) and nodes released by
 * the shell are created at f^eq(rho_bar^k, v_nozzle), with rho_bar^k the mean
 * density over the lattice neighbours that were fluid before and after the
 * move (reading: a node with no such neighbour takes pure air rho_B^0). */
static void update_geometry(lbo_sim *s, unsigned char *newsolid)
{
    const lattice_t *L = &s->L;
    const int Q = L->Q;
    const long N = s->N;
    const lbo_params *p = &s->p;
    geometry(s, s->t, newsolid);
    const double vnoz[3] = {p->noz_v[0], p->noz_v[1], 0.0};
    /* deletions first, serial and in cell order */
    for (long cell = 0; cell < N; ++cell) {
        if (s->solid[cell] || !newsolid[cell]) continue;
        for (int k = 0; k < 2; ++k) {
            double m = 0.0;
            for (int i = 0; i < Q; ++i) m += s->f[k][(long)i * N + cell];
            s->mass_deleted[k] += m;
        }
    }
    /* creations read only nodes fluid before and after, so the order is free */
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long cell = cell_index(s, x, y, z);
                if (!s->solid[cell] || newsolid[cell]) continue;
                double sum[2] = {0.0, 0.0};
                int count = 0;
                for (int i = 1; i < Q; ++i) {
                    int zz = z + L->c[i][2];
                    if (s->p.face_zlo == LBO_PERIODIC) zz = wrapi(zz, s->nz);
                    if (zz < 0 || zz >= s->nz) continue;
                    long nb = cell_index(s, wrapi(x + L->c[i][0], s->nx), wrapi(y + L->c[i][1], s->ny), zz);
                    if (s->solid[nb] || newsolid[nb]) continue;
                    ++count;
                    for (int k = 0; k < 2; ++k)
                        for (int q = 0; q < Q; ++q) sum[k] += s->f[k][(long)q * N + nb];
                }
                double rbar[2];
                rbar[0] = count ? sum[0] / count : 0.0;
                rbar[1] = count ? sum[1] / count : p->rho0[1];
                for (int k = 0; k < 2; ++k) {
                    double feq[QMAX], m = 0.0;
                    feq_site(L, s->phi[k], rbar[k], vnoz, feq);
                    for (int i = 0; i < Q; ++i) {
                        s->f[k][(long)i * N + cell] = feq[i];
                        m += feq[i];
                    }
                    s->mass_created[k] += m;
                }
            }
    for (long cell = 0; cell < N; ++cell) {
        if (!newsolid[cell]) continue;
        for (int k = 0; k < 2; ++k)
            for (int i = 0; i < Q; ++i) s->f[k][(long)i * N + cell] = 0.0;
    }
    memcpy(s->solid, newsolid, (size_t)N);
}

static int validate(const lbo_params *p)
{
    if (p->lattice != LBO_D2Q9 && p->lattice != LBO_D3Q19) return 0;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return 0;
    if (p->lattice == LBO_D2Q9 && p->ny != 1) return 0;
    if (p->tau_b <= 0.5) return 0;
    if (p->rheology == LBO_NEWTONIAN && p->tau_y <= 0.5) return 0;
    if (p->rheology != LBO_NEWTONIAN && !(p->tau_min > 0.5 && p->tau_max >= p->tau_min)) return 0;
    if (p->rheology < 0 || p->rheology > 2) return 0;
    if (p->rho0[0] <= 0.0 || p->rho0[1] <= 0.0) return 0;
    if ((p->face_zlo == LBO_PERIODIC) != (p->face_zhi == LBO_PERIODIC)) return 0;
    if (p->has_nozzle && p->face_zhi == LBO_PERIODIC) return 0;
    if (p->has_nozzle && (p->noz_tip_z < 0.0 || p->noz_tip_z > p->nz - 1)) return 0;
    return 1;
}

int lbo_create(const lbo_params *p, const double *rho_y, const double *rho_b, const double *u, lbo_sim **out)
{
    if (!p || !out || !rho_y || !rho_b || !validate(p)) return LBO_EINVAL;
    lbo_sim *s = (lbo_sim *)calloc(1, sizeof(lbo_sim));
    if (!s) return LBO_ENOMEM;
    s->p = *p;
    lattice_build(p->lattice, &s->L);
    phi_build(&s->L, p->alpha[0], s->phi[0]);
    phi_build(&s->L, p->alpha[1], s->phi[1]);
    B_build(&s->L, s->B);
    s->nx = p->nx;
    s->ny = p->ny;
    s->nz = p->nz;
    s->N = (long)p->nx * p->ny * p->nz;
    const long N = s->N;
    const int Q = s->L.Q;
    int ok = 1;
    for (int k = 0; k < 2; ++k) {
        s->f[k] = (double *)calloc((size_t)Q * N, sizeof(double));
        s->fnew[k] = (double *)calloc((size_t)Q * N, sizeof(double));
        s->fc[k] = (double *)calloc((size_t)Q * N, sizeof(double));
        s->rho[k] = (double *)calloc((size_t)N, sizeof(double));
        ok = ok && s->f[k] && s->fnew[k] && s->fc[k] && s->rho[k];
    }
    for (int a = 0; a < 3; ++a) {
        s->j[a] = (double *)calloc((size_t)N, sizeof(double));
        s->u[a] = (double *)calloc((size_t)N, sizeof(double));
        s->F[a] = (double *)calloc((size_t)N, sizeof(double));
        ok = ok && s->j[a] && s->u[a] && s->F[a];
    }
    s->solid = (unsigned char *)calloc((size_t)N, 1);
    s->plane_acc = (double *)calloc((size_t)s->nz * 4, sizeof(double));
    if (!ok || !s->solid || !s->plane_acc) {
        lbo_destroy(s);
        return LBO_ENOMEM;
    }
    geometry(s, 0, s->solid);
    /* initial state: f = f^eq(rho^k, u) at fluid nodes */
    for (long cell = 0; cell < N; ++cell) {
        if (s->solid[cell]) continue;
        double uc[3] = {0, 0, 0};
        if (u)
            for (int a = 0; a < 3; ++a) uc[a] = u[3 * cell + a];
        double r[2] = {rho_y[cell], rho_b[cell]};
        for (int k = 0; k < 2; ++k) {
            double feq[QMAX];
            feq_site(&s->L, s->phi[k], r[k], uc, feq);
            for (int i = 0; i < Q; ++i) s->f[k][(long)i * N + cell] = feq[i];
        }
    }
    *out = s;
    return LBO_OK;
}

int lbo_step(lbo_sim *s, int nsteps)
{
    if (!s || nsteps < 0) return LBO_EINVAL;
    unsigned char *newsolid = (unsigned char *)malloc((size_t)s->N);
    if (!newsolid) return LBO_ENOMEM;
    for (int n = 0; n < nsteps; ++n) {
        compute_moments(s);
        collide_all(s);
        stream_all(s);
        for (int k = 0; k < 2; ++k) {
            double *tmp = s->f[k];
            s->f[k] = s->fnew[k];
            s->fnew[k] = tmp;
        }
        s->t += 1;
        update_geometry(s, newsolid);
    }
    free(newsolid);
    return LBO_OK;
}

/* Fields at the current step: rho_Y, rho_B and the physical velocity
 * u = (sum f c + F/2) / rho of the exact-difference method; zero at solid
 * nodes.  Conserved sums are over fluid nodes, with the cumulative mass
 * added by each boundary rule and by node creation / deletion. */
int lbo_moments(lbo_sim *s, double *rho_y, double *rho_b, double *u, lbo_conserved *cons)
{
    if (!s) return LBO_EINVAL;
    compute_moments(s);
    const long N = s->N;
    for (long cell = 0; cell < N; ++cell) {
        double rho = s->rho[0][cell] + s->rho[1][cell];
        if (rho_y) rho_y[cell] = s->rho[0][cell];
        if (rho_b) rho_b[cell] = s->rho[1][cell];
        if (u)
            for (int a = 0; a < 3; ++a)
                u[3 * cell + a] = s->solid[cell] ? 0.0 : (s->j[a][cell] + 0.5 * s->F[a][cell]) / rho;
    }
    if (cons) {
        memset(cons, 0, sizeof(*cons));
        double *pl = (double *)calloc((size_t)s->nz * 5, sizeof(double));
        if (!pl) return LBO_ENOMEM;
        long plane = (long)s->nx * s->ny;
        for (int z = 0; z < s->nz; ++z) {
            for (long c = 0; c < plane; ++c) {
                long cell = (long)z * plane + c;
                if (s->solid[cell]) continue;
                pl[5 * z + 0] += s->rho[0][cell];
                pl[5 * z + 1] += s->rho[1][cell];
                for (int a = 0; a < 3; ++a) pl[5 * z + 2 + a] += s->j[a][cell];
            }
        }
        for (int z = 0; z < s->nz; ++z) {
            cons->mass[0] += pl[5 * z + 0];
            cons->mass[1] += pl[5 * z + 1];
            for (int a = 0; a < 3; ++a) cons->mom[a] += pl[5 * z + 2 + a];
        }
        free(pl);
        for (int k = 0; k < 2; ++k) {
            cons->mass_wall[k] = s->mass_wall[k];
            cons->mass_open[k] = s->mass_open[k];
            cons->mass_created[k] = s->mass_created[k];
            cons->mass_deleted[k] = s->mass_deleted[k];
        }
    }
    return LBO_OK;
}

int lbo_get_f(lbo_sim *s, int k, double *out)
{
    if (!s || k < 0 || k > 1 || !out) return LBO_EINVAL;
    memcpy(out, s->f[k], sizeof(double) * (size_t)s->L.Q * s->N);
    return LBO_OK;
}

int lbo_set_f(lbo_sim *s, int k, const double *in)
{
    if (!s || k < 0 || k > 1 || !in) return LBO_EINVAL;
    memcpy(s->f[k], in, sizeof(double) * (size_t)s->L.Q * s->N);
    return LBO_OK;
}

int lbo_solid(lbo_sim *s, unsigned char *out)
{
    if (!s || !out) return LBO_EINVAL;
    memcpy(out, s->solid, (size_t)s->N);
    return LBO_OK;
}

int lbo_velocity_index(lbo_sim *s, int *c)
{
    if (!s || !c) return LBO_EINVAL;
    for (int i = 0; i < s->L.Q; ++i)
        for (int a = 0; a < 3; ++a) c[3 * i + a] = s->L.c[i][a];
    return s->L.Q;
}

long lbo_time(lbo_sim *s) { return s ? s->t : -1; }

/* Threads the OpenMP loops use (1 without OpenMP), and a way to change it
 * (the CPU baseline's single-thread leg). */
int lbo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void lbo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void lbo_destroy(lbo_sim *s)
{
    if (!s) return;
    for (int k = 0; k < 2; ++k) {
        free(s->f[k]);
        free(s->fnew[k]);
        free(s->fc[k]);
        free(s->rho[k]);
    }
    for (int a = 0; a < 3; ++a) {
        free(s->j[a]);
        free(s->u[a]);
        free(s->F[a]);
    }
    free(s->solid);
    free(s->plane_acc);
    free(s);
}
