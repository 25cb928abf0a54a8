/*
 * oracle.c -- plain, slow CPU reference for one implicit-explicit Runge-Kutta
 * step of special/general-relativistic resistive MHD on a fixed (Cowling)
 * Cartesian grid, following Cheong et al., "An extension of Gmunu:
 * general-relativistic resistive magnetohydrodynamics based on staggered-meshed
 * constrained transport with elliptic cleaning" (arXiv:2110.03732).
 *
 * TEST INFRASTRUCTURE ONLY.  The HIP library is tested against this file,
 * which is no part of it: only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header or table with the GPU
 * path.  Everything is FP64, evaluated in the paper's order and notation with a
 * general 3x3 spatial metric gamma_ij = psi^4 delta_ij (conformally flat,
 * beta^i = 0, K_ij = 0), explicit Levi-Civita symbols and plain loops.
 * Build with -O2 -ffp-contract=off.
 *
 * Sections of the paper followed (cited by section / equation name):
 *   Sec 2.1   conserved variables q, fluxes f^i, sources s, Gauss law
 *   Sec 2.2   Ohm's law (eq. ohms_law), stiff / non-stiff current split
 *   Sec 2.3   IMEX-RK scheme and Table imex_ssp2
 *   Sec 2.4   implicit E update (eq. im_E), A_0..A_5, their W-derivatives,
 *             velocity residual (eq. f_u_for_e), Jacobian, Newton iteration
 *   Sec 2.5   maximum-diffusivity characteristic speeds
 *   Sec 2.6   conservative-to-primitive recovery with E and B given
 *   Sec 3.1   GLM hyperbolic divergence cleaning (cell-centred B, Psi, Phi)
 *   Sec 3.2   staggered constrained transport (eq. B_surface, eq. ct) and the
 *             HLL-based upwind EMF, steps (i)-(vii)
 *   App. A    the ideal-MHD form of the upwind EMF (transport velocities)
 *   Sec 4     face fields from an edge vector potential
 *   Sec 5.7   mean-field dynamo (xi != 0) in the implicit update
 * Readings of places where the paper is silent or garbled are stated next to
 * the code that takes them.
 *
 * Rules the paper leaves unstated are taken as readings (the PPM variant,
 * the ghost rules, the time step convention, the atmosphere / failure
 * fallback, the threshold and clamp of eq. sigma_D).  The test-suite pins
 * each of them from outside this file: the rule as the reading states it,
 * evaluated by hand (the decay rate of a cell at rest gives the eta used, the
 * fallback state and field of forced atmosphere and failure cells, the ghost
 * copies, the closed-form time steps), or a property every implementation of
 * the rule has (a limited PPM parabola is monotone and keeps the cell mean).

 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* problem description (mirrored by a ctypes Structure in oracle/__init__.py) */
typedef struct {
    int ndim;            /* 1, 2 or 3 active directions (x, then y, then z)   */
    int n[3];            /* interior cells per direction (1 when inactive)    */
    int ng;              /* ghost width of active directions                  */
    double lo[3], hi[3]; /* domain                                            */
    int bc[3][2];        /* 0 outflow, 1 periodic, 2 fixed                    */
    double gamma_ad;     /* ideal gas p = (Gamma-1) rho eps                   */
    int recon;           /* 0 minmod, 1 MC, 2 PPM                             */
    int imex;            /* 0 IMEX-SSP2(2,2,2), 1 IMEX-SSP3(4,3,3)            */
    double cfl;
    int eta_mode;        /* 0 uniform eta, 1 eta = 1/sigma(D) (eq. sigma_D)   */
    double eta, sigma0, eta_min, eta_max;
    double rho_atm, p_atm;
    int metric;          /* 0 flat, 1 static conformally flat (alpha, psi)    */
    double newton_tol;
    int newton_maxit;
    double xi;           /* mean-field dynamo coefficient of eq. ohms_law     */
    double atm_factor;   /* cells with D <= atm_factor rho_atm are atmosphere */
    int frozen_matter;   /* 1: rho, u~, p stay fixed, only E and B evolve     */
    int glm;             /* 1: cell-centred B with GLM cleaning (Sec 3.1)     */
    double kappa_E, kappa_B; /* GLM damping parameters                        */
    int uct;             /* 0: resistive upwind CT (Sec 3.2), 1: the ideal-MHD
                            form of App. A (edge E from transport velocities)  */
} or_grid;

enum { BC_OUTFLOW = 0, BC_PERIODIC = 1, BC_FIXED = 2 };
enum { RC_MINMOD = 0, RC_MC = 1, RC_PPM = 2 };

/* ------------------------------------------------------------------------- */
/* small tensor helpers on gamma_ij = psi^4 delta_ij                          */
typedef struct { double g[3][3], gi[3][3], sqrtg; } metric3;

static void mk_metric(double psi, metric3 *m)
{
    double p4 = psi * psi * psi * psi;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            m->g[i][j] = (i == j) ? p4 : 0.0;
            m->gi[i][j] = (i == j) ? 1.0 / p4 : 0.0;
        }
    m->sqrtg = p4 * psi * psi; /* sqrt(det gamma) = psi^6 */
}

/* 3-d Levi-Civita symbol eta_{ijk}, indices 0..2 */
static const double LEVI[3][3][3] = {{{0, 0, 0}, {0, 0, 1}, {0, -1, 0}},
                                     {{0, 0, -1}, {0, 0, 0}, {1, 0, 0}},
                                     {{0, 1, 0}, {-1, 0, 0}, {0, 0, 0}}};
static double levi(int i, int j, int k) { return LEVI[i][j][k]; }
static double pow6(double x) { return x * x * x * x * x * x; }
static double pow4(double x) { return x * x * x * x; }

static void lower(const metric3 *m, const double a[3], double out[3])
{
    for (int i = 0; i < 3; i++) {
        out[i] = 0.0;
        for (int j = 0; j < 3; j++) out[i] += m->g[i][j] * a[j];
    }
}
static void raise_(const metric3 *m, const double a[3], double out[3])
{
    for (int i = 0; i < 3; i++) {
        out[i] = 0.0;
        for (int j = 0; j < 3; j++) out[i] += m->gi[i][j] * a[j];
    }
}
/* a^i gamma_ij b^j */
static double dotg(const metric3 *m, const double a[3], const double b[3])
{
    double s = 0.0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) s += a[i] * m->g[i][j] * b[j];
    return s;
}
/* epsilon_{ilm} a^l b^m with epsilon_{ilm} = sqrt(gamma) eta_{ilm} (covariant result) */
static void cross_low(const metric3 *m, const double a[3], const double b[3], double out[3])
{
    for (int i = 0; i < 3; i++) {
        out[i] = 0.0;
        for (int l = 0; l < 3; l++)
            for (int n = 0; n < 3; n++) out[i] += m->sqrtg * levi(i, l, n) * a[l] * b[n];
    }
}
/* epsilon^{ijk} a_j b_k with epsilon^{ijk} = eta^{ijk}/sqrt(gamma), a, b given contravariant */
static void cross_up(const metric3 *m, const double a[3], const double b[3], double out[3])
{
    double al[3], bl[3];
    lower(m, a, al);
    lower(m, b, bl);
    for (int i = 0; i < 3; i++) {
        out[i] = 0.0;
        for (int j = 0; j < 3; j++)
            for (int k = 0; k < 3; k++) out[i] += levi(i, j, k) / m->sqrtg * al[j] * bl[k];
    }
}

/* ------------------------------------------------------------------------- */
/* Sec 2.1: conserved variables from primitives.
 * prim = (rho, u~^1..3, p) with u~^i = W v^i; E^i, B^i contravariant.
 * q = psi^6 (D, S_j, tau, E^j) (sqrt(gamma_bar/gamma_hat) = 1 here). */
void or_prim2cons(double gam, double psi, const double prim[5], const double E[3], const double B[3],
                  double q[8])
{
    metric3 m;
    mk_metric(psi, &m);
    double rho = prim[0], p = prim[4];
    double ut[3] = {prim[1], prim[2], prim[3]};
    double W = sqrt(1.0 + dotg(&m, ut, ut));
    double v[3], vl[3], ExB[3];
    for (int i = 0; i < 3; i++) v[i] = ut[i] / W;
    lower(&m, v, vl);
    double eps = p / ((gam - 1.0) * rho);
    double h = 1.0 + eps + p / rho;
    double E2 = dotg(&m, E, E), B2 = dotg(&m, B, B);
    cross_low(&m, E, B, ExB);
    double D = rho * W;
    double tau = rho * h * W * W - p + 0.5 * (E2 + B2) - D;
    q[0] = m.sqrtg * D;
    for (int j = 0; j < 3; j++) q[1 + j] = m.sqrtg * (rho * h * W * W * vl[j] + ExB[j]);
    q[4] = m.sqrtg * tau;
    for (int j = 0; j < 3; j++) q[5 + j] = m.sqrtg * E[j];
}

/* Sec 2.1: fluxes f^i of (q_D, q_S_j, q_tau, q_E^j) in direction dir, beta = 0. */
void or_flux(int dir, double gam, double alpha, double psi, const double prim[5], const double E[3],
             const double B[3], double f[8])
{
    metric3 m;
    mk_metric(psi, &m);
    double rho = prim[0], p = prim[4];
    double ut[3] = {prim[1], prim[2], prim[3]};
    double W = sqrt(1.0 + dotg(&m, ut, ut));
    double v[3], vl[3], El[3], Bl[3], ExB[3], S[3], Su[3];
    for (int i = 0; i < 3; i++) v[i] = ut[i] / W;
    lower(&m, v, vl);
    lower(&m, E, El);
    lower(&m, B, Bl);
    double eps = p / ((gam - 1.0) * rho);
    double h = 1.0 + eps + p / rho;
    double E2 = dotg(&m, E, E), B2 = dotg(&m, B, B);
    cross_low(&m, E, B, ExB);
    double D = rho * W;
    for (int j = 0; j < 3; j++) S[j] = rho * h * W * W * vl[j] + ExB[j];
    raise_(&m, S, Su);
    int i = dir;
    double vhat = alpha * v[i]; /* v^i_hat = alpha v^i - beta^i */
    f[0] = m.sqrtg * D * vhat;
    for (int j = 0; j < 3; j++) {
        double Sij = (p + 0.5 * (E2 + B2)) * (i == j ? 1.0 : 0.0) + rho * h * W * W * v[i] * vl[j] - E[i] * El[j] -
                     B[i] * Bl[j];
        f[1 + j] = m.sqrtg * alpha * Sij;
    }
    f[4] = m.sqrtg * alpha * (Su[i] - v[i] * D);
    /* (f_E^j)^i = psi^6 [ - epsilon^{jik} Bhat_k ], Bhat_k = alpha B_k */
    for (int j = 0; j < 3; j++) {
        double s = 0.0;
        for (int k = 0; k < 3; k++) s += levi(j, i, k) / m.sqrtg * alpha * Bl[k];
        f[5 + j] = -m.sqrtg * s;
    }
}

/* (f_B^j)^i = psi^6 epsilon^{jik} Ehat_k (used only by the 1-D reduction check) */
void or_flux_B(int dir, double alpha, double psi, const double E[3], double fB[3])
{
    metric3 m;
    mk_metric(psi, &m);
    double El[3];
    lower(&m, E, El);
    for (int j = 0; j < 3; j++) {
        double s = 0.0;
        for (int k = 0; k < 3; k++) s += levi(j, dir, k) / m.sqrtg * alpha * El[k];
        fB[j] = m.sqrtg * s;
    }
}

/* ------------------------------------------------------------------------- */
/* Sec 2.6: primitives from conserved variables when E and B are known.
 * The electromagnetic part is removed (S_f = S - E x B, tau_f = tau - U_EM)
 * and the hydrodynamic recovery is a root in the pressure p of
 *   g(p) = (Gamma-1) rho eps(p) - p,  v = S_f/(tau_f + D + p),  rho = D/W,
 *   rho eps = [tau_f + D(1-W) + p(1-W^2)]/W^2,
 * found by plain bisection (the root, not an iterate sequence, is the result).
 * Returns 0 on success, 1 when no physical root exists. */
static double c2p_g(double gam, double p, double D, double tauf, double Sf2, double *W_out)
{
    double Z = tauf + D + p;
    double v2 = Sf2 / (Z * Z);
    if (v2 >= 1.0) { *W_out = INFINITY; return -INFINITY; }
    double W = 1.0 / sqrt(1.0 - v2);
    double rho = D / W;
    double rhoeps = (tauf + D * (1.0 - W) + p * (1.0 - W * W)) / (W * W);
    (void)rho;
    *W_out = W;
    return (gam - 1.0) * rhoeps - p;
}

int or_c2p(double gam, double psi, const double q[8], const double E[3], const double B[3], double prim[5])
{
    metric3 m;
    mk_metric(psi, &m);
    double D = q[0] / m.sqrtg, tau = q[4] / m.sqrtg;
    double S[3], ExB[3], Sf[3], Sfu[3];
    for (int j = 0; j < 3; j++) S[j] = q[1 + j] / m.sqrtg;
    cross_low(&m, E, B, ExB);
    for (int j = 0; j < 3; j++) Sf[j] = S[j] - ExB[j];
    raise_(&m, Sf, Sfu);
    double Sf2 = 0.0;
    for (int j = 0; j < 3; j++) Sf2 += Sfu[j] * Sf[j];
    double UEM = 0.5 * (dotg(&m, E, E) + dotg(&m, B, B));
    double tauf = tau - UEM;
    if (!(D > 0.0)) return 1;
    double plo = sqrt(Sf2) - tauf - D;
    if (plo < 0.0) plo = 0.0;
    double phi = plo + 2.0 * (gam - 1.0) * fabs(tauf) + 1e-300;
    double Wt;
    /* root must lie in (plo, phi]; g(phi) < 0 because rho eps <= tau_f */
    if (c2p_g(gam, phi, D, tauf, Sf2, &Wt) > 0.0) return 1;
    double glo = c2p_g(gam, plo, D, tauf, Sf2, &Wt);
    if (plo == 0.0 && glo < 0.0) return 1;    /* no root with p >= 0 */
    if (plo == 0.0 && glo == 0.0) phi = 0.0;  /* exact root at p = 0 */
    double a = plo, b = phi;
    for (int it = 0; it < 2000 && b > a; it++) {
        double c = 0.5 * (a + b);
        if (c <= a || c >= b) break;
        if (c2p_g(gam, c, D, tauf, Sf2, &Wt) > 0.0) a = c;
        else b = c;
    }
    double p = (plo == 0.0 && phi == 0.0) ? 0.0 : 0.5 * (a + b);
    double Z = tauf + D + p;
    double v2 = Sf2 / (Z * Z);
    if (!(v2 < 1.0)) return 1;
    double W = 1.0 / sqrt(1.0 - v2);
    prim[0] = D / W;
    for (int i = 0; i < 3; i++) prim[1 + i] = W * Sfu[i] / Z;
    prim[4] = p;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sec 2.4, eq. im_E and the A_0..A_5 coefficients with their W-derivatives.
 * etat = eta/(alpha a_ii dt) inside an IMEX stage (reading of the "n -> n+1"
 * notation of the paper: the implicit sub-step of stage i spans a_ii dt). */
typedef struct { double A[6], Ad[6]; } acoef;

static void or_coeffs(double W, double et, double xi, acoef *c)
{
    double x2 = xi * xi;
    double Wpe = W + et, opW = 1.0 + W * et;
    c->A[0] = W + et + x2 * (W * W - 1.0) / Wpe;
    c->A[1] = et / opW + x2 * et * W / (Wpe * opW);
    c->A[2] = -xi * et / Wpe;
    c->A[3] = xi * opW / Wpe;
    c->A[4] = xi * (1.0 - et * et + x2) / (Wpe * opW);
    c->A[5] = -1.0 - x2 * W / Wpe;
    c->Ad[0] = 1.0 + x2 * (1.0 + W * W + 2.0 * W * et) / (Wpe * Wpe);
    c->Ad[1] = -et * et / (opW * opW) - x2 * et * et * (W * W - 1.0) / (opW * opW * Wpe * Wpe);
    c->Ad[2] = xi * et / (Wpe * Wpe);
    c->Ad[3] = xi * (et * et - 1.0) / (Wpe * Wpe);
    c->Ad[4] = -xi * (1.0 - et * et + x2) * (1.0 + et * et + 2.0 * W * et) / (opW * opW * Wpe * Wpe);
    c->Ad[5] = -x2 * et / (Wpe * Wpe);
}

/* E^{i,n+1}(u~) from eq. im_E */
static void or_E_of_u(const metric3 *m, const double ut[3], const double Es[3], const double B[3], double et,
                      double xi, double W, const acoef *c, double E[3])
{
    double Esu = dotg(m, Es, ut), Bu = dotg(m, B, ut);
    double uxEs[3], uxB[3];
    cross_up(m, ut, Es, uxEs); /* epsilon^{ijk} u~_j E*_k */
    cross_up(m, ut, B, uxB);
    (void)W;
    (void)xi;
    for (int i = 0; i < 3; i++)
        E[i] = (et * Es[i] + c->A[1] * Esu * ut[i] + c->A[2] * uxEs[i] + c->A[3] * B[i] + c->A[4] * Bu * ut[i] +
                c->A[5] * uxB[i]) /
               c->A[0];
}

/* exported for the tests: E(u~) of eq. im_E for a given u~ */
void or_implicit_E(double psi, double etat, double xi, const double ut[3], const double Es[3], const double B[3],
                   double E[3])
{
    metric3 m;
    mk_metric(psi, &m);
    double W = sqrt(1.0 + dotg(&m, ut, ut));
    acoef c;
    or_coeffs(W, etat, xi, &c);
    or_E_of_u(&m, ut, Es, B, etat, xi, W, &c, E);
}

/* residual f_i(u~) of eq. f_u_for_e and its Jacobian J_ij (analytic, Sec 2.4).
 * Readings of the garbled Jacobian (Sec 2.4, eq. f_u_for_e): the Levi-Civita
 * term of dS_EM/du~^j carries the derivative of E^l, contracted with B^m;
 * the electric part of dw~/du~^j is W times the derivative of the field
 * energy, -W E_l dE^l/du~^j; every velocity derivative is taken with respect
 * to u~. */
typedef struct {
    double gam, G1, D, tau, S[3], Es[3], B[3], et, xi;
    const metric3 *m;
} isys;

static void or_residual(const isys *s, const double ut[3], double f[3], double J[3][3], double E_out[3],
                        double *wt_out)
{
    const metric3 *m = s->m;
    double W = sqrt(1.0 + dotg(m, ut, ut));
    acoef c;
    or_coeffs(W, s->et, s->xi, &c);
    double E[3];
    or_E_of_u(m, ut, s->Es, s->B, s->et, s->xi, W, &c, E);
    double UEM = 0.5 * (dotg(m, E, E) + dotg(m, s->B, s->B));
    double den = W * W - 1.0 / s->G1;
    double wt = (W * (s->tau + s->D - UEM) - s->D / s->G1) / den;
    double ul[3], ExB[3];
    lower(m, ut, ul);
    cross_low(m, E, s->B, ExB);
    for (int i = 0; i < 3; i++) f[i] = wt * ul[i] - (s->S[i] - ExB[i]);
    if (E_out) for (int i = 0; i < 3; i++) E_out[i] = E[i];
    if (wt_out) *wt_out = wt;
    if (!J) return;
    /* A_0 W dE^i/du~^j */
    double Esl[3], Bl[3], El[3];
    lower(m, s->Es, Esl);
    lower(m, s->B, Bl);
    lower(m, E, El);
    double Esu = dotg(m, s->Es, ut), Bu = dotg(m, s->B, ut);
    double dE[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double dij = (i == j) ? 1.0 : 0.0; /* gamma^i_j */
            double t = -c.Ad[0] * E[i] * ul[j] + c.A[1] * W * ut[i] * Esl[j] + c.Ad[3] * s->B[i] * ul[j] +
                       c.A[4] * W * ut[i] * Bl[j] + (c.A[1] * W * dij + c.Ad[1] * ut[i] * ul[j]) * Esu +
                       (c.A[4] * W * dij + c.Ad[4] * ut[i] * ul[j]) * Bu;
            for (int l = 0; l < 3; l++)
                for (int n = 0; n < 3; n++) {
                    double eps = levi(i, l, n) / m->sqrtg;
                    if (eps == 0.0) continue;
                    t += eps * (c.A[2] * W * m->g[l][j] + c.Ad[2] * ul[l] * ul[j]) * Esl[n];
                    t += eps * (c.A[5] * W * m->g[l][j] + c.Ad[5] * ul[l] * ul[j]) * Bl[n];
                }
            dE[i][j] = t / (c.A[0] * W);
        }
    for (int j = 0; j < 3; j++) {
        double dU = 0.0;
        for (int l = 0; l < 3; l++) dU += El[l] * dE[l][j];
        double dw = ((s->tau + s->D - UEM) * ul[j] / W - 2.0 * wt * ul[j] - W * dU) / den;
        for (int i = 0; i < 3; i++) {
            double t = wt * m->g[i][j] + ul[i] * dw;
            for (int l = 0; l < 3; l++)
                for (int n = 0; n < 3; n++) t += m->sqrtg * levi(i, l, n) * dE[l][j] * s->B[n];
            J[i][j] = t;
        }
    }
}

/* exported for the finite-difference check of the Jacobian */
void or_implicit_residual(double gam, double psi, const double q[8], const double B[3], double etat, double xi,
                          const double ut[3], double f[3], double J[9])
{
    metric3 m;
    mk_metric(psi, &m);
    isys s;
    s.gam = gam;
    s.G1 = gam / (gam - 1.0);
    s.D = q[0] / m.sqrtg;
    s.tau = q[4] / m.sqrtg;
    for (int i = 0; i < 3; i++) {
        s.S[i] = q[1 + i] / m.sqrtg;
        s.Es[i] = q[5 + i] / m.sqrtg;
        s.B[i] = B[i];
    }
    s.et = etat;
    s.xi = xi;
    s.m = &m;
    double JJ[3][3];
    or_residual(&s, ut, f, J ? JJ : NULL, NULL, NULL);
    if (J)
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) J[3 * i + j] = JJ[i][j];
}

/* 3x3 linear solve by Gaussian elimination with partial pivoting */
static int solve3(double A[3][3], const double b[3], double x[3])
{
    double M[3][4];
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) M[i][j] = A[i][j];
        M[i][3] = b[i];
    }
    for (int c = 0; c < 3; c++) {
        int piv = c;
        for (int r = c + 1; r < 3; r++)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        if (M[piv][c] == 0.0) return 1;
        if (piv != c)
            for (int j = 0; j < 4; j++) {
                double t = M[c][j];
                M[c][j] = M[piv][j];
                M[piv][j] = t;
            }
        for (int r = c + 1; r < 3; r++) {
            double fct = M[r][c] / M[c][c];
            for (int j = c; j < 4; j++) M[r][j] -= fct * M[c][j];
        }
    }
    for (int i = 2; i >= 0; i--) {
        double s = M[i][3];
        for (int j = i + 1; j < 3; j++) s -= M[i][j] * x[j];
        x[i] = s / M[i][i];
    }
    return 0;
}

/* Sec 2.4: fused implicit E update + conservative-to-primitive recovery.
 * Globally convergent multi-dimensional Newton iteration on u~ (backtracking
 * line search on F = f.f/2 with sufficient-decrease constant 1e-4, quadratic
 * backtracking model, step cut never below 0.1 of the previous one).
 * q = densitised (q_D, q_S, q_tau, q_E*) of the explicit stage update.
 * Returns 0 on convergence, 1 on failure.  On success writes prim (rho, u~, p)
 * and the new E^i (contravariant, not densitised). */
int or_implicit(double gam, double psi, const double q[8], const double B[3], double etat, double xi,
                const double guess[3], double tol, int maxit, double prim[5], double Eout[3], int *iters)
{
    metric3 m;
    mk_metric(psi, &m);
    isys s;
    s.gam = gam;
    s.G1 = gam / (gam - 1.0);
    s.D = q[0] / m.sqrtg;
    s.tau = q[4] / m.sqrtg;
    for (int i = 0; i < 3; i++) {
        s.S[i] = q[1 + i] / m.sqrtg;
        s.Es[i] = q[5 + i] / m.sqrtg;
        s.B[i] = B[i];
    }
    s.et = etat;
    s.xi = xi;
    s.m = &m;
    double ut[3] = {guess[0], guess[1], guess[2]};
    double f[3], J[3][3], E[3], wt;
    int conv = 0, it;
    or_residual(&s, ut, f, J, E, &wt);
    double F = 0.5 * (f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (it = 0; it < maxit; it++) {
        double dx[3], mf[3] = {-f[0], -f[1], -f[2]};
        if (solve3(J, mf, dx)) break;
        double dmax = 0.0, umax = 0.0;
        for (int i = 0; i < 3; i++) {
            if (fabs(dx[i]) > dmax) dmax = fabs(dx[i]);
            if (fabs(ut[i]) > umax) umax = fabs(ut[i]);
        }
        /* stopping rule (reading; the paper gives none): the step is below
         * tol [(1 + max|u~|) W^2 + (|S| + |E||B|)/w~], the size to which
         * rounding fixes u~.  Rounding of S and tau fixes v only to a relative
         * eps, and u~ = W v then only to eps W^2; the residual w~ u~ - (S -
         * E x B) carries rounding of size eps (|S| + |E||B|), which a strong
         * field makes large against w~.  A threshold without these factors
         * cannot be met at high Lorentz factor or magnetisation; the step
         * that meets this one is taken, and Newton's quadratic convergence
         * leaves the iterate after it far below the threshold. */
        double W2 = 1.0 + dotg(&m, ut, ut);
        double Sn = sqrt(s.S[0] * s.S[0] + s.S[1] * s.S[1] + s.S[2] * s.S[2]) / (psi * psi);
        double em = sqrt(dotg(&m, E, E) * dotg(&m, s.B, s.B));
        if (dmax <= tol * ((1.0 + umax) * W2 + (wt > 0.0 ? (Sn + em) / wt : 0.0))) {
            /* the full Newton step is below the tolerance: take it and stop */
            for (int i = 0; i < 3; i++) ut[i] += dx[i];
            or_residual(&s, ut, f, J, E, &wt);
            conv = 1;
            it++;
            break;
        }
        double slope = -2.0 * F; /* grad F . dx = f^T J dx = -f.f for the Newton direction */
        double lam = 1.0, un[3], fn[3], Fn;
        int ok = 0;
        for (int ls = 0; ls < 60; ls++) {
            for (int i = 0; i < 3; i++) un[i] = ut[i] + lam * dx[i];
            or_residual(&s, un, fn, NULL, NULL, NULL);
            Fn = 0.5 * (fn[0] * fn[0] + fn[1] * fn[1] + fn[2] * fn[2]);
            if (isfinite(Fn) && Fn <= F + 1e-4 * lam * slope) { ok = 1; break; }
            double lnew = isfinite(Fn) ? -slope * lam * lam / (2.0 * (Fn - F - slope * lam)) : 0.1 * lam;
            if (!(lnew >= 0.1 * lam)) lnew = 0.1 * lam;
            if (lnew > 0.5 * lam) lnew = 0.5 * lam;
            lam = lnew;
        }
        if (!ok) break; /* no acceptable step along the Newton direction */
        for (int i = 0; i < 3; i++) ut[i] += lam * dx[i];
        or_residual(&s, ut, f, J, E, &wt);
        F = 0.5 * (f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    }
    if (iters) *iters = it;
    if (!conv) return 1;
    double W = sqrt(1.0 + dotg(&m, ut, ut));
    double rho = s.D / W;
    double p = (wt / W - rho) / s.G1; /* w~ = rho h W, rho h = rho + Gamma_1 p */
    prim[0] = rho;
    for (int i = 0; i < 3; i++) prim[1 + i] = ut[i];
    prim[4] = p;
    for (int i = 0; i < 3; i++) Eout[i] = E[i];
    return 0;
}

/* ------------------------------------------------------------------------- */
/* reconstruction (one variable, one face, six-point window w[0..5] = cells
 * i-3..i+2 around the face i-1/2 between w[2] and w[3]).  minmod and MC
 * (monotonized central) use w[1..4]; PPM (Colella-Woodward interface value,
 * clipped between neighbours, then the two monotonicity constraints; no
 * steepening or flattening) uses w[0..5]. */
static double minmod2(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return (fabs(a) < fabs(b)) ? a : b;
}
static double minmod3(double a, double b, double c)
{
    if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
    if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
    return 0.0;
}
static double mc_slope(double l, double c, double r) { return minmod3(0.5 * (r - l), 2.0 * (c - l), 2.0 * (r - c)); }
static double ppm_iface(double am1, double a0, double a1, double a2)
{
    double v = 7.0 / 12.0 * (a0 + a1) - 1.0 / 12.0 * (am1 + a2);
    double lo = fmin(a0, a1), hi = fmax(a0, a1);
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}
static void ppm_mono(double a, double *aL, double *aR)
{
    if ((*aR - a) * (a - *aL) <= 0.0) {
        *aL = a;
        *aR = a;
        return;
    }
    double d = *aR - *aL, mm = a - 0.5 * (*aL + *aR);
    if (d * mm > d * d / 6.0) *aL = 3.0 * a - 2.0 * *aR;
    else if (-d * d / 6.0 > d * mm) *aR = 3.0 * a - 2.0 * *aL;
}
void or_recon(int kind, const double w[6], double *L, double *R)
{
    if (kind == RC_MINMOD) {
        *L = w[2] + 0.5 * minmod2(w[2] - w[1], w[3] - w[2]);
        *R = w[3] - 0.5 * minmod2(w[3] - w[2], w[4] - w[3]);
    } else if (kind == RC_MC) {
        *L = w[2] + 0.5 * mc_slope(w[1], w[2], w[3]);
        *R = w[3] - 0.5 * mc_slope(w[2], w[3], w[4]);
    } else {
        double i1 = ppm_iface(w[0], w[1], w[2], w[3]);
        double i2 = ppm_iface(w[1], w[2], w[3], w[4]);
        double i3 = ppm_iface(w[2], w[3], w[4], w[5]);
        double aL = i1, aR = i2;
        ppm_mono(w[2], &aL, &aR);
        *L = aR;
        aL = i2;
        aR = i3;
        ppm_mono(w[3], &aL, &aR);
        *R = aL;
    }
}

/* ------------------------------------------------------------------------- */
/* grid geometry */
typedef struct {
    int N[3], g[3], act[3], n[3];
    double dx[3];
    long ncell;
} geom;

static geom mkgeom(const or_grid *G)
{
    geom q;
    for (int d = 0; d < 3; d++) {
        q.act[d] = d < G->ndim;
        q.n[d] = q.act[d] ? G->n[d] : 1;
        q.g[d] = q.act[d] ? G->ng : 0;
        q.N[d] = q.n[d] + 2 * q.g[d];
        q.dx[d] = q.act[d] ? (G->hi[d] - G->lo[d]) / G->n[d] : 1.0;
    }
    q.ncell = (long)q.N[0] * q.N[1] * q.N[2];
    return q;
}
static long IX(const geom *q, int i, int j, int k) { return i + (long)q->N[0] * (j + (long)q->N[1] * k); }
static long IXv(const geom *q, const int c[3]) { return IX(q, c[0], c[1], c[2]); }

/* ghost fill of cell-centred arrays (zero-gradient copy, periodic copy, or
 * untouched for fixed) and of the three face arrays.  Directions are filled
 * in order x, y, z over the full extent of the other directions so that
 * corner ghosts end up filled. */
void or_ghost_fill(const or_grid *G, double **cells, int ncells, double **faces)
{
    geom q = mkgeom(G);
    for (int d = 0; d < 3; d++) {
        if (!q.act[d]) continue;
        int g = q.g[d], n = q.n[d];
        int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        for (int side = 0; side < 2; side++) {
            int bc = G->bc[d][side];
            if (bc == BC_FIXED) continue;
            for (int b = 0; b < q.N[e2]; b++)
                for (int a = 0; a < q.N[e1]; a++)
                    for (int m = 0; m < g; m++) {
                        int c[3], s[3];
                        c[e1] = s[e1] = a;
                        c[e2] = s[e2] = b;
                        /* cell arrays and transverse face arrays */
                        if (side == 0) {
                            c[d] = m;
                            s[d] = (bc == BC_PERIODIC) ? m + n : g;
                        } else {
                            c[d] = g + n + m;
                            s[d] = (bc == BC_PERIODIC) ? g + m : g + n - 1;
                        }
                        for (int v = 0; v < ncells; v++) cells[v][IXv(&q, c)] = cells[v][IXv(&q, s)];
                        if (faces) {
                            for (int fd = 0; fd < 3; fd++) {
                                if (fd == d) continue;
                                faces[fd][IXv(&q, c)] = faces[fd][IXv(&q, s)];
                            }
                            /* normal face array: faces g..g+n are evolved */
                            int cf[3], sf[3];
                            cf[e1] = sf[e1] = a;
                            cf[e2] = sf[e2] = b;
                            if (side == 0) {
                                cf[d] = m;
                                sf[d] = (bc == BC_PERIODIC) ? m + n : g;
                                faces[d][IXv(&q, cf)] = faces[d][IXv(&q, sf)];
                            } else if (g + n + 1 + m < q.N[d]) {
                                cf[d] = g + n + 1 + m;
                                sf[d] = (bc == BC_PERIODIC) ? g + 1 + m : g + n;
                                faces[d][IXv(&q, cf)] = faces[d][IXv(&q, sf)];
                            }
                        }
                    }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Sec 2.3, Table imex_ssp2 and the cited IMEX-SSP3(4,3,3) tableau of
 * Pareschi & Russo (2005) (the latter is not printed in the paper). */
int or_tableau(int imex, double At[16], double A[16], double wt[4], double w[4])
{
    memset(At, 0, 16 * sizeof(double));
    memset(A, 0, 16 * sizeof(double));
    memset(wt, 0, 4 * sizeof(double));
    memset(w, 0, 4 * sizeof(double));
    if (imex == 0) {
        double g = 1.0 - 1.0 / sqrt(2.0);
        At[1 * 4 + 0] = 1.0;
        A[0 * 4 + 0] = g;
        A[1 * 4 + 0] = 1.0 - 2.0 * g;
        A[1 * 4 + 1] = g;
        wt[0] = wt[1] = 0.5;
        w[0] = w[1] = 0.5;
        return 2;
    }
    double a = 0.24169426078821, b = 0.06042356519705, e = 0.12915286960590;
    At[2 * 4 + 1] = 1.0;
    At[3 * 4 + 1] = 0.25;
    At[3 * 4 + 2] = 0.25;
    wt[1] = 1.0 / 6.0;
    wt[2] = 1.0 / 6.0;
    wt[3] = 2.0 / 3.0;
    A[0 * 4 + 0] = a;
    A[1 * 4 + 0] = -a;
    A[1 * 4 + 1] = a;
    A[2 * 4 + 1] = 1.0 - a;
    A[2 * 4 + 2] = a;
    A[3 * 4 + 0] = b;
    A[3 * 4 + 1] = e;
    A[3 * 4 + 2] = 0.5 - b - e - a;
    A[3 * 4 + 3] = a;
    for (int i = 0; i < 4; i++) w[i] = wt[i];
    return 4;
}

/* ------------------------------------------------------------------------- */
/* spatial operator L(q): Sec 2.1 fluxes and sources, Sec 2.5 speeds, HLL,
 * Sec 3.2 upwind constrained transport.  Inputs are one stage state:
 * primitives (rho, u~, p), the contravariant E^i, face fields q_B^d (face d
 * stored at index (i,j,k) sits half a cell below the cell centre in d), and
 * the static lapse / conformal factor (NULL for flat space).  Ghost cells
 * must already be filled.  Output: Lc[8] on interior cells (for q_D, q_S,
 * q_tau, q_E) and Lf[3] on the evolved faces. */
typedef struct {
    const or_grid *G;
    geom q;
    const double *prim[5], *E[3], *face[3], *alpha, *psi;
    double *Bcc[3];
    double *EfL[3], *EfR[3]; /* covariant E_k at a-faces (left / right states) */
} lctx;

static double A_at(const lctx *c, long id) { return c->alpha ? c->alpha[id] : 1.0; }
static double P_at(const lctx *c, long id) { return c->psi ? c->psi[id] : 1.0; }

/* value of reconstructed variable var at cell id: 0..4 prims, 5..7 E^i, 8..10 B^i (cell-centred) */
static double cellvar(const lctx *c, int var, long id)
{
    if (var < 5) return c->prim[var][id];
    if (var < 8) return c->E[var - 5][id];
    return c->Bcc[var - 8][id];
}

/* left/right states at face (direction d, face index cf) of a cell-centred quantity */
static void recon_cells(const lctx *c, int d, const int cf[3], int var, double *L, double *R)
{
    double w[6];
    int kind = c->G->recon;
    for (int m = 0; m < 6; m++) {
        int cc[3] = {cf[0], cf[1], cf[2]};
        cc[d] += m - 3;
        if (kind != RC_PPM && (m == 0 || m == 5)) { w[m] = 0.0; continue; }
        w[m] = cellvar(c, var, IXv(&c->q, cc));
    }
    or_recon(kind, w, L, R);
}

/* face metric: mean of the two adjacent cell centres (reading: "interpolated") */
static void face_metric(const lctx *c, int d, const int cf[3], double *al, double *ps)
{
    if (!c->q.act[d]) {
        long id = IXv(&c->q, cf);
        *al = A_at(c, id);
        *ps = P_at(c, id);
        return;
    }
    int cm[3] = {cf[0], cf[1], cf[2]};
    cm[d] -= 1;
    long i0 = IXv(&c->q, cm), i1 = IXv(&c->q, cf);
    *al = 0.5 * (A_at(c, i0) + A_at(c, i1));
    *ps = 0.5 * (P_at(c, i0) + P_at(c, i1));
}

/* Sec 2.5: speeds alpha sqrt(gamma^dd) (maximum diffusivity, beta = 0) */
static double face_speed(const lctx *c, int d, const int cf[3])
{
    double al, ps;
    face_metric(c, d, cf, &al, &ps);
    return al / (ps * ps);
}

/* HLL flux at face (d, cf) for the 8 cell-centred conserved fields */
static void hll_face(const lctx *c, int d, const int cf[3], double F[8])
{
    double al, ps;
    face_metric(c, d, cf, &al, &ps);
    double PL[5], PR[5], EL[3], ER[3], BL[3], BR[3];
    for (int v = 0; v < 5; v++) recon_cells(c, d, cf, v, &PL[v], &PR[v]);
    for (int v = 0; v < 3; v++) recon_cells(c, d, cf, 5 + v, &EL[v], &ER[v]);
    for (int t = 0; t < 3; t++) {
        if (t == d) {
            BL[t] = BR[t] = c->face[d][IXv(&c->q, cf)] / pow6(ps);
        } else {
            recon_cells(c, d, cf, 8 + t, &BL[t], &BR[t]);
        }
    }
    double qL[8], qR[8], fL[8], fR[8];
    double gam = c->G->gamma_ad;
    or_prim2cons(gam, ps, PL, EL, BL, qL);
    or_prim2cons(gam, ps, PR, ER, BR, qR);
    or_flux(d, gam, al, ps, PL, EL, BL, fL);
    or_flux(d, gam, al, ps, PR, ER, BR, fR);
    /* lambda_pm = alpha (+-sqrt(gamma^dd)); c+ and c- are the non-negative
     * speeds in the + and - directions, maximised over the L and R states */
    double sp = al * sqrt(1.0 / pow4(ps));
    double cp = fmax(0.0, fmax(sp, sp)), cm = fmax(0.0, fmax(sp, sp));
    for (int v = 0; v < 8; v++) F[v] = (cp * fL[v] + cm * fR[v] - cp * cm * (qR[v] - qL[v])) / (cp + cm);
}

/* covariant E_k at face (a, cf): the primitive E^k reconstructed cell -> face
 * along a, times psi_f^4 at the face; for an inactive direction a the "face"
 * is the cell itself */
static void E_cov_at_aface(const lctx *c, int a, int k, const int cf[3], double *L, double *R)
{
    double al, ps;
    face_metric(c, a, cf, &al, &ps);
    double p4 = pow4(ps);
    if (!c->q.act[a]) {
        double v = c->E[k][IXv(&c->q, cf)] * p4;
        *L = *R = v;
        return;
    }
    double l, r;
    recon_cells(c, a, cf, 5 + k, &l, &r);
    *L = l * p4;
    *R = r * p4;
}

/* reconstruct along direction d a generic array of face / face-derived values */
static void recon_along(const lctx *c, int d, const int ce[3], double (*get)(const lctx *, const int *, void *),
                        void *arg, double *L, double *R)
{
    if (!c->q.act[d]) {
        double v = get(c, ce, arg);
        *L = *R = v;
        return;
    }
    double w[6];
    int kind = c->G->recon;
    for (int m = 0; m < 6; m++) {
        int cc[3] = {ce[0], ce[1], ce[2]};
        cc[d] += m - 3;
        if (kind != RC_PPM && (m == 0 || m == 5)) { w[m] = 0.0; continue; }
        w[m] = get(c, cc, arg);
    }
    or_recon(kind, w, L, R);
}

typedef struct { int a, k, side; } eargs;
static double get_Eface(const lctx *c, const int *cc, void *arg)
{
    eargs *e = (eargs *)arg;
    long id = IXv(&c->q, cc);
    return e->side == 0 ? c->EfL[e->k][id] : c->EfR[e->k][id];
}
static double get_face(const lctx *c, const int *cc, void *arg)
{
    int d = *(int *)arg;
    return c->face[d][IXv(&c->q, cc)];
}

/* App. A steps (i)-(ii): the weighted transverse transport velocity
 * bar-v^j at the d-face cf, from the reconstructed left/right states of u~
 * there: hat-v^j = alpha v^j (beta = 0), v^j = u~^j / W, W^2 = 1 + gamma_ik
 * u~^i u~^k with the face metric; weights c-_d hat-v_R + c+_d hat-v_L. */
static double vbar_at_face(const lctx *c, int d, int j, const int cf[3])
{
    double al, ps;
    face_metric(c, d, cf, &al, &ps);
    double g4 = pow4(ps);
    double uL[3], uR[3];
    for (int i = 0; i < 3; i++) {
        if (c->q.act[d]) {
            recon_cells(c, d, cf, 1 + i, &uL[i], &uR[i]);
        } else {
            uL[i] = uR[i] = c->prim[1 + i][IXv(&c->q, cf)];
        }
    }
    double WL = sqrt(1.0 + g4 * (uL[0] * uL[0] + uL[1] * uL[1] + uL[2] * uL[2]));
    double WR = sqrt(1.0 + g4 * (uR[0] * uR[0] + uR[1] * uR[1] + uR[2] * uR[2]));
    double vL = al * uL[j] / WL, vR = al * uR[j] / WR;
    double cp = face_speed(c, d, cf), cm = cp;
    return (cm * vR + cp * vL) / (cm + cp);
}
static double get_vbar(const lctx *c, const int *cc, void *arg)
{
    const int *dj = (const int *)arg;
    return vbar_at_face(c, dj[0], dj[1], cc);
}

/* edge speeds of Sec 3.2 (vi): c_a maximised over the two a-faces sharing
 * the edge, c_b over the two b-faces */
static void edge_speeds(const lctx *c, int a, int b, const int ce[3], double *ca, double *cb)
{
    int c1[3] = {ce[0], ce[1], ce[2]}, c2[3] = {ce[0], ce[1], ce[2]};
    if (c->q.act[b]) c1[b] -= 1;
    *ca = fmax(face_speed(c, a, c1), face_speed(c, a, c2));
    int c3[3] = {ce[0], ce[1], ce[2]}, c4[3] = {ce[0], ce[1], ce[2]};
    if (c->q.act[a]) c3[a] -= 1;
    *cb = fmax(face_speed(c, b, c3), face_speed(c, b, c4));
}

/* App. A (ideal-MHD upwind CT): hat-E_k = alpha E_k with E_k = -eps_kab v^a
 * B^b, i.e. -eta_kab hat-v^a q_B^b.  (iii) bar-v^a of the b-faces and q_B^b
 * are reconstructed along a to the edge, bar-v^b of the a-faces and q_B^a
 * along b; (iv) the HLL-type combination with the speeds of each direction.
 * Reading: the printed sqrt(gamma) factor is already inside q_B = psi^6 B. */
static double uct_edge_ideal(const lctx *c, int k, const int ce[3])
{
    int a = (k + 1) % 3, b = (k + 2) % 3;
    double vaL, vaR, qbL, qbR, vbL, vbR, qaL, qaR;
    int fb[2] = {b, a}, fa[2] = {a, b};
    recon_along(c, a, ce, get_vbar, fb, &vaL, &vaR);
    recon_along(c, a, ce, get_face, &b, &qbL, &qbR);
    recon_along(c, b, ce, get_vbar, fa, &vbL, &vbR);
    recon_along(c, b, ce, get_face, &a, &qaL, &qaR);
    double ca, cb;
    edge_speeds(c, a, b, ce, &ca, &cb);
    double cap = ca, cam = ca, cbp = cb, cbm = cb;
    double t1 = (cam * vaR * qbR + cap * vaL * qbL - cam * cap * (qbR - qbL)) / (cam + cap);
    double t2 = (cbm * vbR * qaR + cbp * vbL * qaL - cbm * cbp * (qaR - qaL)) / (cbm + cbp);
    return -t1 + t2;
}

/* Sec 3.2 steps (i)-(vii): upwind EMF hat-E_k at the edge with index ce
 * (half a cell below the centre in the two directions a, b other than k;
 * (k, a, b) cyclic).  Reading: in E^{XY} the first letter is the side in a. */
static double uct_edge(const lctx *c, int k, const int ce[3])
{
    if (c->G->uct == 1) return uct_edge_ideal(c, k, ce);
    int a = (k + 1) % 3, b = (k + 2) % 3;
    /* (ii)+(iii): E_k cell -> a-face (L/R), then a-face -> edge along b */
    double ELL, ELR, ERL, ERR;
    eargs eL = {a, k, 0}, eR = {a, k, 1};
    recon_along(c, b, ce, get_Eface, &eL, &ELL, &ELR);
    recon_along(c, b, ce, get_Eface, &eR, &ERL, &ERR);
    /* (iv): q_B^b along a, q_B^a along b */
    double qbL, qbR, qaL, qaR;
    recon_along(c, a, ce, get_face, &b, &qbL, &qbR);
    recon_along(c, b, ce, get_face, &a, &qaL, &qaR);
    /* (vi): speeds, maximised over the two a-faces (b-faces) sharing the edge */
    double ca, cb;
    edge_speeds(c, a, b, ce, &ca, &cb);
    double cap = ca, cam = ca, cbp = cb, cbm = cb;
    /* lapse at the edge: mean of the surrounding cell centres */
    double asum = 0.0;
    int na = 0;
    for (int ia = 0; ia < 2; ia++)
        for (int ib = 0; ib < 2; ib++) {
            if ((ia && !c->q.act[a]) || (ib && !c->q.act[b])) continue;
            int cc[3] = {ce[0], ce[1], ce[2]};
            if (c->q.act[a]) cc[a] -= ia;
            if (c->q.act[b]) cc[b] -= ib;
            asum += A_at(c, IXv(&c->q, cc));
            na++;
        }
    double ae = asum / na;
    /* (v) beta = 0: hat-E^{XY} = alpha E_k^{XY} ; (vii) */
    double Eh = (cap * cbp * ae * ELL + cap * cbm * ae * ELR + cam * cbp * ae * ERL + cam * cbm * ae * ERR) /
                    ((cap + cam) * (cbp + cbm)) +
                cap * cam / (cap + cam) * (qbR - qbL) - cbp * cbm / (cbp + cbm) * (qaR - qaL);
    return Eh;
}

void or_explicit_L(const or_grid *G, double **prim, double **E, double **face, const double *alpha,
                   const double *psi, double **Lc, double **Lf)
{
    lctx c;
    c.G = G;
    c.q = mkgeom(G);
    for (int v = 0; v < 5; v++) c.prim[v] = prim[v];
    for (int v = 0; v < 3; v++) {
        c.E[v] = E[v];
        c.face[v] = face[v];
    }
    c.alpha = G->metric ? alpha : NULL;
    c.psi = G->metric ? psi : NULL;
    geom *q = &c.q;
    /* cell-centred B^d = mean of the two faces / psi^6 (NaN where undefined) */
    for (int d = 0; d < 3; d++) {
        c.Bcc[d] = (double *)malloc(sizeof(double) * q->ncell);
        for (int k = 0; k < q->N[2]; k++)
            for (int j = 0; j < q->N[1]; j++)
                for (int i = 0; i < q->N[0]; i++) {
                    int cc[3] = {i, j, k}, cp[3] = {i, j, k};
                    long id = IXv(q, cc);
                    double p6 = pow6(P_at(&c, id));
                    if (!q->act[d]) { c.Bcc[d][id] = face[d][id] / p6; continue; }
                    cp[d] += 1;
                    if (cp[d] >= q->N[d]) { c.Bcc[d][id] = NAN; continue; }
                    c.Bcc[d][id] = 0.5 * (face[d][id] + face[d][IXv(q, cp)]) / p6;
                }
    }
    /* fluxes on faces of interior cells */
    double *F[3][8];
    for (int d = 0; d < 3; d++)
        for (int v = 0; v < 8; v++) F[d][v] = NULL;
    for (int d = 0; d < 3; d++) {
        if (!q->act[d]) continue;
        for (int v = 0; v < 8; v++) F[d][v] = (double *)calloc(q->ncell, sizeof(double));
        int lo[3], hi[3];
        for (int e = 0; e < 3; e++) {
            lo[e] = q->g[e];
            hi[e] = q->g[e] + q->n[e] + (e == d ? 1 : 0);
        }
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = lo[2]; k < hi[2]; k++)
            for (int j = lo[1]; j < hi[1]; j++)
                for (int i = lo[0]; i < hi[0]; i++) {
                    int cf[3] = {i, j, k};
                    double Fv[8];
                    hll_face(&c, d, cf, Fv);
                    long id = IXv(q, cf);
                    for (int v = 0; v < 8; v++) F[d][v][id] = Fv[v];
                }
    }
    /* steps (ii)-(iii) of the upwind EMF, first half: covariant E_k at every
     * a-face of the edge range along a, over the full extent along b */
    for (int k = 0; k < 3; k++) {
        int a = (k + 1) % 3, b = (k + 2) % 3;
        c.EfL[k] = (double *)calloc(q->ncell, sizeof(double));
        c.EfR[k] = (double *)calloc(q->ncell, sizeof(double));
        if (!q->act[a] && !q->act[b]) continue;
        int lo[3], hi[3];
        for (int e = 0; e < 3; e++) {
            lo[e] = q->g[e];
            hi[e] = q->g[e] + q->n[e] + ((e == a && q->act[e]) ? 1 : 0);
        }
        lo[b] = 0;
        hi[b] = q->N[b];
#pragma omp parallel for collapse(2) schedule(static)
        for (int kk = lo[2]; kk < hi[2]; kk++)
            for (int j = lo[1]; j < hi[1]; j++)
                for (int i = lo[0]; i < hi[0]; i++) {
                    int cf[3] = {i, j, kk};
                    long id = IXv(q, cf);
                    E_cov_at_aface(&c, a, k, cf, &c.EfL[k][id], &c.EfR[k][id]);
                }
    }
    /* EMFs on edges: edge k index range [g, g+n] in its two transverse
     * directions (index 0 when inactive), interior along k */
    double *Ek[3];
    for (int k = 0; k < 3; k++) {
        int a = (k + 1) % 3, b = (k + 2) % 3;
        Ek[k] = (double *)calloc(q->ncell, sizeof(double));
        if (!q->act[a] && !q->act[b]) continue; /* never differentiated */
        int lo[3], hi[3];
        for (int e = 0; e < 3; e++) {
            lo[e] = q->g[e];
            hi[e] = q->g[e] + q->n[e] + ((e != k && q->act[e]) ? 1 : 0);
        }
#pragma omp parallel for collapse(2) schedule(static)
        for (int kk = lo[2]; kk < hi[2]; kk++)
            for (int j = lo[1]; j < hi[1]; j++)
                for (int i = lo[0]; i < hi[0]; i++) {
                    int ce[3] = {i, j, kk};
                    Ek[k][IXv(q, ce)] = uct_edge(&c, k, ce);
                }
    }
    /* face update (eq. ct): d q_B^d/dt = - eta^{d m k} d_m hat-E_k */
    for (int d = 0; d < 3; d++) {
        int lo[3], hi[3];
        for (int e = 0; e < 3; e++) {
            lo[e] = q->g[e];
            hi[e] = q->g[e] + q->n[e] + ((e == d && q->act[e]) ? 1 : 0);
        }
        for (int k = lo[2]; k < hi[2]; k++)
            for (int j = lo[1]; j < hi[1]; j++)
                for (int i = lo[0]; i < hi[0]; i++) {
                    int cf[3] = {i, j, k};
                    long id = IXv(q, cf);
                    double s = 0.0;
                    for (int m = 0; m < 3; m++) {
                        if (!q->act[m]) continue;
                        for (int kk = 0; kk < 3; kk++) {
                            double e = levi(d, m, kk);
                            if (e == 0.0) continue;
                            int cp[3] = {i, j, k};
                            cp[m] += 1;
                            s += e * (Ek[kk][IXv(q, cp)] - Ek[kk][id]) / q->dx[m];
                        }
                    }
                    Lf[d][id] = -s;
                }
    }
    /* cell part: flux divergence + sources */
    double gam = G->gamma_ad;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = q->g[2]; k < q->g[2] + q->n[2]; k++)
        for (int j = q->g[1]; j < q->g[1] + q->n[1]; j++)
            for (int i = q->g[0]; i < q->g[0] + q->n[0]; i++) {
                int cc[3] = {i, j, k};
                long id = IXv(q, cc);
                double L[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                for (int d = 0; d < 3; d++) {
                    if (!q->act[d]) continue;
                    int cp[3] = {i, j, k};
                    cp[d] += 1;
                    long ip = IXv(q, cp);
                    for (int v = 0; v < 8; v++) L[v] -= (F[d][v][ip] - F[d][v][id]) / q->dx[d];
                }
                /* sources (Sec 2.1) with beta = 0, K_ij = 0, Cartesian */
                double al = A_at(&c, id), ps = P_at(&c, id);
                metric3 m;
                mk_metric(ps, &m);
                double dal[3] = {0, 0, 0}, dps[3] = {0, 0, 0}, divqE = 0.0;
                for (int d = 0; d < 3; d++) {
                    if (!q->act[d]) continue;
                    int cp[3] = {i, j, k}, cm[3] = {i, j, k};
                    cp[d] += 1;
                    cm[d] -= 1;
                    long ip = IXv(q, cp), im = IXv(q, cm);
                    dal[d] = (A_at(&c, ip) - A_at(&c, im)) / (2.0 * q->dx[d]);
                    dps[d] = (P_at(&c, ip) - P_at(&c, im)) / (2.0 * q->dx[d]);
                    double qEp = pow6(P_at(&c, ip)) * E[d][ip], qEm = pow6(P_at(&c, im)) * E[d][im];
                    divqE += (qEp - qEm) / (2.0 * q->dx[d]);
                }
                double pr[5], Ev[3], Bv[3];
                for (int v = 0; v < 5; v++) pr[v] = prim[v][id];
                for (int v = 0; v < 3; v++) {
                    Ev[v] = E[v][id];
                    Bv[v] = c.Bcc[v][id];
                }
                double rho = pr[0], p = pr[4];
                double ut[3] = {pr[1], pr[2], pr[3]};
                double W = sqrt(1.0 + dotg(&m, ut, ut));
                double v[3], vl[3], ExB[3], S[3], Su[3];
                for (int a = 0; a < 3; a++) v[a] = ut[a] / W;
                lower(&m, v, vl);
                double eps = p / ((gam - 1.0) * rho), h = 1.0 + eps + p / rho;
                double UEM = 0.5 * (dotg(&m, Ev, Ev) + dotg(&m, Bv, Bv));
                cross_low(&m, Ev, Bv, ExB);
                for (int a = 0; a < 3; a++) S[a] = rho * h * W * W * vl[a] + ExB[a];
                raise_(&m, S, Su);
                double tauD = rho * h * W * W - p + UEM; /* tau + D */
                if (G->metric) {
                    /* S^{jk} and d_i gamma_jk = 4 psi^3 d_i psi delta_jk */
                    double Sjk[3][3];
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            Sjk[a][b] = rho * h * W * W * v[a] * v[b] + (p + UEM) * m.gi[a][b] - Ev[a] * Ev[b] -
                                        Bv[a] * Bv[b];
                    for (int a = 0; a < 3; a++) {
                        double sg = 0.0;
                        for (int jj = 0; jj < 3; jj++)
                            for (int kk = 0; kk < 3; kk++) {
                                double dg = (jj == kk) ? 4.0 * ps * ps * ps * dps[a] : 0.0;
                                sg += 0.5 * al * Sjk[jj][kk] * dg;
                            }
                        L[1 + a] += m.sqrtg * (-tauD * dal[a] + sg);
                    }
                    double st = 0.0;
                    for (int a = 0; a < 3; a++) st -= Su[a] * dal[a];
                    L[4] += m.sqrtg * st;
                }
                /* non-stiff current: s_E = -alpha psi^6 rho_e v^i, rho_e = div(q_E)/psi^6 (Gauss law) */
                double rhoe = divqE / m.sqrtg;
                for (int a = 0; a < 3; a++) L[5 + a] += -al * m.sqrtg * rhoe * v[a];
                for (int vv = 0; vv < 8; vv++) Lc[vv][id] = L[vv];
            }
    for (int d = 0; d < 3; d++) {
        free(c.Bcc[d]);
        free(c.EfL[d]);
        free(c.EfR[d]);
        free(Ek[d]);
        for (int v = 0; v < 8; v++) free(F[d][v]);
    }
}

/* ------------------------------------------------------------------------- */
/* resistivity of a cell: uniform, or eta = 1/sigma_c with eq. sigma_D,
 * sigma_c = sigma_0 max(1 - D_atmo/D, 0)^2, clamped to [eta_min, eta_max].
 * Reading: D_atmo is the density below which a cell is atmosphere,
 * atm_factor rho_atm, so that the conductivity falls continuously to zero
 * where the atmosphere begins. */
static double or_eta(const or_grid *G, double Dund)
{
    if (G->eta_mode == 0) return G->eta;
    double x = 1.0 - G->rho_atm * G->atm_factor / Dund;
    if (x < 0.0) x = 0.0;
    double sig = G->sigma0 * x * x;
    if (sig * G->eta_max <= 1.0) return G->eta_max;
    double e = 1.0 / sig;
    return e < G->eta_min ? G->eta_min : e;
}

/* atmosphere / failure state (reading; the paper gives no fallback rule):
 * rho = rho_atm, u~ = 0, p = p_atm.  A cell is atmosphere when its
 * undensitised D is at most atm_factor rho_atm; a failed or unphysical
 * recovery (no root, p < 0, W > 1e4, rho < rho_atm) falls back to the same
 * state and is counted as a failure. */
static void atmo_prim(const or_grid *G, double prim[5])
{
    prim[0] = G->rho_atm;
    prim[1] = prim[2] = prim[3] = 0.0;
    prim[4] = G->p_atm;
}

/* Electric field of a cell at rest (u~ = 0, W = 1): eq. im_E reduces to
 * (1 + eta~) E = eta~ E* + xi B (A_0 = 1 + eta~, A_3 = xi, the other terms
 * vanish), written with r = 1/eta~ = alpha a_ii dt / eta as
 * (E* + xi r B) / (1 + r). */
static void E_at_rest(double r, double xi, const double Es[3], const double B[3], double E[3])
{
    for (int i = 0; i < 3; i++) E[i] = (Es[i] + xi * r * B[i]) / (1.0 + r);
}

/* The fused implicit solve of one cell within stage with diagonal weight aii.
 * fz != NULL: frozen matter (the paper's dynamo test evolves only the
 * electromagnetic fields): the primitives stay fz and E follows from eq.
 * im_E at the fixed u~.  Returns 0 normal, 1 atmosphere, 2 failure (fallback
 * applied). */
static int cell_implicit(const or_grid *G, double al, double ps, const double qs[8], const double B[3], double aii,
                         double dt, const double guess[3], const double *fz, double prim[5], double E[3])
{
    double p6 = pow6(ps);
    double Dund = qs[0] / p6;
    double Es[3] = {qs[5] / p6, qs[6] / p6, qs[7] / p6};
    if (fz) {
        double eta = or_eta(G, fz[0] * sqrt(1.0 + (fz[1] * fz[1] + fz[2] * fz[2] + fz[3] * fz[3]) * pow4(ps)));
        double ut[3] = {fz[1], fz[2], fz[3]};
        for (int v = 0; v < 5; v++) prim[v] = fz[v];
        or_implicit_E(ps, eta / (al * aii * dt), G->xi, ut, Es, B, E);
        return 0;
    }
    double eta = or_eta(G, Dund);
    double etat = eta / (al * aii * dt);
    if (Dund <= G->rho_atm * G->atm_factor) {
        atmo_prim(G, prim);
        E_at_rest(al * aii * dt / eta, G->xi, Es, B, E);
        return 1;
    }
    int it;
    int bad = or_implicit(G->gamma_ad, ps, qs, B, etat, G->xi, guess, G->newton_tol, G->newton_maxit, prim, E, &it);
    /* p = (w~/W - rho)/Gamma_1 cancels to round-off for a cold gas: a
     * negative value within 1e-12 rho of zero is read as p = 0 */
    if (!bad && prim[4] < 0.0 && prim[4] >= -1e-12 * prim[0]) prim[4] = 0.0;
    if (!bad) {
        metric3 m;
        mk_metric(ps, &m);
        double ut[3] = {prim[1], prim[2], prim[3]};
        double W = sqrt(1.0 + dotg(&m, ut, ut));
        if (!(prim[4] >= 0.0) || !(W <= 1e4) || !(prim[0] >= G->rho_atm)) bad = 1;
    }
    if (bad) {
        atmo_prim(G, prim);
        E_at_rest(al * aii * dt / eta, G->xi, Es, B, E);
        return 2;
    }
    return 0;
}

/* Final recovery with E and B known.  Returns 0, 1 atmosphere, 2 failure;
 * on 1/2 the conserved D, S, tau are rewritten from the atmosphere state. */
static int cell_c2p(const or_grid *G, double ps, double q[8], const double B[3], double prim[5])
{
    double p6 = pow6(ps);
    double E[3] = {q[5] / p6, q[6] / p6, q[7] / p6};
    int r = 0;
    if (q[0] / p6 <= G->rho_atm * G->atm_factor) r = 1;
    else {
        if (or_c2p(G->gamma_ad, ps, q, E, B, prim)) r = 2;
        else {
            metric3 m;
            mk_metric(ps, &m);
            double ut[3] = {prim[1], prim[2], prim[3]};
            double W = sqrt(1.0 + dotg(&m, ut, ut));
            if (!(prim[4] >= 0.0) || !(W <= 1e4) || !(prim[0] >= G->rho_atm)) r = 2;
        }
    }
    if (r) {
        atmo_prim(G, prim);
        double qq[8];
        or_prim2cons(G->gamma_ad, ps, prim, E, B, qq);
        for (int v = 0; v < 5; v++) q[v] = qq[v];
    }
    return r;
}

static void bcc_at(const geom *q, double **face, const double *psi, long id, const int cc[3], double B[3])
{
    double ps = psi ? psi[id] : 1.0;
    double p6 = pow6(ps);
    for (int d = 0; d < 3; d++) {
        if (!q->act[d]) { B[d] = face[d][id] / p6; continue; }
        int cp[3] = {cc[0], cc[1], cc[2]};
        cp[d] += 1;
        B[d] = 0.5 * (face[d][id] + face[d][IXv(q, cp)]) / p6;
    }
}

/* conservative-to-primitive (E, B given) on all interior cells; returns the
 * number of failures */
long or_c2p_grid(const or_grid *G, double **qc, double **face, double **prim, const double *psi)
{
    if (G->frozen_matter) return 0; /* the primitives do not change */
    geom q = mkgeom(G);
    const double *ps_arr = G->metric ? psi : NULL;
    long nfail = 0;
    for (int k = q.g[2]; k < q.g[2] + q.n[2]; k++)
        for (int j = q.g[1]; j < q.g[1] + q.n[1]; j++)
            for (int i = q.g[0]; i < q.g[0] + q.n[0]; i++) {
                int cc[3] = {i, j, k};
                long id = IXv(&q, cc);
                double B[3], qq[8], pr[5];
                bcc_at(&q, face, ps_arr, id, cc, B);
                for (int v = 0; v < 8; v++) qq[v] = qc[v][id];
                int r = cell_c2p(G, ps_arr ? ps_arr[id] : 1.0, qq, B, pr);
                if (r == 2) nfail++;
                for (int v = 0; v < 8; v++) qc[v][id] = qq[v];
                for (int v = 0; v < 5; v++) prim[v][id] = pr[v];
            }
    return nfail;
}

/* ------------------------------------------------------------------------- */
/* One IMEX-RK step (Sec 2.3; reading of the garbled signs/indices: explicit
 * sums over j < i with +dt, implicit over j <= i, final
 * q^{n+1} = q^n + dt sum_i wt_i L(Q^(i)) + dt sum_i w_i R(Q^(i))).
 * State: qc[8] cell conserved (densitised), face[3], prim[5] (rho, u~, p).
 * R(Q) is non-zero only in q_E: R = psi^6 (E^(i) - E*)/(a_ii dt).
 * If stage_out != NULL, the primitives/E of stage `dump_stage` (0-based) are
 * copied there (8 arrays) for stage-level comparisons.  Returns failures. */
long or_step(const or_grid *G, double **qc, double **face, double **prim, const double *alpha, const double *psi,
             double dt, int dump_stage, double **stage_out, double **L_out)
{
    geom q = mkgeom(G);
    const double *al_arr = G->metric ? alpha : NULL;
    const double *ps_arr = G->metric ? psi : NULL;
    double At[16], A[16], wt[4], w[4];
    int s = or_tableau(G->imex, At, A, wt, w);
    long nc = q.ncell;
    long nfail = 0;
    /* stage storage */
    double *sp[4][5], *sE[4][3], *sf[4][3], *Lc[4][8], *Lf[4][3], *R[4][3];
    int Lhave[4] = {0, 0, 0, 0};
    for (int i = 0; i < s; i++) {
        for (int v = 0; v < 5; v++) {
            sp[i][v] = (double *)malloc(nc * sizeof(double));
            memcpy(sp[i][v], prim[v], nc * sizeof(double));
        }
        for (int v = 0; v < 3; v++) {
            sE[i][v] = (double *)malloc(nc * sizeof(double));
            sf[i][v] = (double *)malloc(nc * sizeof(double));
            Lf[i][v] = (double *)calloc(nc, sizeof(double));
            R[i][v] = (double *)calloc(nc, sizeof(double));
            memcpy(sf[i][v], face[v], nc * sizeof(double));
            for (long id = 0; id < nc; id++) sE[i][v][id] = qc[5 + v][id] / pow6(ps_arr ? ps_arr[id] : 1.0);
        }
        for (int v = 0; v < 8; v++) Lc[i][v] = (double *)calloc(nc, sizeof(double));
    }
    double *cells[8];
    for (int i = 0; i < s; i++) {
        /* explicit terms needed by this stage */
        for (int j = 0; j < i; j++) {
            if (At[i * 4 + j] != 0.0 && !Lhave[j]) {
                for (int v = 0; v < 5; v++) cells[v] = sp[j][v];
                for (int v = 0; v < 3; v++) cells[5 + v] = sE[j][v];
                or_ghost_fill(G, cells, 8, sf[j]);
                or_explicit_L(G, sp[j], sE[j], sf[j], al_arr, ps_arr, Lc[j], Lf[j]);
                Lhave[j] = 1;
            }
        }
        double aii = A[i * 4 + i];
        /* faces of the stage state: explicit update only */
        for (int d = 0; d < 3; d++)
            for (long id = 0; id < nc; id++) {
                double acc = face[d][id];
                for (int j = 0; j < i; j++) acc += dt * At[i * 4 + j] * Lf[j][d][id];
                sf[i][d][id] = acc;
            }
        for (int k = q.g[2]; k < q.g[2] + q.n[2]; k++)
            for (int jj = q.g[1]; jj < q.g[1] + q.n[1]; jj++)
                for (int ii = q.g[0]; ii < q.g[0] + q.n[0]; ii++) {
                    int cc[3] = {ii, jj, k};
                    long id = IXv(&q, cc);
                    double qs[8];
                    for (int v = 0; v < 8; v++) {
                        double acc = qc[v][id];
                        for (int j = 0; j < i; j++) {
                            acc += dt * At[i * 4 + j] * Lc[j][v][id];
                            if (v >= 5) acc += dt * A[i * 4 + j] * R[j][v - 5][id];
                        }
                        qs[v] = acc;
                    }
                    double B[3];
                    bcc_at(&q, sf[i], ps_arr, id, cc, B);
                    double al = al_arr ? al_arr[id] : 1.0, ps = ps_arr ? ps_arr[id] : 1.0;
                    double guess[3];
                    double **gp = (i == 0) ? prim : sp[i - 1];
                    for (int a = 0; a < 3; a++) guess[a] = gp[1 + a][id];
                    double pr[5], E[3], fz[5];
                    if (G->frozen_matter)
                        for (int v = 0; v < 5; v++) fz[v] = prim[v][id];
                    int r = cell_implicit(G, al, ps, qs, B, aii, dt, guess, G->frozen_matter ? fz : NULL, pr, E);
                    if (r == 2) nfail++;
                    double p6 = pow6(ps);
                    for (int v = 0; v < 5; v++) sp[i][v][id] = pr[v];
                    for (int a = 0; a < 3; a++) {
                        sE[i][a][id] = E[a];
                        R[i][a][id] = (p6 * E[a] - qs[5 + a]) / (aii * dt);
                    }
                }
    }
    for (int j = 0; j < s; j++) {
        if (wt[j] != 0.0 && !Lhave[j]) {
            for (int v = 0; v < 5; v++) cells[v] = sp[j][v];
            for (int v = 0; v < 3; v++) cells[5 + v] = sE[j][v];
            or_ghost_fill(G, cells, 8, sf[j]);
            or_explicit_L(G, sp[j], sE[j], sf[j], al_arr, ps_arr, Lc[j], Lf[j]);
            Lhave[j] = 1;
        }
    }
    if (stage_out) {
        for (int v = 0; v < 5; v++) memcpy(stage_out[v], sp[dump_stage][v], nc * sizeof(double));
        for (int v = 0; v < 3; v++) memcpy(stage_out[5 + v], sE[dump_stage][v], nc * sizeof(double));
    }
    if (L_out) {
        for (int v = 0; v < 8; v++) memcpy(L_out[v], Lc[dump_stage][v], nc * sizeof(double));
        for (int v = 0; v < 3; v++) memcpy(L_out[8 + v], Lf[dump_stage][v], nc * sizeof(double));
    }
    /* final combination (faces, then cells) */
    for (int d = 0; d < 3; d++) {
        int lo[3], hi[3];
        for (int e = 0; e < 3; e++) {
            lo[e] = q.g[e];
            hi[e] = q.g[e] + q.n[e] + ((e == d && q.act[e]) ? 1 : 0);
        }
        for (int k = lo[2]; k < hi[2]; k++)
            for (int jj = lo[1]; jj < hi[1]; jj++)
                for (int ii = lo[0]; ii < hi[0]; ii++) {
                    long id = IX(&q, ii, jj, k);
                    double acc = face[d][id];
                    for (int j = 0; j < s; j++) acc += dt * wt[j] * Lf[j][d][id];
                    face[d][id] = acc;
                }
    }
    for (int k = q.g[2]; k < q.g[2] + q.n[2]; k++)
        for (int jj = q.g[1]; jj < q.g[1] + q.n[1]; jj++)
            for (int ii = q.g[0]; ii < q.g[0] + q.n[0]; ii++) {
                long id = IX(&q, ii, jj, k);
                for (int v = G->frozen_matter ? 5 : 0; v < 8; v++) {
                    double acc = qc[v][id];
                    for (int j = 0; j < s; j++) {
                        acc += dt * wt[j] * Lc[j][v][id];
                        if (v >= 5) acc += dt * w[j] * R[j][v - 5][id];
                    }
                    qc[v][id] = acc;
                }
            }
    nfail += or_c2p_grid(G, qc, face, prim, psi);
    /* ghost cells of the primitive / E state follow the boundary rule */
    for (int i = 0; i < s; i++) {
        for (int v = 0; v < 5; v++) free(sp[i][v]);
        for (int v = 0; v < 3; v++) {
            free(sE[i][v]);
            free(sf[i][v]);
            free(Lf[i][v]);
            free(R[i][v]);
        }
        for (int v = 0; v < 8; v++) free(Lc[i][v]);
    }
    return nfail;
}

/* ------------------------------------------------------------------------- */
/* Sec 4: face fields q_B^i = eta^{ijk} d_j A_k from an edge vector potential.
 * A_k is given on an edge grid one point larger than the cell grid in each
 * active direction; A_k(i,j,k) sits half a cell below the cell centre in the
 * two directions other than k.  Then conserved variables from primitives on
 * interior cells; q_E = psi^6 E on all cells. */
void or_init(const or_grid *G, double **prim_in, double **E_in, double **Aedge, const double *psi, double **qc,
             double **face, double **prim)
{
    geom q = mkgeom(G);
    const double *ps_arr = G->metric ? psi : NULL;
    int Ne[3];
    for (int d = 0; d < 3; d++) Ne[d] = q.N[d] + (q.act[d] ? 1 : 0);
    for (int d = 0; d < 3; d++)
        for (int k = 0; k < q.N[2]; k++)
            for (int j = 0; j < q.N[1]; j++)
                for (int i = 0; i < q.N[0]; i++) {
                    int cc[3] = {i, j, k};
                    double s = 0.0;
                    for (int m = 0; m < 3; m++) {
                        if (!q.act[m]) continue;
                        for (int kk = 0; kk < 3; kk++) {
                            double e = levi(d, m, kk);
                            if (e == 0.0 || !Aedge) continue;
                            int cp[3] = {i, j, k};
                            cp[m] += 1;
                            long e0 = cc[0] + (long)Ne[0] * (cc[1] + (long)Ne[1] * cc[2]);
                            long e1 = cp[0] + (long)Ne[0] * (cp[1] + (long)Ne[1] * cp[2]);
                            s += e * (Aedge[kk][e1] - Aedge[kk][e0]) / q.dx[m];
                        }
                    }
                    face[d][IXv(&q, cc)] = s;
                }
    for (long id = 0; id < q.ncell; id++) {
        for (int v = 0; v < 5; v++) prim[v][id] = prim_in[v][id];
        double p6 = pow6(ps_arr ? ps_arr[id] : 1.0);
        for (int v = 0; v < 3; v++) qc[5 + v][id] = p6 * E_in[v][id];
    }
    for (int k = q.g[2]; k < q.g[2] + q.n[2]; k++)
        for (int j = q.g[1]; j < q.g[1] + q.n[1]; j++)
            for (int i = q.g[0]; i < q.g[0] + q.n[0]; i++) {
                int cc[3] = {i, j, k};
                long id = IXv(&q, cc);
                double B[3], pr[5], E[3], qq[8];
                bcc_at(&q, face, ps_arr, id, cc, B);
                for (int v = 0; v < 5; v++) pr[v] = prim[v][id];
                for (int v = 0; v < 3; v++) E[v] = E_in[v][id];
                or_prim2cons(G->gamma_ad, ps_arr ? ps_arr[id] : 1.0, pr, E, B, qq);
                for (int v = 0; v < 8; v++) qc[v][id] = qq[v];
            }
}

/* Sec 2.5 / reading: dt = cfl / max_cells sum_d (alpha sqrt(gamma^dd))/dx_d */
double or_cfl_dt(const or_grid *G, const double *alpha, const double *psi)
{
    geom q = mkgeom(G);
    double mx = 0.0;
    for (int k = q.g[2]; k < q.g[2] + q.n[2]; k++)
        for (int j = q.g[1]; j < q.g[1] + q.n[1]; j++)
            for (int i = q.g[0]; i < q.g[0] + q.n[0]; i++) {
                long id = IX(&q, i, j, k);
                double al = (G->metric && alpha) ? alpha[id] : 1.0, ps = (G->metric && psi) ? psi[id] : 1.0;
                double s = 0.0;
                for (int d = 0; d < 3; d++)
                    if (q.act[d]) s += al * sqrt(1.0 / pow4(ps)) / q.dx[d];
                if (s > mx) mx = s;
            }
    return G->cfl / mx;
}

/* discrete divergence of the face field over interior cells: L1 = mean |div|,
 * L2 = sqrt(mean div^2), Linf = max |div| */
void or_divB(const or_grid *G, double **face, double out[3])
{
    geom q = mkgeom(G);
    double s1 = 0.0, s2 = 0.0, mx = 0.0;
    long cnt = 0;
    for (int k = q.g[2]; k < q.g[2] + q.n[2]; k++)
        for (int j = q.g[1]; j < q.g[1] + q.n[1]; j++)
            for (int i = q.g[0]; i < q.g[0] + q.n[0]; i++) {
                int cc[3] = {i, j, k};
                long id = IXv(&q, cc);
                double dv = 0.0;
                for (int d = 0; d < 3; d++) {
                    if (!q.act[d]) continue;
                    int cp[3] = {i, j, k};
                    cp[d] += 1;
                    dv += (face[d][IXv(&q, cp)] - face[d][id]) / q.dx[d];
                }
                s1 += fabs(dv);
                s2 += dv * dv;
                if (fabs(dv) > mx) mx = fabs(dv);
                cnt++;
            }
    out[0] = s1 / cnt;
    out[1] = sqrt(s2 / cnt);
    out[2] = mx;
}


/* ------------------------------------------------------------------------- */
/* GLM hyperbolic divergence cleaning (Sec 3.1): the cell-centred alternative
 * to constrained transport.  Conserved: q_D, q_S, q_tau, q_E (8), q_B^i (3,
 * cell-centred, kept in the face[3] arrays at cell positions) and
 * q_Psi = psi^6 Psi, q_Phi = psi^6 Phi (qc[8], qc[9]).  Fluxes: those of
 * Sec 2.1, f_B of q_B^j along i = psi^6 eps^{jik} alpha E_k (Faraday),
 * f_Psi^i = alpha q_E^i, f_Phi^i = alpha q_B^i (beta = 0).  Sources (K = 0):
 * s_E^i += -alpha psi^6 gamma^{ij} d_j Psi, s_B^i = -alpha psi^6 gamma^{ij}
 * d_j Phi, s_Psi = psi^6 [alpha rho_e - alpha kappa_E Psi + E^i d_i alpha],
 * s_Phi = psi^6 [-alpha kappa_B Phi + B^i d_i alpha]; derivatives of Psi,
 * Phi and alpha by central differences. */
#define GLM_NV 13 /* reconstructed: rho, u~^i, p, E^i, B^i, Psi, Phi */

typedef struct {
    const or_grid *G;
    geom q;
    const double *v[GLM_NV]; /* cell arrays of the reconstructed variables */
    const double *alpha, *psi;
} gctx;

static double gA(const gctx *c, long id) { return c->alpha ? c->alpha[id] : 1.0; }
static double gP(const gctx *c, long id) { return c->psi ? c->psi[id] : 1.0; }

static void glm_hll(const gctx *c, int d, const int cf[3], double F[GLM_NV])
{
    const geom *q = &c->q;
    int cm[3] = {cf[0], cf[1], cf[2]};
    cm[d] -= 1;
    long i0 = IXv(q, cm), i1 = IXv(q, cf);
    double al = 0.5 * (gA(c, i0) + gA(c, i1)), ps = 0.5 * (gP(c, i0) + gP(c, i1));
    double sL[GLM_NV], sR[GLM_NV];
    int kind = c->G->recon;
    for (int v = 0; v < GLM_NV; v++) {
        double w[6];
        for (int m = 0; m < 6; m++) {
            int cc[3] = {cf[0], cf[1], cf[2]};
            cc[d] += m - 3;
            w[m] = (kind != RC_PPM && (m == 0 || m == 5)) ? 0.0 : c->v[v][IXv(q, cc)];
        }
        or_recon(kind, w, &sL[v], &sR[v]);
    }
    double gam = c->G->gamma_ad, p6 = pow6(ps);
    double qL[GLM_NV], qR[GLM_NV], fL[GLM_NV], fR[GLM_NV];
    for (int side = 0; side < 2; side++) {
        const double *st = side ? sR : sL;
        double *qq = side ? qR : qL, *ff = side ? fR : fL;
        const double *pr = st, *E = st + 5, *B = st + 8;
        or_prim2cons(gam, ps, pr, E, B, qq);
        or_flux(d, gam, al, ps, pr, E, B, ff);
        or_flux_B(d, al, ps, E, ff + 8);
        for (int j = 0; j < 3; j++) qq[8 + j] = p6 * B[j];
        qq[11] = p6 * st[11];
        qq[12] = p6 * st[12];
        ff[11] = al * p6 * E[d];
        ff[12] = al * p6 * B[d];
    }
    double sp = al * sqrt(1.0 / pow4(ps));
    for (int v = 0; v < GLM_NV; v++) F[v] = (sp * fL[v] + sp * fR[v] - sp * sp * (qR[v] - qL[v])) / (sp + sp);
}

/* L of the GLM system on the interior cells (cell arrays include ghosts) */
void or_explicit_L_glm(const or_grid *G, double **vars, const double *alpha, const double *psi, double **Lc)
{
    gctx c;
    c.G = G;
    c.q = mkgeom(G);
    for (int v = 0; v < GLM_NV; v++) c.v[v] = vars[v];
    c.alpha = G->metric ? alpha : NULL;
    c.psi = G->metric ? psi : NULL;
    geom *q = &c.q;
    double *F[3][GLM_NV];
    for (int d = 0; d < 3; d++) {
        for (int v = 0; v < GLM_NV; v++) F[d][v] = NULL;
        if (!q->act[d]) continue;
        for (int v = 0; v < GLM_NV; v++) F[d][v] = (double *)calloc(q->ncell, sizeof(double));
        int lo[3], hi[3];
        for (int e = 0; e < 3; e++) {
            lo[e] = q->g[e];
            hi[e] = q->g[e] + q->n[e] + (e == d ? 1 : 0);
        }
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = lo[2]; k < hi[2]; k++)
            for (int j = lo[1]; j < hi[1]; j++)
                for (int i = lo[0]; i < hi[0]; i++) {
                    int cf[3] = {i, j, k};
                    double Fv[GLM_NV];
                    glm_hll(&c, d, cf, Fv);
                    long id = IXv(q, cf);
                    for (int v = 0; v < GLM_NV; v++) F[d][v][id] = Fv[v];
                }
    }
    double gam = G->gamma_ad;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = q->g[2]; k < q->g[2] + q->n[2]; k++)
        for (int j = q->g[1]; j < q->g[1] + q->n[1]; j++)
            for (int i = q->g[0]; i < q->g[0] + q->n[0]; i++) {
                int cc[3] = {i, j, k};
                long id = IXv(q, cc);
                double L[GLM_NV];
                for (int v = 0; v < GLM_NV; v++) L[v] = 0.0;
                for (int d = 0; d < 3; d++) {
                    if (!q->act[d]) continue;
                    int cp[3] = {i, j, k};
                    cp[d] += 1;
                    long ip = IXv(q, cp);
                    for (int v = 0; v < GLM_NV; v++) L[v] -= (F[d][v][ip] - F[d][v][id]) / q->dx[d];
                }
                double al = gA(&c, id), ps = gP(&c, id);
                metric3 m;
                mk_metric(ps, &m);
                double dal[3] = {0, 0, 0}, dps[3] = {0, 0, 0}, dPsi[3] = {0, 0, 0}, dPhi[3] = {0, 0, 0};
                double divqE = 0.0;
                for (int d = 0; d < 3; d++) {
                    if (!q->act[d]) continue;
                    int cp[3] = {i, j, k}, cm[3] = {i, j, k};
                    cp[d] += 1;
                    cm[d] -= 1;
                    long ip = IXv(q, cp), im = IXv(q, cm);
                    double h2 = 2.0 * q->dx[d];
                    dal[d] = (gA(&c, ip) - gA(&c, im)) / h2;
                    dps[d] = (gP(&c, ip) - gP(&c, im)) / h2;
                    dPsi[d] = (vars[11][ip] - vars[11][im]) / h2;
                    dPhi[d] = (vars[12][ip] - vars[12][im]) / h2;
                    divqE += (pow6(gP(&c, ip)) * vars[5 + d][ip] - pow6(gP(&c, im)) * vars[5 + d][im]) / h2;
                }
                double pr[5], Ev[3], Bv[3];
                for (int v = 0; v < 5; v++) pr[v] = vars[v][id];
                for (int v = 0; v < 3; v++) {
                    Ev[v] = vars[5 + v][id];
                    Bv[v] = vars[8 + v][id];
                }
                double Psi = vars[11][id], Phi = vars[12][id];
                double rho = pr[0], p = pr[4];
                double ut[3] = {pr[1], pr[2], pr[3]};
                double W = sqrt(1.0 + dotg(&m, ut, ut));
                double v[3], vl[3], ExB[3], S[3], Su[3];
                for (int a = 0; a < 3; a++) v[a] = ut[a] / W;
                lower(&m, v, vl);
                double eps = p / ((gam - 1.0) * rho), h = 1.0 + eps + p / rho;
                double UEM = 0.5 * (dotg(&m, Ev, Ev) + dotg(&m, Bv, Bv));
                cross_low(&m, Ev, Bv, ExB);
                for (int a = 0; a < 3; a++) S[a] = rho * h * W * W * vl[a] + ExB[a];
                raise_(&m, S, Su);
                double tauD = rho * h * W * W - p + UEM;
                if (G->metric) {
                    double Sjk[3][3];
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            Sjk[a][b] = rho * h * W * W * v[a] * v[b] + (p + UEM) * m.gi[a][b] - Ev[a] * Ev[b] -
                                        Bv[a] * Bv[b];
                    for (int a = 0; a < 3; a++) {
                        double sg = 0.0;
                        for (int jj = 0; jj < 3; jj++)
                            for (int kk = 0; kk < 3; kk++) {
                                double dg = (jj == kk) ? 4.0 * ps * ps * ps * dps[a] : 0.0;
                                sg += 0.5 * al * Sjk[jj][kk] * dg;
                            }
                        L[1 + a] += m.sqrtg * (-tauD * dal[a] + sg);
                    }
                    double st = 0.0;
                    for (int a = 0; a < 3; a++) st -= Su[a] * dal[a];
                    L[4] += m.sqrtg * st;
                }
                double rhoe = divqE / m.sqrtg;
                double Eda = 0.0, Bda = 0.0;
                for (int a = 0; a < 3; a++) {
                    L[5 + a] += -al * m.sqrtg * rhoe * v[a];
                    double gPsi = 0.0, gPhi = 0.0; /* gamma^{ab} d_b */
                    for (int b = 0; b < 3; b++) {
                        gPsi += m.gi[a][b] * dPsi[b];
                        gPhi += m.gi[a][b] * dPhi[b];
                    }
                    L[5 + a] += -al * m.sqrtg * gPsi;
                    L[8 + a] += -al * m.sqrtg * gPhi;
                    Eda += Ev[a] * dal[a];
                    Bda += Bv[a] * dal[a];
                }
                L[11] += m.sqrtg * (al * rhoe - al * G->kappa_E * Psi + Eda);
                L[12] += m.sqrtg * (-al * G->kappa_B * Phi + Bda);
                for (int vv = 0; vv < GLM_NV; vv++) Lc[vv][id] = L[vv];
            }
    for (int d = 0; d < 3; d++)
        for (int v = 0; v < GLM_NV; v++) free(F[d][v]);
}

/* One IMEX step of the GLM system; the conserved set is q (10: D, S, tau,
 * E, Psi, Phi) and qB (3, cell-centred).  Same tableau use as or_step;
 * B, Psi and Phi are explicit (R = 0 for them). */
long or_step_glm(const or_grid *G, double **qc, double **qB, double **prim, const double *alpha, const double *psi,
                 double dt)
{
    geom q = mkgeom(G);
    const double *al_arr = G->metric ? alpha : NULL;
    const double *ps_arr = G->metric ? psi : NULL;
    double At[16], A[16], wt[4], w[4];
    int s = or_tableau(G->imex, At, A, wt, w);
    long nc = q.ncell, nfail = 0;
    /* stage variables (undensitised): prims 5, E 3, B 3, Psi, Phi */
    double *sv[4][GLM_NV], *Lc[4][GLM_NV], *R[4][3];
    int Lhave[4] = {0, 0, 0, 0};
    for (int i = 0; i < s; i++) {
        for (int v = 0; v < GLM_NV; v++) {
            sv[i][v] = (double *)malloc(nc * sizeof(double));
            Lc[i][v] = (double *)calloc(nc, sizeof(double));
        }
        for (int v = 0; v < 3; v++) R[i][v] = (double *)calloc(nc, sizeof(double));
        for (long id = 0; id < nc; id++) {
            double p6 = pow6(ps_arr ? ps_arr[id] : 1.0);
            for (int v = 0; v < 5; v++) sv[i][v][id] = prim[v][id];
            for (int v = 0; v < 3; v++) {
                sv[i][5 + v][id] = qc[5 + v][id] / p6;
                sv[i][8 + v][id] = qB[v][id] / p6;
            }
            sv[i][11][id] = qc[8][id] / p6;
            sv[i][12][id] = qc[9][id] / p6;
        }
    }
    /* conserved-variable index of L component v: L[0..7] -> q[0..7],
     * L[8..10] -> qB, L[11] -> q[8], L[12] -> q[9] */
    for (int i = 0; i < s; i++) {
        for (int j = 0; j < i; j++) {
            if (At[i * 4 + j] != 0.0 && !Lhave[j]) {
                or_ghost_fill(G, sv[j], GLM_NV, NULL);
                or_explicit_L_glm(G, sv[j], al_arr, ps_arr, Lc[j]);
                Lhave[j] = 1;
            }
        }
        double aii = A[i * 4 + i];
        for (int k = q.g[2]; k < q.g[2] + q.n[2]; k++)
            for (int jj = q.g[1]; jj < q.g[1] + q.n[1]; jj++)
                for (int ii = q.g[0]; ii < q.g[0] + q.n[0]; ii++) {
                    long id = IX(&q, ii, jj, k);
                    double qs[GLM_NV];
                    for (int v = 0; v < GLM_NV; v++) {
                        double acc = v < 8 ? qc[v][id] : (v < 11 ? qB[v - 8][id] : qc[v - 3][id]);
                        for (int j = 0; j < i; j++) {
                            acc += dt * At[i * 4 + j] * Lc[j][v][id];
                            if (v >= 5 && v < 8) acc += dt * A[i * 4 + j] * R[j][v - 5][id];
                        }
                        qs[v] = acc;
                    }
                    double ps = ps_arr ? ps_arr[id] : 1.0, al = al_arr ? al_arr[id] : 1.0, p6 = pow6(ps);
                    double B[3] = {qs[8] / p6, qs[9] / p6, qs[10] / p6};
                    double guess[3], pr[5], E[3], fz[5];
                    double **gp = (i == 0) ? prim : sv[i - 1];
                    for (int a = 0; a < 3; a++) guess[a] = gp[1 + a][id];
                    if (G->frozen_matter)
                        for (int v = 0; v < 5; v++) fz[v] = prim[v][id];
                    int r = cell_implicit(G, al, ps, qs, B, aii, dt, guess, G->frozen_matter ? fz : NULL, pr, E);
                    if (r == 2) nfail++;
                    for (int v = 0; v < 5; v++) sv[i][v][id] = pr[v];
                    for (int a = 0; a < 3; a++) {
                        sv[i][5 + a][id] = E[a];
                        sv[i][8 + a][id] = B[a];
                        R[i][a][id] = (p6 * E[a] - qs[5 + a]) / (aii * dt);
                    }
                    sv[i][11][id] = qs[11] / p6;
                    sv[i][12][id] = qs[12] / p6;
                }
    }
    for (int j = 0; j < s; j++) {
        if (wt[j] != 0.0 && !Lhave[j]) {
            or_ghost_fill(G, sv[j], GLM_NV, NULL);
            or_explicit_L_glm(G, sv[j], al_arr, ps_arr, Lc[j]);
            Lhave[j] = 1;
        }
    }
    for (int k = q.g[2]; k < q.g[2] + q.n[2]; k++)
        for (int jj = q.g[1]; jj < q.g[1] + q.n[1]; jj++)
            for (int ii = q.g[0]; ii < q.g[0] + q.n[0]; ii++) {
                long id = IX(&q, ii, jj, k);
                for (int v = G->frozen_matter ? 5 : 0; v < GLM_NV; v++) {
                    double *dst = v < 8 ? &qc[v][id] : (v < 11 ? &qB[v - 8][id] : &qc[v - 3][id]);
                    double acc = *dst;
                    for (int j = 0; j < s; j++) {
                        acc += dt * wt[j] * Lc[j][v][id];
                        if (v >= 5 && v < 8) acc += dt * w[j] * R[j][v - 5][id];
                    }
                    *dst = acc;
                }
                if (G->frozen_matter) continue;
                double ps = ps_arr ? ps_arr[id] : 1.0, p6 = pow6(ps);
                double B[3] = {qB[0][id] / p6, qB[1][id] / p6, qB[2][id] / p6};
                double qq[8], pr[5];
                for (int v = 0; v < 8; v++) qq[v] = qc[v][id];
                int r = cell_c2p(G, ps, qq, B, pr);
                if (r == 2) nfail++;
                for (int v = 0; v < 8; v++) qc[v][id] = qq[v];
                for (int v = 0; v < 5; v++) prim[v][id] = pr[v];
            }
    for (int i = 0; i < s; i++) {
        for (int v = 0; v < GLM_NV; v++) {
            free(sv[i][v]);
            free(Lc[i][v]);
        }
        for (int v = 0; v < 3; v++) free(R[i][v]);
    }
    return nfail;
}

/* cell-centred divergence of the GLM q_B: central differences over the
 * interior cells, with the boundary rule supplying the outer neighbours
 * (L1 = mean |div|, L2, Linf) */
void or_divB_glm(const or_grid *G, double **qB, double out[3])
{
    geom q = mkgeom(G);
    double *tmp[3];
    for (int d = 0; d < 3; d++) {
        tmp[d] = (double *)malloc(q.ncell * sizeof(double));
        memcpy(tmp[d], qB[d], q.ncell * sizeof(double));
    }
    or_ghost_fill(G, tmp, 3, NULL);
    double s1 = 0.0, s2 = 0.0, mx = 0.0;
    long cnt = 0;
    for (int k = q.g[2]; k < q.g[2] + q.n[2]; k++)
        for (int j = q.g[1]; j < q.g[1] + q.n[1]; j++)
            for (int i = q.g[0]; i < q.g[0] + q.n[0]; i++) {
                double dv = 0.0;
                for (int d = 0; d < 3; d++) {
                    if (!q.act[d]) continue;
                    int cp[3] = {i, j, k}, cm[3] = {i, j, k};
                    cp[d] += 1;
                    cm[d] -= 1;
                    dv += (tmp[d][IXv(&q, cp)] - tmp[d][IXv(&q, cm)]) / (2.0 * q.dx[d]);
                }
                s1 += fabs(dv);
                s2 += dv * dv;
                if (fabs(dv) > mx) mx = fabs(dv);
                cnt++;
            }
    for (int d = 0; d < 3; d++) free(tmp[d]);
    out[0] = s1 / cnt;
    out[1] = sqrt(s2 / cnt);
    out[2] = mx;
}

/* OpenMP threads of the per-face / per-edge loops: n > 0 sets them; returns
 * the count in use (the CPU-baseline timing states it) */
int or_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
