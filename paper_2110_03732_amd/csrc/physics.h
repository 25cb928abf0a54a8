// physics.h -- point-wise FP64 device physics of resistive GRMHD for gfx950.
//
// Every local operation is written in the orthonormal frame of the static
// conformally flat metric gamma_ij = psi^4 delta_ij: with u = psi^2 u~,
// E = psi^2 E^i, B = psi^2 B^i and S = S_i / psi^2, the conserved variables,
// fluxes, the implicit Ohm's-law update and the primitive recovery take their
// special-relativistic (flat) form; the metric re-enters only through scale
// factors applied by the callers.  Reference: Cheong et al.,
// arXiv:2110.03732, Sec 2.1 (conserved variables and fluxes), Sec 2.4
// (implicit step), Sec 2.6 (recovery with E, B known).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace gr {

struct Phys {
    double gam;      // adiabatic index Gamma
    double G1;       // Gamma / (Gamma - 1)
    double iG1;      // 1 / G1
    double rho_atm, p_atm, D_atm;  // atmosphere state, D threshold
    double tol;      // Newton tolerance
    int maxit;
    int eta_mode;
    double eta, sigma0, eta_min, eta_max;
    double xi;   // mean-field dynamo coefficient (eq. ohms_law)
    int frozen;  // 1: primitives fixed, only E and B evolve
    double kappa_E, kappa_B;  // GLM damping (Sec 3.1)
};

// flat-frame primitive state -> conserved (D, S, tau, E) and the flux in
// direction d (f_D, f_S, f_tau, f_E); Sec 2.1 with alpha = psi = 1
__device__ __forceinline__ void flat_cons_flux(const Phys &P, int d, double rho, const double u[3], double p,
                                               const double E[3], const double B[3], double q[8], double f[8])
{
    double W = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double iW = frcp(W);
    double v[3] = {u[0] * iW, u[1] * iW, u[2] * iW};
    double rhoh = rho + P.G1 * p;
    double w = rhoh * W * W;   // rho h W^2
    double E2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
    double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    double U = 0.5 * (E2 + B2);
    double ExB[3] = {E[1] * B[2] - E[2] * B[1], E[2] * B[0] - E[0] * B[2], E[0] * B[1] - E[1] * B[0]};
    double D = rho * W;
    double S[3] = {w * v[0] + ExB[0], w * v[1] + ExB[1], w * v[2] + ExB[2]};
    double tau = w - p + U - D;
    q[0] = D;
    q[1] = S[0];
    q[2] = S[1];
    q[3] = S[2];
    q[4] = tau;
    q[5] = E[0];
    q[6] = E[1];
    q[7] = E[2];
    double vd = v[d];
    f[0] = D * vd;
    double pt = p + U;
#pragma unroll
    for (int j = 0; j < 3; j++) f[1 + j] = w * vd * v[j] - E[d] * E[j] - B[d] * B[j] + (j == d ? pt : 0.0);
    f[4] = S[d] - vd * D;
    // f_E^j = eta^{d j k} B^k
    int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    f[5 + d] = 0.0;
    f[5 + d1] = B[d2];
    f[5 + d2] = -B[d1];
}

// HLL with unit speeds, F = (f_L + f_R)/2 - (q_R - q_L)/2, accumulated one
// state at a time: F += (f + sgn q)/2 with sgn = +1 for the left state and -1
// for the right one (only one state's variables are live at a time)
template <int d, bool GLM = false>
__device__ __forceinline__ void hll_accumulate(const Phys &P, double rho, const double u[3], double p,
                                               const double E[3], const double B[3], double sgn, double F[],
                                               double Psi = 0.0, double Phi = 0.0)
{
    constexpr int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    double W = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double iW = frcp(W);
    double v[3] = {u[0] * iW, u[1] * iW, u[2] * iW};
    double w = (rho + P.G1 * p) * W * W;
    double U = 0.5 * (E[0] * E[0] + E[1] * E[1] + E[2] * E[2] + B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    double ExB[3] = {E[1] * B[2] - E[2] * B[1], E[2] * B[0] - E[0] * B[2], E[0] * B[1] - E[1] * B[0]};
    double D = rho * W;
    double S[3] = {w * v[0] + ExB[0], w * v[1] + ExB[1], w * v[2] + ExB[2]};
    double vd = v[d];
    double pt = p + U;
    F[0] += 0.5 * (D * vd + sgn * D);
#pragma unroll
    for (int j = 0; j < 3; j++)
        F[1 + j] += 0.5 * (w * vd * v[j] - E[d] * E[j] - B[d] * B[j] + (j == d ? pt : 0.0) + sgn * S[j]);
    F[4] += 0.5 * (S[d] - vd * D + sgn * (w - p + U - D));
    F[5 + d] += 0.5 * sgn * E[d];
    F[5 + d1] += 0.5 * (B[d2] + sgn * E[d1]);
    F[5 + d2] += 0.5 * (-B[d1] + sgn * E[d2]);
    if (GLM) {
        // GLM (Sec 3.1): Faraday flux of the cell-centred B (the normal
        // component has none), f_Psi = E^d, f_Phi = B^d
        F[8 + d] += 0.5 * sgn * B[d];
        F[8 + d1] += 0.5 * (-E[d2] + sgn * B[d1]);
        F[8 + d2] += 0.5 * (E[d1] + sgn * B[d2]);
        F[11] += 0.5 * (E[d] + sgn * Psi);
        F[12] += 0.5 * (B[d] + sgn * Phi);
    }
}

// resistivity of a cell: uniform, or 1/sigma_c of eq. sigma_D clamped to
// [eta_min, eta_max], with D_atmo the atmosphere threshold D_atm
__device__ __forceinline__ double cell_eta(const Phys &P, double Dund)
{
    if (P.eta_mode == 0) return P.eta;
    double x = 1.0 - P.D_atm / Dund;
    x = x < 0.0 ? 0.0 : x;
    double sig = P.sigma0 * x * x;
    if (sig * P.eta_max <= 1.0) return P.eta_max;
    double e = 1.0 / sig;
    return e < P.eta_min ? P.eta_min : e;
}

// Fused implicit E update + velocity recovery (Sec 2.4, xi = 0), flat frame.
// E(u) = [et E* + A1 (E*.u) u - u x B] / A0, A0 = W + et, A1 = et/(1 + et W);
// f(u) = w~ u - (S - E x B), w~ = [W (tau + D - U) - D/G1]/(W^2 - 1/G1).
// Newton with the analytic Jacobian, 3x3 solve by the adjugate, backtracking
// line search on F = f.f/2 (Armijo 1e-4, quadratic model, cut in [0.1, 0.5]).
struct ImpSys {
    double D, tau, S[3], Es[3], B[3], et, iG1, B2, xi;
};
// everything the Jacobian needs from one residual evaluation
struct ImpEval {
    double f[3], E[3], wt, W, iW, r1, iA0, iden, Esu, U;
};

// the six coefficients of eq. im_E and their W-derivatives (Sec 2.4), for
// xi != 0; with xi = 0 they reduce to A_0 = W + et, A_1 = et/(1 + et W),
// A_5 = -1 and A_2 = A_3 = A_4 = 0, which the solver uses directly
struct ImCoef {
    double A[6], Ad[6];
};
__device__ __forceinline__ void im_coef(double W, double et, double xi, ImCoef &c)
{
    const double x2 = xi * xi;
    const double iWpe = frcp(W + et), iopW = frcp(1.0 + W * et);
    const double iWpe2 = iWpe * iWpe, iopW2 = iopW * iopW;
    c.A[0] = W + et + x2 * (W * W - 1.0) * iWpe;
    c.A[1] = et * iopW + x2 * et * W * iWpe * iopW;
    c.A[2] = -xi * et * iWpe;
    c.A[3] = xi * (1.0 + W * et) * iWpe;
    c.A[4] = xi * (1.0 - et * et + x2) * iWpe * iopW;
    c.A[5] = -1.0 - x2 * W * iWpe;
    c.Ad[0] = 1.0 + x2 * (1.0 + W * W + 2.0 * W * et) * iWpe2;
    c.Ad[1] = -et * et * iopW2 - x2 * et * et * (W * W - 1.0) * iopW2 * iWpe2;
    c.Ad[2] = xi * et * iWpe2;
    c.Ad[3] = xi * (et * et - 1.0) * iWpe2;
    c.Ad[4] = -xi * (1.0 - et * et + x2) * (1.0 + et * et + 2.0 * W * et) * iopW2 * iWpe2;
    c.Ad[5] = -x2 * et * iWpe2;
}

// XI: the mean-field dynamo terms are compiled in (xi != 0); the xi = 0
// instance keeps the short form and its register budget
template <bool XI>
__device__ __forceinline__ void imp_eval(const ImpSys &s, const double u[3], ImpEval &e)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    e.W = sqrt(1.0 + uu);
    e.iW = frcp(e.W);
    e.r1 = frcp(1.0 + s.et * e.W);  // A1 = et r1
    e.iA0 = frcp(e.W + s.et);
    e.Esu = s.Es[0] * u[0] + s.Es[1] * u[1] + s.Es[2] * u[2];
    double uxB[3] = {u[1] * s.B[2] - u[2] * s.B[1], u[2] * s.B[0] - u[0] * s.B[2], u[0] * s.B[1] - u[1] * s.B[0]};
    if (!XI) {
        double A1 = s.et * e.r1;
#pragma unroll
        for (int i = 0; i < 3; i++) e.E[i] = (s.et * s.Es[i] + A1 * e.Esu * u[i] - uxB[i]) * e.iA0;
    } else {
        ImCoef c;
        im_coef(e.W, s.et, s.xi, c);
        e.iA0 = frcp(c.A[0]);
        double Bu = s.B[0] * u[0] + s.B[1] * u[1] + s.B[2] * u[2];
        double uxE[3] = {u[1] * s.Es[2] - u[2] * s.Es[1], u[2] * s.Es[0] - u[0] * s.Es[2],
                         u[0] * s.Es[1] - u[1] * s.Es[0]};
#pragma unroll
        for (int i = 0; i < 3; i++)
            e.E[i] = (s.et * s.Es[i] + c.A[1] * e.Esu * u[i] + c.A[2] * uxE[i] + c.A[3] * s.B[i] +
                      c.A[4] * Bu * u[i] + c.A[5] * uxB[i]) *
                     e.iA0;
    }
    e.U = 0.5 * (e.E[0] * e.E[0] + e.E[1] * e.E[1] + e.E[2] * e.E[2] + s.B2);
    e.iden = frcp(e.W * e.W - s.iG1);
    e.wt = (e.W * (s.tau + s.D - e.U) - s.D * s.iG1) * e.iden;
    double ExB[3] = {e.E[1] * s.B[2] - e.E[2] * s.B[1], e.E[2] * s.B[0] - e.E[0] * s.B[2],
                     e.E[0] * s.B[1] - e.E[1] * s.B[0]};
#pragma unroll
    for (int i = 0; i < 3; i++) e.f[i] = e.wt * u[i] - (s.S[i] - ExB[i]);
}

template <bool XI>
__device__ __forceinline__ void imp_jac(const ImpSys &s, const double u[3], const ImpEval &e, double J[3][3])
{
    double iA0W = e.iA0 * e.iW;
    double dE[3][3];
    if (!XI) {
        double A1 = s.et * e.r1, A1d = -s.et * s.et * e.r1 * e.r1;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                double t = -e.E[i] * u[j] + A1 * e.W * u[i] * s.Es[j] +
                           (A1 * e.W * (i == j ? 1.0 : 0.0) + A1d * u[i] * u[j]) * e.Esu;
                // - W eps_{i j m} B_m
                if (i != j) {
                    int m = 3 - i - j;
                    double sg = ((j - i + 3) % 3 == 1) ? 1.0 : -1.0;
                    t -= e.W * sg * s.B[m];
                }
                dE[i][j] = t * iA0W;
            }
    } else {
        // A_0 W dE^i/du^j = -Ad_0 E^i u_j + A_1 W u^i E*_j + Ad_3 B^i u_j + A_4 W u^i B_j
        //   + (A_1 W d_ij + Ad_1 u^i u_j)(E*.u) + (A_4 W d_ij + Ad_4 u^i u_j)(B.u)
        //   + eps_ijm (A_2 W E*_m + A_5 W B_m) + u_j (Ad_2 (u x E*)^i + Ad_5 (u x B)^i)
        ImCoef c;
        im_coef(e.W, s.et, s.xi, c);
        double Bu = s.B[0] * u[0] + s.B[1] * u[1] + s.B[2] * u[2];
        double uxE[3] = {u[1] * s.Es[2] - u[2] * s.Es[1], u[2] * s.Es[0] - u[0] * s.Es[2],
                         u[0] * s.Es[1] - u[1] * s.Es[0]};
        double uxB[3] = {u[1] * s.B[2] - u[2] * s.B[1], u[2] * s.B[0] - u[0] * s.B[2], u[0] * s.B[1] - u[1] * s.B[0]};
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                double dij = (i == j) ? 1.0 : 0.0;
                double t = -c.Ad[0] * e.E[i] * u[j] + c.A[1] * e.W * u[i] * s.Es[j] + c.Ad[3] * s.B[i] * u[j] +
                           c.A[4] * e.W * u[i] * s.B[j] + (c.A[1] * e.W * dij + c.Ad[1] * u[i] * u[j]) * e.Esu +
                           (c.A[4] * e.W * dij + c.Ad[4] * u[i] * u[j]) * Bu +
                           u[j] * (c.Ad[2] * uxE[i] + c.Ad[5] * uxB[i]);
                if (i != j) {
                    int m = 3 - i - j;
                    double sg = ((j - i + 3) % 3 == 1) ? 1.0 : -1.0;
                    t += e.W * sg * (c.A[2] * s.Es[m] + c.A[5] * s.B[m]);
                }
                dE[i][j] = t * iA0W;
            }
    }
    double tDU = (s.tau + s.D - e.U) * e.iW;
#pragma unroll
    for (int j = 0; j < 3; j++) {
        double dU = e.E[0] * dE[0][j] + e.E[1] * dE[1][j] + e.E[2] * dE[2][j];
        double dw = (tDU * u[j] - 2.0 * e.wt * u[j] - e.W * dU) * e.iden;
        // d(E x B)_i/du_j = eps_{ilm} dE_l/du_j B_m
        double dxB0 = dE[1][j] * s.B[2] - dE[2][j] * s.B[1];
        double dxB1 = dE[2][j] * s.B[0] - dE[0][j] * s.B[2];
        double dxB2 = dE[0][j] * s.B[1] - dE[1][j] * s.B[0];
        J[0][j] = (j == 0 ? e.wt : 0.0) + u[0] * dw + dxB0;
        J[1][j] = (j == 1 ? e.wt : 0.0) + u[1] * dw + dxB1;
        J[2][j] = (j == 2 ? e.wt : 0.0) + u[2] * dw + dxB2;
    }
}

__device__ __forceinline__ bool solve3(const double J[3][3], const double b[3], double x[3])
{
    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (!(det != 0.0) || !isfinite(det)) return false;
    double id = 1.0 / det;
    double c10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    double c12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    double c20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    double c21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    x[0] = (c00 * b[0] + c10 * b[1] + c20 * b[2]) * id;
    x[1] = (c01 * b[0] + c11 * b[1] + c21 * b[2]) * id;
    x[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) * id;
    return true;
}

// returns 0 converged, 1 not converged; u: guess in, root out
template <bool XI>
__device__ __forceinline__ int implicit_solve(const ImpSys &s, double tol, int maxit, double u[3], ImpEval &e)
{
    double J[3][3];
    imp_eval<XI>(s, u, e);
    double F = 0.5 * (e.f[0] * e.f[0] + e.f[1] * e.f[1] + e.f[2] * e.f[2]);
    for (int it = 0; it < maxit; it++) {
        imp_jac<XI>(s, u, e, J);
        double mf[3] = {-e.f[0], -e.f[1], -e.f[2]}, dx[3];
        if (!solve3(J, mf, dx)) return 1;
        double dmax = fmax(fabs(dx[0]), fmax(fabs(dx[1]), fabs(dx[2])));
        double umax = fmax(fabs(u[0]), fmax(fabs(u[1]), fabs(u[2])));
        // stop when the step is below tol [(1 + max|u|) W^2 + (|S| + |E||B|)/w~],
        // the size to which rounding fixes u: S and tau fix v to a relative
        // eps and u = W v only to eps W^2, and the residual w~ u - (S - E x B)
        // carries rounding of size eps (|S| + |E||B|) (the step that meets
        // the threshold is taken)
        const double Sn = sqrt(s.S[0] * s.S[0] + s.S[1] * s.S[1] + s.S[2] * s.S[2]);
        const double em = sqrt((e.E[0] * e.E[0] + e.E[1] * e.E[1] + e.E[2] * e.E[2]) * s.B2);
        if (dmax <= tol * ((1.0 + umax) * (e.W * e.W) + (e.wt > 0.0 ? (Sn + em) / e.wt : 0.0))) {
            u[0] += dx[0];
            u[1] += dx[1];
            u[2] += dx[2];
            imp_eval<XI>(s, u, e);
            return 0;
        }
        double slope = -2.0 * F, lam = 1.0, un[3], Fn = 0.0;
        ImpEval en;
        bool ok = false;
        for (int ls = 0; ls < 60; ls++) {
            un[0] = u[0] + lam * dx[0];
            un[1] = u[1] + lam * dx[1];
            un[2] = u[2] + lam * dx[2];
            imp_eval<XI>(s, un, en);
            Fn = 0.5 * (en.f[0] * en.f[0] + en.f[1] * en.f[1] + en.f[2] * en.f[2]);
            if (isfinite(Fn) && Fn <= F + 1e-4 * lam * slope) {
                ok = true;
                break;
            }
            double lnew = isfinite(Fn) ? -slope * lam * lam / (2.0 * (Fn - F - slope * lam)) : 0.1 * lam;
            if (!(lnew >= 0.1 * lam)) lnew = 0.1 * lam;
            if (lnew > 0.5 * lam) lnew = 0.5 * lam;
            lam = lnew;
        }
        if (!ok) return 1;
        u[0] = un[0];
        u[1] = un[1];
        u[2] = un[2];
        e = en;
        F = Fn;
    }
    return 1;
}

// Recovery with E and B known (Sec 2.6), flat frame: the root in p of
// g(p) = (Gamma-1) rho eps(p) - p with v = S_f/(tau_f + D + p), rho = D/W,
// rho eps = [tau_f + D (1 - W) + p (1 - W^2)]/W^2, by Newton steps kept inside
// a shrinking sign bracket (bisection when a step leaves it).
__device__ __forceinline__ double c2p_g(double gm1, double p, double D, double tauf, double Sf2, double &dg,
                                        double &W)
{
    double Z = tauf + D + p;
    double iZ = 1.0 / Z;
    double v2 = Sf2 * iZ * iZ;
    if (!(v2 < 1.0)) {
        dg = 0.0;
        W = INFINITY;
        return -INFINITY;
    }
    double iW2 = 1.0 - v2;
    double iW = sqrt(iW2);
    W = frcp(iW);
    double rhoeps = (tauf + D) * iW2 - D * iW + p * (iW2 - 1.0);
    double a = 2.0 * Sf2 * iZ * iZ * iZ;  // d(1/W^2)/dp
    double drhoeps = (tauf + D) * a - D * W * 0.5 * a + (iW2 - 1.0) + p * a;
    dg = gm1 * drhoeps - 1.0;
    return gm1 * rhoeps - p;
}

// returns 0 ok (p, W), 1 no physical root
__device__ __forceinline__ int c2p_pressure(double gm1, double D, double tauf, double Sf2, double pguess, double &p,
                                            double &W)
{
    if (!(D > 0.0)) return 1;
    double lo = sqrt(Sf2) - tauf - D;
    lo = lo < 0.0 ? 0.0 : lo;
    double hi = lo + 2.0 * gm1 * fabs(tauf) + 1e-300;
    double dg, Wt;
    if (c2p_g(gm1, hi, D, tauf, Sf2, dg, Wt) > 0.0) return 1;
    if (lo == 0.0) {
        double g0 = c2p_g(gm1, 0.0, D, tauf, Sf2, dg, Wt);
        if (g0 < 0.0) return 1;
        if (g0 == 0.0) {
            p = 0.0;
            W = Wt;
            return 0;
        }
    }
    double x = pguess;
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    for (int it = 0; it < 200; it++) {
        double g = c2p_g(gm1, x, D, tauf, Sf2, dg, Wt);
        if (g > 0.0) lo = x;
        else hi = x;
        double xn = x - g / dg;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        double dx = fabs(xn - x);
        x = xn;
        if (dx <= 1e-15 * x || hi - lo <= 1e-15 * hi) break;
    }
    p = x;
    double Z = tauf + D + p;
    double v2 = Sf2 / (Z * Z);
    if (!(v2 < 1.0)) return 1;
    W = 1.0 / sqrt(1.0 - v2);
    return 0;
}

}  // namespace gr
