// grmhd.hip -- gfx950 kernels and C ABI for one IMEX-RK step of resistive
// GRMHD on a fixed (Cowling) Cartesian grid (Cheong et al., arXiv:2110.03732).
//
// Pass structure of one step (IMEX tableau with s implicit stages):
//   pass p < s : [ghost fill + explicit operator L of stage p-1]
//                -> stage faces -> cell accumulation q* -> fused implicit
//                   E + velocity Newton solve (Sec 2.4)
//   pass p = s : L of stage s-1 -> final combination -> recovery with E, B
//                known (Sec 2.6)
// The explicit operator (Sec 2.1 fluxes and sources, Sec 2.5 speeds, HLL,
// Sec 3.2 upwind constrained transport) is split over kernels that each own
// one kind of location: faces (fluxes), a-faces (edge-bound electric field
// states), edges (EMFs), face fields (CT update), cells (divergence, sources,
// implicit solve).  All data are structure-of-arrays FP64 blocks.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/grmhd.h"
#include "physics.h"

using namespace gr;

namespace {

constexpr int kBlock = 256;

struct Geo {
    int N[3], g[3], n[3], act[3];
    long st[3];   // index stride per direction
    long fs;      // field stride (doubles)
    double dx[3], idx[3];
};

// ---------------------------------------------------------------------------
// reconstruction of one variable at the face between w[2] and w[3]
__device__ __forceinline__ double minmod2(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}
__device__ __forceinline__ double minmod3(double a, double b, double c)
{
    if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
    if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
    return 0.0;
}
__device__ __forceinline__ double ppm_iface(double am1, double a0, double a1, double a2)
{
    double v = 7.0 / 12.0 * (a0 + a1) - 1.0 / 12.0 * (am1 + a2);
    double lo = fmin(a0, a1), hi = fmax(a0, a1);
    return fmin(fmax(v, lo), hi);
}
__device__ __forceinline__ void ppm_mono(double a, double &aL, double &aR)
{
    if ((aR - a) * (a - aL) <= 0.0) {
        aL = a;
        aR = a;
        return;
    }
    double d = aR - aL, m = a - 0.5 * (aL + aR);
    if (d * m > d * d / 6.0) aL = 3.0 * a - 2.0 * aR;
    else if (-d * d / 6.0 > d * m) aR = 3.0 * a - 2.0 * aL;
}
template <int REC>
__device__ __forceinline__ void recon(const double w[6], double &L, double &R)
{
    if (REC == GR_MINMOD) {
        L = w[2] + 0.5 * minmod2(w[2] - w[1], w[3] - w[2]);
        R = w[3] - 0.5 * minmod2(w[3] - w[2], w[4] - w[3]);
    } else if (REC == GR_MC) {
        L = w[2] + 0.5 * minmod3(0.5 * (w[3] - w[1]), 2.0 * (w[2] - w[1]), 2.0 * (w[3] - w[2]));
        R = w[3] - 0.5 * minmod3(0.5 * (w[4] - w[2]), 2.0 * (w[3] - w[2]), 2.0 * (w[4] - w[3]));
    } else {
        double i1 = ppm_iface(w[0], w[1], w[2], w[3]);
        double i2 = ppm_iface(w[1], w[2], w[3], w[4]);
        double i3 = ppm_iface(w[2], w[3], w[4], w[5]);
        double aL = i1, aR = i2;
        ppm_mono(w[2], aL, aR);
        L = aR;
        aL = i2;
        aR = i3;
        ppm_mono(w[3], aL, aR);
        R = aL;
    }
}
template <int REC>
__device__ __forceinline__ void recon_arr(const double *__restrict__ a, long id, long s, double &L, double &R)
{
    double w[6];
    w[1] = a[id - 2 * s];
    w[2] = a[id - s];
    w[3] = a[id];
    w[4] = a[id + s];
    if (REC == GR_PPM) {
        w[0] = a[id - 3 * s];
        w[5] = a[id + 2 * s];
    } else {
        w[0] = w[5] = 0.0;
    }
    recon<REC>(w, L, R);
}

__device__ __forceinline__ void decode(const Geo &G, const int lo[3], const int cnt[3], long t, int c[3])
{
    c[0] = lo[0] + (int)(t % cnt[0]);
    long r = t / cnt[0];
    c[1] = lo[1] + (int)(r % cnt[1]);
    c[2] = lo[2] + (int)(r / cnt[1]);
}
__device__ __forceinline__ long lin(const Geo &G, const int c[3]) { return c[0] + G.st[1] * c[1] + G.st[2] * c[2]; }

struct Region {
    int lo[3], cnt[3];
    long total;
};

// ---------------------------------------------------------------------------
// measurement hook: launches of the selected kernel classes are bracketed by
// HIP events on the stream they are launched on, with the algorithmic bytes
// (every live input field read once, every output written once) of the launch
enum KClass { KC_FACE_FLUX = 0, KC_FACE_E, KC_EDGE_EMF, KC_FACE_UPDATE, KC_CELL_UPDATE, KC_GHOST, KC_COUNT };
struct TRec {
    int cls;
    hipEvent_t a, b;
    double bytes;
};
std::mutex g_tmu;
unsigned g_tmask = 0;
std::vector<TRec> g_trecs;

struct TScope {
    int cls;
    hipStream_t s;
    double bytes;
    hipEvent_t a = nullptr;
    TScope(int c, hipStream_t st, double b) : cls(c), s(st), bytes(b)
    {
        if (g_tmask & (1u << c)) {
            if (hipEventCreate(&a) == hipSuccess) hipEventRecord(a, s);
            else a = nullptr;
        }
    }
    ~TScope()
    {
        if (!a) return;
        hipEvent_t b;
        if (hipEventCreate(&b) != hipSuccess) return;
        hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_tmu);
        g_trecs.push_back({cls, a, b, bytes});
    }
};

// ---------------------------------------------------------------------------
// ghost fill of one direction and side for 8 cell fields and 3 face fields;
// semantics: zero-gradient copy (outflow), periodic copy, untouched (fixed)
__global__ void __launch_bounds__(kBlock) k_ghost(Geo G, int d, int side, int bc, double *__restrict__ cells,
                                                  double *__restrict__ faces)
{
    int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
    long total = (long)G.N[e1] * G.N[e2] * G.g[d];
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        int m = (int)(t % G.g[d]);
        long r = t / G.g[d];
        int a = (int)(r % G.N[e1]);
        int b = (int)(r / G.N[e1]);
        int c[3], s[3];
        c[e1] = s[e1] = a;
        c[e2] = s[e2] = b;
        int g = G.g[d], n = G.n[d];
        if (side == 0) {
            c[d] = m;
            s[d] = (bc == GR_PERIODIC) ? m + n : g;
        } else {
            c[d] = g + n + m;
            s[d] = (bc == GR_PERIODIC) ? g + m : g + n - 1;
        }
        long ic = lin(G, c), is = lin(G, s);
#pragma unroll
        for (int v = 0; v < 8; v++) cells[v * G.fs + ic] = cells[v * G.fs + is];
#pragma unroll
        for (int fd = 0; fd < 3; fd++)
            if (fd != d) faces[fd * G.fs + ic] = faces[fd * G.fs + is];
        // normal face field: faces g .. g+n are evolved
        if (side == 0) {
            faces[d * G.fs + ic] = faces[d * G.fs + is];
        } else if (g + n + 1 + m < G.N[d]) {
            int cf[3] = {c[0], c[1], c[2]}, sf[3] = {c[0], c[1], c[2]};
            cf[d] = g + n + 1 + m;
            sf[d] = (bc == GR_PERIODIC) ? g + 1 + m : g + n;
            faces[d * G.fs + lin(G, cf)] = faces[d * G.fs + lin(G, sf)];
        }
    }
}

// metric helpers (MET = 0: flat)
template <int MET>
__device__ __forceinline__ void face_metric(const Geo &G, const double *__restrict__ met, long id, int d, double &al,
                                            double &ps)
{
    if (!MET) {
        al = 1.0;
        ps = 1.0;
        return;
    }
    if (!G.act[d]) {
        al = met[id];
        ps = met[G.fs + id];
        return;
    }
    long im = id - G.st[d];
    al = 0.5 * (met[im] + met[id]);
    ps = 0.5 * (met[G.fs + im] + met[G.fs + id]);
}

// cell-centred B^t (contravariant) of cell id from the face fields
template <int MET>
__device__ __forceinline__ double bcc(const Geo &G, const double *__restrict__ face, const double *__restrict__ met,
                                      long id, int t)
{
    double v = G.act[t] ? 0.5 * (face[t * G.fs + id] + face[t * G.fs + id + G.st[t]]) : face[t * G.fs + id];
    if (MET) {
        double ps = met[G.fs + id];
        double p2 = ps * ps;
        v /= p2 * p2 * p2;
    }
    return v;
}

// ---------------------------------------------------------------------------
// HLL fluxes on the faces of direction d (Sec 2.1, Sec 2.5, HLL).
// sp: stage primitives + E (8 fields), sf: stage face fields.
// F (8 fields): coordinate flux of the densitised conserved variables.
template <int REC, int MET>
__global__ void __launch_bounds__(kBlock) k_face_flux(Geo G, Phys P, int d, Region R, const double *__restrict__ sp,
                                                      const double *__restrict__ sf, const double *__restrict__ met,
                                                      double *__restrict__ F)
{
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < R.total; t += (long)gridDim.x * blockDim.x) {
        int c[3];
        decode(G, R.lo, R.cnt, t, c);
        long id = lin(G, c);
        long s = G.st[d];
        double al, ps;
        face_metric<MET>(G, met, id, d, al, ps);
        double ps2 = ps * ps;
        double pL[8], pR[8];
#pragma unroll
        for (int v = 0; v < 8; v++) recon_arr<REC>(sp + v * G.fs, id, s, pL[v], pR[v]);
        double BL[3], BR[3];
#pragma unroll
        for (int tt = 0; tt < 3; tt++) {
            if (tt == d) {
                double bn = sf[d * G.fs + id];
                if (MET) bn /= ps2 * ps2 * ps2;
                BL[tt] = BR[tt] = bn;
            } else {
                double w[6];
                w[1] = bcc<MET>(G, sf, met, id - 2 * s, tt);
                w[2] = bcc<MET>(G, sf, met, id - s, tt);
                w[3] = bcc<MET>(G, sf, met, id, tt);
                w[4] = bcc<MET>(G, sf, met, id + s, tt);
                if (REC == GR_PPM) {
                    w[0] = bcc<MET>(G, sf, met, id - 3 * s, tt);
                    w[5] = bcc<MET>(G, sf, met, id + 2 * s, tt);
                } else {
                    w[0] = w[5] = 0.0;
                }
                recon<REC>(w, BL[tt], BR[tt]);
            }
        }
        // orthonormal frame at the face
        double uL[3], uR[3], EL[3], ER[3];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            uL[i] = ps2 * pL[1 + i];
            uR[i] = ps2 * pR[1 + i];
            EL[i] = ps2 * pL[5 + i];
            ER[i] = ps2 * pR[5 + i];
            BL[i] *= ps2;
            BR[i] *= ps2;
        }
        double qL[8], qR[8], fL[8], fR[8];
        flat_cons_flux(P, d, pL[0], uL, pL[4], EL, BL, qL, fL);
        flat_cons_flux(P, d, pR[0], uR, pR[4], ER, BR, qR, fR);
        // HLL with c+ = c- = alpha sqrt(gamma^dd): coordinate flux = scale x flat flux
        double sD = 1.0, sS = 1.0, sE = 1.0;
        if (MET) {
            double p4 = ps2 * ps2;
            sD = al * p4;
            sS = al * p4 * ps2;
            sE = al * ps2;
        }
#pragma unroll
        for (int v = 0; v < 8; v++) {
            double h = 0.5 * (fL[v] + fR[v]) - 0.5 * (qR[v] - qL[v]);
            double sc = (v == 0 || v == 4) ? sD : (v < 4 ? sS : sE);
            F[v * G.fs + id] = sc * h;
        }
    }
}

// covariant E_k (= psi^4 E^k) at the a-faces of edge direction k, left and
// right states of the reconstruction along a (Sec 3.2 steps (ii)-(iii))
template <int REC, int MET>
__global__ void __launch_bounds__(kBlock) k_face_E(Geo G, int k, Region R, const double *__restrict__ sp,
                                                   const double *__restrict__ met, double *__restrict__ EfL,
                                                   double *__restrict__ EfR)
{
    int a = (k + 1) % 3;
    const double *Ek = sp + (5 + k) * G.fs;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < R.total; t += (long)gridDim.x * blockDim.x) {
        int c[3];
        decode(G, R.lo, R.cnt, t, c);
        long id = lin(G, c);
        double al, ps;
        face_metric<MET>(G, met, id, a, al, ps);
        double p4 = MET ? ps * ps * ps * ps : 1.0;
        double L, Rv;
        if (G.act[a]) {
            recon_arr<REC>(Ek, id, G.st[a], L, Rv);
        } else {
            L = Rv = Ek[id];
        }
        EfL[id] = p4 * L;
        EfR[id] = p4 * Rv;
    }
}

// upwind EMF hat-E_k on edges (Sec 3.2 steps (iv)-(vii)), (k, a, b) cyclic
template <int REC, int MET>
__global__ void __launch_bounds__(kBlock) k_edge_emf(Geo G, int k, Region R, const double *__restrict__ sf,
                                                     const double *__restrict__ met, const double *__restrict__ EfL,
                                                     const double *__restrict__ EfR, double *__restrict__ EM)
{
    int a = (k + 1) % 3, b = (k + 2) % 3;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < R.total; t += (long)gridDim.x * blockDim.x) {
        int c[3];
        decode(G, R.lo, R.cnt, t, c);
        long id = lin(G, c);
        double ELL, ELR, ERL, ERR, qbL, qbR, qaL, qaR;
        if (G.act[b]) {
            recon_arr<REC>(EfL, id, G.st[b], ELL, ELR);
            recon_arr<REC>(EfR, id, G.st[b], ERL, ERR);
            recon_arr<REC>(sf + a * G.fs, id, G.st[b], qaL, qaR);
        } else {
            ELL = ELR = EfL[id];
            ERL = ERR = EfR[id];
            qaL = qaR = sf[a * G.fs + id];
        }
        if (G.act[a]) {
            recon_arr<REC>(sf + b * G.fs, id, G.st[a], qbL, qbR);
        } else {
            qbL = qbR = sf[b * G.fs + id];
        }
        double ca = 1.0, cb = 1.0, ae = 1.0;
        if (MET) {
            double al0, ps0, al1, ps1;
            long idb = G.act[b] ? id - G.st[b] : id;
            face_metric<MET>(G, met, idb, a, al0, ps0);
            face_metric<MET>(G, met, id, a, al1, ps1);
            ca = fmax(al0 / (ps0 * ps0), al1 / (ps1 * ps1));
            long ida = G.act[a] ? id - G.st[a] : id;
            face_metric<MET>(G, met, ida, b, al0, ps0);
            face_metric<MET>(G, met, id, b, al1, ps1);
            cb = fmax(al0 / (ps0 * ps0), al1 / (ps1 * ps1));
            double s = met[id];
            int na = 1;
            if (G.act[a]) {
                s += met[id - G.st[a]];
                na++;
            }
            if (G.act[b]) {
                s += met[id - G.st[b]];
                na++;
            }
            if (G.act[a] && G.act[b]) {
                s += met[id - G.st[a] - G.st[b]];
                na++;
            }
            ae = s / na;
        }
        // c+ = c- in every direction (metric-only speeds)
        double Eh = ae * 0.25 * (ELL + ELR + ERL + ERR) + 0.5 * ca * (qbR - qbL) - 0.5 * cb * (qaR - qaL);
        EM[id] = Eh;
    }
}

// ---------------------------------------------------------------------------
struct StageArgs {
    int p, s, fin, withL, storeL;
    double dt, aii_dt;
    double cL[4], cR[4];  // weights of L_j and R_j (j < p), final: wt, w
};

// CT update of the face fields (eq. ct): Lf = -eta^{dmk} d_m hat-E_k, then
// stage face = face^n + dt sum_j cL_j Lf_j
__global__ void __launch_bounds__(kBlock) k_face_update(Geo G, int d, Region R, StageArgs A,
                                                        const double *__restrict__ EM, const double *fn,
                                                        double *__restrict__ Lf_all, double *fout)
{
    // Lf_all: stage j face L at (j*11 + 8 + d)*fs
    int m1 = (d + 1) % 3, m2 = (d + 2) % 3;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < R.total; t += (long)gridDim.x * blockDim.x) {
        int c[3];
        decode(G, R.lo, R.cnt, t, c);
        long id = lin(G, c);
        double acc = fn[d * G.fs + id];
        double Lnew = 0.0;
        if (A.withL) {
            // -(d_{m1} E_{m2} - d_{m2} E_{m1})
            double t1 = G.act[m1] ? (EM[m2 * G.fs + id + G.st[m1]] - EM[m2 * G.fs + id]) * G.idx[m1] : 0.0;
            double t2 = G.act[m2] ? (EM[m1 * G.fs + id + G.st[m2]] - EM[m1 * G.fs + id]) * G.idx[m2] : 0.0;
            Lnew = -(t1 - t2);
            if (A.storeL) Lf_all[((A.p - 1) * 11 + 8 + d) * G.fs + id] = Lnew;
        }
        for (int j = 0; j < A.p && j < 4; j++) {
            if (A.cL[j] == 0.0) continue;
            double l = (A.withL && j == A.p - 1) ? Lnew : Lf_all[(j * 11 + 8 + d) * G.fs + id];
            acc += A.dt * A.cL[j] * l;
        }
        fout[d * G.fs + id] = acc;
    }
}

// cell pass: L of stage p-1 (flux divergence + sources), accumulation of q*,
// then the implicit solve (p < s) or the final recovery (p = s)
template <int MET>
__global__ void __launch_bounds__(kBlock) k_cell_update(Geo G, Phys P, Region R, StageArgs A,
                                                        const double *__restrict__ F,      // 3 x 8 fields
                                                        const double *__restrict__ spm,    // stage p-1 prims+E
                                                        const double *__restrict__ sfm,    // stage p-1 faces
                                                        const double *__restrict__ met,
                                                        double *__restrict__ q,            // state q (8)
                                                        double *__restrict__ Lall,         // s x 11 fields
                                                        double *__restrict__ Rall,         // s x 3 fields
                                                        const double *__restrict__ sfp,    // faces of this pass
                                                        const double *guess,               // prims for the guess
                                                        double *out,                       // stage p prims+E or state prim
                                                        unsigned long long *__restrict__ nfail)
{
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < R.total; t += (long)gridDim.x * blockDim.x) {
        int c[3];
        decode(G, R.lo, R.cnt, t, c);
        long id = lin(G, c);
        double al = 1.0, ps = 1.0;
        if (MET) {
            al = met[id];
            ps = met[G.fs + id];
        }
        double ps2 = ps * ps, ps4 = ps2 * ps2, ps6 = ps4 * ps2;
        double Lc[8];
        if (A.withL) {
#pragma unroll
            for (int v = 0; v < 8; v++) Lc[v] = 0.0;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                if (!G.act[d]) continue;
                const double *Fd = F + d * 8 * G.fs;
#pragma unroll
                for (int v = 0; v < 8; v++) Lc[v] -= (Fd[v * G.fs + id + G.st[d]] - Fd[v * G.fs + id]) * G.idx[d];
            }
            // sources of stage p-1 at the cell (orthonormal frame)
            double rho = spm[id], pr = spm[4 * G.fs + id];
            double u[3] = {ps2 * spm[G.fs + id], ps2 * spm[2 * G.fs + id], ps2 * spm[3 * G.fs + id]};
            double W = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            double v[3] = {u[0] / W, u[1] / W, u[2] / W};
            // Gauss-law charge rho_e = div(q_E)/psi^6, central differences
            double divqE = 0.0;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                if (!G.act[d]) continue;
                long ip = id + G.st[d], im = id - G.st[d];
                double qp = spm[(5 + d) * G.fs + ip], qm = spm[(5 + d) * G.fs + im];
                if (MET) {
                    double a = met[G.fs + ip], b = met[G.fs + im];
                    double a2 = a * a, b2 = b * b;
                    qp *= a2 * a2 * a2;
                    qm *= b2 * b2 * b2;
                }
                divqE += (qp - qm) * 0.5 * G.idx[d];
            }
            double rhoe = divqE / ps6;
            // s_E = -alpha psi^6 rho_e v^i = -alpha psi^4 rho_e v_on
#pragma unroll
            for (int i = 0; i < 3; i++) Lc[5 + i] -= al * ps4 * rhoe * v[i];
            if (MET) {
                double E[3], B[3];
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    E[i] = ps2 * spm[(5 + i) * G.fs + id];
                    B[i] = ps2 * bcc<MET>(G, sfm, met, id, i);
                }
                double rhoh = rho + P.G1 * pr;
                double w = rhoh * W * W;
                double E2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2], B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
                double U = 0.5 * (E2 + B2);
                double S[3] = {w * v[0] + E[1] * B[2] - E[2] * B[1], w * v[1] + E[2] * B[0] - E[0] * B[2],
                               w * v[2] + E[0] * B[1] - E[1] * B[0]};
                double tauD = w - pr + U;
                double trPi = w * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) + 3.0 * pr + U;
                double sdt = 0.0;
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    if (!G.act[d]) continue;
                    long ip = id + G.st[d], im = id - G.st[d];
                    double da = (met[ip] - met[im]) * 0.5 * G.idx[d];
                    double dp = (met[G.fs + ip] - met[G.fs + im]) * 0.5 * G.idx[d];
                    // s_S = psi^6 [-(tau + D) d alpha + 2 alpha (d psi / psi) tr Pi]
                    Lc[1 + d] += ps6 * (-tauD * da + 2.0 * al * dp / ps * trPi);
                    sdt -= S[d] * da;
                }
                // s_tau = -psi^6 S^j d_j alpha = -psi^4 S_on . grad alpha
                Lc[4] += ps4 * sdt;
            }
            if (A.storeL) {
#pragma unroll
                for (int v = 0; v < 8; v++) Lall[((A.p - 1) * 11 + v) * G.fs + id] = Lc[v];
            }
        }
        // accumulation
        double qs[8];
#pragma unroll
        for (int v = 0; v < 8; v++) qs[v] = q[v * G.fs + id];
        for (int j = 0; j < A.p && j < 4; j++) {
            if (A.cL[j] != 0.0) {
                if (A.withL && j == A.p - 1) {
#pragma unroll
                    for (int v = 0; v < 8; v++) qs[v] += A.dt * A.cL[j] * Lc[v];
                } else {
#pragma unroll
                    for (int v = 0; v < 8; v++) qs[v] += A.dt * A.cL[j] * Lall[(j * 11 + v) * G.fs + id];
                }
            }
            if (A.cR[j] != 0.0) {
#pragma unroll
                for (int i = 0; i < 3; i++) qs[5 + i] += A.dt * A.cR[j] * Rall[(j * 3 + i) * G.fs + id];
            }
        }
        // cell-centred B of this pass, orthonormal frame
        double B[3];
#pragma unroll
        for (int i = 0; i < 3; i++) B[i] = ps2 * bcc<MET>(G, sfp, met, id, i);
        double ips6 = 1.0 / ps6;
        double D = qs[0] * ips6, tau = qs[4] * ips6;
        double ips8 = ips6 / ps2;
        double S[3] = {qs[1] * ips8, qs[2] * ips8, qs[3] * ips8};
        double Es[3] = {qs[5] * ips6 * ps2, qs[6] * ips6 * ps2, qs[7] * ips6 * ps2};  // orthonormal E*
        double rho, u[3], pr, E[3];
        int status = 0;  // 0 ok, 1 atmosphere, 2 failure
        if (!A.fin) {
            double eta = cell_eta(P, D);
            if (D <= P.D_atm) {
                status = 1;
            } else {
                ImpSys sy;
                sy.D = D;
                sy.tau = tau;
                sy.G1 = P.G1;
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    sy.S[i] = S[i];
                    sy.Es[i] = Es[i];
                    sy.B[i] = B[i];
                    u[i] = ps2 * guess[(1 + i) * G.fs + id];
                }
                sy.et = eta / (al * A.aii_dt);
                double wt, W;
                int bad = implicit_solve(sy, P.tol, P.maxit, u, E, wt, W);
                if (!bad) {
                    rho = D / W;
                    pr = (wt / W - rho) / P.G1;
                    if (pr < 0.0 && pr >= -1e-12 * rho) pr = 0.0;
                    if (!(pr >= 0.0) || !(W <= 1e4) || !(rho >= P.rho_atm)) bad = 1;
                }
                if (bad) status = 2;
            }
            if (status) {
                rho = P.rho_atm;
                u[0] = u[1] = u[2] = 0.0;
                pr = P.p_atm;
                double fct = 1.0 / (1.0 + al * A.aii_dt / eta);
#pragma unroll
                for (int i = 0; i < 3; i++) E[i] = Es[i] * fct;
            }
            // stage outputs: prims (contravariant), E^i, and R = psi^6 (E - E*)/(a_ii dt)
            double ip2 = 1.0 / ps2;
            out[id] = rho;
#pragma unroll
            for (int i = 0; i < 3; i++) out[(1 + i) * G.fs + id] = u[i] * ip2;
            out[4 * G.fs + id] = pr;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                double Ec = E[i] * ip2;
                out[(5 + i) * G.fs + id] = Ec;
                Rall[(A.p * 3 + i) * G.fs + id] = (ps6 * Ec - qs[5 + i]) / A.aii_dt;
            }
        } else {
            // final recovery with E and B known
#pragma unroll
            for (int i = 0; i < 3; i++) E[i] = Es[i];
            if (D <= P.D_atm) {
                status = 1;
            } else {
                double ExB[3] = {E[1] * B[2] - E[2] * B[1], E[2] * B[0] - E[0] * B[2], E[0] * B[1] - E[1] * B[0]};
                double Sf[3] = {S[0] - ExB[0], S[1] - ExB[1], S[2] - ExB[2]};
                double U = 0.5 * (E[0] * E[0] + E[1] * E[1] + E[2] * E[2] + B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
                double tauf = tau - U;
                double Sf2 = Sf[0] * Sf[0] + Sf[1] * Sf[1] + Sf[2] * Sf[2];
                double W;
                int bad = c2p_pressure(P.gam - 1.0, D, tauf, Sf2, guess[4 * G.fs + id], pr, W);
                if (!bad) {
                    double Z = tauf + D + pr;
                    rho = D / W;
#pragma unroll
                    for (int i = 0; i < 3; i++) u[i] = W * Sf[i] / Z;
                    if (!(pr >= 0.0) || !(W <= 1e4) || !(rho >= P.rho_atm)) bad = 1;
                }
                if (bad) status = 2;
            }
            if (status) {
                rho = P.rho_atm;
                u[0] = u[1] = u[2] = 0.0;
                pr = P.p_atm;
                // conserved variables of the atmosphere state with the known E, B
                double q8[8], f8[8];
                flat_cons_flux(P, 0, rho, u, pr, E, B, q8, f8);
                qs[0] = q8[0] * ps6;
                qs[1] = q8[1] * ps6 * ps2;
                qs[2] = q8[2] * ps6 * ps2;
                qs[3] = q8[3] * ps6 * ps2;
                qs[4] = q8[4] * ps6;
            }
            double ip2 = 1.0 / ps2;
#pragma unroll
            for (int v = 0; v < 8; v++) q[v * G.fs + id] = qs[v];
            out[id] = rho;
#pragma unroll
            for (int i = 0; i < 3; i++) out[(1 + i) * G.fs + id] = u[i] * ip2;
            out[4 * G.fs + id] = pr;
        }
        if (status == 2) atomicAdd(nfail, 1ull);
    }
}

// ---------------------------------------------------------------------------
// initial data
__global__ void __launch_bounds__(kBlock) k_curlA(Geo G, int Ne0, int Ne1, const double *__restrict__ A, long es,
                                                  const double *__restrict__ fadd, double *__restrict__ face)
{
    long total = (long)G.N[0] * G.N[1] * G.N[2];
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        int c[3];
        c[0] = (int)(t % G.N[0]);
        long r = t / G.N[0];
        c[1] = (int)(r % G.N[1]);
        c[2] = (int)(r / G.N[1]);
        long ie = c[0] + (long)Ne0 * (c[1] + (long)Ne1 * c[2]);
        long est[3] = {1, Ne0, (long)Ne0 * Ne1};
#pragma unroll
        for (int d = 0; d < 3; d++) {
            int m1 = (d + 1) % 3, m2 = (d + 2) % 3;
            double s = 0.0;
            if (A) {
                // q_B^d = d_{m1} A_{m2} - d_{m2} A_{m1}
                if (G.act[m1]) s += (A[m2 * es + ie + est[m1]] - A[m2 * es + ie]) * G.idx[m1];
                if (G.act[m2]) s -= (A[m1 * es + ie + est[m2]] - A[m1 * es + ie]) * G.idx[m2];
            }
            face[d * G.fs + t] = fadd ? fadd[d * total + t] + s : s;
        }
    }
}

template <int MET>
__global__ void __launch_bounds__(kBlock) k_init_cons(Geo G, Phys P, Region R, const double *__restrict__ prim,
                                                      const double *__restrict__ E, const double *__restrict__ face,
                                                      const double *__restrict__ met, double *__restrict__ q)
{
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < R.total; t += (long)gridDim.x * blockDim.x) {
        int c[3];
        decode(G, R.lo, R.cnt, t, c);
        long id = lin(G, c);
        double ps = MET ? met[G.fs + id] : 1.0;
        double ps2 = ps * ps, ps6 = ps2 * ps2 * ps2;
        double u[3], Ev[3], B[3];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            u[i] = ps2 * prim[(1 + i) * G.fs + id];
            Ev[i] = ps2 * E[i * G.fs + id];
            B[i] = ps2 * bcc<MET>(G, face, met, id, i);
        }
        double q8[8], f8[8];
        flat_cons_flux(P, 0, prim[id], u, prim[4 * G.fs + id], Ev, B, q8, f8);
        q[id] = ps6 * q8[0];
        q[G.fs + id] = ps6 * ps2 * q8[1];
        q[2 * G.fs + id] = ps6 * ps2 * q8[2];
        q[3 * G.fs + id] = ps6 * ps2 * q8[3];
        q[4 * G.fs + id] = ps6 * q8[4];
    }
}

// q_E = psi^6 E on all cells; copy of prims and E into a stage block
__global__ void __launch_bounds__(kBlock) k_init_qE(Geo G, int met_on, const double *__restrict__ E,
                                                    const double *__restrict__ met, double *__restrict__ q)
{
    long total = (long)G.N[0] * G.N[1] * G.N[2];
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        double ps6 = 1.0;
        if (met_on) {
            double ps = met[G.fs + t];
            double p2 = ps * ps;
            ps6 = p2 * p2 * p2;
        }
#pragma unroll
        for (int i = 0; i < 3; i++) q[(5 + i) * G.fs + t] = ps6 * E[i * G.fs + t];
    }
}

// stage block 8 fields = (prim 5, E = q_E / psi^6)
__global__ void __launch_bounds__(kBlock) k_stage0(Geo G, int met_on, const double *__restrict__ prim,
                                                   const double *__restrict__ q, const double *__restrict__ met,
                                                   double *__restrict__ sp)
{
    long total = (long)G.N[0] * G.N[1] * G.N[2];
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        double ips6 = 1.0;
        if (met_on) {
            double ps = met[G.fs + t];
            double p2 = ps * ps;
            ips6 = 1.0 / (p2 * p2 * p2);
        }
#pragma unroll
        for (int v = 0; v < 5; v++) sp[v * G.fs + t] = prim[v * G.fs + t];
#pragma unroll
        for (int i = 0; i < 3; i++) sp[(5 + i) * G.fs + t] = q[(5 + i) * G.fs + t] * ips6;
    }
}

// ---------------------------------------------------------------------------
// reductions: per-block partials (sum |x|, sum x^2, max |x|), then one block
__device__ __forceinline__ void block_reduce3(double &a, double &b, double &c)
{
    __shared__ double sa[kBlock / 64], sb[kBlock / 64], sc[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
        c = fmax(c, __shfl_down(c, o, 64));
    }
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sa[w] = a;
        sb[w] = b;
        sc[w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; i++) {
            a += sa[i];
            b += sb[i];
            c = fmax(c, sc[i]);
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_divb_partial(Geo G, Region R, const double *__restrict__ face,
                                                         double *__restrict__ part)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < R.total; t += (long)gridDim.x * blockDim.x) {
        int cc[3];
        decode(G, R.lo, R.cnt, t, cc);
        long id = lin(G, cc);
        double dv = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++)
            if (G.act[d]) dv += (face[d * G.fs + id + G.st[d]] - face[d * G.fs + id]) * G.idx[d];
        a += fabs(dv);
        b += dv * dv;
        c = fmax(c, fabs(dv));
    }
    block_reduce3(a, b, c);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = a;
        part[3 * blockIdx.x + 1] = b;
        part[3 * blockIdx.x + 2] = c;
    }
}

__global__ void __launch_bounds__(kBlock) k_reduce_final(int nparts, long count, int mode,
                                                         const double *__restrict__ part, double *__restrict__ out)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        a += part[3 * i];
        b += part[3 * i + 1];
        c = fmax(c, part[3 * i + 2]);
    }
    block_reduce3(a, b, c);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            out[0] = a / count;
            out[1] = sqrt(b / count);
            out[2] = c;
        } else {
            out[0] = c;
        }
    }
}

template <int MET>
__global__ void __launch_bounds__(kBlock) k_cfl_partial(Geo G, Region R, const double *__restrict__ met,
                                                        double *__restrict__ part)
{
    double c = 0.0, z = 0.0, z2 = 0.0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < R.total; t += (long)gridDim.x * blockDim.x) {
        int cc[3];
        decode(G, R.lo, R.cnt, t, cc);
        long id = lin(G, cc);
        double sp = 1.0;
        if (MET) {
            double ps = met[G.fs + id];
            sp = met[id] / (ps * ps);
        }
        double s = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++)
            if (G.act[d]) s += sp * G.idx[d];
        c = fmax(c, s);
    }
    block_reduce3(z, z2, c);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = 0.0;
        part[3 * blockIdx.x + 1] = 0.0;
        part[3 * blockIdx.x + 2] = c;
    }
}

// ---------------------------------------------------------------------------
// host side
Geo make_geo(const gr_grid *g)
{
    Geo G;
    for (int d = 0; d < 3; d++) {
        G.act[d] = d < g->ndim;
        G.n[d] = G.act[d] ? g->n[d] : 1;
        G.g[d] = G.act[d] ? g->ng : 0;
        G.N[d] = G.n[d] + 2 * G.g[d];
        G.dx[d] = G.act[d] ? (g->hi[d] - g->lo[d]) / g->n[d] : 1.0;
        G.idx[d] = 1.0 / G.dx[d];
    }
    G.st[0] = 1;
    G.st[1] = G.N[0];
    G.st[2] = (long)G.N[0] * G.N[1];
    long np = (long)G.N[0] * G.N[1] * G.N[2];
    G.fs = (np + 31) / 32 * 32;
    return G;
}

Phys make_phys(const gr_grid *g)
{
    Phys P;
    P.gam = g->gamma_ad;
    P.G1 = g->gamma_ad / (g->gamma_ad - 1.0);
    P.rho_atm = g->rho_atm;
    P.p_atm = g->p_atm;
    P.D_atm = g->rho_atm * g->atm_factor;
    P.tol = g->newton_tol;
    P.maxit = g->newton_maxit;
    P.eta_mode = g->eta_mode;
    P.eta = g->eta;
    P.sigma0 = g->sigma0;
    P.eta_min = g->eta_min;
    P.eta_max = g->eta_max;
    return P;
}

struct Tableau {
    int s;
    double At[4][4], A[4][4], wt[4], w[4];
};

Tableau tableau(int imex)
{
    Tableau T;
    std::memset(&T, 0, sizeof(T));
    if (imex == GR_SSP2_222) {
        // Table imex_ssp2 of the paper, gamma = 1 - 1/sqrt(2)
        double g = 1.0 - 1.0 / std::sqrt(2.0);
        T.s = 2;
        T.At[1][0] = 1.0;
        T.A[0][0] = g;
        T.A[1][0] = 1.0 - 2.0 * g;
        T.A[1][1] = g;
        T.wt[0] = T.wt[1] = 0.5;
        T.w[0] = T.w[1] = 0.5;
    } else {
        // IMEX-SSP3(4,3,3) of Pareschi & Russo (2005), cited by the paper
        const double a = 0.24169426078821, b = 0.06042356519705, e = 0.12915286960590;
        T.s = 4;
        T.At[2][1] = 1.0;
        T.At[3][1] = 0.25;
        T.At[3][2] = 0.25;
        T.wt[1] = T.wt[2] = 1.0 / 6.0;
        T.wt[3] = 2.0 / 3.0;
        T.A[0][0] = a;
        T.A[1][0] = -a;
        T.A[1][1] = a;
        T.A[2][1] = 1.0 - a;
        T.A[2][2] = a;
        T.A[3][0] = b;
        T.A[3][1] = e;
        T.A[3][2] = 0.5 - b - e - a;
        T.A[3][3] = a;
        for (int i = 0; i < 4; i++) T.w[i] = T.wt[i];
    }
    return T;
}

// is L of stage j used by any later stage or by the final combination?
bool needL(const Tableau &T, int j)
{
    if (T.wt[j] != 0.0) return true;
    for (int m = j + 1; m < T.s; m++)
        if (T.At[m][j] != 0.0) return true;
    return false;
}

// workspace layout (all in fields of fs doubles, after a 1 MiB header)
constexpr size_t kHeader = 1 << 20;  // counters + reduction partials
constexpr int kMaxParts = 4096;

struct Layout {
    size_t sprim, sface, L, R, F, Ef, EM, total_fields;
};

Layout layout(const gr_grid *g)
{
    Tableau T = tableau(g->imex);
    Layout L;
    size_t o = 0;
    L.sprim = o;
    o += 8 * (size_t)T.s;
    L.sface = o;
    o += 3 * (size_t)T.s;
    L.L = o;
    o += 11 * (size_t)T.s;
    L.R = o;
    o += 3 * (size_t)T.s;
    L.F = o;
    o += 24;
    L.Ef = o;
    o += 6;
    L.EM = o;
    o += 3;
    L.total_fields = o;
    return L;
}

inline double *wfield(const gr_state *st, const Geo &G, size_t field)
{
    return (double *)((char *)st->work + kHeader) + field * G.fs;
}
inline unsigned long long *wcounter(const gr_state *st) { return (unsigned long long *)st->work; }
inline double *wparts(const gr_state *st) { return (double *)((char *)st->work + 4096); }

unsigned nblocks(long total)
{
    long b = (total + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (unsigned)b;
}

Region region(const Geo &G, int extra_dim_mask, int full_mask = 0)
{
    Region R;
    R.total = 1;
    for (int d = 0; d < 3; d++) {
        if (full_mask & (1 << d)) {
            R.lo[d] = 0;
            R.cnt[d] = G.N[d];
        } else {
            R.lo[d] = G.g[d];
            R.cnt[d] = G.n[d] + (((extra_dim_mask >> d) & 1) && G.act[d] ? 1 : 0);
        }
        R.total *= R.cnt[d];
    }
    return R;
}

#define HIPCHK(x)                                     \
    do {                                              \
        if ((x) != hipSuccess) return GR_EHIP;         \
    } while (0)
#define LAUNCHCHK()                                   \
    do {                                              \
        if (hipGetLastError() != hipSuccess) return GR_EHIP; \
    } while (0)

gr_status check_state(const gr_grid *g, const gr_state *st)
{
    if (!st || !st->q || !st->face || !st->prim || !st->work) return GR_EINVAL;
    if (g->metric && !st->metric) return GR_EINVAL;
    if (st->work_bytes < gr_workspace_bytes(g)) return GR_ENOMEM;
    return GR_OK;
}

template <int REC, int MET>
gr_status launch_L(const gr_grid *g, const Geo &G, const Phys &P, gr_state *st, const double *sp, const double *sf,
                   hipStream_t s, double *F, double *Ef, double *EM)
{
    const double *met = st->metric;
    const int r = (REC == GR_PPM) ? 3 : 2;
    for (int d = 0; d < 3; d++) {
        if (!G.act[d]) continue;
        Region R = region(G, 1 << d);
        double cells = (double)R.total / R.cnt[d] * (G.n[d] + 2 * r);
        TScope ts(KC_FACE_FLUX, s, 8.0 * (cells * (8 + 2 + 2 * MET) + R.total * (1 + 8)));
        hipLaunchKernelGGL((k_face_flux<REC, MET>), dim3(nblocks(R.total)), dim3(kBlock), 0, s, G, P, d, R, sp, sf,
                           met, F + (size_t)d * 8 * G.fs);
        LAUNCHCHK();
    }
    for (int k = 0; k < 3; k++) {
        int a = (k + 1) % 3, b = (k + 2) % 3;
        if (!G.act[a] && !G.act[b]) continue;
        Region Rf = region(G, 1 << a, 1 << b);
        double *EfL = Ef + (size_t)(2 * k) * G.fs, *EfR = Ef + (size_t)(2 * k + 1) * G.fs;
        {
            TScope ts(KC_FACE_E, s, 8.0 * Rf.total * (1 + 2 * MET + 2));
            hipLaunchKernelGGL((k_face_E<REC, MET>), dim3(nblocks(Rf.total)), dim3(kBlock), 0, s, G, k, Rf, sp, met,
                               EfL, EfR);
            LAUNCHCHK();
        }
        Region Re = region(G, (1 << a) | (1 << b));
        TScope ts(KC_EDGE_EMF, s, 8.0 * (2.0 * Rf.total + Re.total * (2 + 2 * MET + 1)));
        hipLaunchKernelGGL((k_edge_emf<REC, MET>), dim3(nblocks(Re.total)), dim3(kBlock), 0, s, G, k, Re, sf, met,
                           EfL, EfR, EM + (size_t)k * G.fs);
        LAUNCHCHK();
    }
    return GR_OK;
}

gr_status ghost_fill(const gr_grid *g, const Geo &G, double *cells, double *faces, hipStream_t s)
{
    for (int d = 0; d < 3; d++) {
        if (!G.act[d]) continue;
        for (int side = 0; side < 2; side++) {
            int bc = g->bc[d][side];
            if (bc == GR_FIXED) continue;
            long total = (long)G.N[(d + 1) % 3] * G.N[(d + 2) % 3] * G.g[d];
            TScope ts(KC_GHOST, s, 8.0 * total * 11 * 2);
            hipLaunchKernelGGL(k_ghost, dim3(nblocks(total)), dim3(kBlock), 0, s, G, d, side, bc, cells, faces);
            LAUNCHCHK();
        }
    }
    return GR_OK;
}

template <int REC, int MET>
gr_status run_pass(const gr_grid *g, gr_state *st, int p, double dt, hipStream_t s)
{
    Geo G = make_geo(g);
    Phys P = make_phys(g);
    Tableau T = tableau(g->imex);
    Layout Ly = layout(g);
    if (p < 0 || p > T.s) return GR_EINVAL;
    bool fin = (p == T.s);
    bool withL = (p >= 1) && needL(T, p - 1);
    StageArgs A;
    std::memset(&A, 0, sizeof(A));
    A.p = p;
    A.s = T.s;
    A.fin = fin;
    A.withL = withL;
    A.storeL = withL;
    A.dt = dt;
    A.aii_dt = fin ? 0.0 : T.A[p][p] * dt;
    for (int j = 0; j < p && j < 4; j++) {
        A.cL[j] = fin ? T.wt[j] : T.At[p][j];
        A.cR[j] = fin ? T.w[j] : T.A[p][j];
    }
    double *sp_prev = (p >= 1) ? wfield(st, G, Ly.sprim + 8 * (size_t)(p - 1)) : nullptr;
    double *sf_prev = (p >= 1) ? wfield(st, G, Ly.sface + 3 * (size_t)(p - 1)) : nullptr;
    double *F = wfield(st, G, Ly.F), *Ef = wfield(st, G, Ly.Ef), *EM = wfield(st, G, Ly.EM);
    double *Lall = wfield(st, G, Ly.L), *Rall = wfield(st, G, Ly.R);
    if (withL) {
        gr_status r = ghost_fill(g, G, sp_prev, sf_prev, s);
        if (r != GR_OK) return r;
        r = launch_L<REC, MET>(g, G, P, st, sp_prev, sf_prev, s, F, Ef, EM);
        if (r != GR_OK) return r;
    }
    // faces of this pass
    double *fout = fin ? st->face : wfield(st, G, Ly.sface + 3 * (size_t)p);
    int nLst = 0, nRst = 0;
    for (int j = 0; j < p && j < 4; j++) {
        if (A.cL[j] != 0.0 && !(withL && j == p - 1)) nLst++;
        if (A.cR[j] != 0.0) nRst++;
    }
    for (int d = 0; d < 3; d++) {
        Region R = region(G, 1 << d);
        TScope ts(KC_FACE_UPDATE, s, 8.0 * R.total * (2 * (int)withL + 1 + nLst + 1 + (int)withL));
        hipLaunchKernelGGL(k_face_update, dim3(nblocks(R.total)), dim3(kBlock), 0, s, G, d, R, A, EM, st->face, Lall,
                           fout);
        LAUNCHCHK();
    }
    // cells
    Region Rc = region(G, 0);
    double *out = fin ? st->prim : wfield(st, G, Ly.sprim + 8 * (size_t)p);
    const double *guess = (p == 0 || fin) ? st->prim : sp_prev;
    double cb = 8 + 3 + 2 * MET + 8 * nLst + 3 * nRst + (fin ? 1 : 3);           // q, faces, metric, L, R, guess
    if (withL) cb += 3 * 8 + 8 + 3;                                              // fluxes, stage p-1 prims/E, faces
    cb += fin ? (8 + 5) : (8 + 3);                                               // outputs
    if (withL) cb += 8;                                                          // stored L
    TScope ts(KC_CELL_UPDATE, s, 8.0 * Rc.total * cb);
    hipLaunchKernelGGL((k_cell_update<MET>), dim3(nblocks(Rc.total)), dim3(kBlock), 0, s, G, P, Rc, A, F, sp_prev,
                       sf_prev, st->metric, st->q, Lall, Rall, fout, guess, out, wcounter(st));
    LAUNCHCHK();
    return GR_OK;
}

template <int MET>
gr_status dispatch_rec(const gr_grid *g, gr_state *st, int p, double dt, hipStream_t s)
{
    switch (g->recon) {
    case GR_MINMOD: return run_pass<GR_MINMOD, MET>(g, st, p, dt, s);
    case GR_MC: return run_pass<GR_MC, MET>(g, st, p, dt, s);
    default: return run_pass<GR_PPM, MET>(g, st, p, dt, s);
    }
}

}  // namespace

// ===========================================================================
extern "C" {

int gr_abi_version(void) { return GR_ABI_VERSION; }

const char *gr_strerror(gr_status s)
{
    switch (s) {
    case GR_OK: return "ok";
    case GR_EINVAL: return "invalid argument";
    case GR_ENOMEM: return "workspace too small";
    case GR_EHIP: return "HIP runtime error";
    case GR_EUNSUPPORTED: return "unsupported option";
    }
    return "unknown status";
}

gr_status gr_validate(const gr_grid *g)
{
    if (!g) return GR_EINVAL;
    if (g->ndim < 1 || g->ndim > 3) return GR_EINVAL;
    if (g->recon < GR_MINMOD || g->recon > GR_PPM) return GR_EINVAL;
    if (g->imex != GR_SSP2_222 && g->imex != GR_SSP3_433) return GR_EINVAL;
    if (g->ng < (g->recon == GR_PPM ? 3 : 2) || g->ng > 8) return GR_EINVAL;
    for (int d = 0; d < g->ndim; d++) {
        if (g->n[d] < 1 || !(g->hi[d] > g->lo[d])) return GR_EINVAL;
        for (int s = 0; s < 2; s++)
            if (g->bc[d][s] < GR_OUTFLOW || g->bc[d][s] > GR_FIXED) return GR_EINVAL;
        if ((g->bc[d][0] == GR_PERIODIC) != (g->bc[d][1] == GR_PERIODIC)) return GR_EINVAL;
        if (g->bc[d][0] == GR_PERIODIC && g->n[d] < g->ng) return GR_EINVAL;
    }
    if (!(g->gamma_ad > 1.0)) return GR_EINVAL;
    if (g->xi != 0.0) return GR_EUNSUPPORTED;
    if (!(g->newton_tol > 0.0) || g->newton_maxit < 1) return GR_EINVAL;
    if (g->eta_mode == GR_ETA_UNIFORM) {
        if (!(g->eta > 0.0)) return GR_EINVAL;
    } else if (g->eta_mode == GR_ETA_SIGMA_D) {
        if (!(g->eta_min > 0.0) || !(g->eta_max >= g->eta_min)) return GR_EINVAL;
    } else {
        return GR_EINVAL;
    }
    if (!(g->rho_atm > 0.0) || !(g->p_atm >= 0.0) || !(g->atm_factor >= 1.0)) return GR_EINVAL;
    if (g->metric != 0 && g->metric != 1) return GR_EINVAL;
    double cells = 1.0;
    for (int d = 0; d < 3; d++) cells *= (d < g->ndim) ? (g->n[d] + 2.0 * g->ng) : 1.0;
    if (cells > 2.0e9) return GR_EINVAL;
    return GR_OK;
}

size_t gr_field_stride(const gr_grid *g)
{
    if (gr_validate(g) != GR_OK) return 0;
    return (size_t)make_geo(g).fs;
}

size_t gr_workspace_bytes(const gr_grid *g)
{
    if (gr_validate(g) != GR_OK) return 0;
    Geo G = make_geo(g);
    return kHeader + layout(g).total_fields * (size_t)G.fs * sizeof(double);
}

gr_status gr_workspace_offset(const gr_grid *g, int kind, int stage, int field, size_t *off)
{
    gr_status v = gr_validate(g);
    if (v != GR_OK) return v;
    Tableau T = tableau(g->imex);
    Layout L = layout(g);
    Geo G = make_geo(g);
    if (stage < 0 || stage >= T.s || !off) return GR_EINVAL;
    size_t f;
    switch (kind) {
    case 0: if (field < 0 || field >= 8) return GR_EINVAL; f = L.sprim + 8 * (size_t)stage + field; break;
    case 1: if (field < 0 || field >= 3) return GR_EINVAL; f = L.sface + 3 * (size_t)stage + field; break;
    case 2: if (field < 0 || field >= 11) return GR_EINVAL; f = L.L + 11 * (size_t)stage + field; break;
    case 3: if (field < 0 || field >= 3) return GR_EINVAL; f = L.R + 3 * (size_t)stage + field; break;
    default: return GR_EINVAL;
    }
    *off = kHeader + f * (size_t)G.fs * sizeof(double);
    return GR_OK;
}

gr_status gr_init_state(const gr_grid *g, gr_state *st, const double *prim_host, const double *E_host,
                        const double *A_host, const double *face_host, const double *metric_host, hipStream_t s)
{
    gr_status v = gr_validate(g);
    if (v != GR_OK) return v;
    v = check_state(g, st);
    if (v != GR_OK) return v;
    if (!prim_host || !E_host) return GR_EINVAL;
    if (g->metric && !metric_host) return GR_EINVAL;
    Geo G = make_geo(g);
    Phys P = make_phys(g);
    Tableau T = tableau(g->imex);
    Layout Ly = layout(g);
    long np = (long)G.N[0] * G.N[1] * G.N[2];
    size_t cb = (size_t)np * sizeof(double);
    HIPCHK(hipMemsetAsync(st->work, 0, kHeader, s));
    for (int v5 = 0; v5 < 5; v5++)
        HIPCHK(hipMemcpyAsync(st->prim + v5 * G.fs, prim_host + (size_t)v5 * np, cb, hipMemcpyHostToDevice, s));
    if (g->metric)
        for (int v2 = 0; v2 < 2; v2++)
            HIPCHK(hipMemcpyAsync(st->metric + v2 * G.fs, metric_host + (size_t)v2 * np, cb, hipMemcpyHostToDevice, s));
    // E staged in the first stage block, then q_E = psi^6 E
    double *sp0 = wfield(st, G, Ly.sprim);
    for (int i = 0; i < 3; i++)
        HIPCHK(hipMemcpyAsync(sp0 + i * G.fs, E_host + (size_t)i * np, cb, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_init_qE, dim3(nblocks(np)), dim3(kBlock), 0, s, G, g->metric, sp0, st->metric, st->q);
    LAUNCHCHK();
    // faces from the vector potential (+ added face field)
    int Ne0 = G.N[0] + (G.act[0] ? 1 : 0), Ne1 = G.N[1] + (G.act[1] ? 1 : 0), Ne2 = G.N[2] + (G.act[2] ? 1 : 0);
    long es = (long)Ne0 * Ne1 * Ne2;
    double *Ad = nullptr, *fd = nullptr;
    double *scratch = wfield(st, G, Ly.F);  // 24 fields of scratch
    if (A_host) {
        if ((size_t)3 * es > (size_t)24 * G.fs) return GR_EINVAL;
        Ad = scratch;
        HIPCHK(hipMemcpyAsync(Ad, A_host, 3 * es * sizeof(double), hipMemcpyHostToDevice, s));
    }
    if (face_host) {
        fd = scratch + (size_t)12 * G.fs;
        HIPCHK(hipMemcpyAsync(fd, face_host, 3 * cb, hipMemcpyHostToDevice, s));
    }
    hipLaunchKernelGGL(k_curlA, dim3(nblocks(np)), dim3(kBlock), 0, s, G, Ne0, Ne1, Ad, es, fd, st->face);
    LAUNCHCHK();
    Region Rc = region(G, 0);
    if (g->metric)
        hipLaunchKernelGGL(k_init_cons<1>, dim3(nblocks(Rc.total)), dim3(kBlock), 0, s, G, P, Rc, st->prim, sp0,
                           st->face, st->metric, st->q);
    else
        hipLaunchKernelGGL(k_init_cons<0>, dim3(nblocks(Rc.total)), dim3(kBlock), 0, s, G, P, Rc, st->prim, sp0,
                           st->face, st->metric, st->q);
    LAUNCHCHK();
    // every stage block starts as a copy of the state (ghost points of fixed boundaries keep these values)
    for (int j = 0; j < T.s; j++) {
        double *spj = wfield(st, G, Ly.sprim + 8 * (size_t)j);
        hipLaunchKernelGGL(k_stage0, dim3(nblocks(np)), dim3(kBlock), 0, s, G, g->metric, st->prim, st->q, st->metric,
                           spj);
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(wfield(st, G, Ly.sface + 3 * (size_t)j), st->face, 3 * G.fs * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return GR_OK;
}

gr_status gr_imex_stage(const gr_grid *g, gr_state *st, int p, double dt, hipStream_t s)
{
    gr_status v = gr_validate(g);
    if (v != GR_OK) return v;
    v = check_state(g, st);
    if (v != GR_OK) return v;
    if (!(dt > 0.0)) return GR_EINVAL;
    return g->metric ? dispatch_rec<1>(g, st, p, dt, s) : dispatch_rec<0>(g, st, p, dt, s);
}

gr_status gr_step(const gr_grid *g, gr_state *st, double dt, hipStream_t s)
{
    gr_status v = gr_validate(g);
    if (v != GR_OK) return v;
    int ns = tableau(g->imex).s;
    for (int p = 0; p <= ns; p++) {
        v = gr_imex_stage(g, st, p, dt, s);
        if (v != GR_OK) return v;
    }
    return GR_OK;
}

gr_status gr_con2prim(const gr_grid *g, gr_state *st, hipStream_t s)
{
    gr_status v = gr_validate(g);
    if (v != GR_OK) return v;
    v = check_state(g, st);
    if (v != GR_OK) return v;
    Geo G = make_geo(g);
    Phys P = make_phys(g);
    StageArgs A;
    std::memset(&A, 0, sizeof(A));
    A.fin = 1;
    A.dt = 1.0;
    Region Rc = region(G, 0);
    if (g->metric)
        hipLaunchKernelGGL(k_cell_update<1>, dim3(nblocks(Rc.total)), dim3(kBlock), 0, s, G, P, Rc, A, nullptr,
                           nullptr, nullptr, st->metric, st->q, nullptr, nullptr, st->face, st->prim, st->prim,
                           wcounter(st));
    else
        hipLaunchKernelGGL(k_cell_update<0>, dim3(nblocks(Rc.total)), dim3(kBlock), 0, s, G, P, Rc, A, nullptr,
                           nullptr, nullptr, st->metric, st->q, nullptr, nullptr, st->face, st->prim, st->prim,
                           wcounter(st));
    LAUNCHCHK();
    return GR_OK;
}

gr_status gr_divB_norm(const gr_grid *g, const gr_state *st, double *out3, hipStream_t s)
{
    gr_status v = gr_validate(g);
    if (v != GR_OK) return v;
    v = check_state(g, st);
    if (v != GR_OK) return v;
    if (!out3) return GR_EINVAL;
    Geo G = make_geo(g);
    Region Rc = region(G, 0);
    unsigned nb = nblocks(Rc.total);
    if (nb > kMaxParts) nb = kMaxParts;
    double *part = wparts(st);
    hipLaunchKernelGGL(k_divb_partial, dim3(nb), dim3(kBlock), 0, s, G, Rc, st->face, part);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, s, (int)nb, Rc.total, 0, part, out3);
    LAUNCHCHK();
    return GR_OK;
}

gr_status gr_cfl_dt(const gr_grid *g, const gr_state *st, double *dt_host, hipStream_t s)
{
    gr_status v = gr_validate(g);
    if (v != GR_OK) return v;
    v = check_state(g, st);
    if (v != GR_OK) return v;
    if (!dt_host) return GR_EINVAL;
    Geo G = make_geo(g);
    Region Rc = region(G, 0);
    unsigned nb = nblocks(Rc.total);
    if (nb > kMaxParts) nb = kMaxParts;
    double *part = wparts(st);
    double *res = part + 3 * kMaxParts;
    if (g->metric)
        hipLaunchKernelGGL(k_cfl_partial<1>, dim3(nb), dim3(kBlock), 0, s, G, Rc, st->metric, part);
    else
        hipLaunchKernelGGL(k_cfl_partial<0>, dim3(nb), dim3(kBlock), 0, s, G, Rc, st->metric, part);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, s, (int)nb, Rc.total, 1, part, res);
    LAUNCHCHK();
    double mx = 0.0;
    HIPCHK(hipMemcpyAsync(&mx, res, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!(mx > 0.0)) return GR_EINVAL;
    *dt_host = g->cfl / mx;
    return GR_OK;
}

gr_status gr_timing_start(unsigned kernel_class_mask)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &r : g_trecs) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    g_trecs.clear();
    g_tmask = kernel_class_mask;
    return GR_OK;
}

gr_status gr_timing_read(int kernel_class, double *total_ms, long *launches, double *alg_bytes)
{
    if (kernel_class < 0 || kernel_class >= KC_COUNT || !total_ms || !launches || !alg_bytes) return GR_EINVAL;
    std::lock_guard<std::mutex> lk(g_tmu);
    double ms = 0.0, by = 0.0;
    long n = 0;
    for (auto &r : g_trecs) {
        if (r.cls != kernel_class) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return GR_EHIP;
        float e = 0.0f;
        if (hipEventElapsedTime(&e, r.a, r.b) != hipSuccess) return GR_EHIP;
        ms += e;
        by += r.bytes;
        n++;
    }
    *total_ms = ms;
    *launches = n;
    *alg_bytes = by;
    return GR_OK;
}

const char *gr_kernel_class_name(int kernel_class)
{
    static const char *names[KC_COUNT] = {"k_face_flux", "k_face_E", "k_edge_emf", "k_face_update", "k_cell_update",
                                          "k_ghost"};
    if (kernel_class < 0 || kernel_class >= KC_COUNT) return "";
    return names[kernel_class];
}

gr_status gr_fail_count(const gr_grid *g, const gr_state *st, unsigned long long *count, hipStream_t s)
{
    gr_status v = gr_validate(g);
    if (v != GR_OK) return v;
    v = check_state(g, st);
    if (v != GR_OK) return v;
    if (!count) return GR_EINVAL;
    HIPCHK(hipMemcpyAsync(count, wcounter(st), sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return GR_OK;
}

}  // extern "C"
