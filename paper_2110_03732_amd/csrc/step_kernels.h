// step_kernels.h -- gfx950 kernels of one explicit-operator + implicit pass.
//
//   k_ghost_all   one launch over the padded box: outflow / periodic / fixed
//                 ghost points of the stage primitives, E and face fields
//   k_sweep<D>    LDS-staged sweep along direction D: per-cell reconstruction
//                 of the ten face variables, HLL flux on every D-face
//   k_face_E      covariant E_k at the a-faces of edge direction k
//   k_edge_emf    upwind constrained-transport EMF on the edges
//   k_face_update CT update of the face fields + stage accumulation
//   k_cell_update flux divergence, Cowling sources, stage accumulation, fused
//                 implicit E + velocity Newton solve or final recovery
// Paper: Cheong et al., arXiv:2110.03732, Sec 2.1-2.6 and Sec 3.2.
#pragma once
#include "common.h"
#include "physics.h"

namespace gr {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// ghost points: a per-direction index map composed over x, y, z equals
// filling x, then y, then z over the full extent of the other directions
struct BcArgs {
    int bc[3][2];
};

__device__ __forceinline__ int map_cell(const Geo &G, const BcArgs &B, int d, int m)
{
    if (!G.act[d]) return m;
    int g = G.g[d], n = G.n[d];
    if (m < g) {
        int b = B.bc[d][0];
        return b == GR_OUTFLOW ? g : (b == GR_PERIODIC ? m + n : m);
    }
    if (m >= g + n) {
        int b = B.bc[d][1];
        return b == GR_OUTFLOW ? g + n - 1 : (b == GR_PERIODIC ? m - n : m);
    }
    return m;
}
// normal face field of direction d: faces g .. g+n are evolved
__device__ __forceinline__ int map_face(const Geo &G, const BcArgs &B, int d, int m)
{
    if (!G.act[d]) return m;
    int g = G.g[d], n = G.n[d];
    if (m < g) {
        int b = B.bc[d][0];
        return b == GR_OUTFLOW ? g : (b == GR_PERIODIC ? m + n : m);
    }
    if (m > g + n) {
        int b = B.bc[d][1];
        return b == GR_OUTFLOW ? g + n : (b == GR_PERIODIC ? m - n : m);
    }
    return m;
}

__global__ void __launch_bounds__(kBlock) k_ghost_all(Geo G, BcArgs B, Region R, Ptr<8> cells, Ptr<3> faces)
{
    int c[3];
    if (!region_point(R, c)) return;
    int s[3];
    bool move = false;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        s[d] = map_cell(G, B, d, c[d]);
        move |= (s[d] != c[d]);
    }
    unsigned o = (unsigned)lin(G, c) << 3;
    if (move) {
        unsigned os = (unsigned)lin(G, s) << 3;
#pragma unroll
        for (int v = 0; v < 8; v++) stb(cells.p[v], o, ldb(cells.p[v], os));
    }
#pragma unroll
    for (int f = 0; f < 3; f++) {
        int sf[3];
        bool mv = false;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            sf[d] = (d == f) ? map_face(G, B, d, c[d]) : s[d];
            mv |= (sf[d] != c[d]);
        }
        if (mv) stb(faces.p[f], o, ldb(faces.p[f], (unsigned)lin(G, sf) << 3));
    }
}

// ---------------------------------------------------------------------------
// HLL flux at one face of direction D from the reconstructed states of the
// ten face variables (rho, u~^x,y,z, p, E^x,y,z, B^t1, B^t2; reading R9), the
// face metric and the normal face field (Sec 2.1, Sec 2.5).  The orthonormal
// frame makes the flux the special-relativistic one; the coordinate flux of
// the densitised variables is that times alpha psi^4 (D, tau), alpha psi^6
// (S) or alpha psi^2 (E).
template <int MET, int D>
__device__ __forceinline__ void hll_face(const Phys &P, const double sL[10], const double sR[10], double al, double ps,
                                         double bn, double Fout[8])
{
    constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
    double ps2 = MET ? ps * ps : 1.0;
    if (MET) bn *= frcp(ps2 * ps2 * ps2);
    double uL[3], uR[3], EL[3], ER[3], BL[3], BR[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        uL[i] = ps2 * sL[1 + i];
        uR[i] = ps2 * sR[1 + i];
        EL[i] = ps2 * sL[5 + i];
        ER[i] = ps2 * sR[5 + i];
    }
    BL[D] = BR[D] = ps2 * bn;
    BL[t1] = ps2 * sL[8];
    BR[t1] = ps2 * sR[8];
    BL[t2] = ps2 * sL[9];
    BR[t2] = ps2 * sR[9];
    double qL[8], qR[8], gL[8], gR[8];
    flat_cons_flux(P, D, sL[0], uL, sL[4], EL, BL, qL, gL);
    flat_cons_flux(P, D, sR[0], uR, sR[4], ER, BR, qR, gR);
    double sD = 1.0, sS = 1.0, sE = 1.0;
    if (MET) {
        double p4 = ps2 * ps2;
        sD = al * p4;
        sS = al * p4 * ps2;
        sE = al * ps2;
    }
#pragma unroll
    for (int v = 0; v < 8; v++) {
        double h = 0.5 * (gL[v] + gR[v]) - 0.5 * (qR[v] - qL[v]);
        double sc = (v == 0 || v == 4) ? sD : (v < 4 ? sS : sE);
        Fout[v] = sc * h;
    }
}

// transverse cell-centred B^t of the cell at coordinates c (contravariant,
// mean of the two faces / psi^6); the +1 face index is kept inside the array
template <int MET>
__device__ __forceinline__ double bcc_t(const Geo &G, const CPtr<3> &sf, const CPtr<2> &met, const int c[3], int t)
{
    unsigned o = (unsigned)lin(G, c) << 3;
    double b;
    if (G.act[t]) {
        int cc[3] = {c[0], c[1], c[2]};
        if (cc[t] > G.N[t] - 2) cc[t] = G.N[t] - 2;
        unsigned o0 = (unsigned)lin(G, cc) << 3;
        b = 0.5 * (ldb(sf.p[t], o0) + ldb(sf.p[t], o0 + ((unsigned)G.st[t] << 3)));
    } else {
        b = ldb(sf.p[t], o);
    }
    if (MET) {
        double ps = ldb(met.p[1], o);
        double p2 = ps * ps;
        b *= frcp(p2 * p2 * p2);
    }
    return b;
}

// LDS-staged sweep along D.  Tile: TX x TY x TZ cells (one per thread), with a
// halo of 3 cells along D.  Every thread forms the HLL flux on the lower
// D-face of its cell from the six-cell windows in LDS; the upper boundary
// face of each line is done by k_last_face.
template <int D>
struct Tile;
template <>
struct Tile<0> {
    static constexpr int TX = 64, TY = 4, TZ = 1;
};
template <>
struct Tile<1> {
    static constexpr int TX = 16, TY = 16, TZ = 1;
};
template <>
struct Tile<2> {
    static constexpr int TX = 16, TY = 1, TZ = 16;
};

template <int REC, int MET, int D>
__global__ void __launch_bounds__(kBlock) k_sweep(Geo G, Phys P, CPtr<8> sp, CPtr<3> sf, CPtr<2> met, Ptr<8> F)
{
    constexpr int TX = Tile<D>::TX, TY = Tile<D>::TY, TZ = Tile<D>::TZ;
    constexpr int HX = (D == 0) ? 3 : 0, HY = (D == 1) ? 3 : 0, HZ = (D == 2) ? 3 : 0;
    constexpr int EX = TX + 2 * HX, EY = TY + 2 * HY;
    constexpr int NRAW = EX * EY * (TZ + 2 * HZ);
    constexpr int NV = 10 + 2 * MET;
    constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
    constexpr int SD = (D == 0) ? 1 : (D == 1 ? EX : EX * EY);  // LDS stride along D

    __shared__ double raw[NV][NRAW];

    const int tid = threadIdx.x;
    const int ox = G.g[0] + blockIdx.x * TX, oy = G.g[1] + blockIdx.y * TY, oz = G.g[2] + blockIdx.z * TZ;

    // ---- tile + halo of every variable into LDS (clamped at the array ends)
    for (int l = tid; l < NRAW; l += kBlock) {
        int lx = l % EX, ly = (l / EX) % EY, lz = l / (EX * EY);
        int c[3] = {ox + lx - HX, oy + ly - HY, oz + lz - HZ};
#pragma unroll
        for (int d = 0; d < 3; d++) c[d] = c[d] < 0 ? 0 : (c[d] > G.N[d] - 1 ? G.N[d] - 1 : c[d]);
        unsigned o = (unsigned)lin(G, c) << 3;
#pragma unroll
        for (int v = 0; v < 8; v++) raw[v][l] = ldb(sp.p[v], o);
        raw[8][l] = bcc_t<MET>(G, sf, met, c, t1);
        raw[9][l] = bcc_t<MET>(G, sf, met, c, t2);
        if (MET) {
            raw[10][l] = ldb(met.p[0], o);
            raw[10 + MET][l] = ldb(met.p[1], o);
        }
    }
    __syncthreads();

    // ---- flux on the lower D-face of this thread's cell
    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    int c[3] = {ox + lx, oy + ly, oz + lz};
    if (c[0] >= G.g[0] + G.n[0] || c[1] >= G.g[1] + G.n[1] || c[2] >= G.g[2] + G.n[2]) return;
    const int r0 = ((lz + HZ) * EY + (ly + HY)) * EX + (lx + HX);  // LDS index of the cell
    double sL[10], sR[10];
#pragma unroll
    for (int v = 0; v < 10; v++) {
        double w[6];
#pragma unroll
        for (int m = 0; m < 6; m++) w[m] = raw[v][r0 + (m - 3) * SD];
        recon_face<REC>(w, sL[v], sR[v]);
    }
    double al = 1.0, ps = 1.0;
    if (MET) {
        al = 0.5 * (raw[10][r0 - SD] + raw[10][r0]);
        ps = 0.5 * (raw[10 + MET][r0 - SD] + raw[10 + MET][r0]);
    }
    unsigned o = (unsigned)lin(G, c) << 3;
    double Fo[8];
    hll_face<MET, D>(P, sL, sR, al, ps, ldb(sf.p[D], o), Fo);
#pragma unroll
    for (int v = 0; v < 8; v++) stb(F.p[v], o, Fo[v]);
}

// the upper boundary D-face (index g + n) of every line, from global memory
template <int REC, int MET, int D>
__global__ void __launch_bounds__(kBlock) k_last_face(Geo G, Phys P, Region R, CPtr<8> sp, CPtr<3> sf, CPtr<2> met,
                                                      Ptr<8> F)
{
    constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
    int c[3];
    if (!region_point(R, c)) return;
    int id = lin(G, c);
    int s = G.st[D];
    double sL[10], sR[10];
#pragma unroll
    for (int v = 0; v < 8; v++) recon_at<REC>(sp.p[v], id, s, sL[v], sR[v]);
    double w1[6], w2[6];
#pragma unroll
    for (int m = 0; m < 6; m++) {
        int cc[3] = {c[0], c[1], c[2]};
        cc[D] += m - 3;
        if (REC != GR_PPM && (m == 0 || m == 5)) cc[D] += (m == 0) ? 1 : -1;
        w1[m] = bcc_t<MET>(G, sf, met, cc, t1);
        w2[m] = bcc_t<MET>(G, sf, met, cc, t2);
    }
    recon_face<REC>(w1, sL[8], sR[8]);
    recon_face<REC>(w2, sL[9], sR[9]);
    double al = 1.0, ps = 1.0;
    if (MET) {
        al = 0.5 * (met.p[0][id - s] + met.p[0][id]);
        ps = 0.5 * (met.p[1][id - s] + met.p[1][id]);
    }
    double Fo[8];
    hll_face<MET, D>(P, sL, sR, al, ps, sf.p[D][id], Fo);
#pragma unroll
    for (int v = 0; v < 8; v++) F.p[v][id] = Fo[v];
}

// ---------------------------------------------------------------------------
// metric of the face of direction d at index id (mean of the two cells)
template <int MET>
__device__ __forceinline__ void face_metric(const Geo &G, const CPtr<2> &met, unsigned o, int d, double &al,
                                            double &ps)
{
    if (!MET) {
        al = 1.0;
        ps = 1.0;
        return;
    }
    if (!G.act[d]) {
        al = ldb(met.p[0], o);
        ps = ldb(met.p[1], o);
        return;
    }
    unsigned om = o - ((unsigned)G.st[d] << 3);
    al = 0.5 * (ldb(met.p[0], om) + ldb(met.p[0], o));
    ps = 0.5 * (ldb(met.p[1], om) + ldb(met.p[1], o));
}

// covariant E_k = psi^4 E^k at the a-faces of edge direction k, left and right
// states of the reconstruction along a (Sec 3.2 steps (ii)-(iii))
template <int REC, int MET>
__global__ void __launch_bounds__(kBlock) k_face_E(Geo G, int k, Region R, const double *__restrict__ Ek, CPtr<2> met,
                                                   double *__restrict__ EfL, double *__restrict__ EfR)
{
    int c[3];
    if (!region_point(R, c)) return;
    int a = (k + 1) % 3;
    int id = lin(G, c);
    unsigned o = (unsigned)id << 3;
    double al, ps;
    face_metric<MET>(G, met, o, a, al, ps);
    double p4 = MET ? ps * ps * ps * ps : 1.0;
    double L, Rv;
    if (G.act[a]) {
        recon_at<REC>(Ek, id, G.st[a], L, Rv);
    } else {
        L = Rv = ldb(Ek, o);
    }
    stb(EfL, o, p4 * L);
    stb(EfR, o, p4 * Rv);
}

// upwind EMF hat-E_k on the edges (Sec 3.2 steps (iv)-(vii)), (k, a, b) cyclic
template <int REC, int MET>
__global__ void __launch_bounds__(kBlock) k_edge_emf(Geo G, int k, Region R, CPtr<3> sf, CPtr<2> met,
                                                     const double *__restrict__ EfL, const double *__restrict__ EfR,
                                                     double *__restrict__ EM)
{
    int c[3];
    if (!region_point(R, c)) return;
    int a = (k + 1) % 3, b = (k + 2) % 3;
    int id = lin(G, c);
    unsigned o = (unsigned)id << 3;
    double ELL, ELR, ERL, ERR, qbL, qbR, qaL, qaR;
    if (G.act[b]) {
        recon_at<REC>(EfL, id, G.st[b], ELL, ELR);
        recon_at<REC>(EfR, id, G.st[b], ERL, ERR);
        recon_at<REC>(sf.p[a], id, G.st[b], qaL, qaR);
    } else {
        ELL = ELR = ldb(EfL, o);
        ERL = ERR = ldb(EfR, o);
        qaL = qaR = ldb(sf.p[a], o);
    }
    if (G.act[a]) {
        recon_at<REC>(sf.p[b], id, G.st[a], qbL, qbR);
    } else {
        qbL = qbR = ldb(sf.p[b], o);
    }
    double ca = 1.0, cb = 1.0, ae = 1.0;
    if (MET) {
        unsigned sa = G.act[a] ? ((unsigned)G.st[a] << 3) : 0u, sbb = G.act[b] ? ((unsigned)G.st[b] << 3) : 0u;
        double al0, ps0, al1, ps1;
        face_metric<MET>(G, met, o - sbb, a, al0, ps0);
        face_metric<MET>(G, met, o, a, al1, ps1);
        ca = fmax(al0 * frcp(ps0 * ps0), al1 * frcp(ps1 * ps1));
        face_metric<MET>(G, met, o - sa, b, al0, ps0);
        face_metric<MET>(G, met, o, b, al1, ps1);
        cb = fmax(al0 * frcp(ps0 * ps0), al1 * frcp(ps1 * ps1));
        double sm = ldb(met.p[0], o);
        int na = 1;
        if (G.act[a]) {
            sm += ldb(met.p[0], o - sa);
            na++;
        }
        if (G.act[b]) {
            sm += ldb(met.p[0], o - sbb);
            na++;
        }
        if (G.act[a] && G.act[b]) {
            sm += ldb(met.p[0], o - sa - sbb);
            na++;
        }
        ae = sm / na;
    }
    // metric-only speeds: c+ = c- in every direction
    stb(EM, o, ae * 0.25 * (ELL + ELR + ERL + ERR) + 0.5 * ca * (qbR - qbL) - 0.5 * cb * (qaR - qaL));
}

// ---------------------------------------------------------------------------
struct StageArgs {
    int p, s, fin, withL, storeL;
    double dt, aii_dt;
    double cL[4], cR[4];  // weights of L_j and R_j (j < p); final pass: wt, w
};

// CT update of the face fields of direction d (eq. ct):
// Lf = -(d_{m1} E_{m2} - d_{m2} E_{m1}); stage face = face^n + dt sum_j cL_j Lf_j
struct FaceLs {
    const double *Lf[4];  // stored face L of stages j (direction d), may be null
};
__global__ void __launch_bounds__(kBlock) k_face_update(Geo G, int d, Region R, StageArgs A, CPtr<3> EM,
                                                        const double *fn, FaceLs Ls, double *Lstore, double *fout)
{
    int c[3];
    if (!region_point(R, c)) return;
    int m1 = (d + 1) % 3, m2 = (d + 2) % 3;
    unsigned o = (unsigned)lin(G, c) << 3;
    double acc = ldb(fn, o);
    double Lnew = 0.0;
    if (A.withL) {
        double t1 = G.act[m1] ? (ldb(EM.p[m2], o + ((unsigned)G.st[m1] << 3)) - ldb(EM.p[m2], o)) * G.idx[m1] : 0.0;
        double t2 = G.act[m2] ? (ldb(EM.p[m1], o + ((unsigned)G.st[m2] << 3)) - ldb(EM.p[m1], o)) * G.idx[m2] : 0.0;
        Lnew = -(t1 - t2);
        if (A.storeL) stb(Lstore, o, Lnew);
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
        if (j >= A.p || A.cL[j] == 0.0) continue;
        double l = (A.withL && j == A.p - 1) ? Lnew : ldb(Ls.Lf[j], o);
        acc += A.dt * A.cL[j] * l;
    }
    stb(fout, o, acc);
}

// ---------------------------------------------------------------------------
// cell pass
struct CellIO {
    const double *F[3][8];   // fluxes of the three directions (if withL)
    const double *spm[8];    // stage p-1 primitives + E (if withL)
    const double *sfm[3];    // stage p-1 faces (if withL)
    const double *Lc[4][8];  // stored cell L of stages j < p
    const double *Rj[4][3];  // stored R of stages j < p
    const double *sfp[3];    // faces of this pass
    const double *guess[5];  // primitives giving the Newton / recovery guess
    double *q[8];            // state conserved variables (read; written by the final pass)
    double *out[8];          // stage p prims + E, or state prims (final)
    double *Rout[3];         // R of this stage
    double *Lout[8];         // stored cell L of stage p-1 (if storeL)
    const double *met[2];
    unsigned long long *nfail;
};

template <int MET>
__device__ __forceinline__ double bcc_dev(const Geo &G, const double *const *face, double ip6, unsigned o, int t)
{
    double v = G.act[t] ? 0.5 * (ldb(face[t], o) + ldb(face[t], o + ((unsigned)G.st[t] << 3))) : ldb(face[t], o);
    return MET ? v * ip6 : v;
}

template <int MET>
__global__ void __launch_bounds__(kBlock) k_cell_update(Geo G, Phys P, Region R, StageArgs A, CellIO io)
{
    int c[3];
    if (!region_point(R, c)) return;
    const unsigned o = (unsigned)lin(G, c) << 3;
    double al = 1.0, ps = 1.0;
    if (MET) {
        al = ldb(io.met[0], o);
        ps = ldb(io.met[1], o);
    }
    const double ps2 = ps * ps, ps4 = ps2 * ps2, ps6 = ps4 * ps2;
    const double ips6 = MET ? frcp(ps6) : 1.0, ips2 = MET ? frcp(ps2) : 1.0;
    double Lc[8];
    if (A.withL) {
#pragma unroll
        for (int v = 0; v < 8; v++) Lc[v] = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            if (!G.act[d]) continue;
            unsigned op = o + ((unsigned)G.st[d] << 3);
#pragma unroll
            for (int v = 0; v < 8; v++) Lc[v] -= (ldb(io.F[d][v], op) - ldb(io.F[d][v], o)) * G.idx[d];
        }
        double rho = ldb(io.spm[0], o), pr = ldb(io.spm[4], o);
        double u[3] = {ps2 * ldb(io.spm[1], o), ps2 * ldb(io.spm[2], o), ps2 * ldb(io.spm[3], o)};
        double W = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double iW = frcp(W);
        double v[3] = {u[0] * iW, u[1] * iW, u[2] * iW};
        // Gauss-law charge rho_e = div(q_E)/psi^6 (central differences)
        double divqE = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            if (!G.act[d]) continue;
            unsigned sd = (unsigned)G.st[d] << 3;
            double qp = ldb(io.spm[5 + d], o + sd), qm = ldb(io.spm[5 + d], o - sd);
            if (MET) {
                double a = ldb(io.met[1], o + sd), b = ldb(io.met[1], o - sd);
                double a2 = a * a, b2 = b * b;
                qp *= a2 * a2 * a2;
                qm *= b2 * b2 * b2;
            }
            divqE += (qp - qm) * (0.5 * G.idx[d]);
        }
        double rhoe = divqE * ips6;
        // non-stiff current: s_E = -alpha psi^6 rho_e v^i = -alpha psi^4 rho_e v_on
#pragma unroll
        for (int i = 0; i < 3; i++) Lc[5 + i] -= al * ps4 * rhoe * v[i];
        if (MET) {
            double E[3], B[3];
#pragma unroll
            for (int i = 0; i < 3; i++) {
                E[i] = ps2 * ldb(io.spm[5 + i], o);
                B[i] = ps2 * bcc_dev<MET>(G, io.sfm, ips6, o, i);
            }
            double w = (rho + P.G1 * pr) * W * W;
            double U = 0.5 * (E[0] * E[0] + E[1] * E[1] + E[2] * E[2] + B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
            double S[3] = {w * v[0] + E[1] * B[2] - E[2] * B[1], w * v[1] + E[2] * B[0] - E[0] * B[2],
                           w * v[2] + E[0] * B[1] - E[1] * B[0]};
            double tauD = w - pr + U;
            double trPi = w * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) + 3.0 * pr + U;
            double sdt = 0.0, ips = frcp(ps);
#pragma unroll
            for (int d = 0; d < 3; d++) {
                if (!G.act[d]) continue;
                unsigned sd = (unsigned)G.st[d] << 3;
                double da = (ldb(io.met[0], o + sd) - ldb(io.met[0], o - sd)) * (0.5 * G.idx[d]);
                double dp = (ldb(io.met[1], o + sd) - ldb(io.met[1], o - sd)) * (0.5 * G.idx[d]);
                // s_S = psi^6 [-(tau + D) d alpha + 2 alpha (d psi / psi) tr Pi]
                Lc[1 + d] += ps6 * (-tauD * da + 2.0 * al * dp * ips * trPi);
                sdt -= S[d] * da;
            }
            // s_tau = -psi^6 S^j d_j alpha = -psi^4 S_on . grad alpha
            Lc[4] += ps4 * sdt;
        }
        if (A.storeL) {
#pragma unroll
            for (int v8 = 0; v8 < 8; v8++) stb(io.Lout[v8], o, Lc[v8]);
        }
    }
    // accumulation q* = q^n + dt sum_j (cL_j L_j + cR_j R_j)
    double qs[8];
#pragma unroll
    for (int v = 0; v < 8; v++) qs[v] = ldb(io.q[v], o);
#pragma unroll
    for (int j = 0; j < 4; j++) {
        if (j >= A.p) continue;
        if (A.cL[j] != 0.0) {
            double w = A.dt * A.cL[j];
            if (A.withL && j == A.p - 1) {
#pragma unroll
                for (int v = 0; v < 8; v++) qs[v] += w * Lc[v];
            } else {
#pragma unroll
                for (int v = 0; v < 8; v++) qs[v] += w * ldb(io.Lc[j][v], o);
            }
        }
        if (A.cR[j] != 0.0) {
            double w = A.dt * A.cR[j];
#pragma unroll
            for (int i = 0; i < 3; i++) qs[5 + i] += w * ldb(io.Rj[j][i], o);
        }
    }
    // orthonormal frame: B of this pass, D, tau, S, E*
    double B[3];
#pragma unroll
    for (int i = 0; i < 3; i++) B[i] = ps2 * bcc_dev<MET>(G, io.sfp, ips6, o, i);
    const double ips8 = ips6 * ips2;
    double D = qs[0] * ips6, tau = qs[4] * ips6;
    double S[3] = {qs[1] * ips8, qs[2] * ips8, qs[3] * ips8};
    double Es[3] = {qs[5] * ips6 * ps2, qs[6] * ips6 * ps2, qs[7] * ips6 * ps2};
    double rho = P.rho_atm, u[3] = {0.0, 0.0, 0.0}, pr = P.p_atm, E[3];
    int status = 0;  // 0 ok, 1 atmosphere, 2 failure
    if (!A.fin) {
        double eta = cell_eta(P, D);
        if (D <= P.D_atm) {
            status = 1;
        } else {
            ImpSys sy;
            sy.D = D;
            sy.tau = tau;
            sy.iG1 = P.iG1;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                sy.S[i] = S[i];
                sy.Es[i] = Es[i];
                sy.B[i] = B[i];
                u[i] = ps2 * ldb(io.guess[1 + i], o);
            }
            sy.B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
            sy.et = eta / (al * A.aii_dt);
            ImpEval ev;
            int bad = implicit_solve(sy, P.tol, P.maxit, u, ev);
            if (!bad) {
                rho = D * ev.iW;
                pr = (ev.wt * ev.iW - rho) * P.iG1;
                if (pr < 0.0 && pr >= -1e-12 * rho) pr = 0.0;  // cold-gas round-off
                if (!(pr >= 0.0) || !(ev.W <= 1e4) || !(rho >= P.rho_atm)) bad = 1;
#pragma unroll
                for (int i = 0; i < 3; i++) E[i] = ev.E[i];
            }
            if (bad) status = 2;
        }
        if (status) {
            rho = P.rho_atm;
            u[0] = u[1] = u[2] = 0.0;
            pr = P.p_atm;
            double fct = 1.0 / (1.0 + al * A.aii_dt / eta);  // exact v = 0 solution
#pragma unroll
            for (int i = 0; i < 3; i++) E[i] = Es[i] * fct;
        }
        stb(io.out[0], o, rho);
#pragma unroll
        for (int i = 0; i < 3; i++) stb(io.out[1 + i], o, u[i] * ips2);
        stb(io.out[4], o, pr);
        double iadt = 1.0 / A.aii_dt;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            double Ec = E[i] * ips2;
            stb(io.out[5 + i], o, Ec);
            stb(io.Rout[i], o, (ps6 * Ec - qs[5 + i]) * iadt);  // R = psi^6 (E - E*)/(a_ii dt)
        }
    } else {
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
            int bad = c2p_pressure(P.gam - 1.0, D, tauf, Sf2, ldb(io.guess[4], o), pr, W);
            if (!bad) {
                double Z = tauf + D + pr;
                rho = D / W;
                double WZ = W / Z;
#pragma unroll
                for (int i = 0; i < 3; i++) u[i] = WZ * Sf[i];
                if (!(pr >= 0.0) || !(W <= 1e4) || !(rho >= P.rho_atm)) bad = 1;
            }
            if (bad) status = 2;
        }
        if (status) {
            rho = P.rho_atm;
            u[0] = u[1] = u[2] = 0.0;
            pr = P.p_atm;
            // conserved variables of the atmosphere with the known E, B
            double q8[8], f8[8];
            flat_cons_flux(P, 0, rho, u, pr, E, B, q8, f8);
            qs[0] = q8[0] * ps6;
            qs[1] = q8[1] * ps6 * ps2;
            qs[2] = q8[2] * ps6 * ps2;
            qs[3] = q8[3] * ps6 * ps2;
            qs[4] = q8[4] * ps6;
        }
#pragma unroll
        for (int v = 0; v < 8; v++) stb(io.q[v], o, qs[v]);
        stb(io.out[0], o, rho);
#pragma unroll
        for (int i = 0; i < 3; i++) stb(io.out[1 + i], o, u[i] * ips2);
        stb(io.out[4], o, pr);
    }
    if (status == 2) atomicAdd(io.nfail, 1ull);
}

}  // namespace gr
