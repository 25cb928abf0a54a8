// step_kernels.h -- gfx950 kernels of one explicit-operator + implicit pass.
//
//   k_xy          x and y phases of the explicit operator on an LDS-staged
//                 tile: reconstruction of the ten face variables, HLL flux
//                 on every face, flux divergence
//   k_ct          upwind constrained-transport EMF on the edges (Sec 3.2;
//                 the ideal-MHD form of App. A as the CT_IDEAL instances;
//                 one-cell-thick tiles on planes and lines)
//   k_face_update CT update of the face fields + stage accumulation
//   k_cell_update z phase of the explicit operator (3-D), Cowling sources,
//                 stage accumulation, fused implicit E + velocity Newton
//                 solve (with the dynamo terms as the XI instances) or final
//                 recovery; GLM instances carry the cell-centred B, Psi, Phi
// Paper: Cheong et al., arXiv:2110.03732, Sec 2.1-2.6, Sec 3.1-3.2, App. A.
#pragma once
#include "common.h"
#include "physics.h"

namespace gr {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// There is no ghost fill: a read of a stage field at a point beyond the
// interior goes where the boundary rule puts it (stage_cell, common.h); only
// the layer of stage E next to the interior, which the cell pass's charge
// reads with plain offsets, is written (by the face update).

// ---------------------------------------------------------------------------
// HLL flux at one face of direction D from the reconstructed states of the
// face variables (rho, u~^x,y,z, p, E^x,y,z, B^t1, B^t2; reading R9), the
// face metric and the normal face field (Sec 2.1, Sec 2.5).  The orthonormal
// frame makes the flux the special-relativistic one; the coordinate flux of
// the densitised variables is that times alpha psi^4 (D, tau), alpha psi^6
// (S) or alpha psi^2 (E).  GLM (Sec 3.1): three more variables B^D, Psi, Phi
// are reconstructed (the normal B is no longer a face value) and the flux
// has 13 components (+ q_B at alpha psi^2, q_Psi and q_Phi at alpha psi^4).
template <bool GLM>
struct NVar {
    static constexpr int NV = GLM ? 13 : 10;  // reconstructed variables
    static constexpr int NF = GLM ? 13 : 8;   // conserved fields with a flux
};

template <int MET, int D, bool GLM = false>
__device__ __forceinline__ void hll_face(const Phys &P, const double *sL, const double *sR, double al, double ps,
                                         double bn, double *Fout)
{
    constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
    constexpr int NF = NVar<GLM>::NF;
    double ps2 = MET ? ps * ps : 1.0;
    if (MET && !GLM) bn *= frcp(ps2 * ps2 * ps2);
    double h[NF];
#pragma unroll
    for (int v = 0; v < NF; v++) h[v] = 0.0;
#pragma unroll
    for (int side = 0; side < 2; side++) {
        const double *st = side ? sR : sL;
        double u[3], E[3], B[3];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            u[i] = ps2 * st[1 + i];
            E[i] = ps2 * st[5 + i];
        }
        B[D] = ps2 * (GLM ? st[10] : bn);
        B[t1] = ps2 * st[8];
        B[t2] = ps2 * st[9];
        if (GLM) hll_accumulate<D, true>(P, st[0], u, st[4], E, B, side ? -1.0 : 1.0, h, st[11], st[12]);
        else hll_accumulate<D>(P, st[0], u, st[4], E, B, side ? -1.0 : 1.0, h);
    }
    double sD = 1.0, sS = 1.0, sE = 1.0;
    if (MET) {
        double p4 = ps2 * ps2;
        sD = al * p4;
        sS = al * p4 * ps2;
        sE = al * ps2;
    }
#pragma unroll
    for (int v = 0; v < NF; v++) {
        double sc = (v == 0 || v == 4 || v >= 11) ? sD : (v < 4 ? sS : sE);
        Fout[v] = sc * h[v];
    }
}

// cell-centred B^t (contravariant) of the cell at coordinates c: the mean of
// the two faces / psi^6 (the +1 face index kept inside the array), or with
// GLM the cell value / psi^6.  Branch-free: along an inactive t both loads
// read the cell's own value and 0.5 (b + b) = b exactly, so the loads of a
// staging round never wait behind a branch.
template <int MET, bool GLM = false>
__device__ __forceinline__ double bcc_t(const Geo &G, const CPtr<3> &sf, const CPtr<2> &met, const int c[3],
                                        unsigned o, unsigned om, int t)
{
    // face values at byte offset o (the point whose stage values point c
    // takes; the same as c along t), the metric at om (c itself)
    double b;
    if constexpr (!GLM) {
        const bool act = G.act[t];
        const unsigned top = c[t] > G.N[t] - 2 ? (unsigned)G.st[t] << 3 : 0u;  // +1 face kept inside
        const unsigned o0 = act ? o - top : o;
        const unsigned o1 = act ? o0 + ((unsigned)G.st[t] << 3) : o;
        b = 0.5 * (ldb(sf.p[t], o0) + ldb(sf.p[t], o1));
    } else {
        b = ldb(sf.p[t], o);
    }
    if (MET) {
        double ps = ldb(met.p[1], om);
        double p2 = ps * ps;
        b *= frcp(p2 * p2 * p2);
    }
    return b;
}

// One directional phase of the explicit operator over a tile of cells
// [org, org + T), T = (T0, T1, T2) with one thread per cell: the tile plus a
// 3-cell halo along D of the ten face variables goes to LDS; the T_D + 1 faces
// of every line get the HLL flux (a thread takes face tid and, for the few
// faces beyond one per thread, face tid + NT); the fluxes are exchanged
// through the same LDS and each thread returns minus the flux difference of
// its cell divided by dx_D.  Coordinates are clamped into the padded array;
// results for points beyond the interior are computed but never stored.
// threads of a block that owns a tile of n cells: whole wavefronts
constexpr int tile_threads(int n) { return (n + 63) / 64 * 64; }

template <int D, int T0, int T1, int T2, bool GLM = false, bool PCELL = false>
struct PhaseDims {
    static constexpr int NC = T0 * T1 * T2;  // cells of the tile
    static constexpr int NT = tile_threads(NC);
    static constexpr int H = 3;
    static constexpr int E0 = T0 + (D == 0 ? 2 * H : 0), E1 = T1 + (D == 1 ? 2 * H : 0),
                         E2 = T2 + (D == 2 ? 2 * H : 0);
    static constexpr int NRAW = E0 * E1 * E2;
    static constexpr int SD = D == 0 ? 1 : (D == 1 ? E0 : E0 * E1);
    static constexpr int F0 = T0 + (D == 0), F1 = T1 + (D == 1), F2 = T2 + (D == 2);
    static constexpr int NF = F0 * F1 * F2;
    static constexpr int FS = D == 0 ? 1 : (D == 1 ? F0 : F0 * F1);
    static constexpr int NV = NVar<GLM>::NV;
    static constexpr int NFL = NVar<GLM>::NF;
    // PPM: the cells of the tile plus one on each side along D get their
    // left and right interface values once (X0 x X1 x X2 box, stride XS
    // along D), kept in LDS as 2 NV arrays for the faces to read
    static constexpr int X0 = T0 + (D == 0 ? 2 : 0), X1 = T1 + (D == 1 ? 2 : 0), X2 = T2 + (D == 2 ? 2 : 0);
    static constexpr int NE = X0 * X1 * X2;
    static constexpr int XS = D == 0 ? 1 : (D == 1 ? X0 : X0 * X1);
    static constexpr int LR = PCELL ? 2 * NV * NE : 0;
    static constexpr int LDS = NV * NRAW > LR ? NV * NRAW : LR;  // doubles
    static_assert(NF <= 2 * NT, "at most two faces per thread");
    static_assert(NFL * NF <= LDS, "fluxes fit in the staging buffer");
};

// stage block of the sweeps: sp holds rho, u~, p, E (8) and with GLM Psi, Phi
// (fields 8, 9); sf the face fields (GLM: cell-centred q_B)
// PCELL (PPM only): interface values per cell instead of per face
template <int REC, int MET, int D, int T0, int T1, int T2, bool GLM = false, bool PCELL = false>
__device__ __forceinline__ void sweep_phase(const Geo &G, const Phys &P, const CPtr<10> &sp, const CPtr<3> &sf,
                                            const CPtr<2> &met, const int org[3], double *lds, double *Ld)
{
    static_assert(!PCELL || REC == GR_PPM, "per-cell interface values are a PPM form");
    using PD = PhaseDims<D, T0, T1, T2, GLM, PCELL>;
    constexpr int NT = PD::NT, H = PD::H, E0 = PD::E0, E1 = PD::E1, NRAW = PD::NRAW, SD = PD::SD;
    constexpr int F0 = PD::F0, F1 = PD::F1, NF = PD::NF, NV = PD::NV, NFL = PD::NFL;
    constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
    double(*raw)[NRAW] = reinterpret_cast<double(*)[NRAW]>(lds);
    const int tid = threadIdx.x;

    // every load of the staging rounds is issued, unconditionally, before the
    // first LDS store (lanes past the end of the last round load its last
    // point again and store nothing); only a tile whose halo reaches beyond
    // the interior along D maps its points by the boundary rule (the test is
    // the same for the whole block)
    const bool bmap = org[D] - H < G.g[D] || org[D] + (D == 0 ? T0 : (D == 1 ? T1 : T2)) + H > G.g[D] + G.n[D];
    constexpr int NR = (NRAW + NT - 1) / NT;
    double st[NR][NV];
#pragma unroll
    for (int k = 0; k < NR; k++) {
        int l = tid + k * NT;
        if (k == NR - 1 && NRAW % NT != 0) l = l < NRAW ? l : NRAW - 1;
        {
            int c[3] = {org[0] + l % E0, org[1] + (l / E0) % E1, org[2] + l / (E0 * E1)};
            c[D] -= H;
#pragma unroll
            for (int d = 0; d < 3; d++) c[d] = c[d] < 0 ? 0 : (c[d] > G.N[d] - 1 ? G.N[d] - 1 : c[d]);
            // the stage values of a point beyond the interior along D are
            // those the boundary rule gives it
            const unsigned om = (unsigned)lin(G, c) << 3;
            const unsigned o = bmap ? om + ((unsigned)((stage_cell(G, D, c[D]) - c[D]) * G.st[D]) << 3) : om;
#pragma unroll
            for (int v = 0; v < 8; v++) st[k][v] = ldb(sp.p[v], o);
            st[k][8] = bcc_t<MET, GLM>(G, sf, met, c, o, om, t1);
            st[k][9] = bcc_t<MET, GLM>(G, sf, met, c, o, om, t2);
            if (GLM) {
                st[k][10] = bcc_t<MET, GLM>(G, sf, met, c, o, om, D);
                st[k][11] = ldb(sp.p[8], o);
                st[k][12] = ldb(sp.p[9], o);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NR; k++) {
        const int l = tid + k * NT;
        if (l < NRAW) {
#pragma unroll
            for (int v = 0; v < NV; v++) raw[v][l] = st[k][v];
        }
    }
    __syncthreads();

    // PPM: the left and right interface values of every cell of the tile and
    // of one cell beyond it on each side along D, each cell once (two
    // interface values and the monotonicity constraints of that cell): the
    // same arithmetic as per face, where every interface value and every
    // cell's constraints would be evaluated two or three times
    constexpr int X0 = PD::X0, X1 = PD::X1, NE = PD::NE, XS = PD::XS;
    double(*lr)[NE] = reinterpret_cast<double(*)[NE]>(lds);  // [v] aL, [NV + v] aR
    if constexpr (PCELL) {
        constexpr int NRE = (NE + NT - 1) / NT;
        double cl[NRE][NV], cr[NRE][NV];
#pragma unroll
        for (int k = 0; k < NRE; k++) {
            const int e = tid + k * NT;
            if (e < NE) {
                const int x[3] = {e % X0, (e / X0) % X1, e / (X0 * X1)};
                // ext cell x_D = 0 is cell -1 of the tile, raw index H - 1 along D
                const int r = (x[0] + (D == 0 ? H - 1 : 0)) +
                              E0 * ((x[1] + (D == 1 ? H - 1 : 0)) + E1 * (x[2] + (D == 2 ? H - 1 : 0)));
#pragma unroll
                for (int v = 0; v < NV; v++)
                    recon_cell<REC>(raw[v][r - 2 * SD], raw[v][r - SD], raw[v][r], raw[v][r + SD], raw[v][r + 2 * SD],
                                    cl[k][v], cr[k][v]);
            }
        }
        __syncthreads();  // every raw value read: the buffer takes the interface values
#pragma unroll
        for (int k = 0; k < NRE; k++) {
            const int e = tid + k * NT;
            if (e < NE) {
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    lr[v][e] = cl[k][v];
                    lr[NV + v][e] = cr[k][v];
                }
            }
        }
        __syncthreads();
    }

    constexpr int NFR = (NF + NT - 1) / NT;  // faces per thread (1 or 2)
    double Fr[NFR][NFL];
#pragma unroll
    for (int k = 0; k < NFR; k++) {
        const int f = tid + k * NT;
        if (f >= NF) break;
        int e[3] = {f % F0, (f / F0) % F1, f / (F0 * F1)};
        double sL[NV], sR[NV];
        if constexpr (PCELL) {
            // face e_D lies between ext cells e_D (below) and e_D + 1 (above)
            const int xb = e[0] + X0 * (e[1] + X1 * e[2]);
#pragma unroll
            for (int v = 0; v < NV; v++) {
                sL[v] = lr[NV + v][xb];   // right value of the cell below
                sR[v] = lr[v][xb + XS];   // left value of the cell above
            }
        } else {
            const int r0 =
                (e[0] + (D == 0 ? H : 0)) + E0 * ((e[1] + (D == 1 ? H : 0)) + E1 * (e[2] + (D == 2 ? H : 0)));
#pragma unroll
            for (int v = 0; v < NV; v++) {
                double w[6];
#pragma unroll
                for (int m = 0; m < 6; m++) w[m] = raw[v][r0 + (m - 3) * SD];
                recon_face<REC>(w, sL[v], sR[v]);
            }
        }
        int c[3] = {org[0] + e[0], org[1] + e[1], org[2] + e[2]};
#pragma unroll
        for (int d = 0; d < 3; d++) {
            int lo = (d == D) ? 1 : 0;
            c[d] = c[d] < lo ? lo : (c[d] > G.N[d] - 1 ? G.N[d] - 1 : c[d]);
        }
        const unsigned o = (unsigned)lin(G, c) << 3;
        double al = 1.0, ps = 1.0;
        if (MET) {
            const unsigned om = o - ((unsigned)G.st[D] << 3);
            al = 0.5 * (ldb(met.p[0], om) + ldb(met.p[0], o));
            ps = 0.5 * (ldb(met.p[1], om) + ldb(met.p[1], o));
        }
        hll_face<MET, D, GLM>(P, sL, sR, al, ps, GLM ? 0.0 : ldb(sf.p[D], o), Fr[k]);
    }
    __syncthreads();
    double(*fl)[NF] = reinterpret_cast<double(*)[NF]>(lds);
#pragma unroll
    for (int k = 0; k < NFR; k++) {
        const int f = tid + k * NT;
        if (f >= NF) break;
#pragma unroll
        for (int v = 0; v < NFL; v++) fl[v][f] = Fr[k][v];
    }
    __syncthreads();
    if (tid < PD::NC) {
        const int f0 = (tid % T0) + F0 * (((tid / T0) % T1) + F1 * (tid / (T0 * T1)));
#pragma unroll
        for (int v = 0; v < NFL; v++) Ld[v] = -(fl[v][f0 + PD::FS] - fl[v][f0]) * G.idx[D];
    } else {
#pragma unroll
        for (int v = 0; v < NFL; v++) Ld[v] = 0.0;  // threads beyond the tile own no cell
    }
    __syncthreads();  // the buffer is free for the next phase
}

// x and y phases of the explicit operator on a TX x TY tile of one z plane:
// Lxy = -(dF_x/dx) - (dF_y/dy) of every interior cell (the y phase only where
// y is active)
struct XyArgs {
    Geo G;
    Phys P;
    CPtr<10> sp;
    CPtr<3> sf;
    CPtr<2> met;
    Ptr<13> Lxy;
    GridDims gd;
};
template <int REC, int MET, int TX, int TY, bool GLM>
__device__ __forceinline__ void xy_body(const XyArgs &a, Blk blk)
{
    const Geo &G = a.G;
    // TY == 1 tiles serve 1-D grids only: no y phase, LDS for the x phase
    constexpr bool HASY = TY > 1;
    // per-cell PPM interface values in a phase whose arrays fit 40 KiB of
    // LDS (four blocks per compute unit); the other phase keeps the per-face
    // form, so the block's LDS is not raised by the per-cell arrays
    constexpr bool PCX = REC == GR_PPM && PhaseDims<0, TX, TY, 1, GLM, true>::LR * 8 <= 40960;
    constexpr bool PCY = REC == GR_PPM && PhaseDims<1, TX, TY, 1, GLM, true>::LR * 8 <= 40960;
    constexpr int LX = PhaseDims<0, TX, TY, 1, GLM, PCX>::LDS,
                  LY = HASY ? PhaseDims<1, TX, TY, 1, GLM, PCY>::LDS : 1;
    constexpr int NFL = NVar<GLM>::NF;
    __shared__ double lds[LX > LY ? LX : LY];
    const unsigned bx = blk.x, by = blk.y, bz = blk.z;
    const int org[3] = {G.g[0] + (int)bx * TX, G.g[1] + (int)by * TY, G.g[2] + (int)bz};
    double L[NFL];
    sweep_phase<REC, MET, 0, TX, TY, 1, GLM, PCX>(G, a.P, a.sp, a.sf, a.met, org, lds, L);
    if (HASY && G.act[1]) {
        double Ly[NFL];
        sweep_phase<REC, MET, 1, TX, TY, 1, GLM, PCY>(G, a.P, a.sp, a.sf, a.met, org, lds, Ly);
#pragma unroll
        for (int v = 0; v < NFL; v++) L[v] += Ly[v];
    }
    if ((int)threadIdx.x >= TX * TY) return;  // beyond the tile
    const int c[3] = {org[0] + (int)threadIdx.x % TX, org[1] + (int)threadIdx.x / TX, org[2]};
    if (c[0] >= G.g[0] + G.n[0] || c[1] >= G.g[1] + G.n[1]) return;
    const unsigned o = (unsigned)lin(G, c) << 3;
#pragma unroll
    for (int v = 0; v < NFL; v++) stb(a.Lxy.p[v], o, L[v]);
}
template <int REC, int MET, int TX, int TY, bool GLM>
__global__ void __launch_bounds__(tile_threads(TX *TY)) k_xy(XyArgs a)
{
    xy_body<REC, MET, TX, TY, GLM>(a, blk_of(hw_linear<true>(), a.gd));
}
template <int REC, int MET, int TX, int TY, bool GLM>
__global__ void __launch_bounds__(tile_threads(TX *TY)) kb_xy(const XyArgs *__restrict__ aa, const unsigned *__restrict__ start, int n)
{
    unsigned lb;
    const XyArgs &a = aa[batch_locate<true>(start, n, lb)];
    xy_body<REC, MET, TX, TY, GLM>(a, blk_of(lb, a.gd));
}

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

// Upwind constrained-transport EMF hat-E_k on the k-edges (Sec 3.2), (k, a, b)
// cyclic.  One block owns a tile of edges (one edge per thread).  The
// left/right states of the covariant E_k = psi^4 E^k reconstructed along a to
// the a-faces (b widened by the reconstruction halo) are formed first and go
// to LDS; then each edge reconstructs them along b (the LL, LR, RL, RR
// states), q_B^a along b and q_B^b along a, and combines them with the
// metric-only speeds (c+ = c-).  ct_body stages every input in LDS;
// ct_body_direct (x-edges of 3-D grids, and the edges of planes and lines
// along an inactive direction) reads the cell values from memory.
template <int K>
struct CtTile;
template <>
struct CtTile<2> {  // z-edges: a = x, b = y
    static constexpr int T[3] = {16, 16, 1};
};
template <>
struct CtTile<1> {  // y-edges: a = z, b = x
    static constexpr int T[3] = {32, 1, 8};
};
template <>
struct CtTile<0> {  // x-edges: a = y, b = z
    static constexpr int T[3] = {16, 2, 8};
};

// Edge-EMF kernel forms.  CT_BOX: the tiles above (x-edges direct, the others
// staged); CT_IDEAL: the ideal-MHD form of App. A on the same tiles; CT_PLANE
// (z inactive: the x- and y-edges) and CT_LINE (y and z inactive: the y- and
// z-edges): the direct body on one-cell-thick tiles, the inactive directions
// known at compile time so that no halo is staged along them.
enum { CT_BOX = 0, CT_IDEAL = 1, CT_PLANE = 2, CT_LINE = 3 };
template <int K, int F>
struct CtTileF {
    static constexpr int T[3] = {F == CT_PLANE ? 64 : (F == CT_LINE ? 256 : CtTile<K>::T[0]),
                                 F == CT_PLANE ? 4 : (F == CT_LINE ? 1 : CtTile<K>::T[1]),
                                 F == CT_PLANE || F == CT_LINE ? 1 : CtTile<K>::T[2]};
};
// direction d inactive in every grid the form is launched on
template <int F>
__host__ __device__ constexpr bool ct_flat(int d)
{
    return (F == CT_PLANE && d == 2) || (F == CT_LINE && d >= 1);
}

struct CtArgs {
    Geo G;
    Region R;
    const double *Ek;
    CPtr<3> u;  // stage u~ (ideal-MHD form)
    CPtr<3> sf;
    CPtr<2> met;
    double *EM;
    GridDims gd;
};

// transport velocity at a d-face (App. A (i)-(ii)): hat-v^j = alpha v^j of the
// left and right states of u~ reconstructed along d (the cell value along an
// inactive d), weighted by the face speeds; these are equal (metric-only), so
// the weighted velocity is the mean of the two
template <int REC, int MET, int D, int J>
__device__ __forceinline__ double ct_vbar(const Geo &G, const CtArgs &a, const int c[3])
{
    const unsigned o = (unsigned)lin(G, c) << 3;
    double al, ps;
    face_metric<MET>(G, a.met, o, D, al, ps);
    const double p2 = ps * ps;
    // the stage u~ where the boundary rule puts the points (the row mapped
    // across D, the stencil along D point by point)
    int cm[3] = {stage_cell(G, 0, c[0]), stage_cell(G, 1, c[1]), stage_cell(G, 2, c[2])};
    cm[D] = c[D];
    const unsigned om = (unsigned)lin(G, cm) << 3;
    double uL[3], uR[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        if (G.act[D]) {
            recon_stage<REC>(a.u.p[i], G, cm, om, D, uL[i], uR[i]);
        } else {
            uL[i] = uR[i] = ldb(a.u.p[i], om);
        }
    }
    // W^2 = 1 + psi^4 |u~|^2 (orthonormal u = psi^2 u~)
    const double WL = sqrt(1.0 + p2 * p2 * (uL[0] * uL[0] + uL[1] * uL[1] + uL[2] * uL[2]));
    const double WR = sqrt(1.0 + p2 * p2 * (uR[0] * uR[0] + uR[1] * uR[1] + uR[2] * uR[2]));
    return 0.5 * (al * uL[J] / WL + al * uR[J] / WR);
}

// ideal-MHD upwind CT (App. A): hat-E_k = -(hat-v^a q_B^b - hat-v^b q_B^a) at
// the edge, each product in HLL form along the direction it is reconstructed
// in.  Step 1 stages, for the a-faces widened along b, bar-v^b and q_B^a, and
// for the b-faces widened along a, bar-v^a; step 2 reconstructs bar-v^b and
// q_B^a along b, bar-v^a and q_B^b along a, and combines.
template <int REC, int MET, int K>
__device__ __forceinline__ void ct_ideal_body(const CtArgs &args, Blk blk)
{
    const Geo &G = args.G;
    const Region &R = args.R;
    const CPtr<3> &sf = args.sf;
    const CPtr<2> &met = args.met;
    constexpr int A = (K + 1) % 3, B = (K + 2) % 3;
    constexpr int T0 = CtTile<K>::T[0], T1 = CtTile<K>::T[1], T2 = CtTile<K>::T[2];
    constexpr int HB = 3;
    // a-faces widened along b
    constexpr int E0 = T0 + (B == 0 ? 2 * HB : 0), E1 = T1 + (B == 1 ? 2 * HB : 0), E2 = T2 + (B == 2 ? 2 * HB : 0);
    constexpr int NL = E0 * E1 * E2;
    constexpr int SB = (B == 0) ? 1 : (B == 1 ? E0 : E0 * E1);
    // b-faces widened along a
    constexpr int F0 = T0 + (A == 0 ? 2 * HB : 0), F1 = T1 + (A == 1 ? 2 * HB : 0), F2 = T2 + (A == 2 ? 2 * HB : 0);
    constexpr int NLA = F0 * F1 * F2;
    constexpr int SA = (A == 0) ? 1 : (A == 1 ? F0 : F0 * F1);
    static_assert(T0 * T1 * T2 == kBlock, "one edge per thread");
    __shared__ double sVb[NL], sQa[NL], sVa[NLA];

    const int tid = threadIdx.x;
    const int org[3] = {R.lo[0] + (int)blk.x * T0, R.lo[1] + (int)blk.y * T1, R.lo[2] + (int)blk.z * T2};
    const bool actA = G.act[A], actB = G.act[B];
    auto clamp_pos = [&](const int e[3], int W, int c[3]) {
#pragma unroll
        for (int d = 0; d < 3; d++) {
            int lo = R.lo[d], hi = R.lo[d] + R.cnt[d] - 1;
            c[d] = org[d] + e[d];
            if (d == W) {
                c[d] -= HB;
                lo = lo - HB < 0 ? 0 : lo - HB;
                hi = hi + HB > G.N[d] - 1 ? G.N[d] - 1 : hi + HB;
            }
            c[d] = c[d] < lo ? lo : (c[d] > hi ? hi : c[d]);
        }
    };
    for (int l = tid; l < NL; l += kBlock) {
        const int e[3] = {l % E0, (l / E0) % E1, l / (E0 * E1)};
        int c[3];
        clamp_pos(e, B, c);
        sVb[l] = ct_vbar<REC, MET, A, B>(G, args, c);
        // q_B^a of the row where the boundary rule puts it (the a-face itself
        // stays inside the evolved range)
        int cq[3] = {c[0], c[1], c[2]};
        cq[B] = stage_cell(G, B, c[B]);
        sQa[l] = ldb(sf.p[A], (unsigned)lin(G, cq) << 3);
    }
    for (int l = tid; l < NLA; l += kBlock) {
        const int e[3] = {l % F0, (l / F0) % F1, l / (F0 * F1)};
        int c[3];
        clamp_pos(e, A, c);
        sVa[l] = ct_vbar<REC, MET, B, A>(G, args, c);
    }
    __syncthreads();

    const int t[3] = {tid % T0, (tid / T0) % T1, tid / (T0 * T1)};
    int c[3] = {org[0] + t[0], org[1] + t[1], org[2] + t[2]};
    if (c[0] >= R.lo[0] + R.cnt[0] || c[1] >= R.lo[1] + R.cnt[1] || c[2] >= R.lo[2] + R.cnt[2]) return;
    const int r0 = t[0] + (B == 0 ? HB : 0) + E0 * (t[1] + (B == 1 ? HB : 0) + E1 * (t[2] + (B == 2 ? HB : 0)));
    const int r1 = t[0] + (A == 0 ? HB : 0) + F0 * (t[1] + (A == 1 ? HB : 0) + F1 * (t[2] + (A == 2 ? HB : 0)));
    double vbL, vbR, qaL, qaR, vaL, vaR, qbL, qbR;
    if (actB) {
        double w[6];
#pragma unroll
        for (int m = 0; m < 6; m++) w[m] = sVb[r0 + (m - 3) * SB];
        recon_face<REC>(w, vbL, vbR);
#pragma unroll
        for (int m = 0; m < 6; m++) w[m] = sQa[r0 + (m - 3) * SB];
        recon_face<REC>(w, qaL, qaR);
    } else {
        vbL = vbR = sVb[r0];
        qaL = qaR = sQa[r0];
    }
    if (actA) {
        double w[6];
#pragma unroll
        for (int m = 0; m < 6; m++) w[m] = sVa[r1 + (m - 3) * SA];
        recon_face<REC>(w, vaL, vaR);
    } else {
        vaL = vaR = sVa[r1];
    }
    const unsigned o = (unsigned)lin(G, c) << 3;
    // q_B^b along A around the edge, the stencil points where the boundary
    // rule puts them (the edge lies inside the evolved range along B and K)
    if (actA) {
        recon_stage<REC>(sf.p[B], G, c, o, A, qbL, qbR);
    } else {
        qbL = qbR = ldb(sf.p[B], o);
    }
    double ca = 1.0, cb = 1.0;
    if (MET) {
        unsigned sa = actA ? ((unsigned)G.st[A] << 3) : 0u, sbb = actB ? ((unsigned)G.st[B] << 3) : 0u;
        double al0, ps0, al1, ps1;
        face_metric<MET>(G, met, o - sbb, A, al0, ps0);
        face_metric<MET>(G, met, o, A, al1, ps1);
        ca = fmax(al0 * frcp(ps0 * ps0), al1 * frcp(ps1 * ps1));
        face_metric<MET>(G, met, o - sa, B, al0, ps0);
        face_metric<MET>(G, met, o, B, al1, ps1);
        cb = fmax(al0 * frcp(ps0 * ps0), al1 * frcp(ps1 * ps1));
    }
    const double t1 = 0.5 * (vaR * qbR + vaL * qbL) - 0.5 * ca * (qbR - qbL);
    const double t2 = 0.5 * (vbR * qaR + vbL * qaL) - 0.5 * cb * (qaR - qaL);
    stb(args.EM, o, t2 - t1);
}

// Upwind EMF reading its cell values directly (used for the x-edges, whose
// narrow transverse tile would make the staged boxes mostly halo): step 1
// forms, for every a-face the tile needs (b widened by the reconstruction
// halo), the left/right states of psi^4 E_K reconstructed along a and q_B^a
// in LDS; step 2 reconstructs them along b, q_B^b along a from memory, and
// combines them with the metric-only speeds.
template <int REC, int MET, int K, int F>
__device__ __forceinline__ void ct_body_direct(const CtArgs &args, Blk blk)
{
    const Geo &G = args.G;
    const Region &R = args.R;
    const double *__restrict__ Ek = args.Ek;
    const CPtr<3> &sf = args.sf;
    const CPtr<2> &met = args.met;
    constexpr int A = (K + 1) % 3, B = (K + 2) % 3;
    constexpr int T0 = CtTileF<K, F>::T[0], T1 = CtTileF<K, F>::T[1], T2 = CtTileF<K, F>::T[2];
    constexpr int HB = ct_flat<F>(B) ? 0 : 3;
    constexpr int E0 = T0 + (B == 0 ? 2 * HB : 0), E1 = T1 + (B == 1 ? 2 * HB : 0), E2 = T2 + (B == 2 ? 2 * HB : 0);
    constexpr int NL = E0 * E1 * E2;
    constexpr int SB = (B == 0) ? 1 : (B == 1 ? E0 : E0 * E1);  // LDS stride along b
    static_assert(T0 * T1 * T2 == kBlock, "one edge per thread");
    __shared__ double sEL[NL], sER[NL], sQa[NL];

    const int tid = threadIdx.x;
    const int org[3] = {R.lo[0] + (int)blk.x * T0, R.lo[1] + (int)blk.y * T1, R.lo[2] + (int)blk.z * T2};
    // the forms are chosen from the grid's activity: in each of them every
    // direction that is not flat by the form is active
    constexpr bool actA = !ct_flat<F>(A), actB = !ct_flat<F>(B);

    // ---- step 1: a-face states of psi^4 E_k and q_B^a, clamped into range;
    // a lane's loads of all its rounds are issued before the first use (lanes
    // past the end of the last round repeat its last point and store nothing).
    // Only a block whose rows (widened by HB along b) or E stencils (3 along a)
    // leave the interior maps its points by the boundary rule.
    constexpr int TA_ = CtTileF<K, F>::T[A], TB_ = CtTileF<K, F>::T[B];
    const bool bmap = (actA && (org[A] - 3 < G.g[A] || org[A] + TA_ + 2 > G.g[A] + G.n[A] - 1)) ||
                      (actB && (org[B] - HB < G.g[B] || org[B] + TB_ + HB > G.g[B] + G.n[B]));
    constexpr int NR = (NL + kBlock - 1) / kBlock;
    double wE[NR][6], wP[NR][2], wQ[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        int l = tid + r * kBlock;
        if (r == NR - 1 && NL % kBlock != 0) l = l < NL ? l : NL - 1;
        int e[3] = {l % E0, (l / E0) % E1, l / (E0 * E1)};
        int c[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            int lo = R.lo[d], hi = R.lo[d] + R.cnt[d] - 1;
            c[d] = org[d] + e[d];
            if (d == B) {
                c[d] -= HB;
                lo = lo - HB < 0 ? 0 : lo - HB;
                hi = hi + HB > G.N[d] - 1 ? G.N[d] - 1 : hi + HB;
            }
            c[d] = c[d] < lo ? lo : (c[d] > hi ? hi : c[d]);
        }
        const unsigned o = (unsigned)lin(G, c) << 3, sa = (unsigned)G.st[A] << 3;
        // stage values where the boundary rule puts the point: the row mapped
        // along B (the a-face of q_B^a and the stencil centre stay inside the
        // evolved range along A), each E_K stencil point along A by itself;
        // the metric at the point itself
        int cm[3] = {c[0], c[1], c[2]};
        if (bmap) cm[B] = stage_cell(G, B, c[B]);
        const unsigned om = (unsigned)lin(G, cm) << 3;
        if (actA) {
            const int m0 = c[A];
            const bool in = !bmap || (m0 - 3 >= G.g[A] && m0 + 2 <= G.g[A] + G.n[A] - 1);
#pragma unroll
            for (int m = 0; m < 6; m++) {
                // minmod and MC use the four middle points (the outer two are copies)
                const int mm = REC == GR_PPM ? m : (m == 0 ? 1 : (m == 5 ? 4 : m));
                const int dm = in ? mm - 3 : stage_cell(G, A, m0 + mm - 3) - m0;
                wE[r][m] = ldb(Ek, om + ((unsigned)(dm * G.st[A]) << 3));
            }
        } else {
            wE[r][0] = ldb(Ek, om);
        }
        if (MET) {
            wP[r][1] = ldb(met.p[1], o);
            wP[r][0] = actA ? ldb(met.p[1], o - sa) : wP[r][1];
        }
        wQ[r] = ldb(sf.p[A], om);
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int l = tid + r * kBlock;
        if (l < NL) {
            double p4 = 1.0;
            if (MET) {
                const double ps = actA ? 0.5 * (wP[r][0] + wP[r][1]) : wP[r][1];
                p4 = ps * ps * ps * ps;
            }
            double L, Rv;
            if (actA) {
                recon_face<REC>(wE[r], L, Rv);
            } else {
                L = Rv = wE[r][0];
            }
            sEL[l] = p4 * L;
            sER[l] = p4 * Rv;
            sQa[l] = wQ[r];
        }
    }
    __syncthreads();

    // ---- step 2: this thread's edge
    const int t[3] = {tid % T0, (tid / T0) % T1, tid / (T0 * T1)};
    int c[3] = {org[0] + t[0], org[1] + t[1], org[2] + t[2]};
    if (c[0] >= R.lo[0] + R.cnt[0] || c[1] >= R.lo[1] + R.cnt[1] || c[2] >= R.lo[2] + R.cnt[2]) return;
    const int r0 = t[0] + (B == 0 ? HB : 0) + E0 * (t[1] + (B == 1 ? HB : 0) + E1 * (t[2] + (B == 2 ? HB : 0)));
    double ELL, ELR, ERL, ERR, qaL, qaR, qbL, qbR;
    if (actB) {
        double w[6];
#pragma unroll
        for (int m = 0; m < 6; m++) w[m] = sEL[r0 + (m - 3) * SB];
        recon_face<REC>(w, ELL, ELR);
#pragma unroll
        for (int m = 0; m < 6; m++) w[m] = sER[r0 + (m - 3) * SB];
        recon_face<REC>(w, ERL, ERR);
#pragma unroll
        for (int m = 0; m < 6; m++) w[m] = sQa[r0 + (m - 3) * SB];
        recon_face<REC>(w, qaL, qaR);
    } else {
        ELL = ELR = sEL[r0];
        ERL = ERR = sER[r0];
        qaL = qaR = sQa[r0];
    }
    const unsigned o = (unsigned)lin(G, c) << 3;
    // q_B^b along A around the edge, the stencil points where the boundary
    // rule puts them (the edge lies inside the evolved range along B and K)
    if (actA) {
        recon_stage<REC>(sf.p[B], G, c, o, A, qbL, qbR);
    } else {
        qbL = qbR = ldb(sf.p[B], o);
    }
    double ca = 1.0, cb = 1.0, ae = 1.0;
    if (MET) {
        unsigned sa = actA ? ((unsigned)G.st[A] << 3) : 0u, sbb = actB ? ((unsigned)G.st[B] << 3) : 0u;
        double al0, ps0, al1, ps1;
        face_metric<MET>(G, met, o - sbb, A, al0, ps0);
        face_metric<MET>(G, met, o, A, al1, ps1);
        ca = fmax(al0 * frcp(ps0 * ps0), al1 * frcp(ps1 * ps1));
        face_metric<MET>(G, met, o - sa, B, al0, ps0);
        face_metric<MET>(G, met, o, B, al1, ps1);
        cb = fmax(al0 * frcp(ps0 * ps0), al1 * frcp(ps1 * ps1));
        double sm = ldb(met.p[0], o);
        int na = 1;
        if (actA) {
            sm += ldb(met.p[0], o - sa);
            na++;
        }
        if (actB) {
            sm += ldb(met.p[0], o - sbb);
            na++;
        }
        if (actA && actB) {
            sm += ldb(met.p[0], o - sa - sbb);
            na++;
        }
        ae = sm / na;
    }
    stb(args.EM, o, ae * 0.25 * (ELL + ELR + ERL + ERR) + 0.5 * ca * (qbR - qbL) - 0.5 * cb * (qaR - qaL));
}
// An LDS box of the EMF tile of edge direction K: a in [OA, OA + NA), b in
// [OB, OB + NB), k in [0, T_k) relative to the tile origin, stored x fastest
// (consecutive lanes touch consecutive words when they step along x).
template <int K, int NA, int NB, int OA, int OB>
struct CtBox {
    static constexpr int A = (K + 1) % 3, B = (K + 2) % 3;
    static constexpr int TK = CtTile<K>::T[K];
    static constexpr int X[3] = {A == 0 ? NA : (B == 0 ? NB : TK), A == 1 ? NA : (B == 1 ? NB : TK),
                                 A == 2 ? NA : (B == 2 ? NB : TK)};
    static constexpr int O[3] = {A == 0 ? OA : (B == 0 ? OB : 0), A == 1 ? OA : (B == 1 ? OB : 0),
                                 A == 2 ? OA : (B == 2 ? OB : 0)};
    static constexpr int S[3] = {1, X[0], X[0] * X[1]};
    static constexpr int N = NA * NB * TK;
    // index of the point with tile-local coordinates t (x, y, z)
    __device__ static int at(int t0, int t1, int t2)
    {
        return (t0 - O[0]) + S[1] * (t1 - O[1]) + S[2] * (t2 - O[2]);
    }
};

// stage one cell-sized field over a box (coordinates clamped into the padded
// array; clamped points only feed results that are never stored), in two
// halves: ct_load issues a lane's loads unconditionally (lanes past the box
// end load its last point again), ct_store writes them to LDS.  A kernel
// issues the loads of all its boxes before the first store, so a wave keeps
// every load in flight at once.  MAP: the directions (bit d) along which the
// box is widened beyond the tile, where a stage field is read at the point
// the boundary rule gives (the other directions stay inside the evolved
// range; 0 for the metric, read at the point itself).
template <class BX>
struct CtRegs {
    static constexpr int NR = (BX::N + kBlock - 1) / kBlock;
    double v[NR];
};
template <class BX, int MAP>
__device__ __forceinline__ void ct_load(const Geo &G, const double *__restrict__ f, const int org[3], CtRegs<BX> &R)
{
    constexpr int NR = CtRegs<BX>::NR;
    constexpr unsigned X0 = BX::X[0], X1 = BX::X[1];
    const int b[3] = {org[0] + BX::O[0], org[1] + BX::O[1], org[2] + BX::O[2]};
    bool bmap = false;  // the same for the whole block
#pragma unroll
    for (int d = 0; d < 3; d++)
        if (MAP & (1 << d)) bmap |= b[d] < G.g[d] || b[d] + BX::X[d] > G.g[d] + G.n[d];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        unsigned l = threadIdx.x + (unsigned)(r * kBlock);
        if (r == NR - 1 && BX::N % kBlock != 0) l = l < (unsigned)BX::N ? l : (unsigned)BX::N - 1;
        const unsigned e0 = l % X0, q = l / X0, e1 = q % X1, e2 = q / X1;
        int c[3] = {b[0] + (int)e0, b[1] + (int)e1, b[2] + (int)e2};
#pragma unroll
        for (int d = 0; d < 3; d++) {
            c[d] = c[d] < 0 ? 0 : (c[d] > G.N[d] - 1 ? G.N[d] - 1 : c[d]);
            if ((MAP & (1 << d)) && bmap) c[d] = stage_cell(G, d, c[d]);
        }
        R.v[r] = ldb(f, (unsigned)lin(G, c) << 3);
    }
}
template <class BX>
__device__ __forceinline__ void ct_store(const CtRegs<BX> &R, double *dst)
{
#pragma unroll
    for (int r = 0; r < CtRegs<BX>::NR; r++) {
        const int l = (int)threadIdx.x + r * kBlock;
        if (l < BX::N) dst[l] = R.v[r];
    }
}

// Upwind EMF with every input staged in LDS by coalesced loads: E_K over the
// tile widened by the reconstruction halo in a and b, psi and alpha for the
// face and edge metric factors, q_B^a of the a-faces widened along b and q_B^b
// of the b-faces widened along a.  Step 1 reconstructs psi^4 E_K along a to
// the a-faces of the b-widened rows; step 2 reconstructs those along b (LL,
// LR, RL, RR), q_B^a along b and q_B^b along a, and combines them with the
// metric-only speeds.
template <int REC, int MET, int K>
__device__ __forceinline__ void ct_body(const CtArgs &args, Blk blk)
{
    const Geo &G = args.G;
    const Region &R = args.R;
    constexpr int A = (K + 1) % 3, B = (K + 2) % 3;
    constexpr int TA = CtTile<K>::T[A], TB = CtTile<K>::T[B];
    static_assert(CtTile<K>::T[0] * CtTile<K>::T[1] * CtTile<K>::T[2] == kBlock, "one edge per thread");
    using BE = CtBox<K, TA + 5, TB + 5, -3, -3>;  // E_K: a, b in [-3, T + 2)
    using BP = CtBox<K, TA + 1, TB + 5, -1, -3>;  // psi: a in [-1, T_a), b in [-3, T_b + 2)
    using BA = CtBox<K, TA + 1, TB + 1, -1, -1>;  // alpha: a in [-1, T_a), b in [-1, T_b)
    using BQa = CtBox<K, TA, TB + 5, 0, -3>;      // q_B^a and the a-face states of psi^4 E_K
    using BQb = CtBox<K, TA + 5, TB, -3, 0>;      // q_B^b
    __shared__ double sE[BE::N], sP[MET ? BP::N : 1], sAl[MET ? BA::N : 1], sQa[BQa::N], sQb[BQb::N];
    __shared__ double sEL[BQa::N], sER[BQa::N];

    const int org[3] = {R.lo[0] + (int)blk.x * CtTile<K>::T[0], R.lo[1] + (int)blk.y * CtTile<K>::T[1],
                        R.lo[2] + (int)blk.z * CtTile<K>::T[2]};
    constexpr bool actA = true, actB = true;  // the box form runs where both are active
    {
        CtRegs<BE> rE;
        CtRegs<BQa> rQa;
        CtRegs<BQb> rQb;
        CtRegs<BP> rP;
        CtRegs<BA> rA;
        ct_load<BE, (1 << A) | (1 << B)>(G, args.Ek, org, rE);
        ct_load<BQa, 1 << B>(G, args.sf.p[A], org, rQa);
        ct_load<BQb, 1 << A>(G, args.sf.p[B], org, rQb);
        if (MET) {
            ct_load<BP, 0>(G, args.met.p[1], org, rP);
            ct_load<BA, 0>(G, args.met.p[0], org, rA);
        }
        ct_store<BE>(rE, sE);
        ct_store<BQa>(rQa, sQa);
        ct_store<BQb>(rQb, sQb);
        if (MET) {
            ct_store<BP>(rP, sP);
            ct_store<BA>(rA, sAl);
        }
    }
    __syncthreads();

    // ---- step 1: a-face states of psi^4 E_K on the rows b in [-3, T_b + 2)
    for (unsigned l = threadIdx.x; l < (unsigned)BQa::N; l += kBlock) {
        constexpr unsigned Q0 = BQa::X[0], Q1 = BQa::X[1];
        const unsigned q = l / Q0;
        int e[3] = {BQa::O[0] + (int)(l % Q0), BQa::O[1] + (int)(q % Q1),
                    BQa::O[2] + (int)(q / Q1)};  // tile-local face position
        const int e0 = BE::at(e[0], e[1], e[2]);
        double p4 = 1.0;
        if (MET) {
            const int q = BP::at(e[0], e[1], e[2]);  // psi of the cell above the face; below: - S[A]
            const double ps = actA ? 0.5 * (sP[q - BP::S[A]] + sP[q]) : sP[q];
            const double p2 = ps * ps;
            p4 = p2 * p2;
        }
        double L, Rv;
        if (actA) {
            double w[6];
#pragma unroll
            for (int m = 0; m < 6; m++) w[m] = sE[e0 + (m - 3) * BE::S[A]];
            recon_face<REC>(w, L, Rv);
        } else {
            L = Rv = sE[e0];
        }
        sEL[l] = p4 * L;
        sER[l] = p4 * Rv;
    }
    __syncthreads();

    // ---- step 2: this thread's edge
    const int t[3] = {(int)threadIdx.x % CtTile<K>::T[0], ((int)threadIdx.x / CtTile<K>::T[0]) % CtTile<K>::T[1],
                      (int)threadIdx.x / (CtTile<K>::T[0] * CtTile<K>::T[1])};
    int c[3] = {org[0] + t[0], org[1] + t[1], org[2] + t[2]};
    if (c[0] >= R.lo[0] + R.cnt[0] || c[1] >= R.lo[1] + R.cnt[1] || c[2] >= R.lo[2] + R.cnt[2]) return;
    double ELL, ELR, ERL, ERR, qaL, qaR, qbL, qbR;
    const int r0 = BQa::at(t[0], t[1], t[2]);  // a-face row of the edge (b - 1/2 lies below it)
    if (actB) {
        double w[6];
#pragma unroll
        for (int m = 0; m < 6; m++) w[m] = sEL[r0 + (m - 3) * BQa::S[B]];
        recon_face<REC>(w, ELL, ELR);
#pragma unroll
        for (int m = 0; m < 6; m++) w[m] = sER[r0 + (m - 3) * BQa::S[B]];
        recon_face<REC>(w, ERL, ERR);
#pragma unroll
        for (int m = 0; m < 6; m++) w[m] = sQa[r0 + (m - 3) * BQa::S[B]];
        recon_face<REC>(w, qaL, qaR);
    } else {
        ELL = ELR = sEL[r0];
        ERL = ERR = sER[r0];
        qaL = qaR = sQa[r0];
    }
    const int r1 = BQb::at(t[0], t[1], t[2]);  // b-face of the edge
    if (actA) {
        double w[6];
#pragma unroll
        for (int m = 0; m < 6; m++) w[m] = sQb[r1 + (m - 3) * BQb::S[A]];
        recon_face<REC>(w, qbL, qbR);
    } else {
        qbL = qbR = sQb[r1];
    }
    double ca = 1.0, cb = 1.0, ae = 1.0;
    if (MET) {
        // alpha and psi of the cells (a - 1 .. a, b - 1 .. b) around the edge
        const int q11 = BA::at(t[0], t[1], t[2]), p11 = BP::at(t[0], t[1], t[2]);
        const double a11 = sAl[q11], a01 = sAl[q11 - BA::S[A]], a10 = sAl[q11 - BA::S[B]],
                     a00 = sAl[q11 - BA::S[A] - BA::S[B]];
        const double p_11 = sP[p11], p_01 = sP[p11 - BP::S[A]], p_10 = sP[p11 - BP::S[B]],
                     p_00 = sP[p11 - BP::S[A] - BP::S[B]];
        // a-face speeds at rows b - 1 and b, b-face speeds at columns a - 1 and a
        double al0, ps0, al1, ps1;
        al0 = actA ? 0.5 * (a00 + a10) : a10;
        ps0 = actA ? 0.5 * (p_00 + p_10) : p_10;
        al1 = actA ? 0.5 * (a01 + a11) : a11;
        ps1 = actA ? 0.5 * (p_01 + p_11) : p_11;
        if (!actB) {
            al0 = al1;
            ps0 = ps1;
        }
        ca = fmax(al0 * frcp(ps0 * ps0), al1 * frcp(ps1 * ps1));
        al0 = actB ? 0.5 * (a00 + a01) : a01;
        ps0 = actB ? 0.5 * (p_00 + p_01) : p_01;
        al1 = actB ? 0.5 * (a10 + a11) : a11;
        ps1 = actB ? 0.5 * (p_10 + p_11) : p_11;
        if (!actA) {
            al0 = al1;
            ps0 = ps1;
        }
        cb = fmax(al0 * frcp(ps0 * ps0), al1 * frcp(ps1 * ps1));
        double sm = a11;
        int na = 1;
        if (actA) {
            sm += a01;
            na++;
        }
        if (actB) {
            sm += a10;
            na++;
        }
        if (actA && actB) {
            sm += a00;
            na++;
        }
        ae = sm / na;
    }
    const unsigned o = (unsigned)lin(G, c) << 3;
    stb(args.EM, o, ae * 0.25 * (ELL + ELR + ERL + ERR) + 0.5 * ca * (qbR - qbL) - 0.5 * cb * (qaR - qaL));
}

template <int REC, int MET, int K, int F>
__device__ __forceinline__ void ct_dispatch(const CtArgs &a, Blk blk)
{
    if constexpr (F == CT_IDEAL) ct_ideal_body<REC, MET, K>(a, blk);
    else if constexpr (F != CT_BOX || K == 0) ct_body_direct<REC, MET, K, F>(a, blk);
    else ct_body<REC, MET, K>(a, blk);
}
template <int REC, int MET, int K, int F>
__global__ void __launch_bounds__(kBlock) k_ct(CtArgs a)
{
    ct_dispatch<REC, MET, K, F>(a, blk_of(hw_linear<true>(), a.gd));
}
template <int REC, int MET, int K, int F>
__global__ void __launch_bounds__(kBlock) kb_ct(const CtArgs *__restrict__ aa, const unsigned *__restrict__ start, int n)
{
    unsigned lb;
    const CtArgs &a = aa[batch_locate<true>(start, n, lb)];
    ct_dispatch<REC, MET, K, F>(a, blk_of(lb, a.gd));
}

// ---------------------------------------------------------------------------
struct StageArgs {
    int p, s, fin, withL, storeL;
    double dt, aii_dt;
    double cL[4], cR[4];  // weights of L_j and R_j (j < p); final pass: wt, w
    // folded storage (the last implicit pass): the stored L is sum_j fL_j L_j
    // (j < p, the stored ones and the one evaluated here) and the stored R is
    // sum_j fR_j R_j (j <= p), the final combination's part, which then reads
    // one L and one R slot instead of one per stage
    int foldL, foldR;
    double fL[4], fR[4];
};

// CT update of the face fields (eq. ct), all three directions in one pass:
// Lf_d = -(d_{m1} E_{m2} - d_{m2} E_{m1}); stage face = face^n + dt sum_j cL_j Lf_j.
// The region is the interior plus one layer in every active direction; face d
// exists at c when c lies inside the interior in the other two directions.
struct FaceLs {
    const double *Lf[4][3];  // stored face L of stage j, direction d (may be null)
    double *Lst[3];          // where this pass stores its face L (withL)
};
struct FaceArgs {
    Geo G;
    Region R;
    StageArgs A;
    CPtr<3> EM, fn;
    FaceLs Ls;
    Ptr<3> fout;
    // passes with L: the stage E read by this pass, whose ghost layer next to
    // the interior this launch writes (null otherwise)
    Ptr<3> Eg;
    GridDims gd;
};
__device__ __forceinline__ void face_body(const FaceArgs &a, Blk blk)
{
    const Geo &G = a.G;
    const StageArgs &A = a.A;
    const CPtr<3> &EM = a.EM, &fn = a.fn;
    const FaceLs &Ls = a.Ls;
    const Ptr<3> &fout = a.fout;
    int c[3];
    if (!region_point(a.R, blk, c)) return;
    bool in[3];
#pragma unroll
    for (int d = 0; d < 3; d++) in[d] = c[d] < G.g[d] + G.n[d];
    const unsigned o = (unsigned)lin(G, c) << 3;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int m1 = (d + 1) % 3, m2 = (d + 2) % 3;
        if (!in[m1] || !in[m2]) continue;
        double acc = ldb(fn.p[d], o);
        double Lnew = 0.0;
        if (A.withL) {
            double t1 = G.act[m1] ? (ldb(EM.p[m2], o + ((unsigned)G.st[m1] << 3)) - ldb(EM.p[m2], o)) * G.idx[m1] : 0.0;
            double t2 = G.act[m2] ? (ldb(EM.p[m1], o + ((unsigned)G.st[m2] << 3)) - ldb(EM.p[m1], o)) * G.idx[m2] : 0.0;
            Lnew = -(t1 - t2);
        }
        double fold = 0.0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (j >= A.p || A.cL[j] == 0.0) continue;
            const bool fresh = A.withL && j == A.p - 1;
            double l = fresh ? Lnew : ldb(Ls.Lf[j][d], o);
            acc += A.dt * A.cL[j] * l;
            if (A.foldL && !fresh) fold += A.fL[j] * l;
        }
        if (A.storeL) stb(Ls.Lst[d], o, A.foldL ? fold + A.fL[A.p - 1] * Lnew : Lnew);
        stb(fout.p[d], o, acc);
    }
    // The cell pass forms the Gauss-law charge from the stage E of the
    // neighbours of each interior cell, the only reads of a stage field at a
    // ghost point that do not go through the boundary maps (they would keep
    // the cell pass's coordinates in registers through its Newton solve).
    // This launch runs before that cell pass and beside kernels that never
    // read these points: the ghost cell next to the interior along d takes
    // the value the boundary rule gives it (outflow, periodic; a fixed ghost
    // point keeps its value).
    if (a.Eg.p[0]) {
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const int m1 = (d + 1) % 3, m2 = (d + 2) % 3;
            if (!G.act[d] || !in[m1] || !in[m2]) continue;
            const int gp = c[d] == G.g[d] ? G.g[d] - 1 : (c[d] == G.g[d] + G.n[d] ? c[d] : -1);
            if (gp < 0) continue;
            const int src = stage_cell(G, d, gp);
            if (src == gp) continue;
            const unsigned og = o + ((unsigned)((gp - c[d]) * G.st[d]) << 3);
            const unsigned os = o + ((unsigned)((src - c[d]) * G.st[d]) << 3);
#pragma unroll
            for (int i = 0; i < 3; i++) stb(a.Eg.p[i], og, ldb(a.Eg.p[i], os));
        }
    }
}
__global__ void __launch_bounds__(kBlock) k_face_update(FaceArgs a) { face_body(a, blk_of(hw_linear<false>(), a.gd)); }
__global__ void __launch_bounds__(kBlock)
    kb_face_update(const FaceArgs *__restrict__ aa, const unsigned *__restrict__ start, int n)
{
    unsigned lb;
    const FaceArgs &a = aa[batch_locate<false>(start, n, lb)];
    face_body(a, blk_of(lb, a.gd));
}

// ---------------------------------------------------------------------------
// cell pass
// Field counts: 8 cell conserved variables; with GLM also q_B (3, cell
// centred) and q_Psi, q_Phi, i.e. 13 explicit components (L index 8..10 for
// q_B, 11..12 for q_Psi, q_Phi), stage blocks of 10 (prims, E, Psi, Phi).
struct CellIO {
    const double *Lxy[13];    // -(dF_x/dx + dF_y/dy) of stage p-1 (if withL)
    const double *spm[10];    // stage p-1 primitives + E (+ Psi, Phi) (if withL)
    const double *sfm[3];     // stage p-1 faces / GLM cell q_B (if withL)
    const double *Lc[4][13];  // stored cell L of stages j < p
    const double *Rj[4][3];   // stored R of stages j < p
    const double *sfp[3];     // faces of this pass (CT)
    const double *guess[5];   // primitives giving the Newton / recovery guess
    double *q[10];            // state conserved variables (read; written by the final pass)
    double *qB[3];            // GLM: state cell q_B (read; written by the final pass)
    double *sfout[3];         // GLM: stage p cell q_B (not in the final pass)
    double *out[10];          // stage p prims + E (+ Psi, Phi), or state prims (final)
    double *Rout[3];          // R of this stage
    double *Lout[13];         // stored cell L of stage p-1 (if storeL)
    const double *met[2];
    unsigned long long *nfail;
};

template <int MET, bool GLM = false, bool ALLACT = false>
__device__ __forceinline__ double bcc_dev(const Geo &G, const double *const *face, double ip6, unsigned o, int t)
{
    double v = ((ALLACT || G.act[t]) && !GLM) ? 0.5 * (ldb(face[t], o) + ldb(face[t], o + ((unsigned)G.st[t] << 3)))
                                              : ldb(face[t], o);
    return MET ? v * ip6 : v;
}

// cell pass.  SWZ: the z phase of the explicit operator runs first on a
// TX x 1 x TZ tile (one thread per cell), the other variants take one cell per
// thread over the interior.
struct CellArgs {
    Geo G;
    Phys P;
    Region R;
    StageArgs A;
    CellIO io;
    GridDims gd;
    // paired launch (point-wise passes p and p + 1, the PAIR instances):
    // stage p + 1's weights and outputs; stage p's primitives are not stored
    int pair;
    StageArgs A2;
    double *out2[8];
    double *Rout2[3];
};
template <int REC, int MET, int SWZ, int TX, int TZ, bool XI, bool GLM, bool PAIR = false>
__device__ __forceinline__ void cell_body(const CellArgs &args, Blk blk)
{
    const Geo &G = args.G;
    const Phys &P = args.P;
    const Region &R = args.R;
    const StageArgs &A = args.A;
    const CellIO &io = args.io;
    constexpr int NQ = NVar<GLM>::NF;
    // the z-phase instances serve 3-D grids in passes with L: every direction
    // active and L evaluated, known at compile time
    const bool withL = SWZ ? true : (A.withL != 0);
    auto act = [&](int d) { return SWZ ? true : (G.act[d] != 0); };
    int c[3];
    double Lz[NQ];
    if constexpr (SWZ == 1) {
        // the z phase takes the per-cell PPM form (the cell pass is held to
        // three waves per SIMD by its registers, not by this LDS)
        constexpr bool PCZ = REC == GR_PPM;
        __shared__ double lds[PhaseDims<2, TX, 1, TZ, GLM, PCZ>::LDS];
        const int org[3] = {R.lo[0] + (int)blk.x * TX, R.lo[1] + (int)blk.y, R.lo[2] + (int)blk.z * TZ};
        CPtr<10> sp;
        CPtr<3> sf;
        CPtr<2> met;
#pragma unroll
        for (int v = 0; v < 10; v++) sp.p[v] = io.spm[v];
#pragma unroll
        for (int d = 0; d < 3; d++) sf.p[d] = io.sfm[d];
        met.p[0] = io.met[0];
        met.p[1] = io.met[1];
        static_assert(PhaseDims<2, TX, 1, TZ, GLM>::NT == kBlock, "z-phase tile of one block");
        sweep_phase<REC, MET, 2, TX, 1, TZ, GLM, PCZ>(G, P, sp, sf, met, org, lds, Lz);
        if ((int)threadIdx.x >= TX * TZ) return;  // beyond the tile
        c[0] = org[0] + (int)threadIdx.x % TX;
        c[1] = org[1];
        c[2] = org[2] + (int)threadIdx.x / TX;
        if (c[0] >= R.lo[0] + R.cnt[0] || c[2] >= R.lo[2] + R.cnt[2]) return;
    } else {
        if (!region_point(R, blk, c)) return;
    }
    const unsigned o = (unsigned)lin(G, c) << 3;
    double al = 1.0, ps = 1.0;
    if (MET) {
        al = ldb(io.met[0], o);
        ps = ldb(io.met[1], o);
    }
    const double ps2 = ps * ps, ps4 = ps2 * ps2, ps6 = ps4 * ps2;
    const double ips6 = MET ? frcp(ps6) : 1.0, ips2 = MET ? frcp(ps2) : 1.0;
    double Lc[NQ];
    if (withL) {
#pragma unroll
        for (int v = 0; v < NQ; v++) Lc[v] = SWZ ? ldb(io.Lxy[v], o) + Lz[v] : ldb(io.Lxy[v], o);
        double rho = ldb(io.spm[0], o), pr = ldb(io.spm[4], o);
        double u[3] = {ps2 * ldb(io.spm[1], o), ps2 * ldb(io.spm[2], o), ps2 * ldb(io.spm[3], o)};
        double W = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double iW = frcp(W);
        double v[3] = {u[0] * iW, u[1] * iW, u[2] * iW};
        // Gauss-law charge rho_e = div(q_E)/psi^6 (central differences)
        double divqE = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            if (!act(d)) continue;
            unsigned sd = (unsigned)G.st[d] << 3;
            // stage E of the neighbours: the ghost layer next to the interior
            // holds the boundary rule's values (written by this pass's face
            // update; GLM, which has none, maps the neighbours); the metric
            // at the neighbours themselves
            const unsigned op = GLM ? stage_nb(G, c, o, d, 1) : o + sd, om = GLM ? stage_nb(G, c, o, d, -1) : o - sd;
            double qp = ldb(io.spm[5 + d], op), qm = ldb(io.spm[5 + d], om);
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
        if (GLM) {
            // GLM sources (Sec 3.1): -alpha psi^6 gamma^{ij} d_j Psi (q_E) and
            // d_j Phi (q_B), damping and charge of Psi, Phi; the lapse
            // gradient terms follow in the metric block
            const double Psic = ldb(io.spm[8], o), Phic = ldb(io.spm[9], o);
#pragma unroll
            for (int d = 0; d < 3; d++) {
                if (!act(d)) continue;
                const unsigned op = stage_nb(G, c, o, d, 1), om = stage_nb(G, c, o, d, -1);
                double dPsi = (ldb(io.spm[8], op) - ldb(io.spm[8], om)) * (0.5 * G.idx[d]);
                double dPhi = (ldb(io.spm[9], op) - ldb(io.spm[9], om)) * (0.5 * G.idx[d]);
                Lc[5 + d] -= al * ps2 * dPsi;
                Lc[8 + d] -= al * ps2 * dPhi;
            }
            Lc[11] += ps6 * al * (rhoe - P.kappa_E * Psic);
            Lc[12] -= ps6 * al * P.kappa_B * Phic;
        }
        if (MET) {
            double E[3], B[3];
#pragma unroll
            for (int i = 0; i < 3; i++) {
                E[i] = ps2 * ldb(io.spm[5 + i], o);
                B[i] = ps2 * bcc_dev<MET, GLM, SWZ == 1>(G, io.sfm, ips6, o, i);
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
                if (!act(d)) continue;
                unsigned sd = (unsigned)G.st[d] << 3;
                double da = (ldb(io.met[0], o + sd) - ldb(io.met[0], o - sd)) * (0.5 * G.idx[d]);
                double dp = (ldb(io.met[1], o + sd) - ldb(io.met[1], o - sd)) * (0.5 * G.idx[d]);
                // s_S = psi^6 [-(tau + D) d alpha + 2 alpha (d psi / psi) tr Pi]
                Lc[1 + d] += ps6 * (-tauD * da + 2.0 * al * dp * ips * trPi);
                sdt -= S[d] * da;
                if (GLM) {
                    // psi^6 E^i d_i alpha = psi^4 E_on d alpha, likewise for B
                    Lc[11] += ps4 * E[d] * da;
                    Lc[12] += ps4 * B[d] * da;
                }
            }
            // s_tau = -psi^6 S^j d_j alpha = -psi^4 S_on . grad alpha
            Lc[4] += ps4 * sdt;
        }
    }
    // accumulation q* = q^n + dt sum_j (cL_j L_j + cR_j R_j), with the folded
    // sums of the stored L and R where this pass keeps them
    double qs[NQ], Lfold[NQ], Rfold[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < NQ; v++) Lfold[v] = 0.0;
#pragma unroll
    for (int v = 0; v < 8; v++) qs[v] = ldb(io.q[v], o);
    if (GLM) {
#pragma unroll
        for (int i = 0; i < 3; i++) qs[8 + i] = ldb(io.qB[i], o);
        qs[11] = ldb(io.q[8], o);
        qs[12] = ldb(io.q[9], o);
    }
    // the stored R slots this pass reads: loaded before the first is used
    // (the conditions are uniform over the launch); the stored L slots, eight
    // values each, are loaded per stage to bound the live registers
    double rv[4][3];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        if (j < A.p && A.cR[j] != 0.0) {
#pragma unroll
            for (int i = 0; i < 3; i++) rv[j][i] = ldb(io.Rj[j][i], o);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
        if (j >= A.p) continue;
        if (A.cL[j] != 0.0) {
            double w = A.dt * A.cL[j];
            if (withL && j == A.p - 1) {
#pragma unroll
                for (int v = 0; v < NQ; v++) qs[v] += w * Lc[v];
            } else {
#pragma unroll
                for (int v = 0; v < NQ; v++) {
                    const double l = ldb(io.Lc[j][v], o);
                    qs[v] += w * l;
                    if (A.foldL) Lfold[v] += A.fL[j] * l;
                }
            }
        }
        if (A.cR[j] != 0.0) {
            double w = A.dt * A.cR[j];
#pragma unroll
            for (int i = 0; i < 3; i++) {
                qs[5 + i] += w * rv[j][i];
                if (A.foldR) Rfold[i] += A.fR[j] * rv[j][i];
            }
        }
    }
    if (A.storeL) {
        const double wf = A.foldL ? A.fL[A.p - 1] : 1.0;
#pragma unroll
        for (int v8 = 0; v8 < NQ; v8++) stb(io.Lout[v8], o, A.foldL ? Lfold[v8] + wf * Lc[v8] : Lc[v8]);
    }
    // orthonormal frame: B of this pass, D, tau, S, E*
    double B[3];
    if (GLM) {
        // the explicit stage value of the cell-centred q_B; Psi, Phi of the stage
#pragma unroll
        for (int i = 0; i < 3; i++) B[i] = ps2 * qs[8 + i] * ips6;
        if (A.fin) {
#pragma unroll
            for (int i = 0; i < 3; i++) stb(io.qB[i], o, qs[8 + i]);
            stb(io.q[8], o, qs[11]);
            stb(io.q[9], o, qs[12]);
        } else {
#pragma unroll
            for (int i = 0; i < 3; i++) stb(io.sfout[i], o, qs[8 + i]);
            stb(io.out[8], o, qs[11] * ips6);
            stb(io.out[9], o, qs[12] * ips6);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 3; i++) B[i] = ps2 * bcc_dev<MET, false, SWZ == 1>(G, io.sfp, ips6, o, i);
    }
    const double ips8 = ips6 * ips2;
    double D = qs[0] * ips6, tau = qs[4] * ips6;
    double S[3] = {qs[1] * ips8, qs[2] * ips8, qs[3] * ips8};
    double Es[3] = {qs[5] * ips6 * ps2, qs[6] * ips6 * ps2, qs[7] * ips6 * ps2};
    double rho = P.rho_atm, u[3] = {0.0, 0.0, 0.0}, pr = P.p_atm, E[3];
    int status = 0;  // 0 ok, 1 atmosphere, 2 failure
    if (P.frozen && A.fin) {
        // frozen matter: the primitives and q_D, q_S, q_tau stay; only q_E advances
#pragma unroll
        for (int i = 0; i < 3; i++) stb(io.q[5 + i], o, qs[5 + i]);
        return;
    }
    if (P.frozen) {
        // frozen matter: primitives fixed, E from eq. im_E at the fixed u~
        rho = ldb(io.guess[0], o);
        pr = ldb(io.guess[4], o);
        ImpSys sy;
        sy.D = sy.tau = 0.0;
        sy.iG1 = P.iG1;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            sy.S[i] = 0.0;
            sy.Es[i] = Es[i];
            sy.B[i] = B[i];
            u[i] = ps2 * ldb(io.guess[1 + i], o);
        }
        sy.B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
        sy.xi = P.xi;
        const double Wf = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        sy.et = cell_eta(P, rho * Wf) / (al * A.aii_dt);
        ImpEval ev;
        imp_eval<XI>(sy, u, ev);
        stb(io.out[0], o, rho);
#pragma unroll
        for (int i = 0; i < 3; i++) stb(io.out[1 + i], o, u[i] * ips2);
        stb(io.out[4], o, pr);
        const double iadt = 1.0 / A.aii_dt;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            double Ec = ev.E[i] * ips2;
            stb(io.out[5 + i], o, Ec);
            const double Rn = (ps6 * Ec - qs[5 + i]) * iadt;
            stb(io.Rout[i], o, A.foldR ? Rfold[i] + A.fR[A.p] * Rn : Rn);
        }
        return;
    }
    if (!A.fin) {
        const double eta = cell_eta(P, D);
        // one implicit stage (eq. im_E with the velocity Newton solve, Sec
        // 2.4) from E*, the guess u (read from memory when gmem), B and
        // D, S, tau; returns the status and the stage primitives and E
        auto implicit_stage = [&](double aii_dt, const double Es_[3], const double *const *gmem, double u_[3],
                                  double &rho_, double &pr_, double E_[3]) -> int {
            int st = 0;
            if (D <= P.D_atm) {
                st = 1;
            } else {
                ImpSys sy;
                sy.D = D;
                sy.tau = tau;
                sy.iG1 = P.iG1;
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    sy.S[i] = S[i];
                    sy.Es[i] = Es_[i];
                    sy.B[i] = B[i];
                    if (gmem) u_[i] = ps2 * ldb(gmem[1 + i], o);
                }
                sy.B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
                sy.et = eta / (al * aii_dt);
                sy.xi = P.xi;
                ImpEval ev;
                int bad = implicit_solve<XI>(sy, P.tol, P.maxit, u_, ev);
                if (!bad) {
                    rho_ = D * ev.iW;
                    pr_ = (ev.wt * ev.iW - rho_) * P.iG1;
                    if (pr_ < 0.0 && pr_ >= -1e-12 * rho_) pr_ = 0.0;  // cold-gas round-off
                    if (!(pr_ >= 0.0) || !(ev.W <= 1e4) || !(rho_ >= P.rho_atm)) bad = 1;
#pragma unroll
                    for (int i = 0; i < 3; i++) E_[i] = ev.E[i];
                }
                if (bad) st = 2;
            }
            if (st) {
                rho_ = P.rho_atm;
                u_[0] = u_[1] = u_[2] = 0.0;
                pr_ = P.p_atm;
                // exact solution at rest: (1 + et) E = et E* + xi B, as (E* + xi B/et)/(1 + 1/et)
                const double iet = al * aii_dt / eta;
                const double fct = 1.0 / (1.0 + iet);
#pragma unroll
                for (int i = 0; i < 3; i++) E_[i] = (Es_[i] + P.xi * iet * B[i]) * fct;
            }
            return st;
        };
        status = implicit_stage(A.aii_dt, Es, io.guess, u, rho, pr, E);
        static_assert(!PAIR || (SWZ == 0 && !GLM), "paired stages are point-wise, face-centred B");
        constexpr bool pair = PAIR;
        if (!pair) {
            stb(io.out[0], o, rho);
#pragma unroll
            for (int i = 0; i < 3; i++) stb(io.out[1 + i], o, u[i] * ips2);
            stb(io.out[4], o, pr);
        }
        const double iadt = 1.0 / A.aii_dt;
        double Rn[3];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            double Ec = E[i] * ips2;
            if (!pair) stb(io.out[5 + i], o, Ec);
            Rn[i] = (ps6 * Ec - qs[5 + i]) * iadt;  // R = psi^6 (E - E*)/(a_ii dt)
            stb(io.Rout[i], o, A.foldR ? Rfold[i] + A.fR[A.p] * Rn[i] : Rn[i]);
        }
        if constexpr (PAIR) {
            {
                // the next stage in the same launch: its only explicit term is
                // the R just formed (no L, faces of time level n), its guess the
                // primitives of this stage as they would have been stored
                if (status == 2) atomicAdd(io.nfail, 1ull);
                const StageArgs &A2 = args.A2;
                const double w = A2.dt * A2.cR[A.p];
                double Es2[3], u2[3], E2[3], rho2 = P.rho_atm, pr2 = P.p_atm;
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    qs[5 + i] += w * Rn[i];
                    Es2[i] = qs[5 + i] * ips6 * ps2;
                    u2[i] = ps2 * (u[i] * ips2);
                }
                status = implicit_stage(A2.aii_dt, Es2, nullptr, u2, rho2, pr2, E2);
                stb(args.out2[0], o, rho2);
#pragma unroll
                for (int i = 0; i < 3; i++) stb(args.out2[1 + i], o, u2[i] * ips2);
                stb(args.out2[4], o, pr2);
                const double iadt2 = 1.0 / A2.aii_dt;
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    double Ec = E2[i] * ips2;
                    stb(args.out2[5 + i], o, Ec);
                    stb(args.Rout2[i], o, (ps6 * Ec - qs[5 + i]) * iadt2);
                }
            }
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
template <int REC, int MET, int SWZ, int TX, int TZ, bool XI, bool GLM, bool PAIR = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu((SWZ || PAIR) && !XI && !GLM ? 3 : 1)))
    k_cell_update(CellArgs a)
{
    cell_body<REC, MET, SWZ, TX, TZ, XI, GLM, PAIR>(a, blk_of(hw_linear<SWZ != 0>(), a.gd));
}
// the batched form reads its arguments through a pointer; it is held to the
// plain form's 3 waves per SIMD (both take 166 VGPRs for the z-phase instance)
template <int REC, int MET, int SWZ, int TX, int TZ, bool XI, bool GLM, bool PAIR = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu((SWZ || PAIR) && !XI && !GLM ? 3 : 1)))
    kb_cell_update(const CellArgs *__restrict__ aa, const unsigned *__restrict__ start, int n)
{
    unsigned lb;
    const CellArgs &a = aa[batch_locate<SWZ != 0>(start, n, lb)];
    cell_body<REC, MET, SWZ, TX, TZ, XI, GLM, PAIR>(a, blk_of(lb, a.gd));
}

}  // namespace gr
