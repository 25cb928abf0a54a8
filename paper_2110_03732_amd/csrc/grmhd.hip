// grmhd.hip -- host side and C ABI of the gfx950 library for one IMEX-RK step
// of resistive GRMHD on a fixed (Cowling) Cartesian grid (Cheong et al.,
// arXiv:2110.03732).
//
// Pass structure of one step (IMEX tableau with s implicit stages, Sec 2.3):
//   pass p < s : [ghost fill + explicit operator L of stage p-1]
//                -> stage faces -> cell accumulation q* -> fused implicit
//                   E + velocity Newton solve (Sec 2.4)
//   pass p = s : L of stage s-1 -> final combination -> recovery with E, B
//                known (Sec 2.6)
// The explicit operator (Sec 2.1 fluxes and sources, Sec 2.5 speeds, HLL,
// Sec 3.2 upwind constrained transport): one ghost-fill launch, one LDS sweep
// per direction (reconstruction + HLL -> face fluxes), a-face electric field
// states, edge EMFs, the CT face update and the cell pass.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/grmhd.h"
#include "aux_kernels.h"
#include "common.h"
#include "physics.h"
#include "step_kernels.h"

using namespace gr;

namespace {

// ---------------------------------------------------------------------------
// measurement hook: launches of the selected kernel classes are bracketed by
// HIP events on the stream they are launched on, with the algorithmic bytes
// (every live input field read once, every output written once) of the launch
enum KClass { KC_SWEEP = 0, KC_CT, KC_FACE_UPDATE, KC_CELL_UPDATE, KC_GHOST, KC_COUNT };
const char *kClassNames[KC_COUNT] = {"k_xy", "k_ct", "k_face_update", "k_cell_update", "k_ghost_all"};
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
            if (hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
            else a = nullptr;
        }
    }
    ~TScope()
    {
        if (!a) return;
        hipEvent_t b;
        if (hipEventCreate(&b) != hipSuccess) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_tmu);
        g_trecs.push_back({cls, a, b, bytes});
    }
};

// ---------------------------------------------------------------------------
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
    G.st[2] = G.N[0] * G.N[1];
    long np = (long)G.N[0] * G.N[1] * G.N[2];
    G.fs = (np + 31) / 32 * 32;
    return G;
}

Phys make_phys(const gr_grid *g)
{
    Phys P;
    P.gam = g->gamma_ad;
    P.G1 = g->gamma_ad / (g->gamma_ad - 1.0);
    P.iG1 = (g->gamma_ad - 1.0) / g->gamma_ad;
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

// is L of stage j used by a later stage or by the final combination?
bool needL(const Tableau &T, int j)
{
    if (T.wt[j] != 0.0) return true;
    for (int m = j + 1; m < T.s; m++)
        if (T.At[m][j] != 0.0) return true;
    return false;
}
// are the faces of stage p those of time level n (no explicit term yet)?
bool faces_are_n(const Tableau &T, int p)
{
    for (int j = 0; j < p; j++)
        if (T.At[p][j] != 0.0) return false;
    return true;
}

// workspace layout (in fields of fs doubles, after a 1 MiB header)
constexpr size_t kHeader = 1 << 20;  // failure counter + reduction partials
constexpr int kMaxParts = 4096;

struct Layout {
    size_t sprim, sface, L, R, Lxy, EM, total_fields;
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
    L.Lxy = o;
    o += 8;
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

template <int K>
Ptr<K> ptrs(double *base, long fs)
{
    Ptr<K> r;
    for (int i = 0; i < K; i++) r.p[i] = base ? base + i * fs : nullptr;
    return r;
}
template <int K>
CPtr<K> cptrs(const double *base, long fs)
{
    CPtr<K> r;
    for (int i = 0; i < K; i++) r.p[i] = base ? base + i * fs : nullptr;
    return r;
}

// region of points: interior, plus one point in the directions of extra_mask,
// and the full padded extent in the directions of full_mask
Region region(const Geo &G, int extra_mask, int full_mask = 0)
{
    Region R;
    for (int d = 0; d < 3; d++) {
        if (full_mask & (1 << d)) {
            R.lo[d] = 0;
            R.cnt[d] = G.N[d];
        } else {
            R.lo[d] = G.g[d];
            R.cnt[d] = G.n[d] + (((extra_mask >> d) & 1) && G.act[d] ? 1 : 0);
        }
    }
    return R;
}
long rtotal(const Region &R) { return (long)R.cnt[0] * R.cnt[1] * R.cnt[2]; }

void launch_dims(const Region &R, dim3 &grid, dim3 &block)
{
    block = dim3(256, 1, 1);
    long plane = (long)R.cnt[0] * R.cnt[1];
    grid = dim3((unsigned)((plane + 255) / 256), R.cnt[2], 1);
}

FlatBox flatbox(const Geo &G)
{
    FlatBox B;
    B.total = 1;
    for (int d = 0; d < 3; d++) {
        B.lo[d] = G.g[d];
        B.cnt[d] = G.n[d];
        B.total *= B.cnt[d];
    }
    return B;
}

unsigned nblocks(long total)
{
    long b = (total + 255) / 256;
    if (b < 1) b = 1;
    if (b > kMaxParts) b = kMaxParts;
    return (unsigned)b;
}

#define HIPCHK(x)                                     \
    do {                                              \
        if ((x) != hipSuccess) return GR_EHIP;         \
    } while (0)
#define LAUNCHCHK()                                          \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return GR_EHIP; \
    } while (0)

gr_status check_state(const gr_grid *g, const gr_state *st)
{
    if (!st || !st->q || !st->face || !st->prim || !st->work) return GR_EINVAL;
    if (g->metric && !st->metric) return GR_EINVAL;
    if (st->work_bytes < gr_workspace_bytes(g)) return GR_ENOMEM;
    return GR_OK;
}

// ---------------------------------------------------------------------------
gr_status ghost_fill(const gr_grid *g, const Geo &G, double *cells, double *faces, hipStream_t s)
{
    BcArgs B;
    bool any = false;
    for (int d = 0; d < 3; d++)
        for (int e = 0; e < 2; e++) {
            B.bc[d][e] = g->bc[d][e];
            if (G.act[d] && g->bc[d][e] != GR_FIXED) any = true;
        }
    if (!any) return GR_OK;
    Region R = region(G, 0, 7);
    long shell = rtotal(R) - (long)G.n[0] * G.n[1] * G.n[2];
    TScope ts(KC_GHOST, s, 8.0 * shell * 11 * 2);
    dim3 gr, bl;
    launch_dims(R, gr, bl);
    hipLaunchKernelGGL(k_ghost_all, gr, bl, 0, s, G, B, R, ptrs<8>(cells, G.fs), ptrs<3>(faces, G.fs));
    LAUNCHCHK();
    return GR_OK;
}

// x (and y) phases of the explicit operator; 1-D grids take a one-row tile
template <int REC, int MET>
gr_status launch_xy(const Geo &G, const Phys &P, const double *sp, const double *sf, const double *met, double *Lxy,
                    hipStream_t s)
{
    // reads: 8 stage fields, 3 face fields and the metric per cell; writes 8
    TScope ts(KC_SWEEP, s, 8.0 * G.n[0] * G.n[1] * G.n[2] * (8 + 3 + 2 * MET + 8));
    if (G.act[1]) {
        constexpr int TX = 32, TY = 8;
        dim3 grid((G.n[0] + TX - 1) / TX, (G.n[1] + TY - 1) / TY, G.n[2]);
        hipLaunchKernelGGL((k_xy<REC, MET, TX, TY>), grid, dim3(TX * TY), 0, s, G, P, cptrs<8>(sp, G.fs),
                           cptrs<3>(sf, G.fs), cptrs<2>(met, G.fs), ptrs<8>(Lxy, G.fs));
    } else {
        constexpr int TX = 256, TY = 1;
        dim3 grid((G.n[0] + TX - 1) / TX, G.n[1], G.n[2]);
        hipLaunchKernelGGL((k_xy<REC, MET, TX, TY>), grid, dim3(TX * TY), 0, s, G, P, cptrs<8>(sp, G.fs),
                           cptrs<3>(sf, G.fs), cptrs<2>(met, G.fs), ptrs<8>(Lxy, G.fs));
    }
    LAUNCHCHK();
    return GR_OK;
}

// edge EMFs of direction K on the edges of the interior plus one layer in a and b
template <int REC, int MET, int K>
gr_status launch_ct(const Geo &G, const double *met, const double *sp, const double *sf, double *EM, hipStream_t s)
{
    constexpr int a = (K + 1) % 3, b = (K + 2) % 3;
    if (!G.act[a] && !G.act[b]) return GR_OK;
    Region Re = region(G, (1 << a) | (1 << b));
    const int *T = CtTile<K>::T;
    dim3 grid((Re.cnt[0] + T[0] - 1) / T[0], (Re.cnt[1] + T[1] - 1) / T[1], (Re.cnt[2] + T[2] - 1) / T[2]);
    // reads E_k, q_B^a, q_B^b and the metric per edge point; writes one EMF
    TScope ts(KC_CT, s, 8.0 * rtotal(Re) * (3 + 2 * MET + 1));
    hipLaunchKernelGGL((k_ct<REC, MET, K>), grid, dim3(kBlock), 0, s, G, Re, sp + (5 + K) * G.fs, cptrs<3>(sf, G.fs),
                       cptrs<2>(met, G.fs), EM + (size_t)K * G.fs);
    LAUNCHCHK();
    return GR_OK;
}

template <int REC, int MET>
gr_status launch_L(const Geo &G, const Phys &P, const double *met, const double *sp, const double *sf, double *Lxy,
                   double *EM, hipStream_t s)
{
    gr_status r;
    if ((r = launch_xy<REC, MET>(G, P, sp, sf, met, Lxy, s)) != GR_OK) return r;
    if ((r = launch_ct<REC, MET, 2>(G, met, sp, sf, EM, s)) != GR_OK) return r;
    if ((r = launch_ct<REC, MET, 0>(G, met, sp, sf, EM, s)) != GR_OK) return r;
    if ((r = launch_ct<REC, MET, 1>(G, met, sp, sf, EM, s)) != GR_OK) return r;
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
    const bool fin = (p == T.s);
    const bool withL = (p >= 1) && needL(T, p - 1);
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
    // face block of stage j: the state's own faces while no explicit term has entered
    auto stage_face = [&](int j) -> double * {
        return faces_are_n(T, j) ? st->face : wfield(st, G, Ly.sface + 3 * (size_t)j);
    };
    double *sp_prev = (p >= 1) ? wfield(st, G, Ly.sprim + 8 * (size_t)(p - 1)) : nullptr;
    double *sf_prev = (p >= 1) ? stage_face(p - 1) : nullptr;
    double *Lxy = wfield(st, G, Ly.Lxy), *EM = wfield(st, G, Ly.EM);
    const double *met = st->metric;
    if (withL) {
        gr_status r = ghost_fill(g, G, sp_prev, sf_prev, s);
        if (r != GR_OK) return r;
        r = launch_L<REC, MET>(G, P, met, sp_prev, sf_prev, Lxy, EM, s);
        if (r != GR_OK) return r;
    }
    // faces of this pass
    double *fout = fin ? st->face : stage_face(p);
    int nLst = 0, nRst = 0;
    for (int j = 0; j < p && j < 4; j++) {
        if (A.cL[j] != 0.0 && !(withL && j == p - 1)) nLst++;
        if (A.cR[j] != 0.0) nRst++;
    }
    if (fin || !faces_are_n(T, p)) {
        Region R = region(G, 7);
        FaceLs Ls;
        std::memset(&Ls, 0, sizeof(Ls));
        for (int d = 0; d < 3; d++) {
            for (int j = 0; j < 4; j++)
                Ls.Lf[j][d] = (j < T.s) ? wfield(st, G, Ly.L + 11 * (size_t)j + 8 + d) : nullptr;
            Ls.Lst[d] = withL ? wfield(st, G, Ly.L + 11 * (size_t)(p - 1) + 8 + d) : nullptr;
        }
        double nf = 0.0;
        for (int d = 0; d < 3; d++) nf += (double)rtotal(region(G, 1 << d));
        TScope ts(KC_FACE_UPDATE, s, 8.0 * (nf * (1 + nLst + 1 + (int)withL) + (withL ? 3.0 * rtotal(R) : 0.0)));
        dim3 gr, bl;
        launch_dims(R, gr, bl);
        hipLaunchKernelGGL(k_face_update, gr, bl, 0, s, G, R, A, cptrs<3>(EM, G.fs), cptrs<3>(st->face, G.fs), Ls,
                           ptrs<3>(fout, G.fs));
        LAUNCHCHK();
    }
    // cells
    CellIO io;
    std::memset(&io, 0, sizeof(io));
    for (int v = 0; v < 8; v++) io.Lxy[v] = Lxy + (size_t)v * G.fs;
    for (int v = 0; v < 8; v++) io.spm[v] = sp_prev ? sp_prev + v * G.fs : nullptr;
    for (int d = 0; d < 3; d++) io.sfm[d] = sf_prev ? sf_prev + d * G.fs : nullptr;
    for (int j = 0; j < T.s; j++) {
        for (int v = 0; v < 8; v++) io.Lc[j][v] = wfield(st, G, Ly.L + 11 * (size_t)j + v);
        for (int i = 0; i < 3; i++) io.Rj[j][i] = wfield(st, G, Ly.R + 3 * (size_t)j + i);
    }
    for (int d = 0; d < 3; d++) io.sfp[d] = fout + d * G.fs;
    const double *guess = (p == 0 || fin) ? st->prim : sp_prev;
    for (int v = 0; v < 5; v++) io.guess[v] = guess + v * G.fs;
    for (int v = 0; v < 8; v++) io.q[v] = st->q + v * G.fs;
    double *out = fin ? st->prim : wfield(st, G, Ly.sprim + 8 * (size_t)p);
    for (int v = 0; v < (fin ? 5 : 8); v++) io.out[v] = out + v * G.fs;
    if (!fin)
        for (int i = 0; i < 3; i++) io.Rout[i] = wfield(st, G, Ly.R + 3 * (size_t)p + i);
    if (withL)
        for (int v = 0; v < 8; v++) io.Lout[v] = wfield(st, G, Ly.L + 11 * (size_t)(p - 1) + v);
    io.met[0] = met;
    io.met[1] = met ? met + G.fs : nullptr;
    io.nfail = wcounter(st);
    Region Rc = region(G, 0);
    double cb = 8 + 3 + 2 * MET + 8 * nLst + 3 * nRst + (fin ? 1 : 3);  // q, faces, metric, L, R, guess
    if (withL) cb += 8 + 8 + 3;                                          // Lxy, stage p-1 prims/E, faces
    cb += fin ? (8 + 5) : (8 + 3);                                       // outputs
    if (withL) cb += 8;                                                  // stored L
    TScope ts(KC_CELL_UPDATE, s, 8.0 * rtotal(Rc) * cb);
    if (withL && G.act[2]) {
        constexpr int TX = 16, TZ = 16;
        dim3 grid((Rc.cnt[0] + TX - 1) / TX, Rc.cnt[1], (Rc.cnt[2] + TZ - 1) / TZ);
        hipLaunchKernelGGL((k_cell_update<REC, MET, 1, TX, TZ>), grid, dim3(kBlock), 0, s, G, P, Rc, A, io);
    } else {
        dim3 gr, bl;
        launch_dims(Rc, gr, bl);
        hipLaunchKernelGGL((k_cell_update<REC, MET, 0, 1, 1>), gr, bl, 0, s, G, P, Rc, A, io);
    }
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
    // PPM reads 3 cells beyond a face, minmod and MC 2
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
    // 32-bit indices inside a field; the z extent is a launch-grid dimension
    double cells = 1.0;
    for (int d = 0; d < 3; d++) cells *= (d < g->ndim) ? (g->n[d] + 2.0 * g->ng) : 1.0;
    if (cells > 5.0e8) return GR_EINVAL;  // byte offsets inside a field stay below 2^32
    if (g->ndim == 3 && g->n[2] + 2 * g->ng > 65535) return GR_EINVAL;
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
    Region Rall = region(G, 0, 7);
    dim3 gr, bl;
    launch_dims(Rall, gr, bl);
    hipLaunchKernelGGL(k_init_qE, gr, bl, 0, s, G, g->metric, cptrs<3>(sp0, G.fs), cptrs<2>(st->metric, G.fs),
                       ptrs<8>(st->q, G.fs));
    LAUNCHCHK();
    // faces from the vector potential (+ added face field)
    int Ne0 = G.N[0] + (G.act[0] ? 1 : 0), Ne1 = G.N[1] + (G.act[1] ? 1 : 0), Ne2 = G.N[2] + (G.act[2] ? 1 : 0);
    long es = (long)Ne0 * Ne1 * Ne2;
    double *Ad = nullptr, *fd = nullptr;
    double *scratch = wfield(st, G, Ly.L);  // the stored-L block (>= 22 fields) is free before the first step
    if (A_host) {
        if ((size_t)3 * es > (size_t)12 * G.fs) return GR_EINVAL;
        Ad = scratch;
        HIPCHK(hipMemcpyAsync(Ad, A_host, 3 * es * sizeof(double), hipMemcpyHostToDevice, s));
    }
    if (face_host) {
        fd = scratch + (size_t)12 * G.fs;
        HIPCHK(hipMemcpyAsync(fd, face_host, 3 * cb, hipMemcpyHostToDevice, s));
    }
    hipLaunchKernelGGL(k_curlA, gr, bl, 0, s, G, Ne0, Ne1, Ad, es, fd, np, ptrs<3>(st->face, G.fs));
    LAUNCHCHK();
    Region Rc = region(G, 0);
    dim3 grc, blc;
    launch_dims(Rc, grc, blc);
    if (g->metric)
        hipLaunchKernelGGL(k_init_cons<1>, grc, blc, 0, s, G, P, Rc, cptrs<5>(st->prim, G.fs), cptrs<3>(sp0, G.fs),
                           cptrs<3>(st->face, G.fs), cptrs<2>(st->metric, G.fs), ptrs<8>(st->q, G.fs));
    else
        hipLaunchKernelGGL(k_init_cons<0>, grc, blc, 0, s, G, P, Rc, cptrs<5>(st->prim, G.fs), cptrs<3>(sp0, G.fs),
                           cptrs<3>(st->face, G.fs), cptrs<2>(st->metric, G.fs), ptrs<8>(st->q, G.fs));
    LAUNCHCHK();
    // every stage block starts as a copy of the state (ghost points of fixed
    // boundaries keep these values)
    for (int j = 0; j < T.s; j++) {
        double *spj = wfield(st, G, Ly.sprim + 8 * (size_t)j);
        hipLaunchKernelGGL(k_stage_copy, gr, bl, 0, s, G, g->metric, cptrs<5>(st->prim, G.fs), cptrs<8>(st->q, G.fs),
                           cptrs<2>(st->metric, G.fs), ptrs<8>(spj, G.fs));
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
    CellIO io;
    std::memset(&io, 0, sizeof(io));
    for (int d = 0; d < 3; d++) io.sfp[d] = st->face + d * G.fs;
    for (int v5 = 0; v5 < 5; v5++) io.guess[v5] = st->prim + v5 * G.fs;
    for (int v8 = 0; v8 < 8; v8++) io.q[v8] = st->q + v8 * G.fs;
    for (int v5 = 0; v5 < 5; v5++) io.out[v5] = st->prim + v5 * G.fs;
    io.met[0] = st->metric;
    io.met[1] = st->metric ? st->metric + G.fs : nullptr;
    io.nfail = wcounter(st);
    Region Rc = region(G, 0);
    dim3 gr, bl;
    launch_dims(Rc, gr, bl);
    if (g->metric) hipLaunchKernelGGL((k_cell_update<GR_MINMOD, 1, 0, 1, 1>), gr, bl, 0, s, G, P, Rc, A, io);
    else hipLaunchKernelGGL((k_cell_update<GR_MINMOD, 0, 0, 1, 1>), gr, bl, 0, s, G, P, Rc, A, io);
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
    FlatBox B = flatbox(G);
    unsigned nb = nblocks(B.total);
    double *part = wparts(st);
    hipLaunchKernelGGL(k_divb_partial, dim3(nb), dim3(256), 0, s, G, B, cptrs<3>(st->face, G.fs), part);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (int)nb, B.total, 0, part, out3);
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
    FlatBox B = flatbox(G);
    unsigned nb = nblocks(B.total);
    double *part = wparts(st);
    double *res = part + 3 * kMaxParts;
    if (g->metric)
        hipLaunchKernelGGL(k_cfl_partial<1>, dim3(nb), dim3(256), 0, s, G, B, cptrs<2>(st->metric, G.fs), part);
    else
        hipLaunchKernelGGL(k_cfl_partial<0>, dim3(nb), dim3(256), 0, s, G, B, cptrs<2>(st->metric, G.fs), part);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (int)nb, B.total, 1, part, res);
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
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
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
    if (kernel_class < 0 || kernel_class >= KC_COUNT) return "";
    return kClassNames[kernel_class];
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
