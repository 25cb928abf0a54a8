// grmhd.hip -- host side and C ABI of the gfx950 library for one IMEX-RK step
// of resistive GRMHD on a fixed (Cowling) Cartesian grid (Cheong et al.,
// arXiv:2110.03732).
//
// Pass structure of one step (IMEX tableau with s implicit stages, Sec 2.3):
//   pass p < s : [explicit operator L of stage p-1]
//                -> stage faces -> cell accumulation q* -> fused implicit
//                   E + velocity Newton solve (Sec 2.4)
//   pass p = s : L of stage s-1 -> final combination -> recovery with E, B
//                known (Sec 2.6)
// The explicit operator (Sec 2.1 fluxes and sources, Sec 2.5 speeds, HLL,
// Sec 3.2 upwind constrained transport): the x/y LDS sweeps (reconstruction +
// HLL, flux divergence written), one EMF launch per edge direction, the CT
// face update, and the cell pass that runs the z sweep and the sources before
// the accumulation.  The boundary rules enter as index maps in the stencil
// reads (no ghost-fill launch).  GLM cleaning (Sec 3.1) replaces
// the EMF and face-update launches by three more swept components.  A whole
// step runs two consecutive point-wise passes as one cell launch where the
// tableau allows (IMEX-SSP3: passes 0 and 1).  Device fields have rows padded
// to whole 128-byte lines, the first interior point of a row on a line.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <new>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "../../include/grmhd.h"
#include "aux_kernels.h"
#include "common.h"
#include "physics.h"
#include "step_kernels.h"
#include "mg_kernels.h"

using namespace gr;

namespace {

// ---------------------------------------------------------------------------
// measurement hook: launches of the selected kernel classes are bracketed by
// HIP events on the stream they are launched on, with the algorithmic bytes
// (every live input field read once, every output written once) of the launch.
// While it records, passes do not fork (fork_wanted), so that each class is
// timed alone rather than while it shares the device with another.
enum KClass { KC_SWEEP = 0, KC_CT, KC_FACE_UPDATE, KC_CELL_UPDATE, KC_COUNT };
const char *kClassNames[KC_COUNT] = {"k_xy", "k_ct", "k_face_update", "k_cell_update"};
struct TRec {
    int cls;
    hipEvent_t a, b;
    double bytes;
};
std::mutex g_tmu;
unsigned g_tmask = 0;
std::vector<TRec> g_trecs;
thread_local bool g_capturing = false;  // no event records inside a captured graph

struct TScope {
    int cls;
    hipStream_t s;
    double bytes;
    hipEvent_t a = nullptr;
    TScope(int c, hipStream_t st, double b) : cls(c), s(st), bytes(b)
    {
        if ((g_tmask & (1u << c)) && !g_capturing) {
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
// field layout: 16 doubles = one 128-byte line; fields start 256-byte aligned
int row_stride(int nx) { return (nx + 15) / 16 * 16; }
int field_origin(int ng) { return (16 - ng % 16) % 16; }

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
        G.bc[d][0] = g->bc[d][0];
        G.bc[d][1] = g->bc[d][1];
    }
    // rows padded to whole 128-byte lines and the first interior point of
    // every row on a line boundary: a tile row of 16 cells is one line
    G.st[0] = 1;
    G.st[1] = row_stride(G.N[0]);
    G.st[2] = G.st[1] * G.N[1];
    G.o = field_origin(G.g[0]);
    long np = G.o + (long)G.st[2] * G.N[2];
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
    P.xi = g->xi;
    P.frozen = g->frozen_matter;
    P.kappa_E = g->kappa_E;
    P.kappa_B = g->kappa_B;
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
// must pass p store the L it evaluates (L of stage p-1)?  Only when a later
// pass reads it: the final combination evaluates its own and is the last reader
bool storeL_needed(const Tableau &T, int p)
{
    if (p < 1 || p >= T.s) return false;
    const int j = p - 1;
    if (T.wt[j] != 0.0) return true;
    for (int q = p + 1; q < T.s; q++)
        if (T.At[q][j] != 0.0) return true;
    return false;
}
// Folded storage for the final combination.  The last implicit pass
// pf = s - 1 reads the stored L_j / R_j it needs anyway; where these include
// every term of the final combination but its own, it stores the final
// combination's sum of them (L: slot of L_{pf-1}, R: slot of R_pf), and the
// final pass reads that slot with weight 1 instead of one slot per stage.
// Applied when it saves reads (two or more terms); the sums are the same up to
// rounding order.
bool foldL_applies(const Tableau &T)
{
    const int pf = T.s - 1;
    if (!storeL_needed(T, pf)) return false;
    int terms = 0;
    for (int j = 0; j < pf; j++) {
        if (T.wt[j] == 0.0) continue;
        terms++;
        if (j < pf - 1 && T.At[pf][j] == 0.0) return false;  // pf would need an extra read
    }
    return terms >= 2;
}
bool foldR_applies(const Tableau &T)
{
    const int pf = T.s - 1;
    int terms = 0;
    for (int j = 0; j <= pf; j++) {
        if (T.w[j] == 0.0) continue;
        terms++;
        if (j < pf && T.A[pf][j] == 0.0) return false;
    }
    return terms >= 2;
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
    size_t sprim, sface, L, R, Lxy, EM, MG, total_fields;
    int nsp, nL, nLxy;  // fields per stage block / stored L / x-y divergence
};

// multigrid hierarchy of the divergence cleaning: level 0 is the interior,
// each coarser level halves every active direction while all of them are
// even and stay >= 2.  Returns the number of levels and the doubles needed
// (three compact arrays per level); fills lv when given.
constexpr int kMgMaxLevels = kMgLevelsMax;  // the one-block kernel takes them all
int mg_levels(const gr_grid *g, MgLevel *lv, double *base, size_t *doubles)
{
    int n[3], act[3];
    for (int d = 0; d < 3; d++) {
        act[d] = d < g->ndim;
        n[d] = act[d] ? g->n[d] : 1;
    }
    size_t tot = 0;
    int nl = 0;
    while (nl < kMgMaxLevels) {
        size_t cells = (size_t)n[0] * n[1] * n[2];
        if (lv) {
            MgLevel &L = lv[nl];
            for (int d = 0; d < 3; d++) {
                L.n[d] = n[d];
                L.act[d] = act[d];
                L.per[d] = act[d] && g->bc[d][0] == GR_PERIODIC;
                double h = act[d] ? (g->hi[d] - g->lo[d]) / g->n[d] * (double)(g->n[d] / n[d]) : 1.0;
                L.ih2[d] = act[d] ? 1.0 / (h * h) : 0.0;
            }
            L.phi = base + tot;
            L.rhs = base + tot + cells;
            L.res = base + tot + 2 * cells;
        }
        tot += 3 * cells;
        nl++;
        bool more = true;
        for (int d = 0; d < 3; d++)
            if (act[d] && (n[d] % 2 != 0 || n[d] / 2 < 2)) more = false;
        if (!more) break;
        for (int d = 0; d < 3; d++)
            if (act[d]) n[d] /= 2;
    }
    if (doubles) *doubles = tot;
    return nl;
}

Layout layout(const gr_grid *g)
{
    Tableau T = tableau(g->imex);
    Layout L;
    // GLM: stage blocks also hold Psi, Phi; stored L and the x-y divergence
    // carry q_B (cell centred), q_Psi and q_Phi
    L.nsp = g->glm ? 10 : 8;
    L.nL = g->glm ? 13 : 11;
    L.nLxy = g->glm ? 13 : 8;
    size_t o = 0;
    L.sprim = o;
    o += (size_t)L.nsp * T.s;
    L.sface = o;
    o += 3 * (size_t)T.s;
    L.L = o;
    o += (size_t)L.nL * T.s;
    L.R = o;
    o += 3 * (size_t)T.s;
    L.Lxy = o;
    o += (size_t)L.nLxy;
    L.EM = o;
    o += 3;
    L.MG = o;
    {
        size_t mgd = 0;
        mg_levels(g, nullptr, nullptr, &mgd);
        Geo G = make_geo(g);
        o += (mgd + (size_t)G.fs - 1) / (size_t)G.fs;
    }
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
// Kernel variants: the template instance of each tiled kernel a run uses.
// The x/y phase tile and the z-phase tile of the cell pass are the tunables
// (the batch autotuner picks them per class of runs).
// 32x7 leaves one wavefront's worth of lanes without a cell so that every
// face of the tile has its own thread (one HLL evaluation per thread, no
// second partial round); the z-phase tiles of the cell pass are TX x 1 x TZ.
enum XyTile { XY_32x7 = 0, XY_32x8, XY_64x4, XY_16x16, XY_256x1, XY_128x1, XY_64x1, XY_COUNT };
enum CzTile { CZ_16x16 = 0, CZ_32x8, CZ_COUNT };
const int kXyTX[XY_COUNT] = {32, 32, 64, 16, 256, 128, 64}, kXyTY[XY_COUNT] = {7, 8, 4, 16, 1, 1, 1};
const int kCzTX[CZ_COUNT] = {16, 32}, kCzTZ[CZ_COUNT] = {16, 8};
const char *kXyName[XY_COUNT] = {"32x7", "32x8", "64x4", "16x16", "256x1", "128x1", "64x1"};
const char *kCzName[CZ_COUNT] = {"16x16", "32x8"};

struct Variant {
    int rec, met, xy, cz;
    int xi;   // mean-field dynamo terms compiled into the cell pass
    int glm;  // GLM cleaning (cell-centred B): default tiles only
    int uct;  // 1: ideal-MHD edge EMF
};
// tiles a run may use: two-dimensional x/y tiles when y is active, one-row
// tiles otherwise (the metric 1-D case only the 256-wide one)
bool xy_allowed(const gr_grid *g, int t)
{
    if (g->glm) return t == (g->ndim >= 2 ? XY_32x8 : XY_256x1);
    if (g->ndim >= 2) return t <= XY_16x16;
    if (g->metric) return t == XY_256x1;
    return t >= XY_256x1;
}
Variant default_variant(const gr_grid *g)
{
    Variant V;
    V.rec = g->recon;
    V.met = g->metric ? 1 : 0;
    V.xy = g->ndim >= 2 ? (g->glm ? XY_32x8 : XY_32x7) : XY_256x1;
    V.cz = CZ_16x16;
    V.xi = g->xi != 0.0 ? 1 : 0;
    V.glm = g->glm ? 1 : 0;
    V.uct = g->uct ? 1 : 0;
    return V;
}

template <int V>
using IC = std::integral_constant<int, V>;
template <class F>
void with_rm(int rec, int met, F &&f)
{
    auto m = [&](auto R) {
        if (met) f(R, IC<1>{});
        else f(R, IC<0>{});
    };
    if (rec == GR_MINMOD) m(IC<GR_MINMOD>{});
    else if (rec == GR_MC) m(IC<GR_MC>{});
    else m(IC<GR_PPM>{});
}
template <class F>
void with_xy(int t, F &&f)
{
    switch (t) {
    case XY_32x8: f(IC<32>{}, IC<8>{}); break;
    case XY_64x4: f(IC<64>{}, IC<4>{}); break;
    case XY_16x16: f(IC<16>{}, IC<16>{}); break;
    case XY_32x7: f(IC<32>{}, IC<7>{}); break;
    case XY_256x1: f(IC<256>{}, IC<1>{}); break;
    case XY_128x1: f(IC<128>{}, IC<1>{}); break;
    default: f(IC<64>{}, IC<1>{}); break;
    }
}
template <class F>
void with_cz(int t, F &&f)
{
    if (t == CZ_32x8) f(IC<32>{}, IC<8>{});
    else f(IC<16>{}, IC<16>{});
}
// instances that no allowed variant selects are not compiled
template <int MET, int TX, int TY, bool GLM = false>
constexpr bool xy_compiled()
{
    if (GLM) return (TX == 32 && TY == 8) || (TX == 256 && TY == 1);
    return !(MET == 1 && TY == 1 && TX != 256);
}
template <class F>
void with_flag(int flag, F &&f)
{
    if (flag) f(IC<1>{});
    else f(IC<0>{});
}

const int kCtOrder[3] = {2, 0, 1};

// EMF kernel form of edge direction K: the ideal-MHD form when asked for,
// otherwise one-cell-thick tiles when z (and y) are inactive
int ct_form(const Geo &G, int uct, int K)
{
    if (uct) return CT_IDEAL;
    if (!G.act[1]) return CT_LINE;
    if (!G.act[2] && K != 2) return CT_PLANE;
    return CT_BOX;
}
void ct_tile(int K, int F, int T[3])
{
    auto set = [&](auto KK, auto FF) {
        for (int d = 0; d < 3; d++) T[d] = CtTileF<decltype(KK)::value, decltype(FF)::value>::T[d];
    };
    auto byF = [&](auto KK) {
        if (F == CT_PLANE) set(KK, IC<CT_PLANE>{});
        else if (F == CT_LINE) set(KK, IC<CT_LINE>{});
        else set(KK, IC<CT_BOX>{});
    };
    if (K == 0) byF(IC<0>{});
    else if (K == 1) byF(IC<1>{});
    else byF(IC<2>{});
}
// calls f(IC<K>, IC<F>) for the compiled (edge direction, form) pairs: the
// planar form has no z-edge instance (z-edges of a plane use the box form),
// the line form no x-edge one (a line has no x-edges)
template <class Fn>
void with_ct(int K, int F, Fn &&f)
{
    auto byF = [&](auto KK) {
        constexpr int k = decltype(KK)::value;
        if (F == CT_IDEAL) f(KK, IC<CT_IDEAL>{});
        else if (F == CT_PLANE) {
            if constexpr (k != 2) f(KK, IC<CT_PLANE>{});
        } else if (F == CT_LINE) {
            if constexpr (k != 0) f(KK, IC<CT_LINE>{});
        } else f(KK, IC<CT_BOX>{});
    };
    if (K == 0) byF(IC<0>{});
    else if (K == 1) byF(IC<1>{});
    else byF(IC<2>{});
}

// Everything one pass of one run launches, in launch order: x/y phases, the
// three EMF components, the face update, the cell pass.
// a pass forks its EMF and face-update launches to the side stream only on
// grids of at least kForkCells cells, or kForkCellsGraph cells while its
// stream is being captured.  Eager, the fork and the join are host calls on
// each pass, and on a 512^2 plane (launch-bound) they cost more than the
// overlap gains (8% slower); small grids on several caller streams would also
// all queue on the one side stream.  In a graph they are two dependency
// edges and the plane runs 6% faster with them (768^2: 12%).
constexpr long kForkCells = 1L << 20;
constexpr long kForkCellsGraph = 1L << 18;
bool fork_wanted(long cells, hipStream_t s)
{
    if (g_tmask) return false;
    if (cells >= kForkCells) return true;
    // the legacy null stream is never captured (and asking about it while
    // another thread captures in global mode is an error)
    if (cells < kForkCellsGraph || s == nullptr) return false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return cs == hipStreamCaptureStatusActive;
}

struct PassPlan {
    bool xy = false, face = false;
    long cells = 0;  // interior cells of the grid
    bool swz = false;  // cell pass with the z phase
    bool ct[3] = {false, false, false};
    int ctf[3] = {CT_BOX, CT_BOX, CT_BOX};  // EMF kernel form per launch
    XyArgs xya;
    CtArgs cta[3];
    FaceArgs fa;
    CellArgs ca;
    double xy_bytes = 0, ct_bytes[3] = {0, 0, 0}, fa_bytes = 0, ca_bytes = 0;
};

GridDims flat_dims(const Region &R)
{
    long plane = (long)R.cnt[0] * R.cnt[1];
    GridDims d;
    d.x = (unsigned)((plane + kBlock - 1) / kBlock);
    d.y = (unsigned)R.cnt[2];
    d.z = 1;
    return d;
}
unsigned nblk(const GridDims &d) { return d.x * d.y * d.z; }

gr_status plan_pass(const gr_grid *g, gr_state *st, int p, double dt, const Variant &V, PassPlan &pl)
{
    Geo G = make_geo(g);
    Phys P = make_phys(g);
    Tableau T = tableau(g->imex);
    Layout Ly = layout(g);
    if (p < 0 || p > T.s) return GR_EINVAL;
    pl.cells = (long)G.n[0] * G.n[1] * G.n[2];
    const int MET = V.met;
    const bool fin = (p == T.s);
    const bool withL = (p >= 1) && needL(T, p - 1);
    StageArgs A;
    std::memset(&A, 0, sizeof(A));
    A.p = p;
    A.s = T.s;
    A.fin = fin;
    A.withL = withL;
    A.storeL = withL && storeL_needed(T, p);
    A.dt = dt;
    A.aii_dt = fin ? 0.0 : T.A[p][p] * dt;
    for (int j = 0; j < p && j < 4; j++) {
        A.cL[j] = fin ? T.wt[j] : T.At[p][j];
        A.cR[j] = fin ? T.w[j] : T.A[p][j];
    }
    const bool fL = foldL_applies(T), fR = foldR_applies(T);
    if (p == T.s - 1) {
        A.foldL = fL && A.storeL;
        A.foldR = fR;
        for (int j = 0; j < 4; j++) {
            A.fL[j] = j < p ? T.wt[j] : 0.0;
            A.fR[j] = j <= p ? T.w[j] : 0.0;
        }
    }
    if (fin) {
        if (fL) {
            for (int j = 0; j < T.s - 1; j++) A.cL[j] = 0.0;
            A.cL[T.s - 2] = 1.0;  // the folded sum in the slot of L_{s-2}
        }
        if (fR) {
            for (int j = 0; j < T.s; j++) A.cR[j] = 0.0;
            A.cR[T.s - 1] = 1.0;  // the folded sum in the slot of R_{s-1}
        }
    }
    const bool glm = g->glm != 0;
    // face block of stage j: the state's own faces while no explicit term has
    // entered (CT); GLM keeps a stage q_B block per stage, written by the cell pass
    auto stage_face = [&](int j) -> double * {
        return (faces_are_n(T, j) && !glm) ? st->face : wfield(st, G, Ly.sface + 3 * (size_t)j);
    };
    double *sp_prev = (p >= 1) ? wfield(st, G, Ly.sprim + (size_t)Ly.nsp * (p - 1)) : nullptr;
    double *sf_prev = (p >= 1) ? stage_face(p - 1) : nullptr;
    double *Lxy = wfield(st, G, Ly.Lxy), *EM = wfield(st, G, Ly.EM);
    const double *met = st->metric;
    const double ncell = (double)G.n[0] * G.n[1] * G.n[2];

    if (withL) {
        // x/y phases: reads 8 stage fields, 3 face fields, the metric; writes 8
        pl.xy = true;
        XyArgs &x = pl.xya;
        x.G = G;
        x.P = P;
        x.sp = cptrs<10>(sp_prev, G.fs);
        if (!glm) x.sp.p[8] = x.sp.p[9] = nullptr;
        x.sf = cptrs<3>(sf_prev, G.fs);
        x.met = cptrs<2>(met, G.fs);
        x.Lxy = ptrs<13>(Lxy, G.fs);
        if (!glm)
            for (int v = 8; v < 13; v++) x.Lxy.p[v] = nullptr;
        const int TX = kXyTX[V.xy], TY = kXyTY[V.xy];
        x.gd.x = (G.n[0] + TX - 1) / TX;
        x.gd.y = (G.n[1] + TY - 1) / TY;
        x.gd.z = G.n[2];
        pl.xy_bytes = 8.0 * ncell * (Ly.nsp + 3 + 2 * MET + Ly.nLxy);
        // EMFs: reads E_k, two face fields and the metric per edge; writes one
        // (CT only: GLM evolves the cell-centred B with the other fluxes)
        for (int i = 0; i < 3 && !glm; i++) {
            const int K = kCtOrder[i], a = (K + 1) % 3, b = (K + 2) % 3;
            if (!G.act[a] && !G.act[b]) continue;
            pl.ct[i] = true;
            CtArgs &c = pl.cta[i];
            c.G = G;
            c.R = region(G, (1 << a) | (1 << b));
            c.Ek = sp_prev + (size_t)(5 + K) * G.fs;
            c.u = cptrs<3>(sp_prev + G.fs, G.fs);
            c.sf = cptrs<3>(sf_prev, G.fs);
            c.met = cptrs<2>(met, G.fs);
            c.EM = EM + (size_t)K * G.fs;
            pl.ctf[i] = ct_form(G, g->uct, K);
            int Tt[3];
            ct_tile(K, pl.ctf[i], Tt);
            c.gd.x = (c.R.cnt[0] + Tt[0] - 1) / Tt[0];
            c.gd.y = (c.R.cnt[1] + Tt[1] - 1) / Tt[1];
            c.gd.z = (c.R.cnt[2] + Tt[2] - 1) / Tt[2];
            // ideal-MHD form: u~ (3) instead of E_k
            pl.ct_bytes[i] = 8.0 * rtotal(c.R) * ((g->uct ? 5 : 3) + 2 * MET + 1);
        }
    }
    // faces of this pass
    double *fout = fin ? st->face : stage_face(p);
    int nLst = 0, nRst = 0;
    for (int j = 0; j < p && j < 4; j++) {
        if (A.cL[j] != 0.0 && !(withL && j == p - 1)) nLst++;
        if (A.cR[j] != 0.0) nRst++;
    }
    if ((fin || !faces_are_n(T, p)) && !glm) {
        pl.face = true;
        FaceArgs &f = pl.fa;
        f.G = G;
        f.R = region(G, 7);
        f.A = A;
        f.EM = cptrs<3>(EM, G.fs);
        f.fn = cptrs<3>(st->face, G.fs);
        std::memset(&f.Ls, 0, sizeof(f.Ls));
        for (int d = 0; d < 3; d++) {
            for (int j = 0; j < 4; j++)
                f.Ls.Lf[j][d] = (j < T.s) ? wfield(st, G, Ly.L + 11 * (size_t)j + 8 + d) : nullptr;
            f.Ls.Lst[d] = A.storeL ? wfield(st, G, Ly.L + 11 * (size_t)(p - 1) + 8 + d) : nullptr;
        }
        f.fout = ptrs<3>(fout, G.fs);
        std::memset(&f.Eg, 0, sizeof(f.Eg));
        if (withL)
            for (int i = 0; i < 3; i++) f.Eg.p[i] = sp_prev + (size_t)(5 + i) * G.fs;
        f.gd = flat_dims(f.R);
        double nf = 0.0;
        for (int d = 0; d < 3; d++) nf += (double)rtotal(region(G, 1 << d));
        pl.fa_bytes = 8.0 * (nf * (1 + nLst + 1 + (int)A.storeL) + (withL ? 3.0 * rtotal(f.R) : 0.0));
    }
    // the cell pass's charge reads the ghost layer of the stage E that the face
    // update writes: every pass with L must have one (true of both tableaux)
    if (withL && !glm && !pl.face) return GR_EUNSUPPORTED;
    // cells
    CellArgs &c = pl.ca;
    std::memset(&c, 0, sizeof(c));  // no paired stage unless run_pair sets one
    c.G = G;
    c.P = P;
    c.A = A;
    CellIO &io = c.io;
    std::memset(&io, 0, sizeof(io));
    const int nq = glm ? 13 : 8;  // explicit components
    for (int v = 0; v < nq; v++) io.Lxy[v] = Lxy + (size_t)v * G.fs;
    for (int v = 0; v < Ly.nsp; v++) io.spm[v] = sp_prev ? sp_prev + v * G.fs : nullptr;
    for (int d = 0; d < 3; d++) io.sfm[d] = sf_prev ? sf_prev + d * G.fs : nullptr;
    for (int j = 0; j < T.s; j++) {
        for (int v = 0; v < nq; v++) io.Lc[j][v] = wfield(st, G, Ly.L + (size_t)Ly.nL * j + v);
        for (int i = 0; i < 3; i++) io.Rj[j][i] = wfield(st, G, Ly.R + 3 * (size_t)j + i);
    }
    for (int d = 0; d < 3; d++) io.sfp[d] = fout + d * G.fs;
    const double *guess = (p == 0 || fin) ? st->prim : sp_prev;
    for (int v = 0; v < 5; v++) io.guess[v] = guess + v * G.fs;
    for (int v = 0; v < (glm ? 10 : 8); v++) io.q[v] = st->q + v * G.fs;
    if (glm)
        for (int d = 0; d < 3; d++) {
            io.qB[d] = st->face + d * G.fs;
            io.sfout[d] = fin ? nullptr : stage_face(p) + d * G.fs;
        }
    double *out = fin ? st->prim : wfield(st, G, Ly.sprim + (size_t)Ly.nsp * p);
    for (int v = 0; v < (fin ? 5 : Ly.nsp); v++) io.out[v] = out + v * G.fs;
    if (!fin)
        for (int i = 0; i < 3; i++) io.Rout[i] = wfield(st, G, Ly.R + 3 * (size_t)p + i);
    if (A.storeL)
        for (int v = 0; v < nq; v++) io.Lout[v] = wfield(st, G, Ly.L + (size_t)Ly.nL * (p - 1) + v);
    io.met[0] = met;
    io.met[1] = met ? met + G.fs : nullptr;
    io.nfail = wcounter(st);
    c.R = region(G, 0);
    pl.swz = withL && G.act[2];
    if (pl.swz) {
        const int TX = kCzTX[V.cz], TZ = kCzTZ[V.cz];
        c.gd.x = (c.R.cnt[0] + TX - 1) / TX;
        c.gd.y = c.R.cnt[1];
        c.gd.z = (c.R.cnt[2] + TZ - 1) / TZ;
    } else {
        c.gd = flat_dims(c.R);
    }
    const int ng = glm ? 5 : 0;  // GLM: q_B, q_Psi, q_Phi read and written as well
    double cb = 8 + 3 + 2 * MET + nq * nLst + 3 * nRst + (fin ? 1 : 3) + ng;  // q, faces, metric, L, R, guess
    if (withL) cb += nq + Ly.nsp + 3;                                           // Lxy, stage p-1 block, faces
    cb += fin ? (8 + 5 + ng) : (Ly.nsp + 3 + (glm ? 3 : 0));                    // outputs
    if (A.storeL) cb += nq;                                                     // stored L
    pl.ca_bytes = 8.0 * ncell * cb;
    return GR_OK;
}

dim3 d3(const GridDims &g) { return dim3(g.x, g.y, g.z); }

// ---- plain launches (one run, hardware block ids)
void launch_xy(const Variant &V, const XyArgs &a, hipStream_t s)
{
    with_rm(V.rec, V.met, [&](auto R, auto M) {
        with_flag(V.glm, [&](auto GL) {
            with_xy(V.xy, [&](auto TX, auto TY) {
                constexpr bool gl = decltype(GL)::value != 0;
                if constexpr (xy_compiled<decltype(M)::value, decltype(TX)::value, decltype(TY)::value, gl>())
                    hipLaunchKernelGGL((k_xy<decltype(R)::value, decltype(M)::value, decltype(TX)::value,
                                             decltype(TY)::value, gl>),
                                       d3(a.gd), dim3(tile_threads(decltype(TX)::value * decltype(TY)::value)), 0, s, a);
            });
        });
    });
}
void launch_ct(const Variant &V, int K, int F, const CtArgs &a, hipStream_t s)
{
    with_rm(V.rec, V.met, [&](auto R, auto M) {
        with_ct(K, F, [&](auto KK, auto FF) {
            hipLaunchKernelGGL((k_ct<decltype(R)::value, decltype(M)::value, decltype(KK)::value,
                                     decltype(FF)::value>),
                               d3(a.gd), dim3(kBlock), 0, s, a);
        });
    });
}
// cell-pass instances: the dynamo and GLM are not combined (validated), GLM
// uses the default z-phase tile
template <bool XI, bool GLM, int TX, int TZ>
constexpr bool cell_compiled()
{
    return !(XI && GLM) && !(GLM && !(TX == 16 && TZ == 16) && TX != 1);
}
void launch_cell(const Variant &V, int swz, const CellArgs &a, hipStream_t s)
{
    with_rm(V.rec, V.met, [&](auto R, auto M) {
        constexpr int r = decltype(R)::value, m = decltype(M)::value;
        auto go = [&](auto X, auto GL) {
            constexpr bool x = decltype(X)::value != 0, gl = decltype(GL)::value != 0;
            if (!swz) {
                if constexpr (cell_compiled<x, gl, 1, 1>()) {
                    if constexpr (!gl) {
                        if (a.pair) {
                            hipLaunchKernelGGL((k_cell_update<r, m, 0, 1, 1, x, false, true>), d3(a.gd), dim3(kBlock), 0,
                                               s, a);
                            return;
                        }
                    }
                    hipLaunchKernelGGL((k_cell_update<r, m, 0, 1, 1, x, gl>), d3(a.gd), dim3(kBlock), 0, s, a);
                }
                return;
            }
            with_cz(V.cz, [&](auto TX, auto TZ) {
                constexpr int tx = decltype(TX)::value, tz = decltype(TZ)::value;
                if constexpr (cell_compiled<x, gl, tx, tz>())
                    hipLaunchKernelGGL((k_cell_update<r, m, 1, tx, tz, x, gl>), d3(a.gd), dim3(kBlock), 0, s, a);
            });
        };
        if (V.glm) go(IC<0>{}, IC<1>{});
        else if (V.xi) go(IC<1>{}, IC<0>{});
        else go(IC<0>{}, IC<0>{});
    });
}

// a second stream per device for the edge-EMF and face-update launches of a
// pass, which run beside the x/y sweeps (default priority, created once)
std::mutex g_side_mu;
hipStream_t g_side[64] = {};
gr_status side_stream(hipStream_t *out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return GR_EHIP;
    std::lock_guard<std::mutex> lk(g_side_mu);
    if (!g_side[dev]) HIPCHK(hipStreamCreateWithFlags(&g_side[dev], hipStreamNonBlocking));
    *out = g_side[dev];
    return GR_OK;
}

// fork and join events of the calling host thread on the current device,
// created on first use and kept: a wait refers to the record made just
// before it, so one pair serves every pass (per thread, so that two threads
// forking on one device at once never re-record each other's events)
thread_local hipEvent_t t_fork_ev[64][2] = {};
gr_status fork_events(hipEvent_t *fork, hipEvent_t *join)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return GR_EHIP;
    for (int k = 0; k < 2; k++)
        if (!t_fork_ev[dev][k]) HIPCHK(hipEventCreateWithFlags(&t_fork_ev[dev][k], hipEventDisableTiming));
    *fork = t_fork_ev[dev][0];
    *join = t_fork_ev[dev][1];
    return GR_OK;
}

gr_status launch_plan(const Variant &V, const PassPlan &pl, hipStream_t s)
{
    // The EMFs and the face update depend only on the stage block of the
    // previous pass, the x/y sweeps too: with both present the EMFs and the
    // face update go to the side stream (forked at the start of the pass) and
    // the cell pass waits for them, so the memory-bound face update overlaps
    // the sweeps.
    bool ct_any = pl.face;
    for (int i = 0; i < 3; i++) ct_any |= pl.ct[i] != 0;
    hipStream_t s2 = s;
    hipEvent_t fork = nullptr, join = nullptr;
    if (pl.xy && ct_any && fork_wanted(pl.cells, s)) {
        gr_status e = side_stream(&s2);
        if (e == GR_OK) e = fork_events(&fork, &join);
        if (e != GR_OK) return e;
        HIPCHK(hipEventRecord(fork, s));
        HIPCHK(hipStreamWaitEvent(s2, fork, 0));
    }
    for (int i = 0; i < 3; i++) {
        if (!pl.ct[i]) continue;
        TScope ts(KC_CT, s2, pl.ct_bytes[i]);
        launch_ct(V, kCtOrder[i], pl.ctf[i], pl.cta[i], s2);
        LAUNCHCHK();
    }
    if (pl.face) {
        TScope ts(KC_FACE_UPDATE, s2, pl.fa_bytes);
        hipLaunchKernelGGL(k_face_update, d3(pl.fa.gd), dim3(kBlock), 0, s2, pl.fa);
        LAUNCHCHK();
    }
    if (join) HIPCHK(hipEventRecord(join, s2));
    if (pl.xy) {
        TScope ts(KC_SWEEP, s, pl.xy_bytes);
        launch_xy(V, pl.xya, s);
        LAUNCHCHK();
    }
    if (join) HIPCHK(hipStreamWaitEvent(s, join, 0));
    {
        TScope ts(KC_CELL_UPDATE, s, pl.ca_bytes);
        launch_cell(V, pl.swz, pl.ca, s);
        LAUNCHCHK();
    }
    return GR_OK;
}

gr_status run_pass(const gr_grid *g, gr_state *st, int p, double dt, hipStream_t s)
{
    Variant V = default_variant(g);
    PassPlan pl;
    gr_status r = plan_pass(g, st, p, dt, V, pl);
    if (r != GR_OK) return r;
    return launch_plan(V, pl, s);
}

// Passes 0 and 1 of a whole step can run as one point-wise launch when L of
// stage 0 is never used and stage 1 has no explicit term but a_10 R_0 (its
// faces are those of time level n): IMEX-SSP3(4,3,3).  Stage 0's primitives
// are then kept in registers (they only seed stage 1's Newton guess).  Not
// for GLM (stage q_B blocks), frozen matter, or two implicit stages (pass 1
// would be the last implicit pass, which folds the stored sums).
bool pairable(const gr_grid *g)
{
    const Tableau T = tableau(g->imex);
    if (g->glm || g->frozen_matter || T.s < 3) return false;
    return !needL(T, 0) && faces_are_n(T, 1);
}
// p0: the plan of pass 0; adds pass 1 to its cell launch.  GR_EUNSUPPORTED
// when the two passes are not both point-wise (they then run one by one).
gr_status make_pair(const gr_grid *g, gr_state *st, double dt, const Variant &V, PassPlan &p0)
{
    if (!pairable(g)) return GR_EUNSUPPORTED;
    PassPlan p1;
    gr_status r = plan_pass(g, st, 1, dt, V, p1);
    if (r != GR_OK) return r;
    if (p0.xy || p0.face || p0.swz || p1.xy || p1.face || p1.swz || p1.ca.A.storeL || p1.ca.A.foldR)
        return GR_EUNSUPPORTED;
    CellArgs &c = p0.ca;
    c.pair = 1;
    c.A2 = p1.ca.A;
    for (int v = 0; v < 8; v++) c.out2[v] = p1.ca.io.out[v];
    for (int i = 0; i < 3; i++) c.Rout2[i] = p1.ca.io.Rout[i];
    // q, faces, metric and guess read once; R_0, stage 1 block and R_1 written
    const Geo &G = c.G;
    p0.ca_bytes = 8.0 * G.n[0] * G.n[1] * G.n[2] * (8 + 3 + (g->metric ? 2 : 0) + 3 + 3 + 8 + 3);
    return GR_OK;
}
gr_status run_pair(const gr_grid *g, gr_state *st, double dt, hipStream_t s)
{
    Variant V = default_variant(g);
    PassPlan p0;
    gr_status r = plan_pass(g, st, 0, dt, V, p0);
    if (r != GR_OK) return r;
    r = make_pair(g, st, dt, V, p0);
    if (r != GR_OK) return r;
    return launch_plan(V, p0, s);
}

// ---------------------------------------------------------------------------
// Batches of independent runs.  One step of every run is a fixed list of
// batched launches: for each pass and each kernel class, the runs sharing a
// template instance go into one launch whose 1-D grid concatenates their block
// ranges (a prefix array maps a block to its run and to its position in that
// run's own grid; the per-run kernel arguments sit in a device array).  The
// list is captured once into a HIP graph and replayed per step.
struct BLaunch {
    int cls = 0;
    int K = 0, F = 0;  // EMF launches: edge direction and kernel form
    Variant V{};
    bool swz = false;
    bool pair = false;  // cell launches: the paired passes 0 and 1
    size_t args_off = 0, start_off = 0;  // offsets into the batch's device block
    const void *args = nullptr;
    const unsigned *start = nullptr;
    int n = 0;
    unsigned total = 0;
    double bytes = 0.0;
};

}  // namespace

struct gr_batch {
    std::vector<gr_grid> grids;
    std::vector<gr_state> states;
    std::vector<double> dt;
    std::vector<Variant> var;
    int s = 0;
    std::vector<BLaunch> launches;
    void *dev = nullptr;
    size_t dev_bytes = 0, dev_cap = 0;
    // pinned host staging of the argument block, two buffers used in turn;
    // each event marks the end of the last copy out of its buffer
    void *host[2] = {nullptr, nullptr};
    size_t host_cap[2] = {0, 0};
    hipEvent_t host_ev[2] = {nullptr, nullptr};
    int host_next = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;  // capture stream (the caller's may be the null stream)
    hipStream_t side = nullptr;  // the batch's own stream for the EMF and face-update launches
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;  // its fork and join events
    double bytes_step = 0.0;
    long cells = 0;
};

namespace {

// host staging of the device block: 256-byte aligned pieces
struct Staging {
    std::vector<char> buf;
    size_t put(const void *p, size_t n)
    {
        size_t o = (buf.size() + 255) / 256 * 256;
        buf.resize(o + n);
        std::memcpy(buf.data() + o, p, n);
        return o;
    }
};

template <class A>
void add_group(Staging &stg, std::vector<BLaunch> &out, BLaunch proto, const std::vector<const A *> &args,
               const std::vector<double> &bytes)
{
    if (args.empty()) return;
    std::vector<A> arr;
    std::vector<unsigned> start(1, 0u);
    double by = 0.0;
    for (size_t i = 0; i < args.size(); i++) {
        arr.push_back(*args[i]);
        start.push_back(start.back() + nblk(args[i]->gd));
        by += bytes[i];
    }
    proto.n = (int)args.size();
    proto.total = start.back();
    proto.bytes = by;
    proto.args_off = stg.put(arr.data(), arr.size() * sizeof(A));
    proto.start_off = stg.put(start.data(), start.size() * sizeof(unsigned));
    if (proto.total > 0) out.push_back(proto);
}

// build the launch list of one step (or of one pass p, or only some classes
// when tuning) for the runs selected by `use`
gr_status build_launches(gr_batch *b, int p_only, unsigned cls_mask, const std::vector<char> &use, Staging &stg,
                         std::vector<BLaunch> &out)
{
    const int nr = (int)b->grids.size();
    for (int p = 0; p <= b->s; p++) {
        if (p_only >= 0 && p != p_only) continue;
        std::vector<PassPlan> pl(nr);
        // a whole step pairs passes 0 and 1 of the runs where both are point-wise
        std::vector<char> paired(nr, 0), skip(nr, 0);
        for (int r = 0; r < nr; r++) {
            if (!use[r]) continue;
            gr_status e = plan_pass(&b->grids[r], &b->states[r], p, b->dt[r], b->var[r], pl[r]);
            if (e != GR_OK) return e;
            if (p_only < 0 && p <= 1) {
                PassPlan p0 = pl[r];
                if (p == 1) {
                    e = plan_pass(&b->grids[r], &b->states[r], 0, b->dt[r], b->var[r], p0);
                    if (e != GR_OK) return e;
                }
                e = make_pair(&b->grids[r], &b->states[r], b->dt[r], b->var[r], p0);
                if (e == GR_OK) {
                    if (p == 0) {
                        pl[r] = p0;
                        paired[r] = 1;
                    } else {
                        skip[r] = 1;  // pass 1 ran inside pass 0's cell launch
                    }
                } else if (e != GR_EUNSUPPORTED) {
                    return e;
                }
            }
        }
        // x/y phases, grouped by (recon, metric, tile)
        if (cls_mask & (1u << KC_SWEEP)) {
            for (int rec = 0; rec < 3; rec++)
                for (int met = 0; met < 2; met++)
                    for (int gl = 0; gl < 2; gl++)
                        for (int t = 0; t < XY_COUNT; t++) {
                            std::vector<const XyArgs *> a;
                            std::vector<double> by;
                            for (int r = 0; r < nr; r++) {
                                const Variant &V = b->var[r];
                                if (use[r] && pl[r].xy && V.rec == rec && V.met == met && V.glm == gl && V.xy == t) {
                                    a.push_back(&pl[r].xya);
                                    by.push_back(pl[r].xy_bytes);
                                }
                            }
                            BLaunch L;
                            L.cls = KC_SWEEP;
                            L.V = Variant{rec, met, t, 0, 0, gl};
                            add_group(stg, out, L, a, by);
                        }
        }
        // EMFs, grouped by (component, recon, metric, kernel form)
        if (cls_mask & (1u << KC_CT)) {
            for (int i = 0; i < 3; i++)
                for (int rec = 0; rec < 3; rec++)
                    for (int met = 0; met < 2; met++)
                        for (int f = CT_BOX; f <= CT_LINE; f++) {
                            std::vector<const CtArgs *> a;
                            std::vector<double> by;
                            for (int r = 0; r < nr; r++) {
                                const Variant &V = b->var[r];
                                if (use[r] && pl[r].ct[i] && V.rec == rec && V.met == met && pl[r].ctf[i] == f) {
                                    a.push_back(&pl[r].cta[i]);
                                    by.push_back(pl[r].ct_bytes[i]);
                                }
                            }
                            BLaunch L;
                            L.cls = KC_CT;
                            L.K = kCtOrder[i];
                            L.F = f;
                            L.V = Variant{rec, met, 0, 0, 0, 0, f == CT_IDEAL};
                            add_group(stg, out, L, a, by);
                        }
        }
        // face update
        if (cls_mask & (1u << KC_FACE_UPDATE)) {
            std::vector<const FaceArgs *> a;
            std::vector<double> by;
            for (int r = 0; r < nr; r++)
                if (use[r] && pl[r].face) {
                    a.push_back(&pl[r].fa);
                    by.push_back(pl[r].fa_bytes);
                }
            BLaunch L;
            L.cls = KC_FACE_UPDATE;
            add_group(stg, out, L, a, by);
        }
        // cell pass, grouped by (recon, metric, z phase, tile)
        if (cls_mask & (1u << KC_CELL_UPDATE)) {
            for (int rec = 0; rec < 3; rec++)
                for (int met = 0; met < 2; met++)
                    for (int xg = 0; xg < 3; xg++)  // plain, dynamo, GLM
                        for (int sw = 0; sw < 2; sw++)
                            for (int t = 0; t < (sw ? CZ_COUNT : 1); t++)
                                for (int pr = 0; pr < (sw ? 1 : 2); pr++) {
                                    const int xi = xg == 1, gl = xg == 2;
                                    std::vector<const CellArgs *> a;
                                    std::vector<double> by;
                                    for (int r = 0; r < nr; r++) {
                                        const Variant &V = b->var[r];
                                        if (use[r] && !skip[r] && V.rec == rec && V.met == met && V.xi == xi &&
                                            V.glm == gl && (int)pl[r].swz == sw && (!sw || V.cz == t) &&
                                            paired[r] == pr) {
                                            a.push_back(&pl[r].ca);
                                            by.push_back(pl[r].ca_bytes);
                                        }
                                    }
                                    BLaunch L;
                                    L.cls = KC_CELL_UPDATE;
                                    L.V = Variant{rec, met, 0, t, xi, gl};
                                    L.swz = sw;
                                    L.pair = pr;
                                    add_group(stg, out, L, a, by);
                                }
        }
    }
    return GR_OK;
}

gr_status upload(Staging &stg, std::vector<BLaunch> &ls, void **dev, size_t *bytes, hipStream_t s)
{
    *dev = nullptr;
    *bytes = stg.buf.size();
    if (stg.buf.empty()) return GR_OK;
    HIPCHK(hipMalloc(dev, stg.buf.size()));
    if (hipMemcpyAsync(*dev, stg.buf.data(), stg.buf.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipFree(*dev);
        *dev = nullptr;
        return GR_EHIP;
    }
    for (auto &L : ls) {
        L.args = (const char *)*dev + L.args_off;
        L.start = (const unsigned *)((const char *)*dev + L.start_off);
    }
    return GR_OK;
}

// write the argument block of the batch's launch list into its device
// block, stream-ordered on s: from a pinned staging buffer (the one not used
// by the previous upload, whose copy must have finished before it is reused),
// without a host synchronisation.  The device block grows, with spare room,
// only when the list no longer fits; the old one is freed after the work
// queued on s that may read it.
gr_status upload_batch(gr_batch *b, const Staging &stg, hipStream_t s)
{
    const size_t n = stg.buf.size();
    b->dev_bytes = n;
    if (n == 0) return GR_OK;
    if (n > b->dev_cap) {
        if (b->dev) {
            HIPCHK(hipStreamSynchronize(s));
            (void)hipFree(b->dev);
            b->dev = nullptr;
            b->dev_cap = 0;
        }
        const size_t cap = n + n / 2 + 4096;
        HIPCHK(hipMalloc(&b->dev, cap));
        b->dev_cap = cap;
    }
    const int h = b->host_next;
    b->host_next ^= 1;
    if (b->host_ev[h]) HIPCHK(hipEventSynchronize(b->host_ev[h]));
    else HIPCHK(hipEventCreateWithFlags(&b->host_ev[h], hipEventDisableTiming));
    if (n > b->host_cap[h]) {
        if (b->host[h]) (void)hipHostFree(b->host[h]);
        b->host[h] = nullptr;
        b->host_cap[h] = 0;
        const size_t cap = n + n / 2 + 4096;
        HIPCHK(hipHostMalloc(&b->host[h], cap, hipHostMallocDefault));
        b->host_cap[h] = cap;
    }
    std::memcpy(b->host[h], stg.buf.data(), n);
    HIPCHK(hipMemcpyAsync(b->dev, b->host[h], n, hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(b->host_ev[h], s));
    for (auto &L : b->launches) {
        L.args = (const char *)b->dev + L.args_off;
        L.start = (const unsigned *)((const char *)b->dev + L.start_off);
    }
    return GR_OK;
}

gr_status launch_b(const BLaunch &L, hipStream_t s)
{
    if (L.total == 0) return GR_OK;
    const dim3 grid(L.total);
    switch (L.cls) {
    case KC_SWEEP:
        with_rm(L.V.rec, L.V.met, [&](auto R, auto M) {
            with_flag(L.V.glm, [&](auto GL) {
                with_xy(L.V.xy, [&](auto TX, auto TY) {
                    constexpr bool gl = decltype(GL)::value != 0;
                    if constexpr (xy_compiled<decltype(M)::value, decltype(TX)::value, decltype(TY)::value, gl>())
                        hipLaunchKernelGGL((kb_xy<decltype(R)::value, decltype(M)::value, decltype(TX)::value,
                                                  decltype(TY)::value, gl>),
                                           grid, dim3(tile_threads(decltype(TX)::value * decltype(TY)::value)), 0, s,
                                           (const XyArgs *)L.args, L.start, L.n);
                });
            });
        });
        break;
    case KC_CT:
        with_rm(L.V.rec, L.V.met, [&](auto R, auto M) {
            with_ct(L.K, L.F, [&](auto KK, auto FF) {
                hipLaunchKernelGGL((kb_ct<decltype(R)::value, decltype(M)::value, decltype(KK)::value,
                                          decltype(FF)::value>),
                                   grid, dim3(kBlock), 0, s, (const CtArgs *)L.args, L.start, L.n);
            });
        });
        break;
    case KC_FACE_UPDATE:
        hipLaunchKernelGGL(kb_face_update, grid, dim3(kBlock), 0, s, (const FaceArgs *)L.args, L.start, L.n);
        break;
    default:
        with_rm(L.V.rec, L.V.met, [&](auto R, auto M) {
            constexpr int r = decltype(R)::value, m = decltype(M)::value;
            const CellArgs *a = (const CellArgs *)L.args;
            auto go = [&](auto X, auto GLx) {
                constexpr bool x = decltype(X)::value != 0, gl = decltype(GLx)::value != 0;
                if (!L.swz) {
                    if constexpr (cell_compiled<x, gl, 1, 1>()) {
                        if constexpr (!gl) {
                            if (L.pair) {
                                hipLaunchKernelGGL((kb_cell_update<r, m, 0, 1, 1, x, false, true>), grid, dim3(kBlock),
                                                   0, s, a, L.start, L.n);
                                return;
                            }
                        }
                        hipLaunchKernelGGL((kb_cell_update<r, m, 0, 1, 1, x, gl>), grid, dim3(kBlock), 0, s, a,
                                           L.start, L.n);
                    }
                    return;
                }
                with_cz(L.V.cz, [&](auto TX, auto TZ) {
                    constexpr int tx = decltype(TX)::value, tz = decltype(TZ)::value;
                    if constexpr (cell_compiled<x, gl, tx, tz>())
                        hipLaunchKernelGGL((kb_cell_update<r, m, 1, tx, tz, x, gl>), grid, dim3(kBlock), 0, s, a,
                                           L.start, L.n);
                });
            };
            if (L.V.glm) go(IC<0>{}, IC<1>{});
            else if (L.V.xi) go(IC<1>{}, IC<0>{});
            else go(IC<0>{}, IC<0>{});
        });
        break;
    }
    LAUNCHCHK();
    return GR_OK;
}

// The list holds, per pass, x/y sweeps, EMFs and the face update (which all
// depend only on the stage block of the previous pass), then the cell
// launches.
// With a side stream (a batch of as many cells as fork_wanted asks for), as
// in the plain path, where a pass has both sweeps and EMF / face-update
// launches, the latter go to the side stream, forked at the start of the
// pass, and the cell launches wait for them.  side == nullptr: everything on
// s.
gr_status launch_list(const std::vector<BLaunch> &ls, hipStream_t s, hipStream_t side, hipEvent_t fork_ev,
                      hipEvent_t join_ev)
{
    auto one = [](const BLaunch &L, hipStream_t st) {
        TScope ts(L.cls, st, L.bytes);
        return launch_b(L, st);
    };
    auto on_side = [](int c) { return c == KC_CT || c == KC_FACE_UPDATE; };
    const size_t n = ls.size();
    size_t i = 0;
    while (i < n) {
        if (ls[i].cls != KC_SWEEP && !on_side(ls[i].cls)) {
            gr_status e = one(ls[i++], s);
            if (e != GR_OK) return e;
            continue;
        }
        size_t j = i;
        bool sw = false, sd = false;
        for (; j < n && (ls[j].cls == KC_SWEEP || on_side(ls[j].cls)); j++) {
            sw |= ls[j].cls == KC_SWEEP;
            sd |= on_side(ls[j].cls);
        }
        hipStream_t s2 = s;
        hipEvent_t join = nullptr;
        if (side && sw && sd) {
            s2 = side;
            join = join_ev;
            HIPCHK(hipEventRecord(fork_ev, s));
            HIPCHK(hipStreamWaitEvent(s2, fork_ev, 0));
        }
        gr_status e = GR_OK;
        for (size_t k = i; k < j && e == GR_OK; k++)
            if (on_side(ls[k].cls)) e = one(ls[k], s2);
        if (join) {
            // the join is recorded and waited for even after a failed launch,
            // so the side stream never runs ahead of the launch stream
            const bool ok = hipEventRecord(join, s2) == hipSuccess;
            if (e == GR_OK && !ok) e = GR_EHIP;
        }
        for (size_t k = i; k < j && e == GR_OK; k++)
            if (ls[k].cls == KC_SWEEP) e = one(ls[k], s);
        if (join && hipStreamWaitEvent(s, join, 0) != hipSuccess && e == GR_OK) e = GR_EHIP;
        if (e != GR_OK) return e;
        i = j;
    }
    return GR_OK;
}

void drop_graph(gr_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

gr_status rebuild(gr_batch *b, hipStream_t s)
{
    drop_graph(b);
    b->launches.clear();
    b->bytes_step = 0.0;
    Staging stg;
    std::vector<char> all(b->grids.size(), 1);
    std::vector<BLaunch> ls;
    gr_status e = build_launches(b, -1, ~0u, all, stg, ls);
    if (e != GR_OK) return e;
    b->launches.swap(ls);
    e = upload_batch(b, stg, s);
    if (e != GR_OK) {
        b->launches.clear();
        return e;
    }
    for (const auto &L : b->launches) b->bytes_step += L.bytes;
    return GR_OK;
}

// the runs' interior cells
long batch_cells(const gr_batch *b)
{
    long c = 0;
    for (const auto &g : b->grids) {
        Geo G = make_geo(&g);
        c += (long)G.n[0] * G.n[1] * G.n[2];
    }
    return c;
}

// ---- autotuner.  Runs are classed by (recon, metric, dimensionality); for
// each class the x/y tile (and for 3-D runs the z-phase tile of the cell
// pass) is timed over the batch's own runs of that class and the fastest kept.
// A cache file holds one line per decision: "xy|cz rec met ndim tile".
struct TuneKey {
    int what, rec, met, ndim;
    bool operator==(const TuneKey &o) const
    {
        return what == o.what && rec == o.rec && met == o.met && ndim == o.ndim;
    }
};

double time_list(const std::vector<BLaunch> &ls, hipStream_t s, int reps)
{
    hipEvent_t a, e;
    if (hipEventCreate(&a) != hipSuccess) return -1.0;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1.0;
    }
    double ms = -1.0;
    if (launch_list(ls, s, nullptr, nullptr, nullptr) == GR_OK && hipEventRecord(a, s) == hipSuccess) {
        bool ok = true;
        for (int i = 0; i < reps && ok; i++) ok = launch_list(ls, s, nullptr, nullptr, nullptr) == GR_OK;
        float f = 0.0f;
        if (ok && hipEventRecord(e, s) == hipSuccess && hipEventSynchronize(e) == hipSuccess &&
            hipEventElapsedTime(&f, a, e) == hipSuccess)
            ms = f / reps;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(e);
    return ms;
}

gr_status tune(gr_batch *b, const char *cache, hipStream_t s)
{
    const int nr = (int)b->grids.size();
    std::vector<std::pair<TuneKey, int>> known;
    if (cache && cache[0]) {
        if (FILE *f = std::fopen(cache, "r")) {
            char w[8], t[16];
            int rec, met, nd;
            while (std::fscanf(f, "%7s %d %d %d %15s", w, &rec, &met, &nd, t) == 5) {
                TuneKey k{w[0] == 'x' ? 0 : 1, rec, met, nd};
                int tile = -1;
                for (int i = 0; i < (k.what == 0 ? XY_COUNT : CZ_COUNT); i++)
                    if (!std::strcmp(t, k.what == 0 ? kXyName[i] : kCzName[i])) tile = i;
                if (tile >= 0) known.push_back({k, tile});
            }
            std::fclose(f);
        }
    }
    // the first pass that evaluates the explicit operator
    Tableau T = tableau(b->grids[0].imex);
    int pL = 1;
    while (pL <= T.s && !needL(T, pL - 1)) pL++;
    // the failure counters are restored after the timing launches
    std::vector<unsigned long long> cnt(nr);
    for (int r = 0; r < nr; r++)
        HIPCHK(hipMemcpyAsync(&cnt[r], wcounter(&b->states[r]), sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<std::pair<TuneKey, int>> fresh;
    gr_status status = GR_OK;
    for (int what = 0; what < 2 && status == GR_OK; what++) {
        std::vector<TuneKey> keys;
        for (int r = 0; r < nr; r++) {
            const gr_grid &g = b->grids[r];
            if ((what == 1 && g.ndim < 3) || g.glm) continue;  // GLM runs keep the default tiles
            TuneKey k{what, (int)g.recon, g.metric ? 1 : 0, g.ndim};
            bool seen = false;
            for (auto &q : keys) seen |= q == k;
            if (!seen) keys.push_back(k);
        }
        for (const TuneKey &k : keys) {
            std::vector<char> use(nr, 0);
            for (int r = 0; r < nr; r++) {
                const gr_grid &g = b->grids[r];
                use[r] = ((int)g.recon == k.rec && (g.metric ? 1 : 0) == k.met && g.ndim == k.ndim && !g.glm);
            }
            int r0 = 0;
            while (!use[r0]) r0++;
            int best = -1;
            for (auto &q : known)
                if (q.first == k && (what == 1 || xy_allowed(&b->grids[r0], q.second))) best = q.second;
            if (best < 0) {
                double bms = 1e300;
                const int nc = what == 0 ? XY_COUNT : CZ_COUNT;
                for (int t = 0; t < nc && status == GR_OK; t++) {
                    if (what == 0 && !xy_allowed(&b->grids[r0], t)) continue;
                    for (int r = 0; r < nr; r++)
                        if (use[r]) (what == 0 ? b->var[r].xy : b->var[r].cz) = t;
                    Staging stg;
                    std::vector<BLaunch> ls;
                    status = build_launches(b, pL, what == 0 ? (1u << KC_SWEEP) : (1u << KC_CELL_UPDATE), use, stg,
                                            ls);
                    if (status != GR_OK) break;
                    void *dev = nullptr;
                    size_t nb = 0;
                    status = upload(stg, ls, &dev, &nb, s);
                    if (status != GR_OK) break;
                    double ms = time_list(ls, s, 5);
                    (void)hipFree(dev);
                    if (ms < 0.0) {
                        status = GR_EHIP;
                        break;
                    }
                    if (ms < bms) {
                        bms = ms;
                        best = t;
                    }
                }
                if (best >= 0) fresh.push_back({k, best});
            }
            for (int r = 0; r < nr; r++)
                if (use[r] && best >= 0) (what == 0 ? b->var[r].xy : b->var[r].cz) = best;
        }
    }
    for (int r = 0; r < nr; r++)
        HIPCHK(hipMemcpyAsync(wcounter(&b->states[r]), &cnt[r], sizeof(unsigned long long), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (status == GR_OK && cache && cache[0] && !fresh.empty()) {
        if (FILE *f = std::fopen(cache, "a")) {
            for (auto &q : fresh)
                std::fprintf(f, "%s %d %d %d %s\n", q.first.what == 0 ? "xy" : "cz", q.first.rec, q.first.met,
                             q.first.ndim, q.first.what == 0 ? kXyName[q.second] : kCzName[q.second]);
            std::fclose(f);
        }
    }
    return status;
}

// ---------------------------------------------------------------------------
// measurement hooks: a streaming read and a streaming copy with 16-byte
// loads and stores, four per thread issued before any is used; the practical
// HBM ceiling that the stencil kernels are compared with
constexpr int kStreamPer = 4;
__global__ void __launch_bounds__(kBlock) k_stream_read(const double2 *__restrict__ src, size_t n2, double *sink)
{
    const size_t base = (size_t)blockIdx.x * (kBlock * kStreamPer) + threadIdx.x;
    double2 v[kStreamPer];
#pragma unroll
    for (int k = 0; k < kStreamPer; k++) {
        const size_t i = base + (size_t)k * kBlock;
        v[k] = i < n2 ? src[i] : make_double2(0.0, 0.0);
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kStreamPer; k++) acc += v[k].x + v[k].y;
    if (acc == -1.0e308) sink[0] = acc;  // never for the finite data read here: keeps the loads live
}
__global__ void __launch_bounds__(kBlock) k_stream_copy(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                        size_t n2)
{
    const size_t base = (size_t)blockIdx.x * (kBlock * kStreamPer) + threadIdx.x;
    double2 v[kStreamPer];
#pragma unroll
    for (int k = 0; k < kStreamPer; k++) {
        const size_t i = base + (size_t)k * kBlock;
        if (i < n2) v[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < kStreamPer; k++) {
        const size_t i = base + (size_t)k * kBlock;
        if (i < n2) dst[i] = v[k];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of the allocation-free divergence norm: the reduction partials
// (three per block, at most kMaxParts blocks) in a file-scope device array,
// one copy per GPU the library runs on, held until the process ends.  Host
// code uses only the device address looked up per device (the array's name
// is a host-side stand-in there), never the name itself.
constexpr int kScratchDoubles = 3 * kMaxParts;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device, looked up on the first
// call per device (the library's init call, gr_init_state, does it first)
gr_status scratch_ptr(double **out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return GR_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return GR_EHIP;
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return GR_OK;
}

// the divergence norms (both entry points): partials into `part`, then the
// fixed-order final reduction
gr_status divb_norm_into(const gr_grid *g, const gr_state *st, double *part, double *out3, hipStream_t s)
{
    Geo G = make_geo(g);
    FlatBox B = flatbox(G);
    unsigned nb = nblocks(B.total);
    if (g->glm) {
        hipLaunchKernelGGL(k_divb_cc_partial, dim3(nb), dim3(256), 0, s, G, B, cptrs<3>(st->face, G.fs), part);
    } else {
        hipLaunchKernelGGL(k_divb_partial, dim3(nb), dim3(256), 0, s, G, B, cptrs<3>(st->face, G.fs), part);
    }
    LAUNCHCHK();
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (int)nb, B.total, 0, part, out3);
    LAUNCHCHK();
    return GR_OK;
}
}  // namespace

// ===========================================================================
extern "C" {

gr_status gr_stream_read(const void *src, size_t bytes, double *sink, hipStream_t s)
{
    if (!src || !sink || bytes % 16 || ((uintptr_t)src & 15)) return GR_EINVAL;
    const size_t n2 = bytes / 16;
    if (n2 == 0) return GR_OK;
    const size_t nb = (n2 + kBlock * kStreamPer - 1) / (kBlock * kStreamPer);
    if (nb > 0x7fffffffu) return GR_EINVAL;
    hipLaunchKernelGGL(k_stream_read, dim3((unsigned)nb), dim3(kBlock), 0, s, (const double2 *)src, n2, sink);
    LAUNCHCHK();
    return GR_OK;
}

gr_status gr_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    if (!src || !dst || bytes % 16 || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return GR_EINVAL;
    const size_t n2 = bytes / 16;
    if (n2 == 0) return GR_OK;
    const size_t nb = (n2 + kBlock * kStreamPer - 1) / (kBlock * kStreamPer);
    if (nb > 0x7fffffffu) return GR_EINVAL;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)nb), dim3(kBlock), 0, s, (const double2 *)src, (double2 *)dst,
                       n2);
    LAUNCHCHK();
    return GR_OK;
}

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
    if (!std::isfinite(g->xi)) return GR_EINVAL;
    if (g->frozen_matter != 0 && g->frozen_matter != 1) return GR_EINVAL;
    if (g->glm != 0 && g->glm != 1) return GR_EINVAL;
    if (g->glm && (!(g->kappa_E >= 0.0) || !(g->kappa_B >= 0.0))) return GR_EINVAL;
    if (g->glm && g->xi != 0.0) return GR_EUNSUPPORTED;  // GLM with the dynamo term: not built
    if (g->uct != 0 && g->uct != 1) return GR_EINVAL;
    if (g->glm && g->uct) return GR_EUNSUPPORTED;  // GLM has no edge EMF
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
    double cells = row_stride(g->n[0] + 2 * g->ng);  // padded rows
    for (int d = 1; d < 3; d++) cells *= (d < g->ndim) ? (g->n[d] + 2.0 * g->ng) : 1.0;
    cells += field_origin(g->ng);
    if (cells > 5.0e8) return GR_EINVAL;  // byte offsets inside a field stay below 2^32
    if (g->ndim == 3 && g->n[2] + 2 * g->ng > 65535) return GR_EINVAL;
    return GR_OK;
}

size_t gr_field_stride(const gr_grid *g)
{
    if (gr_validate(g) != GR_OK) return 0;
    return (size_t)make_geo(g).fs;
}

size_t gr_row_stride(const gr_grid *g)
{
    if (gr_validate(g) != GR_OK) return 0;
    return (size_t)make_geo(g).st[1];
}

size_t gr_field_origin(const gr_grid *g)
{
    if (gr_validate(g) != GR_OK) return 0;
    return (size_t)make_geo(g).o;
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
    case 0: if (field < 0 || field >= L.nsp) return GR_EINVAL; f = L.sprim + (size_t)L.nsp * stage + field; break;
    case 1: if (field < 0 || field >= 3) return GR_EINVAL; f = L.sface + 3 * (size_t)stage + field; break;
    case 2: if (field < 0 || field >= L.nL) return GR_EINVAL; f = L.L + (size_t)L.nL * stage + field; break;
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
    double *scr = nullptr;
    v = scratch_ptr(&scr);  // set-up of the allocation-free entry point on this device
    if (v != GR_OK) return v;
    hipStream_t side = nullptr;
    v = side_stream(&side);  // created here, so that a step under graph capture never creates it
    if (v != GR_OK) return v;
    Geo G = make_geo(g);
    Phys P = make_phys(g);
    Tableau T = tableau(g->imex);
    Layout Ly = layout(g);
    long np = (long)G.N[0] * G.N[1] * G.N[2];
    size_t cb = (size_t)np * sizeof(double);
    Region Rall = region(G, 0, 7);
    dim3 gr, bl;
    launch_dims(Rall, gr, bl);
    double *staging = wfield(st, G, Ly.L);  // the stored-L block (>= 22 fields) is free before the first step
    // host fields are compact: one contiguous copy into staging, then spread
    // into the padded rows of the device layout
    auto put = [&](double *field, const double *host) -> gr_status {
        HIPCHK(hipMemcpyAsync(staging, host, cb, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_unpack, gr, bl, 0, s, G, staging, field);
        LAUNCHCHK();
        return GR_OK;
    };
    HIPCHK(hipMemsetAsync(st->work, 0, kHeader, s));
    gr_status e;
    for (int v5 = 0; v5 < 5; v5++)
        if ((e = put(st->prim + v5 * G.fs, prim_host + (size_t)v5 * np)) != GR_OK) return e;
    if (g->metric)
        for (int v2 = 0; v2 < 2; v2++)
            if ((e = put(st->metric + v2 * G.fs, metric_host + (size_t)v2 * np)) != GR_OK) return e;
    // E staged in the first stage block, then q_E = psi^6 E
    double *sp0 = wfield(st, G, Ly.sprim);
    for (int i = 0; i < 3; i++)
        if ((e = put(sp0 + i * G.fs, E_host + (size_t)i * np)) != GR_OK) return e;
    hipLaunchKernelGGL(k_init_qE, gr, bl, 0, s, G, g->metric, cptrs<3>(sp0, G.fs), cptrs<2>(st->metric, G.fs),
                       ptrs<8>(st->q, G.fs));
    LAUNCHCHK();
    // faces from the vector potential (+ added face field)
    int Ne0 = G.N[0] + (G.act[0] ? 1 : 0), Ne1 = G.N[1] + (G.act[1] ? 1 : 0), Ne2 = G.N[2] + (G.act[2] ? 1 : 0);
    long es = (long)Ne0 * Ne1 * Ne2;
    double *Ad = nullptr, *fd = nullptr;
    if (A_host) {
        if ((size_t)3 * es > (size_t)12 * G.fs) return GR_EINVAL;
        Ad = staging;
        HIPCHK(hipMemcpyAsync(Ad, A_host, 3 * es * sizeof(double), hipMemcpyHostToDevice, s));
    }
    if (face_host) {
        fd = staging + (size_t)12 * G.fs;
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
    if (g->glm) {
        // cell-centred q_B from the faces; q_Psi = q_Phi = 0
        HIPCHK(hipMemcpyAsync(staging, st->face, 3 * G.fs * sizeof(double), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_face_to_cell, gr, bl, 0, s, G, cptrs<3>(staging, G.fs), ptrs<3>(st->face, G.fs));
        LAUNCHCHK();
        HIPCHK(hipMemsetAsync(st->q + 8 * G.fs, 0, 2 * G.fs * sizeof(double), s));
    }
    // every stage block starts as a copy of the state (ghost points of fixed
    // boundaries keep these values: no kernel writes them)
    for (int j = 0; j < T.s; j++) {
        double *spj = wfield(st, G, Ly.sprim + (size_t)Ly.nsp * j);
        hipLaunchKernelGGL(k_stage_copy, gr, bl, 0, s, G, g->metric, cptrs<5>(st->prim, G.fs), cptrs<8>(st->q, G.fs),
                           cptrs<2>(st->metric, G.fs), ptrs<8>(spj, G.fs));
        LAUNCHCHK();
        if (g->glm) HIPCHK(hipMemsetAsync(spj + 8 * G.fs, 0, 2 * G.fs * sizeof(double), s));  // Psi, Phi
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
    return run_pass(g, st, p, dt, s);
}

gr_status gr_step(const gr_grid *g, gr_state *st, double dt, hipStream_t s)
{
    gr_status v = gr_validate(g);
    if (v != GR_OK) return v;
    v = check_state(g, st);
    if (v != GR_OK) return v;
    if (!(dt > 0.0)) return GR_EINVAL;
    int ns = tableau(g->imex).s;
    int p0 = 0;
    if (pairable(g)) {
        v = run_pair(g, st, dt, s);
        if (v == GR_OK) p0 = 2;
        else if (v != GR_EUNSUPPORTED) return v;
    }
    for (int p = p0; p <= ns; p++) {
        v = run_pass(g, st, p, dt, s);
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
    for (int v8 = 0; v8 < (g->glm ? 10 : 8); v8++) io.q[v8] = st->q + v8 * G.fs;
    if (g->glm)
        for (int d = 0; d < 3; d++) io.qB[d] = st->face + d * G.fs;
    for (int v5 = 0; v5 < 5; v5++) io.out[v5] = st->prim + v5 * G.fs;
    io.met[0] = st->metric;
    io.met[1] = st->metric ? st->metric + G.fs : nullptr;
    io.nfail = wcounter(st);
    CellArgs ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.G = G;
    ca.P = P;
    ca.R = region(G, 0);
    ca.A = A;
    ca.io = io;
    ca.gd = flat_dims(ca.R);
    if (g->glm) {
        if (g->metric)
            hipLaunchKernelGGL((k_cell_update<GR_MINMOD, 1, 0, 1, 1, false, true>), d3(ca.gd), dim3(kBlock), 0, s, ca);
        else
            hipLaunchKernelGGL((k_cell_update<GR_MINMOD, 0, 0, 1, 1, false, true>), d3(ca.gd), dim3(kBlock), 0, s, ca);
    } else if (g->metric) {
        hipLaunchKernelGGL((k_cell_update<GR_MINMOD, 1, 0, 1, 1, false, false>), d3(ca.gd), dim3(kBlock), 0, s, ca);
    } else {
        hipLaunchKernelGGL((k_cell_update<GR_MINMOD, 0, 0, 1, 1, false, false>), d3(ca.gd), dim3(kBlock), 0, s, ca);
    }
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
    return divb_norm_into(g, st, wparts(st), out3, s);
}

gr_status gr_divB_norm_noalloc(const gr_grid *g, const gr_state *st, double *out3, hipStream_t s)
{
    gr_status v = gr_validate(g);
    if (v != GR_OK) return v;
    if (!st || !st->face || !out3) return GR_EINVAL;  // only the face fields are read; work may be NULL
    const Geo G = make_geo(g);
    if (3 * (long)nblocks(flatbox(G).total) > kScratchDoubles) return GR_ENOMEM;  // partials beyond the array
    double *part = nullptr;
    v = scratch_ptr(&part);
    if (v != GR_OK) return v;
    return divb_norm_into(g, st, part, out3, s);
}

gr_status gr_clean_divB(const gr_grid *g, gr_state *st, int vcycles, double *out6, hipStream_t s)
{
    gr_status v = gr_validate(g);
    if (v != GR_OK) return v;
    v = check_state(g, st);
    if (v != GR_OK) return v;
    if (vcycles < 0 || vcycles > 1000) return GR_EINVAL;
    if (g->glm) return GR_EUNSUPPORTED;  // the projection acts on face fields
    Geo G = make_geo(g);
    Layout Ly = layout(g);
    MgLevel lv[kMgMaxLevels];
    const int nl = mg_levels(g, lv, wfield(st, G, Ly.MG), nullptr);
    if (out6) {
        v = gr_divB_norm(g, st, out6, s);
        if (v != GR_OK) return v;
    }
    auto blocks = [](const MgLevel &L) {
        long t = (long)L.n[0] * L.n[1] * L.n[2];
        return dim3((unsigned)((t + 255) / 256));
    };
    hipLaunchKernelGGL(k_mg_div, blocks(lv[0]), dim3(256), 0, s, G, cptrs<3>(st->face, G.fs), lv[0]);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_mg_zero, blocks(lv[0]), dim3(256), 0, s, lv[0]);
    LAUNCHCHK();
    // coarsest level: Gauss-Seidel sweeps in proportion to its size
    int nmax = 1;
    for (int d = 0; d < 3; d++) nmax = lv[nl - 1].n[d] > nmax ? lv[nl - 1].n[d] : nmax;
    const int coarse_sweeps = nmax * nmax > 512 ? 512 : (nmax * nmax < 4 ? 4 : nmax * nmax);
    auto smooth = [&](const MgLevel &L, int sweeps) -> gr_status {
        const bool half = L.act[0] && L.n[0] % 2 == 0;  // one thread per cell of the color
        const long cells = (long)L.n[0] * L.n[1] * L.n[2];
        const dim3 hb((unsigned)((cells / 2 + 255) / 256));
        for (int i = 0; i < sweeps; i++)
            for (int col = 0; col < 2; col++) {
                if (half) hipLaunchKernelGGL(k_mg_smooth_color, hb, dim3(256), 0, s, L, col);
                else hipLaunchKernelGGL(k_mg_smooth, blocks(L), dim3(256), 0, s, L, col);
                LAUNCHCHK();
            }
        return GR_OK;
    };
    // levels from ls on are small enough for one workgroup: that part of
    // each V-cycle is one launch (k_mg_small_cycle) instead of a launch per
    // stage; the arithmetic and its order are the same
    int ls = nl;
    long small = 0;
    while (ls > 0) {
        const long c = (long)lv[ls - 1].n[0] * lv[ls - 1].n[1] * lv[ls - 1].n[2];
        if (c > kMgOneBlockCells || small + c > kMgSmallCells) break;
        small += c;
        ls--;
    }
    MgStack stk;
    for (int l = 0, off = 0; l < nl; l++) {
        stk.lv[l] = lv[l];
        stk.sh_off[l] = l >= ls ? off : 0;
        if (l >= ls) off += 2 * lv[l].n[0] * lv[l].n[1] * lv[l].n[2];
    }
    for (int cyc = 0; cyc < vcycles; cyc++) {
        for (int l = 0; l < ls && l < nl - 1; l++) {
            if ((v = smooth(lv[l], 2)) != GR_OK) return v;
            hipLaunchKernelGGL(k_mg_restrict, blocks(lv[l + 1]), dim3(256), 0, s, lv[l], lv[l + 1]);
            LAUNCHCHK();
        }
        if (ls < nl) {
            hipLaunchKernelGGL(k_mg_small_cycle, dim3(1), dim3(kMgBlockThreads), 0, s, stk, ls, nl, coarse_sweeps);
            LAUNCHCHK();
        } else if ((v = smooth(lv[nl - 1], coarse_sweeps)) != GR_OK) {
            return v;
        }
        for (int l = (ls < nl ? ls : nl - 1) - 1; l >= 0; l--) {
            hipLaunchKernelGGL(k_mg_prolong, blocks(lv[l]), dim3(256), 0, s, lv[l + 1], lv[l]);
            LAUNCHCHK();
            if ((v = smooth(lv[l], 2)) != GR_OK) return v;
        }
    }
    Region R = region(G, 7);
    dim3 gr, bl;
    launch_dims(R, gr, bl);
    hipLaunchKernelGGL(k_mg_apply, gr, bl, 0, s, G, lv[0], ptrs<3>(st->face, G.fs), R);
    LAUNCHCHK();
    if (out6) return gr_divB_norm(g, st, out6 + 3, s);
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

// ---------------------------------------------------------------------------
gr_status gr_batch_create(gr_batch **out, const gr_grid *grids, const gr_state *states, const double *dt, int nruns,
                          const char *tune_cache, hipStream_t s)
{
    if (!out || !grids || !states || !dt || nruns < 1) return GR_EINVAL;
    *out = nullptr;
    for (int r = 0; r < nruns; r++) {
        gr_status v = gr_validate(&grids[r]);
        if (v != GR_OK) return v;
        v = check_state(&grids[r], &states[r]);
        if (v != GR_OK) return v;
        if (!(dt[r] > 0.0)) return GR_EINVAL;
        if (grids[r].imex != grids[0].imex) return GR_EUNSUPPORTED;
    }
    gr_batch *b = new (std::nothrow) gr_batch;
    if (!b) return GR_ENOMEM;
    if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess) {
        b->side = nullptr;
        delete b;
        return GR_EHIP;
    }
    if (hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join_ev, hipEventDisableTiming) != hipSuccess) {
        gr_batch_destroy(b);
        return GR_EHIP;
    }
    b->grids.assign(grids, grids + nruns);
    b->states.assign(states, states + nruns);
    b->dt.assign(dt, dt + nruns);
    b->s = tableau(grids[0].imex).s;
    for (int r = 0; r < nruns; r++) b->var.push_back(default_variant(&grids[r]));
    b->cells = batch_cells(b);
    gr_status e = GR_OK;
    if (tune_cache) e = tune(b, tune_cache, s);
    if (e == GR_OK) e = rebuild(b, s);
    if (e == GR_OK && hipStreamSynchronize(s) != hipSuccess) e = GR_EHIP;
    if (e != GR_OK) {
        gr_batch_destroy(b);
        return e;
    }
    *out = b;
    return GR_OK;
}

gr_status gr_batch_set_dt(gr_batch *b, const double *dt, hipStream_t s)
{
    if (!b || !dt) return GR_EINVAL;
    for (size_t r = 0; r < b->dt.size(); r++)
        if (!(dt[r] > 0.0)) return GR_EINVAL;
    b->dt.assign(dt, dt + b->dt.size());
    return rebuild(b, s);  // the block is rewritten after the work already queued on s
}

gr_status gr_batch_update(gr_batch *b, const gr_grid *grids, const gr_state *states, const double *dt, int nruns,
                          hipStream_t s)
{
    if (!b || !grids || !states || !dt || nruns < 1 || b->grids.empty()) return GR_EINVAL;
    for (int r = 0; r < nruns; r++) {
        gr_status v = gr_validate(&grids[r]);
        if (v != GR_OK) return v;
        v = check_state(&grids[r], &states[r]);
        if (v != GR_OK) return v;
        if (!(dt[r] > 0.0)) return GR_EINVAL;
        if (grids[r].imex != b->grids[0].imex) return GR_EUNSUPPORTED;
    }
    // runs of a class the batch already holds keep that class's tiles
    std::vector<Variant> var;
    for (int r = 0; r < nruns; r++) {
        const gr_grid &g = grids[r];
        Variant V = default_variant(&g);
        for (size_t o = 0; o < b->grids.size() && !g.glm; o++) {
            const gr_grid &h = b->grids[o];
            if (!h.glm && h.recon == g.recon && (h.metric ? 1 : 0) == (g.metric ? 1 : 0) && h.ndim == g.ndim) {
                V.xy = b->var[o].xy;
                V.cz = b->var[o].cz;
                break;
            }
        }
        var.push_back(V);
    }
    b->grids.assign(grids, grids + nruns);
    b->states.assign(states, states + nruns);
    b->dt.assign(dt, dt + nruns);
    b->var.swap(var);
    b->cells = batch_cells(b);
    return rebuild(b, s);
}

gr_status gr_batch_step(gr_batch *b, hipStream_t s)
{
    if (!b) return GR_EINVAL;
    return launch_list(b->launches, s, fork_wanted(b->cells, s) ? b->side : nullptr, b->fork_ev, b->join_ev);
}

gr_status gr_batch_run(gr_batch *b, int nsteps, hipStream_t s)
{
    if (!b || nsteps < 0) return GR_EINVAL;
    if (!b->exec) {
        if (!b->cap) HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        g_capturing = true;
        hipError_t c = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        gr_status e = GR_OK;
        if (c == hipSuccess) {
            e = launch_list(b->launches, b->cap, b->cells >= kForkCellsGraph ? b->side : nullptr, b->fork_ev,
                            b->join_ev);
            c = hipStreamEndCapture(b->cap, &b->graph);
        }
        g_capturing = false;
        if (c != hipSuccess || e != GR_OK) {
            drop_graph(b);
            return GR_EHIP;
        }
        if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(b);
            return GR_EHIP;
        }
    }
    for (int i = 0; i < nsteps; i++) HIPCHK(hipGraphLaunch(b->exec, s));
    return GR_OK;
}

gr_status gr_batch_stats(const gr_batch *b, int *launches_per_step, double *alg_bytes_per_step, long *cells)
{
    if (!b) return GR_EINVAL;
    if (launches_per_step) *launches_per_step = (int)b->launches.size();
    if (alg_bytes_per_step) *alg_bytes_per_step = b->bytes_step;
    if (cells) *cells = b->cells;
    return GR_OK;
}

gr_status gr_batch_tiles(const gr_batch *b, int run, int *xy_tile, int *cz_tile)
{
    if (!b || run < 0 || run >= (int)b->var.size() || !xy_tile || !cz_tile) return GR_EINVAL;
    *xy_tile = b->var[run].xy;
    *cz_tile = b->var[run].cz;
    return GR_OK;
}

const char *gr_tile_name(int which, int tile)
{
    if (which == 0 && tile >= 0 && tile < XY_COUNT) return kXyName[tile];
    if (which == 1 && tile >= 0 && tile < CZ_COUNT) return kCzName[tile];
    return "";
}

gr_status gr_batch_destroy(gr_batch *b)
{
    if (!b) return GR_OK;
    drop_graph(b);
    if (b->side) (void)hipStreamSynchronize(b->side);  // its launches read the argument block
    if (b->dev) (void)hipFree(b->dev);
    for (int h = 0; h < 2; h++) {
        if (b->host_ev[h]) {
            (void)hipEventSynchronize(b->host_ev[h]);
            (void)hipEventDestroy(b->host_ev[h]);
        }
        if (b->host[h]) (void)hipHostFree(b->host[h]);
    }
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    if (b->join_ev) (void)hipEventDestroy(b->join_ev);
    delete b;
    return GR_OK;
}

}  // extern "C"
