// common.h -- grid geometry, launch regions and reconstructions shared by the
// gfx950 kernels.  32-bit indices inside one field (a field holds < 2^31
// points), uniform (scalar) field base pointers.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/grmhd.h"

namespace gr {

struct Geo {
    int N[3], g[3], n[3], act[3];
    int st[3];   // index stride per direction: 1, row stride P, P Ny
    int o;       // offset of point (0, 0, 0) from the start of its field
    long fs;     // field stride (doubles) of a field block
    double dx[3], idx[3];
    int bc[3][2];  // boundary rule per direction and side (GR_OUTFLOW, ...)
};

template <int K>
struct Ptr {
    double *p[K];
};
template <int K>
struct CPtr {
    const double *p[K];
};

// a box of points [lo, lo + cnt): 1-D blocks run over the (x, y) plane
// (x fastest, so consecutive lanes touch consecutive addresses) and
// blockIdx.y runs over z
struct Region {
    int lo[3], cnt[3];
};

// Block coordinates.  A kernel body sees its block as Blk inside a grid of
// GridDims.  For a plain launch these are the hardware ids; for a batched
// launch (one 1-D grid over the concatenated block ranges of many runs) the
// body sees the block's position inside its own run's grid.
struct GridDims {
    unsigned x, y, z;
};
struct Blk {
    unsigned x, y, z;
};

// XCD-aware block order.  Workgroups are dealt round-robin to the 8 XCDs
// (dispatch id i runs on XCD i mod 8), each with its own L2.  Renumbering so
// that XCD x receives the contiguous run [x P, (x + 1) P) of logical blocks
// keeps stencil neighbours (adjacent rows, planes and tiles) in one L2.  The
// tail of a grid that does not divide by 8 keeps its order.
constexpr int kXcd = 8;
template <bool XCD>
__device__ __forceinline__ unsigned hw_linear()
{
    unsigned gx = gridDim.x, gy = gridDim.y;
    unsigned L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    if (XCD) {
        unsigned total = gx * gy * gridDim.z;
        unsigned per = total / kXcd;
        if (L < per * kXcd) L = (L % kXcd) * per + L / kXcd;
    }
    return L;
}
__device__ __forceinline__ Blk blk_of(unsigned L, const GridDims &g)
{
    Blk b;
    b.x = L % g.x;
    unsigned r = L / g.x;
    b.y = r % g.y;
    b.z = r / g.y;
    return b;
}
// batched launch: start[r] is the first block of run r (start[n] = total);
// returns the run of this block and its linear index inside that run's grid
template <bool XCD>
__device__ __forceinline__ int batch_locate(const unsigned *__restrict__ start, int n, unsigned &local)
{
    unsigned L = hw_linear<XCD>();
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= L) lo = mid;
        else hi = mid - 1;
    }
    local = L - start[lo];
    return lo;
}

// flat kernels: 1-D blocks run over the (x, y) plane of a region, Blk.y over z
__device__ __forceinline__ bool region_point(const Region &R, const Blk &b, int c[3])
{
    int t = b.x * blockDim.x + threadIdx.x;
    if (t >= R.cnt[0] * R.cnt[1]) return false;
    int y = t / R.cnt[0];
    c[0] = R.lo[0] + (t - y * R.cnt[0]);
    c[1] = R.lo[1] + y;
    c[2] = R.lo[2] + (int)b.y;
    return true;
}

__device__ __forceinline__ int lin(const Geo &G, const int c[3])
{
    return G.o + c[0] + G.st[1] * c[1] + G.st[2] * c[2];
}

// loads / stores at a 32-bit byte offset from a uniform base pointer: the
// address is formed by the memory instruction (scalar base + vector offset)
// instead of a 64-bit vector add per pointer.  Every array these kernels
// touch through them is device global memory; the pointer is taken into the
// global address space explicitly, so that pointers read from memory (the
// batched kernels' argument arrays) give global instead of flat loads and
// stores, as kernel arguments do.
typedef const __attribute__((address_space(1))) char g_cchar;
typedef __attribute__((address_space(1))) char g_char;
__device__ __forceinline__ double ldb(const double *p, unsigned off)
{
    return *(const __attribute__((address_space(1))) double *)((g_cchar *)p + off);
}
__device__ __forceinline__ void stb(double *p, unsigned off, double v)
{
    *(__attribute__((address_space(1))) double *)((g_char *)p + off) = v;
}

// reciprocal: hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r); for the positive, bounded denominators of the
// point-wise solvers (a few ulp, no IEEE special-case handling)
__device__ __forceinline__ double frcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// ---------------------------------------------------------------------------
// reconstruction (Sec 5: minmod, MC, PPM).  Per-cell form: the left and right
// interface values (aL, aR) of cell 0 from its neighbours a[-2..2].
//
// Rounding policy: the limiters and their switch predicates are evaluated
// without contraction (no fused multiply-add), each product and sum rounded
// as written, in the expression order of the plain definition; the one
// deliberate difference is the CW threshold d^2/6, formed as d^2 * (1/6).
// Every switch of these limiters is continuous at its threshold (the value
// on either side agrees there), so a decision that a rounding difference
// moves changes the result by an amount of the order of that difference.
__device__ __forceinline__ double minmod2(double a, double b)
{
#pragma clang fp contract(off)
    if (a * b <= 0.0) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}
__device__ __forceinline__ double minmod3(double a, double b, double c)
{
    if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
    if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
    return 0.0;
}
// Colella-Woodward fourth-order interface value, clipped between neighbours
__device__ __forceinline__ double ppm_iface(double am1, double a0, double a1, double a2)
{
#pragma clang fp contract(off)
    double v = 7.0 / 12.0 * (a0 + a1) - 1.0 / 12.0 * (am1 + a2);
    double lo = fmin(a0, a1), hi = fmax(a0, a1);
    return fmin(fmax(v, lo), hi);
}
// the two CW monotonicity constraints (no steepening, no flattening)
__device__ __forceinline__ void ppm_mono(double a, double &aL, double &aR)
{
#pragma clang fp contract(off)
    if ((aR - a) * (a - aL) <= 0.0) {
        aL = a;
        aR = a;
        return;
    }
    // the two tests are continuous at their thresholds (the modified value
    // equals the unmodified one there), so d^2/6 may be formed as d^2 * (1/6)
    double d = aR - aL, m = a - 0.5 * (aL + aR);
    double d26 = d * d * (1.0 / 6.0);
    if (d * m > d26) aL = 3.0 * a - 2.0 * aR;
    else if (-d26 > d * m) aR = 3.0 * a - 2.0 * aL;
}

template <int REC>
__device__ __forceinline__ void recon_cell(double am2, double am1, double a0, double ap1, double ap2, double &aL,
                                          double &aR)
{
#pragma clang fp contract(off)
    if (REC == GR_MINMOD) {
        double s = minmod2(a0 - am1, ap1 - a0);
        aL = a0 - 0.5 * s;
        aR = a0 + 0.5 * s;
    } else if (REC == GR_MC) {
        double s = minmod3(0.5 * (ap1 - am1), 2.0 * (a0 - am1), 2.0 * (ap1 - a0));
        aL = a0 - 0.5 * s;
        aR = a0 + 0.5 * s;
    } else {
        aL = ppm_iface(am2, am1, a0, ap1);
        aR = ppm_iface(am1, a0, ap1, ap2);
        ppm_mono(a0, aL, aR);
    }
}

// face form: the left state (right value of the cell below) and the right
// state (left value of the cell above) at the face between w[2] and w[3];
// PPM shares the interface value of the face itself between the two cells
template <int REC>
__device__ __forceinline__ void recon_face(const double w[6], double &L, double &R)
{
    if (REC == GR_PPM) {
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
    } else {
        double t;
        recon_cell<REC>(w[0], w[1], w[2], w[3], w[4], t, L);
        recon_cell<REC>(w[1], w[2], w[3], w[4], w[5], R, t);
    }
}

// ---------------------------------------------------------------------------
// boundary rules as index maps: the point whose value a ghost point takes
// (outflow: the nearest interior point; periodic: the image; fixed: itself).
// The stencil kernels read the stage fields (primitives, E, face fields)
// through these maps, so their ghost points need no fill: a read at a ghost
// point goes to the point whose value the rule gives it (fixed ghost points
// hold their initial values, set at initialisation and never written; the
// one layer of stage E next to the interior, which the cell pass's charge
// reads with plain offsets, is written by the face update).  Composing the
// maps of x, y and z gives the values that filling the ghost points along x,
// then y, then z over the full extent of the other directions would give.
// The metric is static and read at the point itself.

// index along d of the cell whose stage value cell m takes (m inside the
// padded box; m itself inside the interior and along an inactive direction)
__device__ __forceinline__ int stage_cell(const Geo &G, int d, int m)
{
    const int g = G.g[d], n = G.n[d];
    if (m < g) {
        const int b = G.bc[d][0];
        return b == GR_OUTFLOW ? g : (b == GR_PERIODIC ? m + n : m);
    }
    if (m >= g + n) {
        const int b = G.bc[d][1];
        return b == GR_OUTFLOW ? g + n - 1 : (b == GR_PERIODIC ? m - n : m);
    }
    return m;
}
// byte offset of the stage value of the neighbour delta = +-1 along d of an
// interior cell c at byte offset o: the neighbour leaves the interior only
// from the first (delta -1) or the last (+1) interior cell, where the rule
// moves it by the same number of cells for every such cell
__device__ __forceinline__ unsigned stage_nb(const Geo &G, const int c[3], unsigned o, int d, int delta)
{
    const int g = G.g[d], n = G.n[d];
    const int edge = delta > 0 ? g + n - 1 : g;  // the cell whose neighbour leaves
    const int step = c[d] == edge ? stage_cell(G, d, edge + delta) - edge : delta;
    return o + ((unsigned)(step * G.st[d]) << 3);
}
// reconstruction along d at the d-face below point c from the stage field a
// (a cell field, or a face field whose normal is not d), the stencil points
// mapped by the boundary rule along d (o: the byte offset of c, whose other
// coordinates are already those of a stage value)
template <int REC>
__device__ __forceinline__ void recon_stage(const double *__restrict__ a, const Geo &G, const int c[3], unsigned o,
                                            int d, double &L, double &R)
{
    const int m = c[d], g = G.g[d], n = G.n[d];
    double w[6];
    if (m - 3 >= g && m + 2 <= g + n - 1) {
        const unsigned sb = (unsigned)G.st[d] << 3;
        w[1] = ldb(a, o - 2 * sb);
        w[2] = ldb(a, o - sb);
        w[3] = ldb(a, o);
        w[4] = ldb(a, o + sb);
        if (REC == GR_PPM) {
            w[0] = ldb(a, o - 3 * sb);
            w[5] = ldb(a, o + 2 * sb);
        }
    } else {
#pragma unroll
        for (int k = (REC == GR_PPM ? 0 : 1); k < (REC == GR_PPM ? 6 : 5); k++) {
            w[k] = ldb(a, o + ((unsigned)((stage_cell(G, d, m + k - 3) - m) * G.st[d]) << 3));
        }
    }
    if (REC != GR_PPM) {
        w[0] = w[1];
        w[5] = w[4];
    }
    recon_face<REC>(w, L, R);
}

}  // namespace gr
