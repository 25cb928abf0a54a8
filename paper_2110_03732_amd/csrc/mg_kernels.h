// mg_kernels.h -- elliptic divergence cleaning of the face fields (Sec 3.3,
// eq. poisson and eq. update_bfield) by a cell-centred geometric multigrid
// V-cycle: L Phi = div q_B on the interior cells, then q_B^d -= dPhi/dx_d on
// every d-face.  L is the 3/5/7-point Laplacian consistent with the face
// divergence and the face gradient; outside the domain Phi is the periodic
// image or minus the boundary cell's value (Phi = 0 on the boundary face).
// Level arrays are compact (no ghost points), x fastest.
#pragma once
#include "common.h"

namespace gr {

struct MgLevel {
    int n[3];        // cells per direction (1 when inactive)
    int act[3];      // active direction
    int per[3];      // periodic direction
    double ih2[3];   // 1/dx^2 (active directions)
    double *phi, *rhs, *res;
};

__device__ __forceinline__ int mg_lin(const MgLevel &L, int i, int j, int k) { return i + L.n[0] * (j + L.n[1] * k); }

// one thread per cell of a level (32-bit: a level holds < 2^31 cells)
__device__ __forceinline__ bool mg_point(const MgLevel &L, int c[3])
{
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned n0 = (unsigned)L.n[0], n1 = (unsigned)L.n[1];
    if (t >= n0 * n1 * (unsigned)L.n[2]) return false;
    const unsigned r = t / n0;
    c[0] = (int)(t - r * n0);
    c[1] = (int)(r % n1);
    c[2] = (int)(r / n1);
    return true;
}

// sum over the two neighbours along d of Phi inside (or its periodic image),
// and the number of neighbours outside a non-periodic boundary (each stands
// for -Phi(c))
__device__ __forceinline__ double mg_nbsum(const MgLevel &L, const double *__restrict__ a, const int c[3], int d,
                                           int &nout)
{
    double s = 0.0;
#pragma unroll
    for (int sg = -1; sg <= 1; sg += 2) {
        int cc[3] = {c[0], c[1], c[2]};
        cc[d] += sg;
        if (cc[d] < 0 || cc[d] >= L.n[d]) {
            if (!L.per[d]) {
                nout++;
                continue;
            }
            cc[d] = (cc[d] + L.n[d]) % L.n[d];
        }
        s += a[mg_lin(L, cc[0], cc[1], cc[2])];
    }
    return s;
}

// right-hand side: the divergence of the face fields on the interior cells
__global__ void __launch_bounds__(256) k_mg_div(Geo G, CPtr<3> face, MgLevel L)
{
    int c[3];
    if (!mg_point(L, c)) return;
    int p[3] = {c[0] + G.g[0], c[1] + G.g[1], c[2] + G.g[2]};
    const unsigned o = (unsigned)lin(G, p) << 3;
    double dv = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++)
        if (G.act[d]) dv += (ldb(face.p[d], o + ((unsigned)G.st[d] << 3)) - ldb(face.p[d], o)) * G.idx[d];
    L.rhs[mg_lin(L, c[0], c[1], c[2])] = dv;
}

// red-black Gauss-Seidel update of one cell (the caller picks the color)
__device__ __forceinline__ void mg_smooth_pt(const MgLevel &L, const int c[3])
{
    double off = 0.0, diag = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        if (!L.act[d]) continue;
        int nout = 0;
        off += L.ih2[d] * mg_nbsum(L, L.phi, c, d, nout);
        diag += L.ih2[d] * (2 + nout);
    }
    const int id = mg_lin(L, c[0], c[1], c[2]);
    L.phi[id] = (off - L.rhs[id]) / diag;
}
__global__ void __launch_bounds__(256) k_mg_smooth(MgLevel L, int color)
{
    int c[3];
    if (!mg_point(L, c)) return;
    if (((c[0] + c[1] + c[2]) & 1) != color) return;
    mg_smooth_pt(L, c);
}
// the same half sweep with one thread per cell of the color (n[0] even: the
// cells of a color are every second cell of each x row, starting at the
// row's parity)
__global__ void __launch_bounds__(256) k_mg_smooth_color(MgLevel L, int color)
{
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned h = (unsigned)L.n[0] >> 1, n1 = (unsigned)L.n[1];
    if (t >= h * n1 * (unsigned)L.n[2]) return;
    const unsigned r = t / h;
    int c[3];
    c[1] = (int)(r % n1);
    c[2] = (int)(r / n1);
    c[0] = 2 * (int)(t - r * h) + ((color + c[1] + c[2]) & 1);
    mg_smooth_pt(L, c);
}

// rhs - L Phi at one cell
__device__ __forceinline__ double mg_residual_pt(const MgLevel &L, const int c[3])
{
    const int id = mg_lin(L, c[0], c[1], c[2]);
    const double pc = L.phi[id];
    double lap = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        if (!L.act[d]) continue;
        int nout = 0;
        double s = mg_nbsum(L, L.phi, c, d, nout);
        lap += L.ih2[d] * (s - (2 + nout) * pc);
    }
    return L.rhs[id] - lap;
}

// coarse right-hand side at one coarse cell: the mean of its children's
// residuals (formed here, not stored); coarse Phi = 0
__device__ __forceinline__ void mg_restrict_pt(const MgLevel &F, const MgLevel &C, const int c[3])
{
    double s = 0.0;
    int m = 0;
    for (int dz = 0; dz <= C.act[2]; dz++)
        for (int dy = 0; dy <= C.act[1]; dy++)
            for (int dx = 0; dx <= C.act[0]; dx++) {
                const int f[3] = {C.act[0] ? 2 * c[0] + dx : c[0], C.act[1] ? 2 * c[1] + dy : c[1],
                                  C.act[2] ? 2 * c[2] + dz : c[2]};
                s += mg_residual_pt(F, f);
                m++;
            }
    const int id = mg_lin(C, c[0], c[1], c[2]);
    C.rhs[id] = s / m;
    C.phi[id] = 0.0;
}
__global__ void __launch_bounds__(256) k_mg_restrict(MgLevel F, MgLevel C)
{
    int c[3];
    if (!mg_point(C, c)) return;
    mg_restrict_pt(F, C, c);
}

// coarse value at (possibly outside) coarse index, boundary rule applied
// relative to the inside cell q
__device__ __forceinline__ double mg_coarse_at(const MgLevel &C, int I[3], const int q[3])
{
    double sign = 1.0;
    int J[3] = {I[0], I[1], I[2]};
#pragma unroll
    for (int d = 0; d < 3; d++) {
        if (J[d] < 0 || J[d] >= C.n[d]) {
            if (C.per[d]) {
                J[d] = (J[d] + C.n[d]) % C.n[d];
            } else {
                J[d] = q[d];  // mirror: minus the boundary cell
                sign = -sign;
            }
        }
    }
    return sign * C.phi[mg_lin(C, J[0], J[1], J[2])];
}

// fine Phi += cell-centred (bi/tri)linear interpolation of the coarse Phi
// (weights 3/4 for the parent, 1/4 for the neighbour across the child's side)
__device__ __forceinline__ void mg_prolong_pt(const MgLevel &C, const MgLevel &F, const int c[3])
{
    int P[3], S[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        P[d] = C.act[d] ? c[d] >> 1 : c[d];
        S[d] = C.act[d] ? ((c[d] & 1) ? 1 : -1) : 0;
    }
    double v = 0.0;
    for (int bz = 0; bz <= C.act[2]; bz++)
        for (int by = 0; by <= C.act[1]; by++)
            for (int bx = 0; bx <= C.act[0]; bx++) {
                int I[3] = {P[0] + bx * S[0], P[1] + by * S[1], P[2] + bz * S[2]};
                double w = (C.act[0] ? (bx ? 0.25 : 0.75) : 1.0) * (C.act[1] ? (by ? 0.25 : 0.75) : 1.0) *
                           (C.act[2] ? (bz ? 0.25 : 0.75) : 1.0);
                v += w * mg_coarse_at(C, I, P);
            }
    F.phi[mg_lin(F, c[0], c[1], c[2])] += v;
}
__global__ void __launch_bounds__(256) k_mg_prolong(MgLevel C, MgLevel F)
{
    int c[3];
    if (!mg_point(F, c)) return;
    mg_prolong_pt(C, F, c);
}

// The part of the V-cycle on the levels l0 .. nl - 1, all small enough for one
// workgroup: the same stages as the per-level launches (two red-black sweeps,
// restriction down to the coarsest level, its sweeps, prolongation and two
// sweeps back up), each a loop over the level's cells separated by block
// barriers, in one launch of one block.  Phi and the right-hand sides of these
// levels live in LDS for the launch (level l0's are read in first and its
// Phi written back at the end), so every stage runs at LDS latency.
constexpr int kMgBlockThreads = 1024;
constexpr int kMgOneBlockCells = 512;  // levels at most this large run in the one-block kernel
constexpr int kMgSmallCells = 2 * kMgOneBlockCells;  // all of them together (at most 512 + 256 + ... in 1-D)
constexpr int kMgLevelsMax = 24;
struct MgStack {
    MgLevel lv[kMgLevelsMax];
    int sh_off[kMgLevelsMax];  // LDS offsets (doubles) of the small levels' Phi; rhs follows Phi
};
__device__ __forceinline__ void mg_cell_of(const MgLevel &L, int t, int c[3])
{
    c[0] = t % L.n[0];
    const int r = t / L.n[0];
    c[1] = r % L.n[1];
    c[2] = r / L.n[1];
}
__device__ __forceinline__ int mg_cells(const MgLevel &L) { return L.n[0] * L.n[1] * L.n[2]; }
__device__ void mg_sweeps_block(const MgLevel &L, int sweeps)
{
    const int n = mg_cells(L);
    for (int s = 0; s < sweeps; s++)
        for (int col = 0; col < 2; col++) {
            for (int t = threadIdx.x; t < n; t += blockDim.x) {
                int c[3];
                mg_cell_of(L, t, c);
                if (((c[0] + c[1] + c[2]) & 1) == col) mg_smooth_pt(L, c);
            }
            __syncthreads();
        }
}
// level l of the stack with Phi and rhs in LDS (the kernel argument holds the
// levels; a uniform index reads them without a private copy)
__device__ __forceinline__ MgLevel mg_small(const MgStack &S, int l, double *sh)
{
    MgLevel L = S.lv[l];
    const int n = mg_cells(L);
    L.phi = sh + S.sh_off[l];
    L.rhs = sh + S.sh_off[l] + n;
    L.res = nullptr;
    return L;
}
__global__ void __launch_bounds__(kMgBlockThreads) k_mg_small_cycle(MgStack S, int l0, int nl, int coarse_sweeps)
{
    __shared__ double sh[2 * kMgSmallCells];  // the host checked that the small levels fit
    {
        const MgLevel G0 = S.lv[l0], L0 = mg_small(S, l0, sh);
        const int n = mg_cells(G0);
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            L0.phi[t] = G0.phi[t];
            L0.rhs[t] = G0.rhs[t];
        }
        __syncthreads();
    }
    for (int l = l0; l < nl - 1; l++) {
        const MgLevel F = mg_small(S, l, sh), C = mg_small(S, l + 1, sh);
        mg_sweeps_block(F, 2);
        const int n = mg_cells(C);
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            int c[3];
            mg_cell_of(C, t, c);
            mg_restrict_pt(F, C, c);
        }
        __syncthreads();
    }
    mg_sweeps_block(mg_small(S, nl - 1, sh), coarse_sweeps);
    for (int l = nl - 2; l >= l0; l--) {
        const MgLevel F = mg_small(S, l, sh), C = mg_small(S, l + 1, sh);
        const int n = mg_cells(F);
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            int c[3];
            mg_cell_of(F, t, c);
            mg_prolong_pt(C, F, c);
        }
        __syncthreads();
        mg_sweeps_block(F, 2);
    }
    const MgLevel G0 = S.lv[l0], L0 = mg_small(S, l0, sh);
    const int n = mg_cells(G0);
    for (int t = threadIdx.x; t < n; t += blockDim.x) G0.phi[t] = L0.phi[t];
}

__global__ void __launch_bounds__(256) k_mg_zero(MgLevel L)
{
    int c[3];
    if (!mg_point(L, c)) return;
    L.phi[mg_lin(L, c[0], c[1], c[2])] = 0.0;
}

// q_B^d -= (Phi(c) - Phi(c - e_d)) / dx_d on the d-faces g .. g+n of the
// interior; one thread per point of the interior plus one layer
__global__ void __launch_bounds__(256) k_mg_apply(Geo G, MgLevel L, Ptr<3> face, Region R)
{
    int c[3];
    if (!region_point(R, Blk{blockIdx.x, blockIdx.y, blockIdx.z}, c)) return;
    int q[3] = {c[0] - G.g[0], c[1] - G.g[1], c[2] - G.g[2]};  // cell index of the face's upper cell
    const unsigned o = (unsigned)lin(G, c) << 3;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        if (!G.act[d]) continue;
        bool ok = true;
#pragma unroll
        for (int e = 0; e < 3; e++)
            if (e != d && q[e] >= L.n[e]) ok = false;
        if (!ok) continue;
        // Phi of the cells on both sides of the face, boundary rule outside
        int up[3] = {q[0], q[1], q[2]}, dn[3] = {q[0], q[1], q[2]};
        dn[d] -= 1;
        double pu, pd;
        if (up[d] >= L.n[d]) {
            int in[3] = {q[0], q[1], q[2]};
            in[d] = L.per[d] ? 0 : L.n[d] - 1;
            pu = (L.per[d] ? 1.0 : -1.0) * L.phi[mg_lin(L, in[0], in[1], in[2])];
        } else {
            pu = L.phi[mg_lin(L, up[0], up[1], up[2])];
        }
        if (dn[d] < 0) {
            int in[3] = {q[0], q[1], q[2]};
            in[d] = L.per[d] ? L.n[d] - 1 : 0;
            pd = (L.per[d] ? 1.0 : -1.0) * L.phi[mg_lin(L, in[0], in[1], in[2])];
        } else {
            pd = L.phi[mg_lin(L, dn[0], dn[1], dn[2])];
        }
        stb(face.p[d], o, ldb(face.p[d], o) - (pu - pd) * G.idx[d]);
    }
}

}  // namespace gr
