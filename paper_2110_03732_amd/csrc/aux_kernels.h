// aux_kernels.h -- initial data and reductions (not on the per-step path,
// except the div B / dt reductions when requested).
#pragma once
#include "common.h"
#include "physics.h"

namespace gr {

// flat index over a box region (used by grid-stride reduction kernels)
struct FlatBox {
    int lo[3], cnt[3];
    long total;
};
__device__ __forceinline__ void flat_coords(const FlatBox &R, long t, int c[3])
{
    c[0] = R.lo[0] + (int)(t % R.cnt[0]);
    long r = t / R.cnt[0];
    c[1] = R.lo[1] + (int)(r % R.cnt[1]);
    c[2] = R.lo[2] + (int)(r / R.cnt[1]);
}
__device__ __forceinline__ int flat_point(const Geo &G, const FlatBox &R, long t)
{
    int c[3];
    flat_coords(R, t, c);
    return lin(G, c);
}

// Sec 4: face fields q_B^d = d_{m1} A_{m2} - d_{m2} A_{m1} from the edge
// vector potential (+ an optional added face field), every padded point
__global__ void __launch_bounds__(256) k_curlA(Geo G, int Ne0, int Ne1, const double *__restrict__ A, long es,
                                               const double *__restrict__ fadd, long np, Ptr<3> face)
{
    int c[3];
    int tt = blockIdx.x * blockDim.x + threadIdx.x;
    if (tt >= G.N[0] * G.N[1]) return;
    c[1] = tt / G.N[0];
    c[0] = tt - c[1] * G.N[0];
    c[2] = blockIdx.y;
    int t = lin(G, c);
    long tc = c[0] + (long)G.N[0] * (c[1] + (long)G.N[1] * c[2]);  // the added field is compact
    long ie = c[0] + (long)Ne0 * (c[1] + (long)Ne1 * c[2]);
    long est[3] = {1, Ne0, (long)Ne0 * Ne1};
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int m1 = (d + 1) % 3, m2 = (d + 2) % 3;
        double s = 0.0;
        if (A) {
            if (G.act[m1]) s += (A[m2 * es + ie + est[m1]] - A[m2 * es + ie]) * G.idx[m1];
            if (G.act[m2]) s -= (A[m1 * es + ie + est[m2]] - A[m1 * es + ie]) * G.idx[m2];
        }
        face.p[d][t] = fadd ? fadd[d * np + tc] + s : s;
    }
}

// a compact field (index i + Nx (j + Ny k), as the host passes it) into the
// padded device layout; every padded point
__global__ void __launch_bounds__(256) k_unpack(Geo G, const double *__restrict__ src, double *__restrict__ dst)
{
    int c[3];
    int tt = blockIdx.x * blockDim.x + threadIdx.x;
    if (tt >= G.N[0] * G.N[1]) return;
    c[1] = tt / G.N[0];
    c[0] = tt - c[1] * G.N[0];
    c[2] = blockIdx.y;
    dst[lin(G, c)] = src[c[0] + (long)G.N[0] * (c[1] + (long)G.N[1] * c[2])];
}

// conserved D, S, tau of the interior cells from primitives, E and faces
template <int MET>
__global__ void __launch_bounds__(256) k_init_cons(Geo G, Phys P, Region R, CPtr<5> prim, CPtr<3> E, CPtr<3> face,
                                                   CPtr<2> met, Ptr<8> q)
{
    int c[3];
    if (!region_point(R, Blk{blockIdx.x, blockIdx.y, blockIdx.z}, c)) return;
    int id = lin(G, c);
    double ps = MET ? met.p[1][id] : 1.0;
    double ps2 = ps * ps, ps6 = ps2 * ps2 * ps2;
    double u[3], Ev[3], B[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        u[i] = ps2 * prim.p[1 + i][id];
        Ev[i] = ps2 * E.p[i][id];
        double b = G.act[i] ? 0.5 * (face.p[i][id] + face.p[i][id + G.st[i]]) : face.p[i][id];
        B[i] = ps2 * b / ps6;
    }
    double q8[8], f8[8];
    flat_cons_flux(P, 0, prim.p[0][id], u, prim.p[4][id], Ev, B, q8, f8);
    q.p[0][id] = ps6 * q8[0];
    q.p[1][id] = ps6 * ps2 * q8[1];
    q.p[2][id] = ps6 * ps2 * q8[2];
    q.p[3][id] = ps6 * ps2 * q8[3];
    q.p[4][id] = ps6 * q8[4];
}

// q_E = psi^6 E on every padded point
__global__ void __launch_bounds__(256) k_init_qE(Geo G, int met_on, CPtr<3> E, CPtr<2> met, Ptr<8> q)
{
    int c[3];
    int tt = blockIdx.x * blockDim.x + threadIdx.x;
    if (tt >= G.N[0] * G.N[1]) return;
    c[1] = tt / G.N[0];
    c[0] = tt - c[1] * G.N[0];
    c[2] = blockIdx.y;
    int t = lin(G, c);
    double ps6 = 1.0;
    if (met_on) {
        double ps = met.p[1][t];
        double p2 = ps * ps;
        ps6 = p2 * p2 * p2;
    }
#pragma unroll
    for (int i = 0; i < 3; i++) q.p[5 + i][t] = ps6 * E.p[i][t];
}

// stage block (prim 5, E = q_E / psi^6) on every padded point
__global__ void __launch_bounds__(256) k_stage_copy(Geo G, int met_on, CPtr<5> prim, CPtr<8> q, CPtr<2> met,
                                                    Ptr<8> sp)
{
    int c[3];
    int tt = blockIdx.x * blockDim.x + threadIdx.x;
    if (tt >= G.N[0] * G.N[1]) return;
    c[1] = tt / G.N[0];
    c[0] = tt - c[1] * G.N[0];
    c[2] = blockIdx.y;
    int t = lin(G, c);
    double ips6 = 1.0;
    if (met_on) {
        double ps = met.p[1][t];
        double p2 = ps * ps;
        ips6 = 1.0 / (p2 * p2 * p2);
    }
#pragma unroll
    for (int v = 0; v < 5; v++) sp.p[v][t] = prim.p[v][t];
#pragma unroll
    for (int i = 0; i < 3; i++) sp.p[5 + i][t] = q.p[5 + i][t] * ips6;
}

// GLM initial data (Sec 3.1): cell-centred q_B^d = mean of the cell's two
// d-faces (the face value itself along an inactive direction and at the last
// point of the padded array); every padded point
__global__ void __launch_bounds__(256) k_face_to_cell(Geo G, CPtr<3> face, Ptr<3> cell)
{
    int c[3];
    int tt = blockIdx.x * blockDim.x + threadIdx.x;
    if (tt >= G.N[0] * G.N[1]) return;
    c[1] = tt / G.N[0];
    c[0] = tt - c[1] * G.N[0];
    c[2] = blockIdx.y;
    int t = lin(G, c);
#pragma unroll
    for (int d = 0; d < 3; d++) {
        double f = face.p[d][t];
        if (G.act[d] && c[d] + 1 < G.N[d]) f = 0.5 * (f + face.p[d][t + G.st[d]]);
        cell.p[d][t] = f;
    }
}

// ---------------------------------------------------------------------------
// reductions: per-block partials (sum |x|, sum x^2, max |x|), then one block;
// fixed tree order, so the result does not depend on scheduling
__device__ __forceinline__ void block_reduce3(double &a, double &b, double &c)
{
    __shared__ double sa[4], sb[4], sc[4];
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
        for (int i = 1; i < 4; i++) {
            a += sa[i];
            b += sb[i];
            c = fmax(c, sc[i]);
        }
    }
}

__global__ void __launch_bounds__(256) k_divb_partial(Geo G, FlatBox R, CPtr<3> face, double *__restrict__ part)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < R.total; t += (long)gridDim.x * blockDim.x) {
        int id = flat_point(G, R, t);
        double dv = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++)
            if (G.act[d]) dv += (face.p[d][id + G.st[d]] - face.p[d][id]) * G.idx[d];
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

// GLM: central-difference divergence of the cell-centred q_B over the
// interior, the boundary rule supplying the neighbour outside
__global__ void __launch_bounds__(256) k_divb_cc_partial(Geo G, FlatBox R, CPtr<3> qB, double *__restrict__ part)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < R.total; t += (long)gridDim.x * blockDim.x) {
        int p[3];
        flat_coords(R, t, p);
        const int id = lin(G, p);
        double dv = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            if (!G.act[d]) continue;
            int up = stage_cell(G, d, p[d] + 1), dn = stage_cell(G, d, p[d] - 1);
            dv += (qB.p[d][id + (up - p[d]) * G.st[d]] - qB.p[d][id + (dn - p[d]) * G.st[d]]) * (0.5 * G.idx[d]);
        }
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

__global__ void __launch_bounds__(256) k_reduce_final(int nparts, long count, int mode, const double *__restrict__ part,
                                                      double *__restrict__ out)
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
__global__ void __launch_bounds__(256) k_cfl_partial(Geo G, FlatBox R, CPtr<2> met, double *__restrict__ part)
{
    double c = 0.0, z = 0.0, z2 = 0.0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < R.total; t += (long)gridDim.x * blockDim.x) {
        int id = flat_point(G, R, t);
        double sp = 1.0;
        if (MET) {
            double ps = met.p[1][id];
            sp = met.p[0][id] / (ps * ps);
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

}  // namespace gr
