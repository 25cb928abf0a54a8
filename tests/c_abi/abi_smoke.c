/* A plain C99 consumer of the library's C ABI (no C++, no PyTorch): the
 * 400-cell relativistic resistive shock tube (Gamma = 2, (rho, p, B^y) =
 * (1, 1, 0.5) | (0.125, 0.1, -0.5), B^x = 0.5, eta = 1e-3, minmod, IMEX-SSP2)
 * advanced to t = 0.4 through gr_init_state / gr_cfl_dt / gr_step /
 * gr_divB_norm / gr_fail_count, with device memory from hipMalloc.  Writes
 * the final interior primitives (5 x 400 doubles) to the file named by argv[1]
 * and prints one summary line; exits non-zero on any error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "grmhd.h"

#define CHECK(call)                                                                          \
    do {                                                                                     \
        gr_status st_ = (call);                                                              \
        if (st_ != GR_OK) {                                                                  \
            fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #call, gr_strerror(st_)); \
            return 1;                                                                        \
        }                                                                                    \
    } while (0)
#define HCHECK(call)                                                  \
    do {                                                              \
        if ((call) != hipSuccess) {                                   \
            fprintf(stderr, "%s:%d %s failed\n", __FILE__, __LINE__, #call); \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main(int argc, char **argv)
{
    if (argc < 2) {
        fprintf(stderr, "usage: %s output.bin\n", argv[0]);
        return 2;
    }
    if (gr_abi_version() != GR_ABI_VERSION) {
        fprintf(stderr, "ABI version %d, header %d\n", gr_abi_version(), GR_ABI_VERSION);
        return 1;
    }
    gr_grid g;
    memset(&g, 0, sizeof(g));
    g.ndim = 1;
    g.n[0] = 400;
    g.n[1] = g.n[2] = 1;
    g.ng = 2;
    g.lo[0] = -0.5;
    g.hi[0] = 0.5;
    g.lo[1] = g.lo[2] = 0.0;
    g.hi[1] = g.hi[2] = 1.0;
    g.bc[0][0] = g.bc[0][1] = GR_OUTFLOW;
    g.gamma_ad = 2.0;
    g.recon = GR_MINMOD;
    g.imex = GR_SSP2_222;
    g.cfl = 0.4;
    g.eta_mode = GR_ETA_UNIFORM;
    g.eta = 1e-3;
    g.eta_max = 1.0;
    g.rho_atm = 1e-14;
    g.p_atm = 1e-14;
    g.newton_tol = 1e-13;
    g.newton_maxit = 60;
    g.atm_factor = 1.001;
    g.kappa_E = g.kappa_B = 1.0;
    gr_grid bad = g;
    bad.ng = 1;
    if (gr_validate(&bad) != GR_EINVAL || gr_validate(&g) != GR_OK) {
        fprintf(stderr, "validation\n");
        return 1;
    }
    const int N = g.n[0] + 2 * g.ng;
    const size_t fs = gr_field_stride(&g);
    double *prim = calloc(5 * (size_t)N, sizeof(double));
    double *E = calloc(3 * (size_t)N, sizeof(double));
    double *face = calloc(3 * (size_t)N, sizeof(double));
    if (!prim || !E || !face) return 1;
    const double dx = (g.hi[0] - g.lo[0]) / g.n[0];
    for (int i = 0; i < N; i++) {
        const double x = g.lo[0] + (i - g.ng + 0.5) * dx;
        const int left = x < 0.0;
        prim[0 * N + i] = left ? 1.0 : 0.125;
        prim[4 * N + i] = left ? 1.0 : 0.1;
        face[0 * N + i] = 0.5;                /* B^x on the x-faces */
        face[1 * N + i] = left ? 0.5 : -0.5;  /* B^y (y inactive: cell values) */
    }
    gr_state s;
    memset(&s, 0, sizeof(s));
    HCHECK(hipMalloc((void **)&s.q, 8 * fs * sizeof(double)));
    HCHECK(hipMalloc((void **)&s.face, 3 * fs * sizeof(double)));
    HCHECK(hipMalloc((void **)&s.prim, 5 * fs * sizeof(double)));
    s.work_bytes = gr_workspace_bytes(&g);
    HCHECK(hipMalloc(&s.work, s.work_bytes));
    CHECK(gr_init_state(&g, &s, prim, E, NULL, face, NULL, 0));
    double dt = 0.0;
    CHECK(gr_cfl_dt(&g, &s, &dt, 0));
    const int nsteps = (int)(0.4 / dt + 0.5);
    for (int k = 0; k < nsteps; k++) CHECK(gr_step(&g, &s, dt, 0));
    double *d3;
    HCHECK(hipMalloc((void **)&d3, 3 * sizeof(double)));
    CHECK(gr_divB_norm(&g, &s, d3, 0));
    double div[3];
    HCHECK(hipMemcpy(div, d3, sizeof(div), hipMemcpyDeviceToHost));
    unsigned long long fails = 0;
    CHECK(gr_fail_count(&g, &s, &fails, 0));
    double *out = malloc(5 * (size_t)g.n[0] * sizeof(double));
    if (!out) return 1;
    for (int v = 0; v < 5; v++)
        HCHECK(hipMemcpy(out + (size_t)v * g.n[0], s.prim + (size_t)v * fs + gr_field_origin(&g) + g.ng,
                         g.n[0] * sizeof(double),
                         hipMemcpyDeviceToHost));
    int ok = fails == 0 && div[2] <= 1e-12;
    for (int i = 0; i < 5 * g.n[0]; i++) ok = ok && isfinite(out[i]);
    for (int i = 0; i < g.n[0]; i++) ok = ok && out[i] > 0.05 && out[i] < 1.5;  /* density */
    FILE *f = fopen(argv[1], "wb");
    if (!f || fwrite(out, sizeof(double), 5 * (size_t)g.n[0], f) != 5 * (size_t)g.n[0]) return 1;
    fclose(f);
    printf("abi_smoke: %d steps of dt %.6g, div B linf %.3g, failures %llu, rho range ok %d\n", nsteps, dt, div[2],
           fails, ok);
    hipFree(d3);
    hipFree(s.q);
    hipFree(s.face);
    hipFree(s.prim);
    hipFree(s.work);
    free(prim);
    free(E);
    free(face);
    free(out);
    return ok ? 0 : 1;
}
