/*
 * grmhd.h -- C ABI of the MI355X (gfx950) library for one implicit-explicit
 * Runge-Kutta step of special/general-relativistic resistive MHD on a fixed
 * (Cowling) Cartesian grid, after Cheong et al., arXiv:2110.03732.
 *
 * All arithmetic is FP64.  All array arguments named *_dev are DEVICE
 * pointers owned by the caller; *_host arguments are host pointers read
 * during the call.  Every call is asynchronous on the given stream unless
 * it says it synchronises.  The library never allocates device memory in
 * these calls: stage storage lives in the caller's workspace.
 *
 * Layouts (shared with the caller):
 *   - cell arrays have N_d = n_d + 2 ng points per active direction (1 for an
 *     inactive one), x fastest, rows padded: point (i,j,k) of a field sits at
 *     index o + i + P (j + Ny k) from the field's start, with row stride
 *     P = gr_row_stride(grid) (Nx rounded up to 16 doubles, one 128-byte line)
 *     and origin o = gr_field_origin(grid) (< 16), chosen so that the first
 *     interior point of every row (i = ng) starts a 128-byte line when the
 *     field starts on one.  The padding points are never read or written.  A
 *     "field block" holds F such arrays back to back, field f starting at
 *     f * stride with stride = gr_field_stride(grid) doubles
 *     (>= o + P Ny Nz, a multiple of 32); allocate blocks 256-byte aligned.
 *     Host arrays passed to gr_init_state are compact instead: index
 *     i + Nx (j + Ny k), fields back to back;
 *   - q: 8 fields, the densitised conserved variables of Sec 2.1,
 *     (q_D, q_S_x, q_S_y, q_S_z, q_tau, q_E^x, q_E^y, q_E^z), q = psi^6 (...);
 *   - face: 3 fields, face-centred q_B^d = psi^6 B^d (Sec 3.2); field d at
 *     index (i,j,k) sits half a cell below the cell centre in direction d.
 *     With glm = 1 (Sec 3.1) the same 3 fields hold the cell-centred q_B^d
 *     and q holds 10 fields: the 8 above, then q_Psi = psi^6 Psi and
 *     q_Phi = psi^6 Phi;
 *   - prim: 5 fields (rho, u~^x, u~^y, u~^z, p), u~^i = W v^i (Sec 2.4);
 *   - metric: NULL (flat) or 2 fields (lapse alpha, conformal factor psi) of
 *     a static conformally flat metric, gamma_ij = psi^4 delta_ij, beta = 0.
 *   - an edge array (vector potential A_k) is one point longer than a cell
 *     array in every active direction; A_k at (i,j,k) sits half a cell below
 *     the cell centre in the two directions other than k.
 *
 * Errors: host-detectable problems return a negative gr_status; numerical
 * trouble inside a cell never fails a call: the cell falls back to the
 * atmosphere state and a device counter is incremented (gr_fail_count).
 */
#ifndef GRMHD_H
#define GRMHD_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GR_ABI_VERSION 6

typedef enum {
    GR_OK = 0,
    GR_EINVAL = -1,        /* bad argument, shape or parameter            */
    GR_ENOMEM = -2,        /* workspace too small                         */
    GR_EHIP = -3,          /* a HIP runtime call or kernel launch failed   */
    GR_EUNSUPPORTED = -4   /* valid but not implemented (e.g. mixed IMEX tableaux in a batch) */
} gr_status;

enum { GR_OUTFLOW = 0, GR_PERIODIC = 1, GR_FIXED = 2 };   /* boundary rules  */
enum { GR_MINMOD = 0, GR_MC = 1, GR_PPM = 2 };             /* reconstruction  */
enum { GR_SSP2_222 = 0, GR_SSP3_433 = 1 };                 /* IMEX tableaux   */
enum { GR_ETA_UNIFORM = 0, GR_ETA_SIGMA_D = 1 };           /* resistivity law */

/* Problem description.  Field order is part of the ABI. */
typedef struct gr_grid {
    int ndim;             /* 1..3; active directions are x, then y, then z      */
    int n[3];             /* interior cells per direction (1 when inactive)     */
    int ng;               /* ghost width: >= 2 (minmod, MC), >= 3 (PPM)         */
    double lo[3], hi[3];  /* domain                                            */
    int bc[3][2];         /* GR_OUTFLOW / GR_PERIODIC / GR_FIXED per side       */
    double gamma_ad;      /* ideal gas p = (Gamma - 1) rho eps                  */
    int recon;            /* GR_MINMOD / GR_MC / GR_PPM                         */
    int imex;             /* GR_SSP2_222 / GR_SSP3_433                          */
    double cfl;           /* dt = cfl / max sum_d alpha sqrt(gamma^dd) / dx_d   */
    int eta_mode;         /* GR_ETA_UNIFORM: eta; GR_ETA_SIGMA_D: eq. sigma_D    */
    double eta, sigma0, eta_min, eta_max;
    double rho_atm, p_atm;/* atmosphere state                                  */
    int metric;           /* 0 flat, 1 static conformally flat (alpha, psi)     */
    double newton_tol;    /* Newton stop: |du~|_inf <= tol (1 + |u~|_inf)       */
    int newton_maxit;
    double xi;            /* mean-field dynamo coefficient of eq. ohms_law      */
    double atm_factor;    /* cells with D <= atm_factor rho_atm are atmosphere  */
    int frozen_matter;    /* 1: rho, u~, p stay fixed and only E and B evolve   */
    int glm;              /* 1: cell-centred B with GLM cleaning (Sec 3.1)      */
    double kappa_E, kappa_B; /* GLM damping parameters                          */
    int uct;              /* edge EMF of the CT update: 0 the resistive upwind
                             form (Sec 3.2, reconstructed E), 1 the ideal-MHD
                             form (App. A, transport velocities x face fields;
                             the eta -> 0 limit); GR_EUNSUPPORTED with glm     */
} gr_grid;

/* Device state of one run (all pointers caller-owned device memory). */
typedef struct gr_state {
    double *q;            /* 8-field block                                     */
    double *face;         /* 3-field block                                     */
    double *prim;         /* 5-field block                                     */
    double *metric;       /* 2-field block or NULL when grid->metric == 0       */
    void *work;           /* workspace of gr_workspace_bytes(grid) bytes        */
    size_t work_bytes;
} gr_state;

int gr_abi_version(void);
const char *gr_strerror(gr_status s);

/* Checks a grid description; GR_OK when every other call accepts it. */
gr_status gr_validate(const gr_grid *grid);

/* Doubles between consecutive fields of a field block. */
size_t gr_field_stride(const gr_grid *grid);

/* Doubles between consecutive rows (j to j + 1) of a device cell array; rows
 * are Nx points padded to a multiple of 16.  0 for an invalid grid. */
size_t gr_row_stride(const gr_grid *grid);

/* Doubles from the start of a device field to its point (0, 0, 0).  0 for
 * an invalid grid (also a valid origin: check gr_validate first). */
size_t gr_field_origin(const gr_grid *grid);

/* Bytes of workspace the stage calls need (stage states, stored L and R
 * terms of the IMEX tableau, scratch, counters). */
size_t gr_workspace_bytes(const gr_grid *grid);

/* Byte offset inside the workspace of one field of stage storage, for
 * inspection: kind 0 = stage primitives + E (8 fields: rho, u~, p, E^i;
 * with glm 10: + Psi, Phi), 1 = stage face fields (3; with glm the cell q_B),
 * 2 = stored L (11: 8 cell + 3 face; with glm 13: 8 cell, q_B, q_Psi,
 * q_Phi), 3 = stored R (3, q_E rows).  stage is 0-based (< number of
 * implicit stages); a field index beyond the kind's count is GR_EINVAL. */
gr_status gr_workspace_offset(const gr_grid *grid, int kind, int stage, int field, size_t *offset_bytes);

/* Initial state (Sec 4 and Sec 2.1): face fields q_B^i = eta^{ijk} d_j A_k
 * from the edge vector potential A_host (3 edge arrays back to back, or
 * NULL), plus face_host (3 cell-sized arrays, densitised, or NULL); q_E =
 * psi^6 E everywhere; D, S, tau from the primitives on interior cells.
 * prim_host: 5 cell arrays, E_host: 3 cell arrays, metric_host: 2 cell arrays
 * (alpha, psi) or NULL; all host arrays are compact (index i + Nx (j + Ny k),
 * stride Nx Ny Nz between fields) and are copied into the padded device
 * layout.  Also resets the failure counter and sets every stage block of
 * the workspace to a copy of the state, ghost points included.  With glm the
 * face fields are then turned into the cell-centred q_B^d (mean of the
 * cell's two d-faces; the face value itself along an inactive direction and
 * at the last point of the array) and q_Psi = q_Phi = 0 (Sec 3.1).
 * Synchronises the stream. */
gr_status gr_init_state(const gr_grid *grid, gr_state *state, const double *prim_host, const double *E_host,
                        const double *A_host, const double *face_host, const double *metric_host,
                        hipStream_t stream);

/* One pass of the IMEX-RK step (Sec 2.3): pass p = 0 .. s-1 is implicit
 * stage p+1 (it first evaluates the explicit operator L of stage p when the
 * tableau needs it, then accumulates q* and solves the stiff Ohm's-law
 * update fused with the primitive recovery, Sec 2.4); pass p = s is the
 * final combination followed by the recovery with E and B known (Sec 2.6).
 * s = 2 for GR_SSP2_222, 4 for GR_SSP3_433.  Passes must run in order.
 * No pass writes a ghost point of the state: the boundary rules (outflow,
 * periodic) are applied where a stencil reads beyond the interior, and ghost
 * points of fixed boundaries keep the values they were initialised with (in
 * the workspace, a pass with L writes the layer of stage E next to the
 * interior, which its cell pass reads for the Gauss-law charge).
 * In a pass that evaluates L on a grid of at least 2^20 interior cells (2^18
 * while `stream` is being captured into a graph), the edge-EMF and
 * face-update launches run on a second stream the library owns (one per
 * device, default priority, created by gr_init_state), forked from `stream`
 * with an event at the start of the pass and joined back before the cell
 * pass: the call stays ordered on `stream` and can be captured into a graph
 * from it.  Smaller grids launch everything on `stream`.  The second stream
 * is shared by every call on the device: forked calls from several host
 * threads queue their EMF launches on it one after another, and a call being
 * captured must not overlap a forked call from another thread. */
gr_status gr_imex_stage(const gr_grid *grid, gr_state *state, int pass, double dt, hipStream_t stream);

/* All passes of one step (Sec 2.3).  Where passes 0 and 1 are both
 * point-wise (IMEX-SSP3(4,3,3): L of stage 0 is never used and stage 1's only
 * explicit term is a_10 R_0; face-centred B, matter not frozen) they run as
 * one launch: stage 0's primitives then only seed stage 1's Newton guess and
 * its workspace block is not written (gr_imex_stage writes it; a batch step
 * pairs the same passes). */
gr_status gr_step(const gr_grid *grid, gr_state *state, double dt, hipStream_t stream);

/* Primitive recovery with E and B known (Sec 2.6) on the interior cells of
 * the state; atmosphere and failure rules as in the step.  B is the cell
 * mean of the face fields, or the cell q_B with glm. */
gr_status gr_con2prim(const gr_grid *grid, gr_state *state, hipStream_t stream);

/* Discrete divergence of the face field on interior cells,
 * div = sum_d (q_B^d(+1/2) - q_B^d(-1/2)) / dx_d (Sec 3, eq. divb_0):
 * out3_dev[0] = mean |div|, [1] = sqrt(mean div^2), [2] = max |div|.
 * With glm: central differences of the cell q_B, sum_d (q_B^d(+1) -
 * q_B^d(-1)) / (2 dx_d), the boundary rule giving the outside neighbour.
 * Uses the workspace scratch; deterministic reduction order. */
gr_status gr_divB_norm(const gr_grid *grid, const gr_state *state, double *out3_dev, hipStream_t stream);

/* gr_divB_norm for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * same norms, bit for bit, with the reduction partials in a file-scope
 * device array of the library (3 x 4096 doubles = 96 KiB on every GPU the
 * library runs on, held until the process ends) instead of the workspace;
 * only grid, state->face and out3_dev are used (state->work may be NULL).
 * Allocates nothing; the array's device address is looked up once per device
 * (gr_init_state does it; otherwise the first call on that device).  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams) race and must be ordered by the caller.  GR_ENOMEM if
 * the partials would not fit the array (no grid reaches it: the partial
 * count is capped at 4096 blocks); otherwise errors as gr_divB_norm. */
gr_status gr_divB_norm_noalloc(const gr_grid *grid, const gr_state *state, double *out3_dev, hipStream_t stream);

/* Elliptic divergence cleaning of the face fields (Sec 3.3, eq. poisson and
 * eq. update_bfield): solve L Phi = div q_B on the interior cells with
 * `vcycles` multigrid V-cycles (red-black Gauss-Seidel 2+2, mean
 * restriction, linear prolongation), then q_B^d -= dPhi/dx_d on every
 * d-face of the interior, boundary faces included.  Outside a non-periodic
 * boundary Phi is minus the boundary cell's value (Phi = 0 on the boundary
 * face); periodic directions wrap.  Coarsening stops at the first level with
 * an odd active size, which is then smoothed n^2 (<= 512) times per cycle, so
 * grids whose sizes carry few factors of 2 converge slowly.  Scratch lives
 * in the workspace.  out6_dev: NULL, or 6 device doubles receiving the
 * (L1, L2, Linf) norms of div q_B before and after.  A GLM grid (cell-centred
 * q_B) returns GR_EUNSUPPORTED. */
gr_status gr_clean_divB(const gr_grid *grid, gr_state *state, int vcycles, double *out6_dev, hipStream_t stream);

/* Time step of Sec 2.5 (maximum-diffusivity speeds depend on the metric
 * only).  Synchronises the stream; result written to *dt_host. */
gr_status gr_cfl_dt(const gr_grid *grid, const gr_state *state, double *dt_host, hipStream_t stream);

/* Cells that fell back to the atmosphere after a failed or unphysical
 * recovery since gr_init_state.  Synchronises the stream. */
gr_status gr_fail_count(const gr_grid *grid, const gr_state *state, unsigned long long *count_host,
                        hipStream_t stream);

/* Measurement hook (not part of the method): while the bit of a kernel
 * class is set in kernel_class_mask, every launch of that class is
 * bracketed by two HIP events recorded on the stream it is launched on,
 * together with the algorithmic bytes of the launch (each live input field
 * read once, each output field written once).  While any bit is set, passes
 * launch every kernel on the caller's stream (no fork to the second stream),
 * so that each class is timed alone and not while it shares the device with
 * another.  gr_timing_start clears earlier records; mask 0 switches
 * recording off.  Host-side state shared by all calls of the process. */
gr_status gr_timing_start(unsigned kernel_class_mask);

/* Totals of the records of one kernel class: summed event time (ms), number
 * of launches, summed algorithmic bytes.  Waits for the recorded events. */
gr_status gr_timing_read(int kernel_class, double *total_ms, long *launches, double *alg_bytes);

/* Name of a kernel class ("" when out of range). */
const char *gr_kernel_class_name(int kernel_class);

/* ------------------------------------------------------------------------
 * Batches of independent runs (not a construct of the paper: the same step
 * of Sec 2.3 applied to many grids at once).
 *
 * A batch advances nruns independent runs -- any mix of sizes, dimensions,
 * reconstructions, metrics and resistivities, all with the same IMEX
 * tableau -- by one full step each per call.  Every kernel launch of a step
 * serves all runs that share its template instance: its grid concatenates
 * the runs' block ranges, and each block finds its run through a prefix
 * array.  The batch copies grids, state descriptors and time steps; the
 * arrays they point to stay owned by the caller and must outlive the batch.
 * The batch owns one device block of kernel arguments and, after the first
 * gr_batch_run, one captured HIP graph of a step.  Results of a run do not
 * depend on the other runs of the batch: every cell of a run is computed by
 * the same arithmetic as in gr_step.
 */
typedef struct gr_batch gr_batch;

/* Build a batch.  dt: one time step per run (host array).  tune_cache: NULL
 * keeps the default tiles; "" times the tile candidates of every class of
 * runs (recon, metric, ndim) on these runs and keeps the fastest; a path
 * does the same for the classes not yet listed in that text file and
 * appends its decisions to it.  Allocates the argument block (hipMalloc,
 * with spare room for later updates) and its pinned host staging
 * (hipHostMalloc), a second stream and two events for the forked launches
 * of gr_batch_step and gr_batch_run, and synchronises the stream.
 * GR_EUNSUPPORTED if the runs mix IMEX tableaux. */
gr_status gr_batch_create(gr_batch **batch, const gr_grid *grids, const gr_state *states, const double *dt,
                          int nruns, const char *tune_cache, hipStream_t stream);

/* Replace the time steps (host array of nruns) and rewrite the argument
 * block, ordered on the stream after the work already queued there (a later
 * gr_batch_run captures a new graph). */
gr_status gr_batch_set_dt(gr_batch *batch, const double *dt, hipStream_t stream);

/* Replace the batch's runs by nruns others (a continuous-batching loop
 * admits and retires runs this way; not in the paper, which has no many-run
 * mode).  Same conventions as gr_batch_create, with the batch's IMEX
 * tableau (GR_EUNSUPPORTED otherwise); runs of a class the batch already
 * holds keep that class's tiles, others get the default ones.  The launch
 * list is re-planned on the host and the argument block is rewritten in the
 * batch's device block, ordered on the stream after the work already queued
 * there, without a host synchronisation; the device block is reallocated
 * (after synchronising the stream) only when the new list does not fit its
 * spare room.  Launch the batch on the same stream afterwards (or order the
 * other stream after it).  A captured graph is dropped.  On error the batch
 * holds no launches until the next successful update. */
gr_status gr_batch_update(gr_batch *batch, const gr_grid *grids, const gr_state *states, const double *dt,
                          int nruns, hipStream_t stream);

/* One step of every run, launched eagerly on the stream.  When the runs
 * hold at least 2^20 interior cells together (2^18 while `stream` is being
 * captured), the EMF and face-update launches of each pass run on a second
 * stream the batch owns (created by gr_batch_create, default priority)
 * beside the x/y sweeps, forked from and joined back into `stream` as in
 * gr_imex_stage. */
gr_status gr_batch_step(gr_batch *batch, hipStream_t stream);

/* nsteps steps of every run: on the first call the step is captured into a
 * HIP graph (on a capture stream the batch creates; the launches are never
 * executed there; the fork to the batch's second stream from 2^18 cells)
 * and the graph is then launched nsteps times on the given stream, which may
 * be the null stream.  Asynchronous. */
gr_status gr_batch_run(gr_batch *batch, int nsteps, hipStream_t stream);

/* Launches per step, algorithmic bytes per step (summed over runs, same
 * count as the measurement hook), interior cells summed over runs. */
gr_status gr_batch_stats(const gr_batch *batch, int *launches_per_step, double *alg_bytes_per_step,
                         long *cells);

/* Tiles chosen for one run: x/y-phase tile and z-phase tile indices, named
 * by gr_tile_name(0, xy) and gr_tile_name(1, cz). */
gr_status gr_batch_tiles(const gr_batch *batch, int run, int *xy_tile, int *cz_tile);
const char *gr_tile_name(int which, int tile);

/* Free the batch (argument block, staging buffers, graph and its streams).
 * Waits for the batch's own argument copies and its second stream;
 * otherwise does not synchronise: the caller makes sure no launch of the
 * batch is still pending. */
gr_status gr_batch_destroy(gr_batch *batch);

/* Measurement hooks (not part of the method): a streaming read of `bytes`
 * bytes at src, and a streaming copy of `bytes` bytes from src to dst, with
 * 16-byte loads and stores (device pointers, 16-byte aligned, bytes a
 * multiple of 16, GR_EINVAL otherwise).  sink is one device double that the
 * read never writes for finite data.  Their bandwidth is the practical HBM
 * ceiling the stencil kernels are measured against; asynchronous. */
gr_status gr_stream_read(const void *src, size_t bytes, double *sink, hipStream_t stream);
gr_status gr_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
