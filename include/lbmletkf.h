/*
 * lbmletkf.h -- C ABI of the MI355X (gfx950) forecast-analysis cycle of
 * LBM-LETKF (Hasegawa et al., "Continuous data assimilation of large eddy
 * simulation by lattice Boltzmann method and local ensemble transform Kalman
 * filter").
 *
 * The library runs the continuous-DA workflow of Sec. 3 on one GPU:
 *   (ii) forecast: every ensemble member advances s steps of the D2Q9
 *        lattice Boltzmann equation with BGK relaxation, Smagorinsky eddy
 *        viscosity and a body force (Sec. 2);
 *  (iii) observation: y_m = H(x_m), the macroscopic variables (u, v) or
 *        (rho, u, v) at the observation nodes (Sec. 3, state and
 *        observation vectors);
 *   (iv) analysis: the LETKF of Sec. 3.2.1 with R-localization by the
 *        Gaspari-Cohn weight and multiplicative inflation (Sec. 3.2.2),
 *        solved independently at every grid node and applied directly to
 *        the nine populations.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers named d_* are DEVICE pointers; all other pointers are host.
 * Every device buffer is allocated and owned by the caller; the library never
 * allocates or frees device memory.  `stream` is a hipStream_t passed as
 * void* (NULL = the default stream).  All calls are stream-ordered and return
 * without waiting for the GPU, except lbmletkf_create (which uploads its
 * tables and waits once) and lbmletkf_profile_collect.
 *
 * Lattice units: dx = dt = c = 1.  D2Q9 velocity order
 *   0:(0,0) 1:(1,0) 2:(-1,0) 3:(0,1) 4:(0,-1) 5:(1,1) 6:(-1,-1) 7:(1,-1) 8:(-1,1).
 *
 * State layouts (M x 9 x ny x nx values):
 *   canonical  FP64 f[m][a][y][x] = f_a(x, y) of member m, x fastest: the
 *              pre-collision population of the lattice Boltzmann equation --
 *              the state vector x(xi) = [f_0 .. f_8] the LETKF updates.
 *   storage    the layout the kernels keep between calls (element type per
 *              lbmletkf_storage): f[y][x][a][m], members fastest, where slot
 *              (node (x, y), a, m) holds the canonical f_a of node
 *              (x + c_ax, y + c_ay) of member m, i.e. the post-collision value
 *              streamed by a pull step.  Convert with lbmletkf_import /
 *              lbmletkf_export.
 * Observation vector index q = nvar * k + var, k = observation point,
 * var = (u, v) for nvar = 2 and (rho, u, v) for nvar = 3.
 *
 * Errors: every function returns a status and never aborts.  Arguments are
 * validated on the host before any launch; a failed launch maps to
 * LBMLETKF_EHIP.  lbmletkf_last_error() gives a thread-local message.
 * A context is not thread-safe; two contexts may share a device.
 */
#ifndef LBMLETKF_H
#define LBMLETKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBMLETKF_OK = 0,
    LBMLETKF_EINVAL = -1,      /* invalid parameter value */
    LBMLETKF_ESHAPE = -2,      /* sizes the kernels cannot take */
    LBMLETKF_EHIP = -3,        /* a HIP runtime call or launch failed */
    LBMLETKF_ENONFINITE = -4,  /* non-finite value found by the diagnostics */
    LBMLETKF_EDIVERGED = -5,   /* spread or RMSE above the divergence limit */
    LBMLETKF_EEIG = -6,        /* eigensolver did not converge */
    LBMLETKF_EWORKSPACE = -7,  /* workspace missing, misaligned or too small */
    LBMLETKF_EUNSUPPORTED = -8 /* a valid request the library does not implement */
} lbmletkf_status;

/* Storage of the populations in every state buffer d_f:
 *   F64      FP64 values f_a;
 *   F32_DEV  FP32 deviations f_a - w_a from the lattice weights (the precision
 *            form: half the bytes per step).
 * Canonical buffers (import/export) are always FP64 values f_a.  With F32_DEV
 * the forecast relaxes the deviations in FP32 arithmetic (rho = 1 + sum of
 * the deviations); the analysis forms its Gram matrices on FP32 matrix cores
 * and keeps the eigensolve, the weights and their square root in FP64. */
typedef enum { LBMLETKF_F64 = 0, LBMLETKF_F32_DEV = 1 } lbmletkf_storage;

/* Which eigenproblem the analysis solves (both give the same analysis):
 *   ENSEMBLE     the M x M matrix (M-1)/beta I + dY^T R_loc^-1 dY of Sec. 3.2.2;
 *   OBSERVATION  its l x l dual Z Z^T, Z = R_loc^-1/2 dY (l = local
 *                observations), whose eigenpairs give those of the M x M
 *                matrix: eigenvalue (M-1)/beta + lambda_i with vector
 *                Z^T u_i / sqrt(lambda_i), and (M-1)/beta on the rest;
 *   AUTO         the one with the smaller estimated cost: a per-node cost
 *                table measured on MI355X for each eigenproblem size, summed
 *                over the nodes (the observation route sizes each node's
 *                problem by its own local count, the ensemble route solves
 *                M x M at every node). */
typedef enum {
    LBMLETKF_ROUTE_AUTO = 0,
    LBMLETKF_ROUTE_ENSEMBLE = 1,
    LBMLETKF_ROUTE_OBSERVATION = 2
} lbmletkf_route;

/* Forecast model parameters (Sec. 2). */
typedef struct {
    int32_t nx, ny;    /* grid, doubly periodic; nx, ny >= 3 */
    int32_t members;   /* ensemble size M, 1..64 (M >= 2 for an analysis) */
    double tau0;       /* molecular relaxation time, > 1/2 (nu = (tau0 - 1/2)/3) */
    double cs;         /* Smagorinsky constant C_s >= 0, filter width = dx */
    double mu;         /* linear friction coefficient >= 0 (force -mu u) */
    int32_t storage;   /* lbmletkf_storage */
} lbmletkf_lbm_params;

/* Observing network and analysis parameters (Sec. 3.2, Sec. 4.3). */
typedef struct {
    int32_t n_points;        /* observation points, >= 1 */
    const int32_t* points;   /* host, [n_points][2] = (x, y) node indices; copied */
    int32_t nvar;            /* 2: (u, v); 3: (rho, u, v) */
    double sigma[3];         /* observation-error std per variable (> 0), var order */
    double d_cut;            /* Gaspari-Cohn cutoff in cells; <= 0 or inf: no localization */
    double beta;             /* multiplicative inflation > 0 */
    int32_t route;           /* lbmletkf_route */
} lbmletkf_obs_params;

/* Opaque host-side handles: a context (one ensemble with its observing
 * network, holding parameters and pointers into the caller's workspace) and a
 * batch of contexts (batching form). */
typedef struct lbmletkf_ctx lbmletkf_ctx;
typedef struct lbmletkf_batch lbmletkf_batch;

/* Size of the device workspace a context needs (bytes, 256-byte aligned base). */
lbmletkf_status lbmletkf_workspace_bytes(const lbmletkf_lbm_params* lbm,
                                         const lbmletkf_obs_params* obs, size_t* bytes);

/* Create a context.  d_force: device [2][ny][nx] external acceleration
 * (F_x, F_y) or NULL for none; it is copied into the workspace.  The
 * workspace (caller-owned, >= lbmletkf_workspace_bytes) must stay valid until
 * lbmletkf_destroy.  Builds the per-node local-observation table on the GPU
 * (observations with Gaspari-Cohn weight > 0) and waits for it. */
lbmletkf_status lbmletkf_create(const lbmletkf_lbm_params* lbm, const lbmletkf_obs_params* obs,
                                const double* d_force, void* d_workspace, size_t bytes,
                                void* stream, lbmletkf_ctx** ctx_out);

/* Free the host context (the workspace stays with the caller). */
lbmletkf_status lbmletkf_destroy(lbmletkf_ctx* ctx);

/* Equilibrium state f^eq(rho, u) (Sec. 2 equilibrium) in storage layout.
 * d_rho: [M][ny][nx] or NULL for rho = 1; d_uv: [M][2][ny][nx]. */
lbmletkf_status lbmletkf_init_equilibrium(lbmletkf_ctx* ctx, const double* d_rho, const double* d_uv,
                                          void* d_f, void* stream);

/* canonical -> storage and storage -> canonical (buffers must not overlap). */
lbmletkf_status lbmletkf_import(lbmletkf_ctx* ctx, const double* d_canonical, void* d_f, void* stream);
lbmletkf_status lbmletkf_export(lbmletkf_ctx* ctx, const void* d_f, double* d_canonical, void* stream);

/* Forecast (Sec. 2 LBE): advance every member nsteps >= 0 steps of
 * fused pull-stream + collide, in place on d_f (storage layout; the
 * workspace holds the ping-pong partner).  With FP64 storage and 16 | M,
 * pairs of steps run in one launch (spatial tiles, the intermediate state on
 * chip); the result is bit-identical to nsteps single-step calls. */
lbmletkf_status lbm_ensemble_step(lbmletkf_ctx* ctx, void* d_f, int32_t nsteps, void* stream);

/* Observation operator y = H x (Sec. 3): d_yf[M][nvar * n_points]. */
lbmletkf_status observe(lbmletkf_ctx* ctx, const void* d_f, double* d_yf, void* stream);

/* LETKF analysis (Sec. 3.2.1, Sec. 3.2.2), in place on d_f:
 * ensemble statistics of d_yf against d_yo[nvar * n_points], then at every
 * node the localized ensemble-space problem, its symmetric
 * eigendecomposition, w_bar, dW = [(M-1) P~a]^(1/2) and
 * x_m^a = x_bar + dX (w_bar + dW[:, m]) applied to the nine populations. */
lbmletkf_status letkf_analyze(lbmletkf_ctx* ctx, void* d_f, const double* d_yf, const double* d_yo,
                              void* stream);

/* Ensemble diagnostics into d_diag[LBMLETKF_DIAG_LEN]: RMSE of the
 * ensemble-mean velocity against d_truth_uv ([2][ny][nx]; Sec. 4.3.1), spread,
 * non-finite count, min/max density.  d_truth_uv may be NULL (RMSE = 0). */
#define LBMLETKF_DIAG_LEN 8
#define LBMLETKF_DIAG_RMSE 0
#define LBMLETKF_DIAG_SPREAD 1
#define LBMLETKF_DIAG_NONFINITE 2
#define LBMLETKF_DIAG_RHO_MIN 3
#define LBMLETKF_DIAG_RHO_MAX 4
lbmletkf_status lbmletkf_diagnostics(lbmletkf_ctx* ctx, const void* d_f, const double* d_truth_uv,
                                     double* d_diag, void* stream);

/* Allocation-free variant of lbmletkf_diagnostics, for callers that cannot
 * allocate device memory or hand over a workspace: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  It needs no
 * context: lbm gives the grid, members and storage of d_f (the other fields
 * are validated but unused).  Same kernels and output (bit for bit) as
 * lbmletkf_diagnostics; the per-block partial sums go to a static device array
 * of 4 MiB that the library holds on every GPU it runs on until the process
 * ends, so grids of at most 6,710,848 nodes (LBMLETKF_ESHAPE beyond; 40 bytes
 * per 64 nodes).  Calls no allocator.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (different streams, threads) race;
 * calls ordered on one stream do not.  The first call on a device resolves
 * the array's address there. */
lbmletkf_status lbmletkf_diagnostics_noalloc(const lbmletkf_lbm_params* lbm, const void* d_f,
                                             const double* d_truth_uv, double* d_diag,
                                             void* stream);

/* One forecast-analysis cycle (Sec. 3 workflow (ii)-(iv)):
 * lbm_ensemble_step(nsteps) -> observe -> letkf_analyze.  d_yo: this
 * cycle's observations.  If d_diag is not NULL it receives the forecast
 * diagnostics in d_diag[0..7] and the analysis diagnostics in d_diag[8..15]
 * (d_truth_uv as in lbmletkf_diagnostics): the same quantities as
 * lbmletkf_diagnostics, computed by the analysis kernels from each node's
 * forecast and analysis (no extra pass over the state) and summed over the
 * nodes in a fixed order of their own, so they agree with separate
 * lbmletkf_diagnostics calls to rounding.  The ensemble must have >= 2
 * members (LBMLETKF_EINVAL before any launch otherwise).  With
 * check_every_cycle set (lbmletkf_set_checks) and d_diag != NULL, run_cycle
 * waits for the cycle and returns the status of lbmletkf_check. */
lbmletkf_status run_cycle(lbmletkf_ctx* ctx, void* d_f, int32_t nsteps, const double* d_yo,
                          const double* d_truth_uv, double* d_diag, void* stream);

/* ---- health checks (failure detection) -------------------------------------
 *
 * The failure mode the paper reports is catastrophic filter divergence
 * (Sec. 4.3.3); numerically an ensemble can also turn non-finite, and a node's
 * Jacobi eigensolver can stop at its sweep cap without converging.
 *   max_sweeps         cap of the analysis eigensolvers' Jacobi sweeps, 1..100
 *                      (default 30; converged solves take 4-8); a node that
 *                      reaches it is counted and its weights are used as they are;
 *   diverge_limit      run_cycle's divergence threshold on the analysis RMSE and
 *                      spread (same units as the velocity; <= 0 or inf: none,
 *                      the default);
 *   check_every_cycle  1: run_cycle with d_diag != NULL waits for its
 *                      diagnostics and returns the health status below (one
 *                      stream synchronisation per cycle); 0 (default): no wait,
 *                      call lbmletkf_check when convenient.
 * The batching form takes max_sweeps from each context at lbmletkf_batch_create. */
lbmletkf_status lbmletkf_set_checks(lbmletkf_ctx* ctx, int32_t max_sweeps, double diverge_limit,
                                    int32_t check_every_cycle);

/* Waits for `stream`, then returns the health of the analyses since the last
 * check, in this order: LBMLETKF_ENONFINITE if d_diag (NULL, or a run_cycle
 * diagnostics record of 16 doubles) counts members with a non-finite density
 * or velocity or holds a non-finite RMSE/spread; LBMLETKF_EEIG if any node's
 * eigensolver reached the sweep cap; LBMLETKF_EDIVERGED if the record's
 * analysis RMSE or spread exceeds the divergence limit; else LBMLETKF_OK.  The
 * counts are in lbmletkf_last_error().  Clears the sweep-cap counter. */
lbmletkf_status lbmletkf_check(lbmletkf_ctx* ctx, const double* d_diag, void* stream);

/* Precision form (F32_DEV storage) only: enable = 1 runs the observation
 * route's two per-node ensemble-space contractions of Sec. 3.2.1 -- B = dX Z^T
 * (populations x local observations, summed over the members) and the
 * transform dX (w_bar + dW) written as (B G) Z -- on the BF16 matrix cores
 * with FP32 accumulation, each FP32 operand split into two BF16 parts (three
 * products per tile, ~2^-16 relative per product); 0 (default) keeps them on
 * the FP64 vector units, which is faster on MI355X for these shapes (the
 * per-node products are 9 x l x M with l <= 32).  Nodes with more than 32 local
 * observations always take the vector path.  LBMLETKF_EUNSUPPORTED for FP64
 * storage.  A batch takes the setting at lbmletkf_batch_create (all its
 * contexts must agree). */
lbmletkf_status lbmletkf_set_matrix_core_transform(lbmletkf_ctx* ctx, int32_t enable);

/* Energy spectrum of the ensemble at a report time (Sec. 4.1 shell spectrum;
 * the ensemble's spectrum is the mean of the members' spectra, Sec. 4.3.2):
 * d_E[k] (device, kmax + 1 doubles) for k = 0 .. kmax (0 <= kmax <= n) =
 * M^-1 sum_m sum over the integer wavevectors k' with k - 1/2 <= |k'| < k + 1/2
 * of (|u_hat_m(k')|^2 + |v_hat_m(k')|^2) / 2, u_hat = n^-2 sum_xi u e^{-i k'.xi}
 * (xi in cells, k' in units of 2 pi / n), u = j / rho of member m.  Square
 * grids n <= 2048 only (LBMLETKF_ESHAPE otherwise).  Uses the workspace's
 * ping-pong buffer as scratch (free between calls).  Direct DFT sums in FP64,
 * deterministic; not for the hot loop (about 1 ms at 256^2 x 64 members). */
lbmletkf_status lbmletkf_energy_spectrum(lbmletkf_ctx* ctx, const void* d_f, double* d_E, int32_t kmax,
                                         void* stream);

/* rho, u, v of every node of every member: d_out[M][3][ny][nx]. */
lbmletkf_status lbmletkf_moments(lbmletkf_ctx* ctx, const void* d_f, double* d_out, void* stream);

/* Synthetic observations y^o_q = y_q + sigma_q * eps_q for q < n (OSSE,
 * Sec. 4.3); all three arrays and d_yo are device [n]. */
lbmletkf_status lbmletkf_synth_obs(const double* d_y, const double* d_eps, const double* d_sigma,
                                   double* d_yo, int32_t n, void* stream);

/* Host-only plan (no GPU call): the largest number of observation points in
 * any node's localization support (squared distance < (2 d_cut)^2), the
 * eigenproblem size the analysis will use and its route after AUTO. */
lbmletkf_status lbmletkf_plan(const lbmletkf_lbm_params* lbm, const lbmletkf_obs_params* obs,
                              int32_t* max_local_points, int32_t* eig_size, int32_t* route);

/* Introspection: local-observation points per node (max over nodes), the
 * eigenproblem size the analysis uses and its route (after AUTO). */
lbmletkf_status lbmletkf_info(lbmletkf_ctx* ctx, int32_t* max_local_points, int32_t* eig_size,
                              int32_t* route);

/* Host-only: hist[k] = number of nodes with exactly k observation points in
 * their localization support, for k < len (larger counts are not reported). */
lbmletkf_status lbmletkf_local_histogram(lbmletkf_ctx* ctx, int32_t* hist, int32_t len);

/* ---- differentiation form: reverse mode of the Sec. 2 forecast -----------
 *
 * Observation misfit of a forecast started from d_f0 (storage layout) with
 * n_times observation times, steps_per_obs steps apart:
 *   J(f0, C_s) = sum_{c=1..n_times} sum_m sum_q (H_q(f_m(c steps_per_obs)) - y^o_{c,q})^2,
 * unweighted, H the observation operator of `observe` (the context's points
 * and nvar), f(t) the pre-collision state after t steps of the Sec. 2 LBE with
 * the context's tau0, mu and force.  `cs` is the Smagorinsky constant of the
 * call -- the parameter J is differentiated with respect to -- and replaces
 * the context's value for these two calls only.  d_yo: device
 * [n_times][nvar * n_points] (index q as for letkf_analyze).
 *
 * The adjoint workspace (device, caller-owned, 256-byte aligned, at least
 * lbmletkf_adjoint_workspace_bytes; separate from the context's workspace)
 * holds the state at every observation time (the checkpoints; a checkpoint
 * every steps_per_obs steps), two sets of the steps_per_obs - 1 states between
 * two checkpoints that the reverse sweep recomputes (one interval is
 * recomputed on a library-owned stream while the caller's stream runs the
 * adjoint steps of the next), two FP64 adjoint states and the partial sums.  lbmletkf_misfit_forward writes the checkpoints;
 * lbmletkf_misfit_backward reads them, so call it after a forward call with
 * the same d_f0, cs, steps_per_obs, n_times and workspace (checked; the
 * contents of d_f0, d_yo and the workspace must not change in between, which
 * is not checked).  A backward call leaves the checkpoints intact and may be
 * repeated. */
lbmletkf_status lbmletkf_adjoint_workspace_bytes(const lbmletkf_lbm_params* lbm,
                                                 int32_t n_points, int32_t steps_per_obs,
                                                 int32_t n_times, size_t* bytes);

/* Forward sweep: J into d_J[0] (device) and the checkpoints into d_work.
 * d_f0 is not modified.  steps_per_obs >= 1, n_times >= 1, cs >= 0. */
lbmletkf_status lbmletkf_misfit_forward(lbmletkf_ctx* ctx, const void* d_f0, double cs,
                                        int32_t steps_per_obs, int32_t n_times,
                                        const double* d_yo, double* d_J, void* d_work,
                                        size_t work_bytes, void* stream);

/* Reverse sweep (the adjoint of every step, taken at the recomputed forward
 * states; at |Pi^neq| = 0 the subgradient 0 of the Smagorinsky term is
 * used): d_grad_f0 (device, canonical FP64 [M][9][ny][nx], overwritten) =
 * dJ/df0 with respect to the canonical populations of d_f0, and, if
 * d_grad_cs is not NULL, d_grad_cs[0] = dJ/dC_s.  For F32_DEV storage the
 * derivative is that of the FP64 step evaluated at the stored states (the
 * rounding of the stored deviations counts as the identity).  d_grad_f0 must
 * not overlap d_f0, d_yo or the workspace.  The observation points must be
 * distinct (LBMLETKF_EUNSUPPORTED otherwise). */
lbmletkf_status lbmletkf_misfit_backward(lbmletkf_ctx* ctx, const void* d_f0, double cs,
                                         int32_t steps_per_obs, int32_t n_times,
                                         const double* d_yo, void* d_work, size_t work_bytes,
                                         double* d_grad_f0, double* d_grad_cs, void* stream);

/* ---- batching form: many independent problems per cycle -----------------
 *
 * A batch binds n contexts (problems of any grid, ensemble size and observing
 * network; members >= 2 must divide 256 and every context must have the same
 * storage) to their state buffers d_f[k] and advances all of them one cycle
 * (Sec. 3 workflow (ii)-(iv), as run_cycle without diagnostics) per call:
 *   - the forecast of all problems is one launch per step over the
 *     concatenated (problem, node tile) list, or one launch per pair of steps
 *     over the concatenated (problem, tile, member group) blocks;
 *   - H and the observation statistics run per problem;
 *   - the analyses are grouped across problems by eigenproblem size (one
 *     eigen + one apply launch, or one ensemble-route launch, per size),
 *     spread over the launch stream and three batch-owned side streams;
 *   - with use_graph, the whole cycle is captured once as a hipGraph and
 *     replayed by every lbmletkf_batch_run_cycle.
 * The results are those of run_cycle on each context (same kernels' per-node
 * arithmetic).  The batch uses each context's workspace (ping-pong partner,
 * tables, statistics) and its own workspace (caller-owned, 256-byte aligned,
 * >= lbmletkf_batch_workspace_bytes) for the per-problem parameters, forecast
 * task lists, observation slots, the analysis node lists, wave lists and G
 * buffers.  The contexts, state buffers and both workspaces must outlive the
 * batch; a context must not run other calls concurrently with its batch. */
typedef struct {
    int32_t forecast_blocks;    /* blocks of the forecast launch, 1..2^20 walking the tile
                                   list with a fixed stride, or 0: one block per tile */
    int32_t tile_rows;          /* forecast tile = tile_rows x 256 / (M / V) nodes, 1..64; V = 2
                                   members per thread with FP32 storage and even M, else 1 */
    int32_t bucket_granularity; /* eigenproblem sizes rounded up to multiples of 2, 4 or 8 */
    int32_t use_graph;          /* 1: capture the cycle once as a hipGraph and replay it */
    int32_t steps_per_launch;   /* 1: the launch above per step; 2: pairs of steps in one launch
                                   over every problem's (6 x 6 tile, 16-member group) blocks, the
                                   first step's results kept on chip (needs 16 | members in every
                                   problem; the same bits as single steps) */
    int32_t analysis_queue;     /* 0: per observation-route group one eigen and one apply launch
                                   with a block per (problem, node tile) item; 1: persistent
                                   launches (16 wavefronts per CU) whose blocks take the items
                                   from per-XCD queues in the batch workspace, four at a time;
                                   the same bits (measured ~4x slower on the twelve-problem
                                   batch: the loop costs the eigen kernels occupancy) */
} lbmletkf_batch_config;

lbmletkf_status lbmletkf_batch_workspace_bytes(lbmletkf_ctx* const* ctxs, int32_t n, size_t* bytes);

/* Create a batch of n contexts with states d_f[k] (device, storage layout) and
 * nsteps forecast steps per cycle.  ctxs and d_f are host arrays of n pointers.
 * cfg may be NULL: {one block per tile, 4 tile rows, granularity 2, graph, two steps per
 * launch where every problem allows it, else one, no analysis queue}.  Waits for its setup copies and,
 * with use_graph, captures the cycle. */
lbmletkf_status lbmletkf_batch_create(lbmletkf_ctx* const* ctxs, void* const* d_f, int32_t n,
                                      int32_t nsteps, const lbmletkf_batch_config* cfg,
                                      void* d_workspace, size_t bytes, void* stream,
                                      lbmletkf_batch** batch_out);

/* One cycle of every problem.  d_yo: host array of n device pointers, d_yo[k]
 * = this cycle's observations of problem k ([nvar * n_points], copied in on
 * `stream` before the cycle). */
lbmletkf_status lbmletkf_batch_run_cycle(lbmletkf_batch* batch, const double* const* d_yo, void* stream);

lbmletkf_status lbmletkf_batch_get_config(lbmletkf_batch* batch, lbmletkf_batch_config* cfg);

/* Re-tile, re-group and (with use_graph) re-capture; waits for its setup. */
lbmletkf_status lbmletkf_batch_set_config(lbmletkf_batch* batch, const lbmletkf_batch_config* cfg,
                                          void* stream);

/* Autotuner: times every (forecast_blocks in {256, 512, 1024, 2048, 0}) x
 * (tile_rows in {1, 2, 4, 8}) forecast step, the two-step launch (per step, when
 * every problem allows it) and every bucket granularity {2, 4, 8} of the analysis
 * (reps timed runs each, HIP events; analysis_queue keeps its setting), then applies
 * the fastest with use_graph = 1.  Runs on the contexts' ping-pong partner
 * buffers: the bound states are not modified.  Outputs (any may be NULL): the
 * chosen configuration, its forecast ms per step and analysis ms per cycle. */
lbmletkf_status lbmletkf_batch_tune(lbmletkf_batch* batch, int32_t reps, lbmletkf_batch_config* best,
                                    double* forecast_ms, double* analysis_ms, void* stream);

lbmletkf_status lbmletkf_batch_destroy(lbmletkf_batch* batch);

/* Per-stage GPU timing with HIP events on the launch stream.  enable = 1:
 * every launch is bracketed by an event pair; enable = 2: one pair around the
 * forecast steps of each lbm_ensemble_step call (its launch count = the
 * steps) and one around each analysis, nothing else (an event pair costs
 * the stream a few microseconds, so level 2 keeps the timing live at a small
 * fraction of the per-launch cost; its per-launch figure includes the gaps
 * between the back-to-back launches); 0 turns timing off.  Other values:
 * LBMLETKF_EINVAL.  lbmletkf_profile_collect waits for the pairs and returns,
 * per stage, the summed milliseconds and launch counts (stage 0 counts
 * forecast steps: a launch that takes two steps counts 2), then clears the
 * record.  Stages: 0 stream-collide (also the steps of the misfit sweeps),
 * 1 observe, 2 obs statistics, 3 analysis (all node groups of one call),
 * 4 diagnostics, 5 adjoint step, 6 misfit terms. */
#define LBMLETKF_NSTAGES 7
lbmletkf_status lbmletkf_set_profiling(lbmletkf_ctx* ctx, int32_t enable);
lbmletkf_status lbmletkf_profile_collect(lbmletkf_ctx* ctx, double* ms, int64_t* counts);

const char* lbmletkf_status_string(int32_t status);
const char* lbmletkf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBMLETKF_H */
