/*
 * sdd.h -- C ABI of the MI355X (gfx950) Monte-Carlo interface solver for the
 * 2-D TE magnetotelluric equation.
 *
 * Method (Bihlo, Farquharson, Haynes, Loredo-Osti, arXiv:1603.09311):
 *   TE mode of the quasi-static Maxwell equations (Sec. 2.1, Eq. 1) in model
 *   length units L:  Laplace(E) = i alpha(y, z) E,  alpha = omega mu0 sigma L^2,
 *   with Dirichlet data g on the rectangle Omega (Sec. 2.1).  At each
 *   interface node x the library evaluates the Feynman-Kac representation
 *   (Sec. 2.2, Eqs. 5a/5b, 7-8)
 *       E(x) = Exp[ g(X_tau) exp(-i S) ],  S = (1/2) int_0^tau alpha(X_s) ds,
 *   by Monte-Carlo over Euler-Maruyama Brownian walks (Sec. 3.1, Eq. 13) that
 *   stop at the first exit from Omega, detected with the Brownian-bridge
 *   hitting test (Sec. 3.1, Eq. 14, applied to the outer boundary), and
 *   reduces each node's samples to the MC estimate (Sec. 3.1, estimator) with
 *   its variance and standard error.
 *
 * Conventions: y to the right, z downward; walls are named top (z = z_lo),
 * right (y = y_hi), bottom (z = z_hi), left (y = y_lo).
 *
 * Every call returns an sdd_status; no exception crosses the ABI; a failing
 * call leaves a thread-local message readable with sdd_last_error().
 * Ownership: the caller owns every host buffer; inputs are copied before a
 * call returns; result buffers passed to sdd_submit must stay valid until
 * sdd_wait/sdd_poll report completion (or cancellation).  Device memory is
 * the caller's workspace given to sdd_create: the library never allocates
 * device memory itself, and its HBM admission budget is that workspace.
 */
#ifndef SDD_H
#define SDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdd_ctx *sdd_ctx_t;
typedef uint32_t sdd_model_t;
typedef uint64_t sdd_ticket_t;

typedef enum {
    SDD_OK = 0,
    SDD_E_INVALID = -1,    /* bad argument; see sdd_last_error() */
    SDD_E_NOMEM = -2,      /* the request does not fit in the workspace */
    SDD_E_DEVICE = -3,     /* a HIP call failed */
    SDD_E_BUSY = -4,       /* model in use / ticket not finished */
    SDD_E_NOTFOUND = -5,   /* unknown model or ticket */
    SDD_E_TIMEOUT = -6,    /* sdd_wait timed out */
    SDD_E_CANCELLED = -7   /* the ticket was cancelled */
} sdd_status;

/* Arithmetic of the walk.  SDD_FP64: every step in FP64 (the plain form:
 * the decisions of an FP64 reference on the same streams, its logarithm and
 * sine/cosine of the uniforms within 2 ulp of the exact values).
 * SDD_FP32_MIXED: positions, normals, exit test and region lookup in FP32,
 * the phase integral as exact per-region step counts formed in FP64 (models
 * of air plus at most one half-space, box or triangle) or as an exact 64-bit
 * fixed-point sum of each region's phase per step (other models; each
 * region's phase rounded once, to within 2^-30 of the largest), the per-path weight
 * and the per-node reduction in FP64.  Both precisions draw the same random
 * numbers. */
typedef enum { SDD_FP64 = 0, SDD_FP32_MIXED = 1 } sdd_precision;

/* Conductivity primitives (Sec. 2.2: piecewise-constant sub-domains).
 * A model is an ordered list; a point belongs to the first primitive that
 * contains it, else to the background.
 *   SDD_HALF_Z_LT : z < v[0]                         (e.g. air above z = 0)
 *   SDD_HALF_Y_LT : y < v[0]
 *   SDD_BOX       : v[0] <= y < v[1] and v[2] <= z < v[3]
 *   SDD_TRIANGLE  : closed triangle (v[0],v[1]), (v[2],v[3]), (v[4],v[5]) */
typedef enum { SDD_HALF_Z_LT = 0, SDD_HALF_Y_LT = 1, SDD_BOX = 2, SDD_TRIANGLE = 3 } sdd_region_kind;

#define SDD_MAX_REGIONS 16

typedef struct {
    int32_t kind;          /* sdd_region_kind */
    int32_t reserved;      /* 0 */
    double v[6];           /* geometry, model length units */
    double sigma;          /* conductivity, S/m (>= 0; 0 = air) */
} sdd_region;

/* A conductivity model on Omega = [y_lo, y_hi] x [z_lo, z_hi]. */
typedef struct {
    double y_lo, y_hi, z_lo, z_hi;
    double length_unit_m;      /* metres per model length unit (> 0) */
    double sigma_background;   /* S/m, >= 0 */
    uint32_t n_regions;        /* <= SDD_MAX_REGIONS */
    const sdd_region *regions; /* copied by sdd_model_create */
} sdd_model_desc;

/* One interface solve: the paper's problem statement (model, frequency,
 * boundary data, nodes, paths per node, time step) plus the random streams.
 *   alpha_r = (2 pi freq_hz) mu0 sigma_r L^2 with mu0 = 4 pi 1e-7 H/m, or,
 *   when freq_hz == 0, alpha_r = alpha_direct * sigma_r (non-dimensional).
 * Random numbers: Philox4x32-10 keyed by `seed`; the normal pair of step n of
 * path p at node j comes from the call with counter (n/2, p, j, 2 stream)
 * (words 0,1 for even n, 2,3 for odd n); the bridge uniforms of step n from
 * counter (n, p, j, 2 stream + 1).  A node's paths are therefore the same
 * realisations in every batch, mix, precision and kernel. */
typedef struct {
    sdd_model_t model;
    int32_t precision;          /* sdd_precision */
    double freq_hz;
    double alpha_direct;
    /* Dirichlet data: 4 walls (top, right, bottom, left) x g_samples x
     * (re, im), each wall sampled at g_samples equispaced points from its
     * low to its high end (top/bottom along y, left/right along z);
     * linear interpolation in between. */
    const double *g_tables;
    uint32_t g_samples;         /* >= 2 */
    uint32_t n_nodes;
    const double *nodes_yz;     /* n_nodes x (y, z), strictly inside Omega */
    const uint32_t *path_begin; /* nullable: first path index per node (default 0) */
    const uint32_t *path_count; /* nullable: paths per node (default paths_uniform) */
    uint32_t paths_uniform;
    double dt;                  /* Euler-Maruyama step; 7 sqrt(dt) < half the shorter side */
    uint64_t seed;
    uint32_t stream;            /* < 2^31 */
    uint32_t max_steps;         /* proposals per path before it counts as unfinished; 0 = 2e9 */
    uint32_t flags;             /* 0, or SDD_FLAG_NO_SIGMA_GRID | SDD_FLAG_EXIT_NAIVE | SDD_FLAG_NO_LDS_GRID */
    uint32_t reserved;          /* 0 */
    double target_rel_se;       /* 0: fixed paths.  > 0: a 4096-path pilot per node, then
                                   extended on the same streams to N = ceil((s/(target*|g|inf))^2)
                                   (capped at 2^20), s^2 = var_re + var_im of the pilot.  The
                                   target is relative to |g|inf, the largest modulus in g_tables,
                                   not to each node's own estimate: SE <= target |g|inf */
} sdd_request;

/* Request flags.  SDD_FLAG_NO_SIGMA_GRID: an FP32-mixed request whose model
 * has no specialised walker (more than two primitives, or other than air plus
 * one half-space, box or triangle) looks regions up by the loop over its
 * primitives instead of the sigma grid: a grid of 256 cells along the longer
 * side, each holding its region or the boundary inequality that crosses it
 * (a cell crossed by two holds both, one crossed by more uses the loop).
 * When every request of a launch shares one grid (the same model, time step
 * and frequency) and the grid has at most 255 distinct cells, each block of
 * the walker stages it in LDS (a byte per cell and a table of the distinct
 * cells); otherwise the walker reads it from global memory.  SDD_FLAG_NO_LDS_GRID keeps a request's
 * grid in global memory.  All three give the same region for every point,
 * hence the same results; LDS is the fastest, the loop the slowest. */
enum { SDD_FLAG_NO_SIGMA_GRID = 1, SDD_FLAG_EXIT_NAIVE = 2, SDD_FLAG_NO_LDS_GRID = 4 };

/* SDD_FLAG_EXIT_NAIVE: an ablation of the exit rule of Sec. 3.1.  A path
 * leaves the domain only when a proposal lands outside it (the crossing case
 * of Eq. 14); the Brownian-bridge test for a path that left and came back
 * within a step is skipped.  Exit times are then biased late by O(sqrt(dt))
 * and so is the field; the default (flag clear) applies both cases.  Both
 * precisions, all request kinds. */

/* Per-path record (node-major, path order), for inspection and tests. */
typedef struct {
    double w_re, w_im;   /* g(X_tau) exp(-i S) */
    double tau;          /* exit-time estimate (n + f) dt; -1 if unfinished */
    uint32_t steps;      /* proposals drawn */
    int32_t wall;        /* 0 top, 1 right, 2 bottom, 3 left; -1 unfinished */
} sdd_path_record;

/* Diagnostics of one solve, written when sdd_result.diag is not NULL.
 *   rho_dt        the largest phase one full step adds, max over regions of
 *                 alpha_r dt / 2 (kappa walk: max_i |lambda_i| dt).  The
 *                 paper chooses dt proportional to dx^2 (Sec. 4.1) so that
 *                 the phase is resolved; rho_dt > 0.1 sets
 *                 SDD_DIAG_DT_UNRESOLVED: the result carries a time-step bias
 *                 that the Monte-Carlo error does not show.
 *   g_norm        |g|inf, the largest modulus in the request's tables (the
 *                 scale of target_rel_se).
 *   se_over_gnorm the largest se (third column of sdd_result.se) over the
 *                 nodes divided by g_norm. */
typedef struct {
    double rho_dt;
    uint32_t flags;          /* SDD_DIAG_* */
    uint32_t reserved;
    double g_norm;
    double se_over_gnorm;
} sdd_diag;
#define SDD_DIAG_DT_UNRESOLVED 1u

/* Results per node (arrays of n_nodes rows; every pointer but `mean` is nullable). */
typedef struct {
    double *mean;            /* n x 2: re, im */
    double *var;             /* n x 3: var_re, var_im, cov (divisor N - 1) */
    double *se;              /* n x 3: se_re, se_im, se = sqrt((var_re + var_im)/N) */
    uint64_t *paths_done;    /* n: finished paths N */
    uint64_t *steps;         /* n: proposals drawn, all paths */
    uint64_t *unfinished;    /* n: paths that reached max_steps */
    double *mean_exit_time;  /* n */
    sdd_path_record *path_records; /* sum of path counts; fixed-path requests only */
    sdd_diag *diag;          /* one per request */
} sdd_result;

/* Launch shape of the persistent walker (0 = automatic). */
typedef struct {
    uint32_t block_threads;   /* multiple of 64, <= 256 */
    uint32_t blocks_per_cu;
    uint32_t tile_paths;      /* paths per tile (work unit claimed by a wave) */
    uint32_t slice_iters;     /* served mode: pairs of steps per wave per slice (the FP32
                                 walker takes two pairs per iteration: rounded up to even) */
    uint32_t refill_every;    /* refill idle lanes every k pairs of steps (power of 2, <= 64;
                                 the FP32 walker at most every second pair) */
} sdd_tuning;

/* Context on device `device` (HIP ordinal) with a caller-owned device
 * workspace of workspace_bytes (256-byte aligned) and a HIP stream
 * (hipStream_t, may be NULL for the default stream). */
sdd_status sdd_create(int device, void *workspace_dev, size_t workspace_bytes, void *hip_stream,
                      sdd_ctx_t *out);
sdd_status sdd_destroy(sdd_ctx_t ctx);

/* Copy a conductivity model into the workspace, where it stays resident
 * until sdd_model_destroy (SDD_E_BUSY while a submitted request uses it). */
sdd_status sdd_model_create(sdd_ctx_t ctx, const sdd_model_desc *desc, sdd_model_t *out);
sdd_status sdd_model_destroy(sdd_ctx_t ctx, sdd_model_t model);

/* Blocking solve of one request by the persistent walker. */
sdd_status sdd_solve(sdd_ctx_t ctx, const sdd_request *req, sdd_result *res);

/* Blocking solve of n requests with uneven node counts, path counts,
 * frequencies, models and precisions in one persistent launch. */
sdd_status sdd_solve_batch(sdd_ctx_t ctx, uint32_t n, const sdd_request *reqs, sdd_result *res);

/* The plain form: FP64, one kernel launch per node, one thread per path,
 * no refill (req->precision is ignored).  Same streams, same records. */
sdd_status sdd_solve_plain(sdd_ctx_t ctx, const sdd_request *req, sdd_result *res);

/* Served mode: requests are queued, admitted while the workspace has room,
 * and walked together in time slices of the persistent kernel (continuous
 * batching); a request that arrives while others run joins at the next
 * slice. */
sdd_status sdd_submit(sdd_ctx_t ctx, const sdd_request *req, sdd_result *res, sdd_ticket_t *out);
sdd_status sdd_poll(sdd_ctx_t ctx, sdd_ticket_t t, int *done);
sdd_status sdd_wait(sdd_ctx_t ctx, sdd_ticket_t t, int64_t timeout_ns);   /* < 0: forever */
sdd_status sdd_cancel(sdd_ctx_t ctx, sdd_ticket_t t);

/* Set or read the context's tuning.  set: block_threads not a multiple of
 * 64 or above 256, blocks_per_cu above 64, tile_paths above 2^24 or
 * refill_every not a power of 2 up to 64 give SDD_E_INVALID; zeros select
 * the defaults (256, occupancy, 512, 4096, 1).  Waits for the running launch
 * sequence; served requests pick the new tuning up at their next slice. */
sdd_status sdd_set_tuning(sdd_ctx_t ctx, const sdd_tuning *t);
sdd_status sdd_get_tuning(sdd_ctx_t ctx, sdd_tuning *t);

/* One timed trial of sdd_autotune. */
typedef struct {
    sdd_tuning tuning;
    double walk_ms;            /* walk kernel duration (HIP events) */
    double walk_steps_per_s;   /* proposals drawn / walk_ms */
} sdd_tune_trial;

/* Autotuner: times the persistent walker on a sample of *req (the request's
 * nodes, at most sample_paths paths each; 0 = enough paths to occupy every
 * resident lane about four times) under a sequence of tunings and keeps the
 * fastest.  Starting from the context's tuning it sweeps block_threads
 * {256, 128, 64}, then tile_paths {128, 512, 2048, 8192}, then refill_every
 * {1, 2, 4, 8}, each with the others held at the best so far.  Results of
 * every solve are bitwise the same under any tuning (a path's random numbers
 * are indexed by seed, stream, node, path and step, its record has a fixed
 * slot, and each node is reduced in path order), so tuning changes speed
 * only.  On success the context keeps the chosen tuning and copies it to
 * *chosen (may be NULL); slice_iters is not touched.  Up to max_trials
 * trials are written to trials (may be NULL when max_trials is 0) and their
 * count to *n_trials (may be NULL).  On failure the previous tuning is
 * restored.  Blocks the calling thread for the trials (each about one
 * sample solve). */
sdd_status sdd_autotune(sdd_ctx_t ctx, const sdd_request *req, uint32_t sample_paths, sdd_tuning *chosen,
                        sdd_tune_trial *trials, uint32_t max_trials, uint32_t *n_trials);

/* Timing of the most recent walk launch on this context, measured with HIP
 * events on the context's stream around the walk kernel alone (for a batch
 * replay: around the whole replayed graph, of which the walks are all but a
 * fraction of a percent). */
typedef struct {
    double last_walk_ms;          /* duration of the last walk kernel (persistent or plain) */
    double last_reduce_ms;        /* duration of the last reduction kernel */
    uint64_t last_walk_steps;     /* proposals drawn by that walk launch */
    uint64_t last_walk_paths;     /* paths walked by that launch */
    uint32_t last_blocks, last_threads;  /* launch shape of the last persistent walk */
    uint64_t launches;            /* walk launches since sdd_create */
    /* served mode, since sdd_create */
    uint32_t served_in_flight_max;  /* most requests walked together in one slice */
    uint32_t served_waits;          /* requests that waited in the queue for workspace */
    uint32_t served_requeues;       /* target-SE requests whose extension did not fit next to the
                                       others: they gave their workspace back and were walked again
                                       in one pass, all paths, once admitted (same results) */
    uint32_t reserved;
    double served_walk_ms;          /* walk kernel time of every served slice so far (HIP events),
                                       for the GPU-busy fraction of a served stream */
    uint64_t served_slices;         /* served slices launched so far */
} sdd_stats;

sdd_status sdd_get_stats(sdd_ctx_t ctx, sdd_stats *out);

/* A prepared batch: the requests' inputs stay resident in the workspace and
 * the launch sequence (counter reset, one persistent walk per precision, the
 * per-node reduction, the copy of the results to pinned host memory) is
 * captured once into a HIP graph; sdd_batch_run replays it on the context's
 * stream and blocks until the results are in `res` (one sdd_result per
 * request, as for sdd_solve_batch).  Fixed-path requests only.  The batch
 * holds its workspace until sdd_batch_destroy.  Every replay gives bitwise
 * the results of sdd_solve_batch on the same requests. */
typedef struct sdd_batch *sdd_batch_t;
sdd_status sdd_batch_create(sdd_ctx_t ctx, uint32_t n, const sdd_request *reqs, sdd_batch_t *out);
sdd_status sdd_batch_run(sdd_batch_t batch, sdd_result *res);
sdd_status sdd_batch_destroy(sdd_batch_t batch);

/* Multi-frequency solve (one walk, many frequencies).  In the TE equation
 * the walk itself does not depend on the frequency: only the phase rate
 * alpha = omega mu0 sigma L^2 does, and the phase of a path is linear in it
 * (Feynman-Kac weight exp(-i S), S = 1/2 int alpha ds: Sec. 2.2, and the
 * estimator of Sec. 3.1).  So one walk at the request's frequency, recording
 * each path's phase S and exit point, gives for every frequency f_k the
 * weight g_k(exit point) exp(-i S f_k / f) of the same path: the per-node
 * estimates at all frequencies come from the same paths (correlated across
 * frequencies) and each equals, up to rounding, what sdd_solve returns for
 * the request at f_k with the same seed and stream.
 *   req        fixed-path request; its freq_hz (or alpha_direct when that is
 *              > 0) must be > 0 and sets the walk's phase scale; its own
 *              g_tables are validated but not used for any result.
 *   freqs      n_freq frequencies in Hz (alpha values when the request gives
 *              alpha directly), each finite and > 0.
 *   g_tables   n_freq tables, each laid out as sdd_request.g_tables with the
 *              request's g_samples.
 *   res        n_freq results (per node as sdd_solve; path_records must be
 *              NULL).
 * Errors: SDD_E_INVALID for the above, SDD_E_NOMEM, SDD_E_DEVICE. */
sdd_status sdd_solve_multi_freq(sdd_ctx_t ctx, const sdd_request *req, uint32_t n_freq, const double *freqs,
                                const double *const *g_tables, sdd_result *res);

/* TE apparent resistivity and phase at n sites from the field at three
 * points per site: (y, z - h), (y, z), (y, z + h), z positive down (Sec. 2.1,
 * Eqs. 2-3): H^x = -(1 / (i omega mu0)) dE/dz with the centred difference
 * (E(z + h) - E(z - h)) / (2 h L), then rho_a = |E / H^x|^2 / (omega mu0) in
 * ohm m and phi = arg(E / H^x) in degrees, E = E(z).
 *   e_minus, e_mid, e_plus  n x (re, im) each (host, caller-owned);
 *   h                       offset in model length units (> 0);
 *   length_unit_m           metres per model length unit (> 0);
 *   freq_hz                 > 0;
 *   rho_a, phase_deg        n each (host, caller-owned), written.
 * Host arithmetic only (no device work).  SDD_E_INVALID for NULL arrays with
 * n > 0 or a non-positive h, length unit or frequency.  A site whose
 * difference is exactly zero gets rho_a = +inf and phase NaN. */
sdd_status sdd_mt_te_response(uint32_t n, const double *e_minus, const double *e_mid, const double *e_plus, double h,
                              double length_unit_m, double freq_hz, double *rho_a, double *phase_deg);

/* sdd_mt_te_response for sites on a horizontal conductivity jump (the
 * air-ground surface: sigma_jump = the ground's sigma).  On either side of
 * the jump Laplace E = i omega mu0 sigma E (Sec. 2.1, Eq. 1 with z in
 * metres) and d2E/dy2 is continuous along it, so d2E/dz2 jumps by
 * i omega mu0 sigma_jump E(z), sigma_jump = sigma(below) - sigma(above) in
 * S/m.  The centred difference across the jump then carries the first-order
 * term (h L / 4) i omega mu0 sigma_jump E(z); it is subtracted:
 *   dE/dz = (E(z + h) - E(z - h)) / (2 h L) - (h L / 4) i omega mu0 sigma_jump E(z),
 * which leaves an error of second order in h (on an exact half-space under
 * air at 10 Hz, 100 ohm m: rho_a -0.13% and phase -0.57 degrees at
 * h = 400 m, against +13% and +3.2 degrees uncorrected), so that a larger h
 * (a Monte-Carlo difference quotient whose noise falls like 1 / h) keeps a
 * small bias.  The two outer points must lie in the two layers next to the
 * jump.  Arguments, errors and outputs as sdd_mt_te_response; sigma_jump
 * must be finite (SDD_E_INVALID otherwise); sigma_jump = 0 gives
 * sdd_mt_te_response's results bit for bit.  Host arithmetic only. */
sdd_status sdd_mt_te_response_jump(uint32_t n, const double *e_minus, const double *e_mid, const double *e_plus,
                                   double h, double length_unit_m, double freq_hz, double sigma_jump, double *rho_a,
                                   double *phase_deg);

/* Sub-domain solver (Sec. 3.2): RBF-FD on a rectangular grid of ny x nz
 * nodes (y[0..ny), z[0..nz) strictly increasing, model length units) with the
 * multiquadric phi(r) = sqrt(1 + (eps r)^2) and, at every interior node, the
 * 9-node stencil of the node and its 8 grid neighbours; separate weights for
 * d2/dy2 and d2/dz2 (exact on phi centred at each stencil node).  Solves
 * Laplace E = i alpha E (the TE equation in model units, alpha = omega mu0
 * sigma L^2 of the sub-domain) for the interior values, the boundary values
 * (the grid's first and last rows and columns: walk results on interfaces,
 * Dirichlet data on the outer boundary) given.
 *   field  ny * nz complex values, (re, im) interleaved, y fastest:
 *          node (i, j) at field[2 (j ny + i)]; boundary entries are read,
 *          interior entries are written.  Host memory, caller-owned.
 *   eps    > 0: the shape parameter, in inverse model length units, at every
 *          node (the paper's choice, 1/2000 per metre for 50-300 m cells);
 *          < 0: eps h = |eps| at every node, h the largest grid spacing next
 *          to it (for graded grids).  The stencil systems are solved in
 *          extended precision; eps h below about 0.01 is ill-conditioned.
 * Host only.  SDD_E_INVALID for a grid smaller than 3 x 3 or above 2^24
 * interior nodes, non-increasing coordinates, a non-finite boundary value,
 * alpha < 0, eps = 0 or not finite, or a singular system. */
sdd_status sdd_rbffd_solve(uint32_t ny, uint32_t nz, const double *y, const double *z, double alpha, double eps,
                           double *field);

/* The stencil weights sdd_rbffd_solve uses: for interior node (i, j) (row
 * r = (j - 1)(ny - 2) + (i - 1)) the 9 weights of d2/dy2 and of d2/dz2 at
 * w[9 r + k], k = 3 (dj + 1) + (di + 1) for the neighbour (i + di, j + dj).
 * Host only; errors as above. */
sdd_status sdd_rbffd_weights(uint32_t ny, uint32_t nz, const double *y, const double *z, double eps, double *w_yy,
                             double *w_zz);

/* Discontinuous kappa (Secs. 2.2 and 3.1): the walk for
 *   (1/2) div(kappa grad u) - lambda u = 0 in Omega, u = g on its boundary
 * (Eq. 9), kappa > 0 and lambda constant on each side of one vertical
 * interface y = y_if (the configuration of Eqs. 10-12; with kappa = 2/sigma
 * and lambda = i omega mu it is the TM mode, with kappa constant the TE mode
 * in the form of Eq. 9).  FP64.  A step that reaches the interface resumes
 * from a uniform point of a disc of radius h = sqrt(kappa_i dt), kappa_i of
 * the side the step started on, that touches the interface from side i
 * (probability kappa_i / (kappa_i + kappa_j), Eq. 12) or from side j; the
 * step's time is split between the occupation times T_0, T_1 as in Sec. 3.1
 * (shares summing to dt), and a path's value is
 * g(exit point) exp(-(lambda_0 T_0 + lambda_1 T_1)).  A disc point outside
 * Omega ends the walk at the nearest boundary point.  With equal kappa the
 * proposal is kept and the step's time goes to the side of the proposal.
 * Random numbers: Philox4x32-10 keyed by `seed`; step n of path p at node j
 * takes its normals from counter (n/2, p, j, 4 stream) (words 0,1 for even
 * n, 2,3 for odd n), its bridge and side uniforms from (n, p, j,
 * 4 stream + 1) (outer bridge y, z: words 0, 1; interface bridge: word 2;
 * side: word 3) and its disc point from (n, p, j, 4 stream + 2) (radius:
 * word 0, angle: word 1). */
typedef struct {
    double y_lo, y_hi, z_lo, z_hi;  /* Omega; z_lo is the top wall */
    double y_if;                    /* y_lo < y_if < y_hi */
    double kappa[2];                /* side 0: y < y_if, side 1: y >= y_if; finite, > 0 */
    double lambda_re[2];            /* finite, >= 0 */
    double lambda_im[2];            /* finite */
    const double *g_tables;         /* host: 4 walls x g_samples x (re, im), as in sdd_request */
    uint32_t g_samples;             /* >= 2 */
    uint32_t n_nodes;
    const double *nodes_yz;         /* host: n_nodes x (y, z), strictly inside Omega */
    const uint32_t *path_begin;     /* host, nullable: first path index per node (default 0) */
    const uint32_t *path_count;     /* host, nullable: paths per node (default paths_uniform) */
    uint32_t paths_uniform;
    uint32_t max_steps;             /* steps before a path counts as unfinished; 0 = 2e9 */
    double dt;                      /* 7 sqrt(max kappa dt) < half the shorter side */
    uint64_t seed;
    uint32_t stream;                /* < 2^30 */
    uint32_t precision;             /* SDD_FP64, or SDD_FP32_MIXED: positions, normals and tests in FP32
                                       (hardware log2, sqrt, sin, cos), the same random numbers, full
                                       steps counted per side, interface time shares and the weight in
                                       FP64 */
} sdd_kappa_request;

/* Solve a discontinuous-kappa request on the context's stream.  Results per
 * node in `res` as for sdd_solve (path_records, when not NULL, receive every
 * path's record: w = the path's value).  Inputs are host memory and are
 * copied; the call returns when the results are on the host.  SDD_FP64 is
 * the parity form (the arithmetic of a plain FP64 reading of the scheme);
 * SDD_FP32_MIXED walks the same paths up to FP32 rounding.
 * Errors: SDD_E_INVALID (NULL pointers, a value outside the ranges above, a
 * node not strictly inside Omega, a node with no paths or whose path range
 * passes 2^32, more than 2^40 paths), SDD_E_NOMEM (workspace), SDD_E_DEVICE. */
sdd_status sdd_solve_kappa(sdd_ctx_t ctx, const sdd_kappa_request *req, sdd_result *res);

/* For callers that cannot allocate device memory while they run (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): sdd_solve without the context's workspace.  Every device
 * buffer the solve needs beyond the request's inputs and the results (the
 * request descriptor, claim and done counters, boundary tables, nodes, sigma
 * grid, tiles, one 32-byte record per path, reduction jobs and rows) is
 * carved from a static device array of SDD_NOALLOC_SCRATCH_BYTES (64 MiB)
 * that the library holds on each GPU it runs on until the process ends; the
 * call makes no hipMalloc, hipFree or other allocating call.  The same
 * kernels run in the same order as in sdd_solve, so the results are bitwise
 * those of sdd_solve on the same request.
 *   req   fixed-path request (target_rel_se == 0), host memory, validated
 *         and copied as for sdd_solve;
 *   res   as for sdd_solve (path_records allowed).
 * Errors: SDD_E_INVALID as sdd_solve, and for target_rel_se > 0;
 * SDD_E_NOMEM when the request needs more than the scratch holds (about 2
 * million paths in all; the message gives the bytes needed); SDD_E_DEVICE.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (counters are zeroed by a kernel at the start of each
 * call): calls on one GPU, from any context or thread of the process, are
 * serialised by a per-device lock held until the call's results are on the
 * host; calls that overlapped on one GPU would race. */
#define SDD_NOALLOC_SCRATCH_BYTES (64u << 20)
sdd_status sdd_solve_noalloc(sdd_ctx_t ctx, const sdd_request *req, sdd_result *res);

/* Bytes of workspace a request needs (tables, nodes, tiles, records; for a
 * target-SE request the pilot and the largest extension). */
sdd_status sdd_request_footprint(sdd_ctx_t ctx, const sdd_request *req, uint64_t *bytes);

const char *sdd_status_string(sdd_status s);
const char *sdd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SDD_H */
