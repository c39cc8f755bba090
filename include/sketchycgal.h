/*
 * sketchycgal.h -- C ABI of the MI355X (gfx950) SketchyCGAL library for the
 * MaxCut SDP.
 *
 * The library solves the model problem of Section 2.1 (eqn model-problem)
 *
 *     minimize <C, X>  subject to  diag(X) = b,  X psd,  tr X = alpha,
 *
 * which for C = -L/4 (L the weighted graph Laplacian, eqn comb-laplacian)
 * and b = 1 is the MaxCut SDP (Section 1.1, eqn maxcut-sdp) with
 * alpha = sum(b) = n.  It runs SketchyCGAL (Section 6, alg:sketchy-cgal):
 * the n x n variable is never formed; the iteration keeps z = diag(X)
 * (primitive 3 of eqn primitives), the dual y, the objective tracker p and a
 * Nystrom sketch S = X Omega (Section 5).  C is touched only through sparse
 * matrix-vector products (primitives 1 and 2).
 *
 * The same engine runs the general template of Appendix D (eqn
 * general-problem, alg:full-sketchy-cgal-supp) with the diagonal constraint
 * map: diag(X) in a box K = {lo <= u <= hi} (params.constraint_set = 1 and
 * sketchycgal_set_constraints), and tr X <= alpha in place of tr X = alpha
 * (params.trace_mode = 1).  Equality rows have lo_i = hi_i.
 *
 * Conventions for every entry point:
 *   - Arrays marked "device" are hipMalloc'd (or torch CUDA) pointers on the
 *     current HIP device; arrays marked "host" are ordinary host memory.
 *   - Every function returns scg_status and never throws across the ABI.
 *   - A context is used by one host thread at a time; all its GPU work is
 *     enqueued on the stream given to sketchycgal_init.
 *   - The library never calls hipMalloc/hipFree after init: the caller owns
 *     every device buffer, including the workspace.
 *   - Values inside the iteration are in scaled units (Section 7.1.1, eqn
 *     problem-scaling: ||C||_F = 1, alpha = 1, b <- b / alpha) when
 *     params.scale = 1; sketchycgal_summary converts back.
 */
#ifndef SKETCHYCGAL_H
#define SKETCHYCGAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCG_OK = 0,
    SCG_EINVAL = 1,    /* bad argument or malformed CSR                          */
    SCG_ENOMEM = 2,    /* workspace smaller than scg_workspace_size reports      */
    SCG_EHIP = 3,      /* a HIP runtime call failed                             */
    SCG_ENUMERIC = 4,  /* NaN/Inf in the iteration, or Cholesky failed (reconstruct) */
    SCG_ESTATE = 5     /* stepping past T, or a call out of order               */
} scg_status;

typedef enum {
    SCG_FP64 = 0,         /* every stream and accumulator in FP64 ("plain FP64")                */
    SCG_FP32_STREAM = 1   /* matrix, Lanczos basis, Omega, S stored/streamed in FP32 with FP32
                             SpMV accumulation; tridiagonal eigensolve, z, y, p, dot products and
                             the reconstruction in FP64 */
} scg_precision;

/* Solver parameters; scg_default_params fills the paper's defaults
 * (Section 7.1.2: beta0 = 1, K = +inf, Gaussian Omega, trace correction on,
 * scaling on; q_t = t^(1/4) log n from alg:sketchy-cgal). */
typedef struct {
    int32_t  R;             /* sketch size, 1 <= R <= min(n, 32)                           */
    int32_t  T;             /* iteration budget (sizes logs and the Lanczos basis), >= 1    */
    double   beta0;         /* initial smoothing beta0 > 0 (beta_t = beta0 sqrt(t+1))        */
    double   K;             /* dual bound K >= 0; +INF disables the guard                   */
    double   alpha;         /* trace alpha > 0; <= 0 selects sum(b)                          */
    uint64_t seed;          /* Philox4x64-10 key for Omega and the Lanczos start vectors     */
    int32_t  q_mode;        /* 0: q_t = ceil(t^(1/4) ln n); 1: q_t = q_fixed                 */
    int32_t  q_fixed;       /* used when q_mode = 1                                          */
    int32_t  scale;         /* 1: scale the problem (Section 7.1.1); 0: solve as given       */
    int32_t  trace_correct; /* 1: trace-correct Lambda in reconstruct (alg:sketchy-cgal)     */
    int32_t  reorth;        /* 0: Lanczos as in alg:rand-lanczos; 1: local reorthogonalisation
                               (one Gram-Schmidt pass against v_{i-1}, v_i); 2: full (against
                               every stored vector)                                           */
    int32_t  precision;     /* scg_precision                                                 */
    int32_t  instance;      /* Philox counter word selecting this problem's random streams   */
    int32_t  matrix_format; /* 0: compress the off-diagonal values when they share one
                               magnitude (columns only, sign in bit 31); 1: always store values */
    int32_t  autotune;      /* 1: time the SpMV variants (lanes per row, column segments, grid
                               size, the quad- or entry-chunk product when the matrix qualifies,
                               and the column slices in entry chunks when the row-block form of
                               the eight segments beats the single launches) at init on the
                               product of Lanczos step 1, and keep the fastest (in
                               a fixed order; a later candidate must be at least 3% faster to
                               replace an earlier one); runs when the matrix has at least 2^20
                               off-diagonal entries or segments is set.  The chosen shape is
                               reported by sketchycgal_summary and can be forced with
                               segments, spmv_lanes and spmv_grid                             */
    int32_t  segments;      /* column segments of the SpMV: 0 = chosen by the autotuner
                               (1 below 1M nonzeros), or 1, 2, 4 (one launch per segment,
                               each adding into the product), or 8 (all eight in one launch,
                               segment s on the workgroups the s-th XCD dispatches, so each
                               XCD gathers from one eighth of x; their raw row sums go to a
                               workspace buffer and a second pass adds them up)               */
    int32_t  spmv_lanes;    /* lanes per row of the SpMV reduction: 0 = autotuned / by mean
                               row length, or 2, 4, 8, 16, 32; 1 = a chunk product (one chunk
                               of 256 entries per wave, 4 per lane, rows summed by a scan
                               across the lanes): for compressed formats (one off-diagonal
                               magnitude) the quad-chunk layout (each row's column words
                               padded to 16-byte quads, rows of at most 128 off-diagonal
                               entries); with stored values the entry-chunk layout (column
                               words and values unpadded, a row starting anywhere in a quad,
                               rows of at most 64 off-diagonal entries); one column segment,
                               or eight (segments = 8: each column slice's row segments in
                               entry chunks, segments of more than 64 entries summed by a
                               wave of their own, any matrix); init returns SCG_EINVAL when
                               the matrix does not qualify                                    */
    int32_t  spmv_grid;     /* SpMV workgroups: 0 = autotuned / one row-block range per wave,
                               or a cap (rounded to a multiple of 8, at most 2048)            */
    int32_t  basis_mode;    /* Lanczos basis storage: 0 = all q+1 vectors kept (ld x (q+1)),
                               1 = three rotating vectors; the Ritz vector is rebuilt by a
                               second Lanczos pass that regenerates the basis bitwise (the
                               storage-optimal randomized Lanczos of Section 4.2, alg
                               rand-lanczos; 0 is the time-storage trade-off its remark
                               describes).  1 requires reorth 0 or 1 (singleton engine only)  */
    int32_t  omega_mode;    /* test matrix: 0 = stored n x R (from Philox or the caller),
                               1 = regenerated from the Philox counters wherever it is used
                               (no n x R array; the caller may not pass omega).  Singleton
                               engine only                                                    */
    int32_t  trace_mode;    /* 0: tr X = alpha (the set alpha Delta_n of eqn model-problem);
                               1: tr X <= alpha: the linear minimisation returns H = alpha
                               v v^T when xi < 0 and H = 0 otherwise (Appendix D.2).
                               Singleton engine only                                          */
    int32_t  constraint_set;/* 0: diag X = b; 1: lo <= diag X <= hi (Appendix D.3; every use
                               of b in the iteration becomes the projection onto the box),
                               bounds from sketchycgal_set_constraints (until then lo = hi =
                               b), b then only gives the default alpha = sum(b); 2: the l2
                               ball ||diag X - b|| <= r (the norm-constraint example of
                               Appendix D.3), r from sketchycgal_set_ball (until then 0).
                               Singleton engine only                                          */
    int32_t  batch_kernel;  /* batched engine only (0 for the single-problem engine): the
                               iteration kernel.  0 = chosen at init: with autotune = 1 every
                               form that fits is timed on one iteration (after a warm-up one)
                               and the fastest kept, in the order 1, 2, 3, a later form only
                               when at least 3% faster; with autotune = 0 the first that fits;
                               1 = the vector being multiplied held whole in LDS (it fits when
                               the largest problem's vector and slice table do); 2 = held in
                               LDS one column tile of half the largest vector at a time, each
                               product making one pass over the slices per tile; 3 = products
                               gathering from global memory.  A form that does not fit gives
                               SCG_EINVAL                                                    */
} scg_params;

/* One record per iteration t, in scaled units (see file comment).  Gap and
 * stopping quantities use the state before the update (Section 6.2 and
 * Appendix E, eqn scgal-stopping-supp, with lambda_min(D_t) ~ xi_t). */
typedef struct {
    int32_t t, q, k, flags;   /* iteration, Lanczos cap q_t, Lanczos steps taken, bit0 = breakdown */
    double xi;                /* Ritz value (approximate lambda_min(D_t))                          */
    double cv;                /* v^T C v                                                           */
    double p;                 /* p_{t+1} = <C, X_{t+1}>                                            */
    double infeas;            /* ||z_{t+1} - b||; box or ball constraints: dist_K(z_{t+1})         */
    double gamma;             /* dual step taken (0 when the K guard refused it)                   */
    double gap;               /* surrogate duality gap g_t = <D_t, X_t - H_t>                      */
    double stop_obj;          /* relative-gap stopping quantity (NaN unless diag X = b, tr X = a)  */
    double stop_feas;         /* ||z_t - b|| / (1 + ||b||)      (NaN unless diag X = b, tr X = a)  */
    double resid;             /* ||D_t v - xi v||                                                  */
    double beta, eta;
} scg_iter_log;

/* Result summary in ORIGINAL units (objective <C, X_T>, infeasibility
 * ||diag X_T - b||) plus the scaling constants. */
typedef struct {
    int32_t t_done;           /* iterations completed                       */
    int32_t status_flags;     /* bit0: NaN/Inf seen                         */
    double objective;         /* <C, X>                                     */
    double infeasibility;     /* ||diag X - b|| (box or ball: dist_K)       */
    double p_scaled, tau_scaled, c_F, alpha, alpha_scaled;
    int32_t spmv_lanes;       /* lanes per row chosen for the SpMV row reduction (1: a chunk
                                 product: quad-chunk or entry-chunk by matrix_format, or with
                                 spmv_segments = 8 the column slices in entry chunks)          */
    int32_t spmv_segments;    /* column segments of the SpMV (8: the concurrent form)          */
    int32_t matrix_format;    /* storage of the off-diagonal values: 0 values, 1 columns only
                                 (common value), 2 columns with sign bit (common magnitude)  */
    int32_t spmv_grid;        /* workgroups of the SpMV launch                                 */
    int32_t batch_kernel;     /* batched engine: the iteration kernel form in use (1, 2, 3);
                                 0 for the single-problem engine                              */
} scg_summary;

typedef struct scg_ctx scg_ctx;

/* Fill *p with the defaults above (R = 10, T = 100, seed = 0, FP64). */
void scg_default_params(scg_params* p);

/* Bytes of device workspace sketchycgal_init needs for an n x n matrix with
 * at most nnz stored entries (diagonal included). */
scg_status scg_workspace_size(const scg_params* p, int64_t n, int64_t nnz, size_t* bytes);

/* Create a context and run the initialisation of alg:sketchy-cgal:
 * validate and scale the data, split the diagonal of C from its off-diagonal
 * part, draw Omega (NystromSketch.Init), zero z, y, S, tau, p.
 *   row_ptr  device int64[n+1], row_ptr[0] = 0, nondecreasing, row_ptr[n] = nnz
 *   col      device int32[nnz], 0 <= col < n (order within a row is free)
 *   val      device double[nnz], finite; C must be symmetric (not checked)
 *   b        device double[n], finite
 *   omega    device double[n*R] row-major test matrix, or NULL to draw it from
 *            the Philox stream (seed; column c, instance, purpose 1)
 *   workspace device, at least scg_workspace_size bytes, 256-byte aligned,
 *            owned by the caller and kept alive until sketchycgal_destroy
 *   stream   hipStream_t (NULL = default stream)
 * Inputs are copied; they may be freed after init returns.  init
 * synchronises the stream once (validation).  Errors: SCG_EINVAL for bad
 * sizes/parameters/CSR/non-finite data, SCG_ENOMEM for a short workspace,
 * SCG_EHIP for runtime failures; *out is NULL on error. */
scg_status sketchycgal_init(scg_ctx** out, const scg_params* p, int64_t n, int64_t nnz,
                            const int64_t* row_ptr, const int32_t* col, const double* val,
                            const double* b, const double* omega, void* workspace,
                            size_t ws_bytes, void* stream);

/* Box constraint set K = {u : lo <= u <= hi} of the general template
 * (Appendix D.3) for a context initialised with params.constraint_set = 1.
 *   lo, hi   device double[n] in original units (the scaling divides them by
 *            alpha like b), or NULL for an unbounded side; -inf / +inf entries
 *            are allowed; copied, may be freed after the call returns.
 * Must be called before the first sketchycgal_step (SCG_ESTATE otherwise).
 * SCG_EINVAL if constraint_set != 1, or any lo_i > hi_i or NaN bound
 * (synchronises the stream once for that check). */
scg_status sketchycgal_set_constraints(scg_ctx* ctx, const double* lo, const double* hi);

/* Radius r >= 0 (original units; scaled by 1/alpha like b) of the ball
 * constraint set K = {u : ||u - b||_2 <= r} for a context initialised with
 * params.constraint_set = 2; the projection is b + (u - b) min(1, r/||u - b||).
 * Before the first sketchycgal_step (SCG_ESTATE otherwise); SCG_EINVAL for
 * another constraint set or a negative or non-finite r.  Host-side only. */
scg_status sketchycgal_set_ball(scg_ctx* ctx, double radius);

/* Enqueue `iters` iterations of alg:sketchy-cgal (loop body: ApproxMinEvec by
 * randomized Lanczos, z, y and sketch updates).  Asynchronous: never
 * synchronises.  SCG_ESTATE if it would run past T.
 * On a non-null stream (and constraint_set != 2) runs of iterations with the
 * same Lanczos step count q_t replay a HIP graph captured once per q (the
 * kernels read the iteration counter from device memory, advanced by the
 * graph's last node); on the null stream the kernels are launched one by one.
 * Both give bit-identical results.  The graphs are owned by the context and
 * freed by sketchycgal_destroy. */
scg_status sketchycgal_step(scg_ctx* ctx, int32_t iters);

/* NystromSketch.Reconstruct (alg:nystrom-sketch-supp) of the current sketch,
 * in FP64 on the device, with the optional trace correction of
 * alg:sketchy-cgal (to alpha; with trace_mode = 1 to the tracked trace
 * tau = tr X_T).  X_hat = U diag(lambda) U^T approximates X in SCALED
 * units (multiply lambda by alpha/alpha_scaled for the original X).
 *   U       device double[n*R] column-major (column j contiguous), orthonormal
 *   lambda  device double[R], nonincreasing, >= 0 (trace-corrected if enabled)
 *   err     device double[R] or NULL: err_r = tau - sum_{j<=r} lambda_raw_j
 *           (eqn sketch-err-supp)
 * Synchronises the stream.  SCG_ENUMERIC if Cholesky fails after three
 * tenfold increases of the shift. */
scg_status sketchycgal_reconstruct(scg_ctx* ctx, double* U, double* lambda, double* err);

/* MaxCut rounding (Section 7.2, sec:maxcut-rounding) of a reconstruction:
 * the columns of sgn(U) (sgn 0 taken as +1) are R cut indicators chi_j; their
 * weights -chi_j^T C chi_j (original units; the total weight of the cut
 * edges when C = -L/4, the MaxCut data) are returned and the heaviest is kept.
 *   U        device double[n*R] column-major, as written by sketchycgal_reconstruct
 *   chi      device int8[n]: the heaviest cut (+1 / -1 per vertex), or NULL
 *   weights  host double[R]: every cut weight
 *   best     host int32: index of the heaviest (lowest index on ties)
 * Evaluated on the matrix as stored (values rounded to FP32 in the FP32-stream
 * precision when they are stored).  Synchronises. */
scg_status sketchycgal_round(scg_ctx* ctx, const double* U, int8_t* chi, double* weights, int32_t* best);

/* MaxCut rounding for callers that cannot allocate device memory (code under
 * stream capture, serving loops, harnesses that forbid hipMalloc): the cut
 * weights of sketchycgal_round computed from the caller's matrix with no
 * context and no workspace.  The partial sums live in a static device array of
 * 1024 x 33 doubles (264 KiB) that the library keeps on every device it has
 * run this call on until the process ends; nothing in it needs clearing.
 *   n, nnz   sizes of C (n >= 1, nnz >= 0)
 *   row_ptr  device int64[n+1], col device int32[nnz], val device double[nnz]:
 *            C in CSR with its diagonal, as for sketchycgal_init; a row pointer
 *            or column outside its range is reported, never followed
 *   R        columns of U, 1 <= R <= min(n, 32)
 *   U        device double[n*R] column-major (as sketchycgal_reconstruct writes)
 *   chi      device int8[n]: the heaviest cut, or NULL
 *   weights  host double[R]: -chi_j^T C chi_j for every column (C as given, FP64)
 *   best     host int32: index of the heaviest (lowest index on ties)
 *   stream   hipStream_t (NULL = default stream) on the current device
 * Synchronises the stream.  SCG_EINVAL for bad sizes or pointers and for a
 * malformed CSR.  Calls that overlap on one device share the array and race:
 * issue them one at a time per device. */
scg_status scg_round_csr(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col, const double* val,
                         int32_t R, const double* U, int8_t* chi, double* weights, int32_t* best, void* stream);

/* Copy up to `max` iteration records into host memory (synchronises). */
scg_status sketchycgal_log(scg_ctx* ctx, scg_iter_log* host_out, int32_t max, int32_t* count);

/* Summary in original units (synchronises).  SCG_ENUMERIC if NaN/Inf seen. */
scg_status sketchycgal_summary(scg_ctx* ctx, scg_summary* host_out);

/* Checkpoint / resume of the iteration state (scaled units; device arrays):
 * z, y double[n]; S double[n*R] row-major; t_next is the next iteration
 * index (1 = fresh).  get_state synchronises. */
scg_status sketchycgal_get_state(scg_ctx* ctx, int32_t* t_next, double* z, double* y, double* S,
                                 double* p, double* tau);
scg_status sketchycgal_set_state(scg_ctx* ctx, int32_t t_next, const double* z, const double* y,
                                 const double* S, double p, double tau);

/* Tridiagonal coefficients of the last Lanczos run (host arrays of length
 * >= *k on return): omega[0..k), rho[0..k-1), and its Ritz value.
 * Synchronises. */
scg_status sketchycgal_lanczos_coeffs(scg_ctx* ctx, double* omega, double* rho, int32_t cap,
                                      int32_t* k, double* xi);

/* x -> D x with D = C_s + diag(y + beta_t (z - b)) for the next iteration t
 * (primitives 1 and 2 of eqn primitives; device double[n] in and out), using
 * the same SpMV kernel as the Lanczos loop.  Synchronises. */
scg_status sketchycgal_apply(scg_ctx* ctx, const double* x, double* y);

/* Average duration (ms) of `reps` back-to-back launches of the Lanczos SpMV
 * kernel on the context's stream, timed with HIP events on that stream.  The
 * launches are the product of Lanczos step 1 (the form every step after the
 * first takes: it reduces the preceding update's partial sums), after the
 * shift, the start vector, one product and one update of the next iteration
 * have been formed.  Overwrites the per-iteration scratch (Lanczos vectors,
 * product, coefficients); z, y, S, p and tau are untouched.  Synchronises. */
scg_status sketchycgal_time_spmv(scg_ctx* ctx, int32_t reps, double* avg_ms);

void sketchycgal_destroy(scg_ctx* ctx);
const char* scg_status_string(scg_status s);

/* ------------------------------------------------------------------------
 * Batched engine: many independent MaxCut-type problems of uneven size, each
 * solved by alg:sketchy-cgal with its own scaling (Section 7.1.1), its own
 * random streams (Philox counter word params.instance + i for problem i) and
 * its own iteration state, advanced together by ONE kernel launch per
 * iteration.  The problems are given as one block-diagonal CSR matrix: rows
 * of problem i are rows [r_i, r_i + inst_n[i]) with r_i = sum_{j<i} inst_n[j],
 * and every column index of such a row must lie in the same range (checked).
 * Result per problem i is identical (up to rounding order) to sketchycgal_init
 * + step on that problem alone with params.instance + i.
 * Limits: q_t <= 128 for every problem and t; n_i >= R;
 * sum of n_i < 2^31.  Conventions as for the single-problem entry points.
 * ---------------------------------------------------------------------- */
typedef struct scg_batch scg_batch;

/* Workspace bytes for problems of sizes inst_n[0..n_inst) with nnz stored
 * entries in total (diagonals included). */
scg_status scg_batch_workspace_size(const scg_params* p, int32_t n_inst, const int64_t* inst_n,
                                    int64_t nnz, size_t* bytes);

/* Initialise every problem (alg:sketchy-cgal, Init):
 *   inst_n   host int64[n_inst], sizes n_i >= R
 *   row_ptr  device int64[N+1] (N = sum n_i), as in sketchycgal_init
 *   col      device int32[nnz], global column numbers inside the row's block
 *   val, b   device double[nnz], double[N], finite
 *   workspace device, scg_batch_workspace_size bytes, 256-byte aligned, owned
 *            by the caller until sketchycgal_batch_destroy
 *   stream   hipStream_t; on a non-null stream step() replays captured HIP
 *            graphs of 16 iterations, on the null stream it launches eagerly
 * The value format (values, or columns only when all off-diagonal entries
 * of all problems share one value / one magnitude) is chosen once for the
 * batch.  Synchronises.  Errors as sketchycgal_init. */
scg_status sketchycgal_batch_init(scg_batch** out, const scg_params* p, int32_t n_inst,
                                  const int64_t* inst_n, int64_t nnz, const int64_t* row_ptr,
                                  const int32_t* col, const double* val, const double* b,
                                  void* workspace, size_t ws_bytes, void* stream);

/* Enqueue `iters` iterations for every problem; asynchronous.  SCG_ESTATE
 * past T. */
scg_status sketchycgal_batch_step(scg_batch* ctx, int32_t iters);

/* Per-problem initial penalty: problem k runs with beta_t = beta0[k] sqrt(t + 1)
 * and the dual step bound of eqn sketchy-cgal-dual-step with beta0[k]
 * (alg:sketchy-cgal; every problem keeps its own iteration counter).
 *   beta0  host double[n_inst], each > 0 and finite (SCG_EINVAL otherwise);
 *          copied.  Until it is called every problem takes params.beta0.
 * Must come before the first sketchycgal_batch_step or set_state
 * (SCG_ESTATE otherwise).  Synchronises the stream. */
scg_status sketchycgal_batch_set_beta0(scg_batch* ctx, const double* beta0);

/* Per-problem iteration records, summary (original units), checkpoint state
 * (z, y device double[n_i]; S device double[n_i*R] row-major; any pointer of
 * get_state may be NULL; set_state puts problem `inst` at iteration t_next,
 * 1 <= t_next <= T+1, and step() then requires every problem to have `iters`
 * iterations left) and reconstruction (U device double[n_i*R] column-major,
 * lambda and err device double[R]; as sketchycgal_reconstruct).  All
 * synchronise. */
scg_status sketchycgal_batch_log(scg_batch* ctx, int32_t inst, scg_iter_log* host_out, int32_t max,
                                 int32_t* count);
scg_status sketchycgal_batch_summary(scg_batch* ctx, int32_t inst, scg_summary* host_out);
scg_status sketchycgal_batch_get_state(scg_batch* ctx, int32_t inst, int32_t* t_next, double* z,
                                       double* y, double* S, double* p, double* tau);
scg_status sketchycgal_batch_set_state(scg_batch* ctx, int32_t inst, int32_t t_next, const double* z,
                                       const double* y, const double* S, double p, double tau);
scg_status sketchycgal_batch_reconstruct(scg_batch* ctx, int32_t inst, double* U, double* lambda,
                                         double* err);
/* MaxCut rounding of problem `inst` from its reconstruction U (device
 * double[n_i*R]); as sketchycgal_round. */
scg_status sketchycgal_batch_round(scg_batch* ctx, int32_t inst, const double* U, int8_t* chi,
                                   double* weights, int32_t* best);
void sketchycgal_batch_destroy(scg_batch* ctx);

/* ======================================================================
 * Phase retrieval (Section 7.3, eqn numerics-phase-retrieval-sdp): minimise
 * tr X over complex Hermitian psd X subject to A X = b and tr X <= alpha,
 * with coded diffraction measurements (Appendix F.1):
 *     (A X)_{j,l} = a_{j,l}^* X a_{j,l},  a_{j,l}^* x = (DFT_n (conj(psi_j) x))_l,
 * DFT_n unnormalised (entry (l, m) = exp(-2 pi i l m / n)), j < L waveforms.
 * The solver is alg:sketchy-cgal over the trace-bounded set of Appendix D.2
 * (H = alpha v v^* when the Ritz value xi < 0, else H = 0) in complex FP64:
 * randomized Lanczos (alg:rand-lanczos) on the Hermitian D_t = C + A^*(w),
 * the Nystrom sketch (alg:nystrom-sketch-supp) with a complex test matrix,
 * and the rounding of Section 7.3.2 (chi = sqrt(lambda_1) u_1) with the
 * relative error of Section 7.3.3.
 *
 * Scaling (eqn problem-scaling): C = I becomes I / sqrt(n); the A_i of
 * waveform j are divided by ||psi_j||^2 (equal ||A_i||_F) and all by the
 * norm N of the result, N^2 = n lambda_max(Q Q^T), Q_{j,m} =
 * |psi_j(m)|^2 / ||psi_j||^2 (the Gram matrix of the A_i is block-circulant
 * in l and its zero-frequency block holds the top eigenvalue), so ||A|| = 1;
 * b is scaled the same way and by 1/alpha, alpha <- 1.
 *
 * Complex arrays are interleaved (re, im) doubles.  Measurement-indexed
 * arrays (b, z, y, w, measure output) are L x n, entry j * n + l.  Random
 * draws: the Lanczos start vector of iteration t and column c of Omega are
 * complex with independent standard normal parts, complex element m being
 * the Box-Muller pair (2m, 2m+1) of the Philox stream (seed; t, instance,
 * purpose 2) and (seed; c, instance, purpose 3).
 *
 * Supported n: n = n1 n2 with n1, n2 <= 4096 and both products of 2, 3, 5
 * (every n = 10^k, 2 <= k <= 7, qualifies); L <= 32; R <= 16.
 * ====================================================================== */
typedef struct {
    int32_t  R;             /* sketch size, 1 <= R <= min(n, 16)                        */
    int32_t  T;             /* iteration budget, >= 1                                     */
    double   beta0;         /* beta0 > 0                                                  */
    double   K;             /* dual bound K >= 0; +INF disables the guard                */
    double   alpha;         /* trace bound alpha > 0; 0 selects 3 n (Section 7.3.3)       */
    uint64_t seed;          /* Philox key                                                 */
    int32_t  q_mode;        /* 0: q_t = ceil(t^(1/4) ln n); 1: q_t = q_fixed             */
    int32_t  q_fixed;
    int32_t  scale;         /* 1: the scaling above; 0: solve as given                    */
    int32_t  trace_correct; /* 1: reconstruct corrects the trace to tau = tr X_T          */
    int32_t  instance;      /* Philox counter word                                        */
    int32_t  mask_groups;   /* inverse column pass: the waveforms are split into this many
                               groups, each summed by its own workgroups into its own
                               partial product; 0 = chosen at init (with autotune = 1 one
                               product is timed for 1, 2, 3, 4, 6, 12 and L groups and the
                               fastest kept, a later candidate only when at least 3% faster;
                               with autotune = 0 one group), else 1 .. L                   */
    int32_t  tile_cols;     /* columns per column-pass tile: 0 = chosen, else a power of
                               two with n1 * tile_cols <= 4096                             */
    int32_t  mask_format;   /* 0: waveforms stored as one-byte codes into a dictionary when
                               they take at most 256 distinct values (bitwise; the coded
                               diffraction waveforms take 8), else whole; 1: always whole */
    int32_t  autotune;      /* 1: choose mask_groups by timing at init (when it is 0)      */
} scg_pr_params;

/* Summary in ORIGINAL units: objective tr X, infeasibility ||A X - b||. */
typedef struct {
    int32_t t_done;
    int32_t status_flags;     /* bit0: NaN/Inf seen                                       */
    double objective;
    double infeasibility;
    double p_scaled, tau_scaled, alpha, alpha_scaled, c_F;
    double op_norm;           /* N of the scaling (1 when unscaled)                       */
    int32_t n1, n2;           /* the four-step split n = n1 n2                            */
    int32_t tile_cols, row_tile, mask_groups;   /* launch shape of the DFT passes         */
    int32_t mask_codes;       /* 1: waveforms stored as dictionary codes                  */
} scg_pr_info;

typedef struct scg_pr_ctx scg_pr_ctx;

/* Defaults: R = 5, T = 100, beta0 = 1, K = +inf, alpha = 3n, q_t schedule,
 * scaling and trace correction on. */
void scg_pr_default_params(scg_pr_params* p);

/* Device workspace bytes for an n-dimensional signal and L waveforms;
 * SCG_EINVAL for unsupported n or parameters. */
scg_status scg_pr_workspace_size(const scg_pr_params* p, int64_t n, int32_t L, size_t* bytes);

/* Create a context: copy psi, compute the scaling, scale b into the solver's
 * order, draw (or copy) Omega, zero z, y, S, p, tau.
 *   psi       device complex[L*n] waveforms (row j = psi_j)
 *   b         device double[L*n] measurements, original units
 *   omega     device complex[R*n] test matrix (column c contiguous) or NULL
 *             to draw it from the Philox stream
 *   workspace device, >= scg_pr_workspace_size bytes, 256-byte aligned, owned
 *             by the caller until scg_pr_destroy
 * Inputs are copied.  Synchronises.  SCG_EINVAL (sizes, parameters, a zero
 * waveform), SCG_ENOMEM (short workspace), SCG_EHIP. */
scg_status scg_pr_init(scg_pr_ctx** out, const scg_pr_params* p, int64_t n, int32_t L, const double* psi,
                       const double* b, const double* omega, void* workspace, size_t bytes, void* stream);

/* Enqueue `iters` iterations (asynchronous).  SCG_ESTATE past T.  On a
 * non-null stream runs of iterations with the same Lanczos step count replay
 * one HIP graph per count (captured on first use, owned by the context; the
 * kernels read t from a device counter); on the null stream the kernels are
 * launched one by one.  Both give bit-identical results. */
scg_status scg_pr_step(scg_pr_ctx* ctx, int32_t iters);

/* y = (C + A^*(w)) x in scaled units: w device double[L*n] (dual weights,
 * scaled units), x and y device complex[n].  Overwrites the iteration's
 * dual weights (recomputed at the next step).  Synchronises. */
scg_status scg_pr_apply(scg_pr_ctx* ctx, const double* w, const double* x, double* y);

/* m = A(x x^*) in scaled units (s_j |DFT_n(conj(psi_j) x)_l|^2): x device
 * complex[n], m device double[L*n].  Synchronises. */
scg_status scg_pr_measure(scg_pr_ctx* ctx, const double* x, double* m);

/* Iteration records (scg_iter_log; stop_obj, stop_feas, resid are NaN). */
scg_status scg_pr_log(scg_pr_ctx* ctx, scg_iter_log* host_out, int32_t max, int32_t* count);

/* Summary; with check_numeric, SCG_ENUMERIC once a NaN/Inf was seen. */
scg_status scg_pr_summary(scg_pr_ctx* ctx, scg_pr_info* host_out, int32_t check_numeric);

/* Checkpoint state in scaled units: z, y device double[L*n]; S device
 * complex[R*n] (column c contiguous); any output may be NULL.  set_state
 * puts the context before iteration t_next (1 <= t_next <= T+1).  Both
 * synchronise. */
scg_status scg_pr_get_state(scg_pr_ctx* ctx, int32_t* t_next, double* z, double* y, double* S, double* p,
                            double* tau);
scg_status scg_pr_set_state(scg_pr_ctx* ctx, int32_t t_next, const double* z, const double* y,
                            const double* S, double p, double tau);

/* NystromSketch.Reconstruct of the current sketch, FP64, scaled units:
 * X_hat = U diag(lambda) U^*, U device complex[R*n] (column c contiguous,
 * orthonormal), lambda device double[R] nonincreasing (trace-corrected to tau
 * when enabled), err device double[R] or NULL (eqn sketch-err-supp).
 * sigma = sqrt(n) eps(||S||_2); B = Omega^* S_sigma made Hermitian; on a
 * Cholesky failure sigma grows tenfold, at most three times, then
 * SCG_ENUMERIC.  The R x R steps run on the host.  Synchronises. */
scg_status scg_pr_reconstruct(scg_pr_ctx* ctx, double* U, double* lambda, double* err);

/* Rounding (Section 7.3.2): chi = sqrt(alpha lambda_j) u_j (original units)
 * for the largest lambda_j (lowest index on ties).  U, lambda as written by
 * scg_pr_reconstruct; chi device complex[n] or NULL; with chi_true (device
 * complex[n]) rel_err (host) receives min_phi ||e^{i phi} chi - chi_true|| /
 * ||chi_true|| (Section 7.3.3).  Synchronises. */
scg_status scg_pr_round(scg_pr_ctx* ctx, const double* U, const double* lambda, const double* chi_true,
                        double* chi, double* rel_err);

/* Average times (ms) of the three passes of one D v product, each launched
 * `reps` times back to back on the context's stream (ms[0] column DFT pass,
 * ms[1] fused row pass, ms[2] inverse column pass) and of the whole product
 * (ms[3]), measured with HIP events; the operands are the dual weights and
 * start vector of the next iteration.  Synchronises. */
scg_status scg_pr_time_apply(scg_pr_ctx* ctx, int32_t reps, double* ms);

scg_status scg_pr_destroy(scg_pr_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SKETCHYCGAL_H */
