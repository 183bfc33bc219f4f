/*
 * pins.h -- C ABI of the MI355X (gfx950) PINS solver library, libpins.so.
 *
 * PINS (Wu, Liang, Yang, arXiv 2502.03749) solves the Kantorovich problem of
 * eq. (ot):   min <C, X>  s.t.  X e_n = a,  X^T e_m = b,  X >= 0,
 * with a in R^m_{++}, b in R^n_{++}, e^T a = e^T b = 1, by the two-loop method
 * of Alg. 2: an entropic proximal-point (EPPA) outer loop, eq. (x_inner), whose
 * k-th subproblem is entropic OT on the shifted cost C^k = C - eta log X^k,
 * eq. (eppa-sub); each subproblem is solved by a log-domain Sinkhorn warm-up
 * (Alg. 1 sweeps) and sparse-Newton refinement on the dual, eqs.
 * (eppa-sub-dual) and (eppa-hess): Sparsify, truncated preconditioned CG and
 * Armijo backtracking.
 *
 * All arithmetic that decides the result runs in hand-written HIP kernels on
 * the GPU; the host side only validates, allocates and sequences launches.
 *
 * Conventions
 *  - Every array is row-major, double precision, unless stated otherwise.
 *  - The library never frees memory it did not allocate.  Inputs stay owned
 *    by the caller; outputs are written into caller-owned arrays.
 *  - No exception crosses this boundary; every call returns a pins_status.
 *  - One pins_ctx per host thread.  A ctx owns its device workspace and
 *    reuses it across calls; calls on one ctx must not overlap.
 *  - Errors leave a message retrievable with pins_last_error().
 */
#ifndef PINS_H
#define PINS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PINS_ABI_VERSION 2

typedef struct pins_ctx pins_ctx;

typedef enum {
    PINS_OK = 0,
    PINS_NOT_CONVERGED = 1, /* outputs valid; the last subproblem hit the Newton cap T2 */
    PINS_EINVAL = -1,       /* invalid argument; nothing written */
    PINS_ENOMEM = -2,       /* device allocation failed / workspace limit exceeded */
    PINS_EDEVICE = -3,      /* HIP runtime error */
    PINS_ENUMERIC = -4,     /* non-finite value met (NaN/Inf in C or in an iterate) */
    PINS_EUNSUPPORTED = -5  /* combination of options not implemented */
} pins_status;

/* How the cost C of eq. (ot) is given. */
typedef enum {
    PINS_COST_DENSE = 0,  /* C: m*n array */
    PINS_COST_POINTS = 1, /* C_ij = ||x_i - y_j||^2 * scale; x: m*d, y: n*d */
    PINS_COST_GRID = 2    /* s x s pixel grid, m = n = s*s, pixel p = row*s + col,
                             C_pq = ((row_p-row_q)^2 + (col_p-col_q)^2) * scale;
                             computed on the fly, never materialised */
} pins_cost_kind;

typedef enum {
    PINS_FP64 = 0,      /* every step in double precision */
    PINS_MIXED = 1,     /* Sinkhorn warm-up sweeps evaluate exp and accumulate the
                           log-sum-exp in float (exponent formed in double);
                           everything else -- the Newton passes and gradients,
                           the sparsified Hessian and its CG, line search,
                           potentials and outputs -- in double */
    PINS_MIXED_FAST = 2 /* PINS_MIXED, and in addition the CG stores the kept
                           entries of the sparsified Hessian in float and
                           matrix-free products evaluate X~ with a float exp
                           (CG vectors and sums stay double) */
} pins_precision;

typedef enum {
    PINS_SHIFT_IMPLICIT = 0,    /* C^k kept as (k+1) C minus a row and a column vector
                                   (exact algebraic form of C - eta log X^k); O(m+n) per shift */
    PINS_SHIFT_MATERIALIZED = 1 /* C^k stored as an m*n array and updated elementwise,
                                   C^{k+1} = C^k + C - f (+) g + eta */
} pins_shift_mode;

/* Solver parameters.  pins_params_default() fills the paper's defaults
 * (numerical appendix, "Implementation Details"): K = 250, T1 = 100,
 * T2 = 50, Armijo beta = 0.5, c1 = 1e-4, CG relative residual 1e-6,
 * marginal tolerance 1e-9. */
typedef struct {
    double eta;           /* proximal/entropic parameter, > 0 */
    int32_t max_outer;    /* K, number of EPPA outer iterations (fixed; >= 1) */
    int32_t max_sinkhorn; /* T1, warm-up cap per subproblem */
    int32_t max_newton;   /* T2, Newton cap per subproblem */
    int32_t cg_max_iter;  /* CG iteration cap */
    double warm_tol;      /* warm-up ends when the row-marginal L1 error <= warm_tol */
    double inner_tol;     /* Newton ends at ||Xe-a||_1 + ||X^Te-b||_1 <= inner_tol (subproblems < K-1) */
    double final_tol;     /* same for the last subproblem */
    double cg_rtol;       /* CG stops at ||res||_2 <= cg_rtol ||rhs||_2 */
    double ls_beta;       /* Armijo backtracking factor */
    double ls_c1;         /* Armijo constant */
    int32_t ls_max;       /* number of trial steps 1, beta, ..., beta^(ls_max-1) */
    int32_t rho_levels;   /* Sparsify levels tried: thresholds rho * 10^l, l < rho_levels */
    double rho;           /* Sparsify keeps Xt_ij >= rho*10^l*min(a_i,b_j) for the smallest */
    double budget;        /* level l whose count is <= budget*(m+n-1); when no level is
                             within that budget no entry is kept (the Newton system is its
                             diagonal) */
    int32_t precision;    /* pins_precision */
    int32_t shift_mode;   /* pins_shift_mode */
    int32_t profile;      /* nonzero: time every kernel launch with HIP events (pins_result.kern_*) */
    int32_t streams;      /* batch entry point: number of concurrent lanes (own HIP stream and host
                             thread each, instances split into contiguous groups, at most
                             PINS_MAX_LANES);
                             0 or 1 = one lane on the caller's stream; results do not depend on it */
    int32_t profile_mask; /* with profile: bit k set = time the launches of kernel class k
                             (PINS_K_*); 0 = every class.  Fewer timed classes, less overhead */
    int32_t hvp;          /* Hessian-vector products of the Newton CG: 0 = the sparsified
                             Hessian (Sparsify, CSR/CSC products; the default), 1 = matrix-free
                             products with the full Hessian, X~ recomputed tile by tile from
                             the potentials and the streamed cost (no Sparsify), 2 = matrix-free
                             in the outer iterations k < hvp_switch, sparsified after */
    int32_t hvp_switch;   /* hvp = 2: first outer iteration with sparsified products */
    int32_t graphs;       /* nonzero: an outer iteration that starts with a single warm-up
                             iteration and a first Newton round of one-block CGs (the common case
                             once the warm start settles) is replayed as one captured HIP graph
                             (shift, warm-up iteration, Newton pass, Sparsify, CG, first Armijo
                             trial) instead of being launched kernel by kernel.  Needs a non-null
                             stream and profile = 0 (otherwise ignored); results are bitwise
                             those of the kernel-by-kernel launches */
    int32_t tile_rows[4]; /* rows per tile of the dense passes (the tiles are 256 columns wide) for
                             instances with m in [1, 64), [64, 256), [256, 1024), [1024, ...);
                             0 = 16, 32, 32, 64 for the four classes, else 1..64.  The order in which column partials are summed
                             follows it, so results depend on it (last bits), but only through each
                             instance's own m: an instance gets the same result alone and in any
                             batch solved with the same parameters */
} pins_params;

/* One problem instance.  For pins_solve the pointers are host pointers, for
 * the *_device entry points they are device pointers. */
typedef struct {
    int32_t kind;      /* pins_cost_kind */
    int32_t m, n;      /* sizes (>= 1, m*n < 2^31, m+n < 2^28, else PINS_EUNSUPPORTED); GRID: m = n = grid_s^2 */
    int32_t d;         /* POINTS: dimension */
    int32_t grid_s;    /* GRID: side */
    int32_t reserved;
    const double* C;   /* DENSE: m*n */
    const double* x;   /* POINTS: m*d */
    const double* y;   /* POINTS: n*d */
    double cost_scale; /* multiplies C; <= 0 means 1/max C (GRID: 1/(2(s-1)^2)) */
    const double* a;   /* m, positive, sums to 1 (|sum-1| <= 1e-10) */
    const double* b;   /* n, positive, sums to 1 */
} pins_problem;

#define PINS_NKERN 16
#define PINS_MAX_LANES 8 /* most concurrent lanes of one batch call (params.streams) */

/* Results.  alpha/beta/X point to caller-owned arrays (host for pins_solve,
 * device for the *_device entry points); X may be NULL (not written).
 * Outputs are the standard-form potentials at eps = eta/K:
 *   X_ij = exp((alpha_i + beta_j - C_ij)/eps),  gauge <a,alpha> = <b,beta>,
 * which is the plan X^K of Alg. 2 after K outer iterations. */
typedef struct {
    double* alpha;        /* m */
    double* beta;         /* n */
    double* X;            /* m*n or NULL */
    double cost;          /* <C, X^K> (C as scaled) */
    double eps;           /* eta / K */
    double resid;         /* ||X^K e - a||_1 + ||X^K^T e - b||_1 */
    double dual;          /* <a,alpha> + <b,beta>, an LP dual value when the marginals hold */
    double gap;           /* cost - dual */
    double entropy;       /* -sum X log X */
    double cost_scale;    /* scale actually applied to C */
    double time_ms;       /* wall time of the call */
    int32_t status;       /* pins_status of this instance */
    int32_t flags;        /* bit0: last subproblem hit T2; bit1: an earlier one did; bit2: non-finite */
    int32_t outer_iters, sinkhorn_iters, newton_iters, cg_iters, fallbacks, nnz_last;
    double kern_ms[PINS_NKERN];   /* summed kernel time per kernel class (profile != 0) */
    int32_t kern_calls[PINS_NKERN];
    double kern_work[PINS_NKERN]; /* work per kernel class by this instance, always filled:
                                     dense passes: matrix entries visited;
                                     CG classes: stored CSR+CSC entries read (2 nnz per CG
                                     iteration), by the class that ran this instance's CG */
    int32_t group;        /* batch entry point: lane that solved this instance (kern_* are that
                             lane's totals, shared by the instances of the group) */
    int32_t reserved;
} pins_result;

/* Kernel classes reported in kern_ms / kern_calls. */
#define PINS_K_ROW_LSE 0   /* Sinkhorn f-update (row log-sum-exp sweep) */
#define PINS_K_COL_LSE 1   /* Sinkhorn g-update, column partials */
#define PINS_K_COL_MERGE 2 /* Sinkhorn g-update, merge + warm-up control */
#define PINS_K_GRAD 3      /* Newton pass: Xt row/col sums, Sparsify histogram */
#define PINS_K_GRAD_MERGE 4 /* gradient merge, convergence, Sparsify level, CSR row pointers */
#define PINS_K_FILL 5      /* Sparsify: counts, pointer scans, CSR+CSC fill */
#define PINS_K_PCG_ROWS 6  /* one-block CG over row-contiguous S (instances whose S has too many
                              row pieces for the jagged-diagonal form) */
#define PINS_K_PCG 7       /* preconditioned CG, one block per instance (jagged-diagonal S) */
#define PINS_K_LS 8        /* Armijo trial pass */
#define PINS_K_UPDATE 9    /* dual update */
#define PINS_K_SHIFT 10    /* outer shift */
#define PINS_K_FINAL 11    /* potentials and outputs */
#define PINS_K_SETUP 12    /* cost preparation, initialisation */
#define PINS_K_PCG_WIDE 13 /* CG with products over many blocks: large instances, matrix-free */

int pins_abi_version(void);

/* Fill *p with the defaults above (eta = 1e-2). */
void pins_params_default(pins_params* p);

/* Create a context on HIP device `device`.  *out receives the handle.
 * Returns PINS_EDEVICE if the device cannot be used. */
int pins_create(int device, pins_ctx** out);
void pins_destroy(pins_ctx* ctx);

/* Message of the last failing call on ctx (never NULL). */
const char* pins_last_error(const pins_ctx* ctx);

/* Device bytes a solve of `count` problems needs (workspace; inputs and
 * outputs excluded).  Used for admission by HBM footprint. */
int pins_workspace_bytes(const pins_problem* probs, int count, const pins_params* p, size_t* bytes);

/* Solve one problem given by HOST pointers; synchronous.  Copies the inputs
 * to the device, runs Alg. 2, writes alpha, beta (and X if non-NULL) to host
 * arrays and fills the scalars of *res. */
int pins_solve(pins_ctx* ctx, const pins_problem* prob, const pins_params* p, pins_result* res);

/* Solve one problem given by DEVICE pointers on HIP stream `stream` (NULL =
 * the null stream).  Outputs res->alpha/beta/X are device pointers.  The
 * call returns when the solve has finished (the host sequences the
 * data-dependent loops). */
int pins_solve_device(pins_ctx* ctx, const pins_problem* prob, const pins_params* p, pins_result* res,
                      void* stream);

/* ---- Solving without allocation ----
 * For callers that cannot allocate device or pinned memory (code between HIP
 * graph captures, tight serving loops, harnesses that forbid hipMalloc):
 * pins_solve_device with its workspace in a fixed device array that the
 * library holds on each GPU it runs on, PINS_NOALLOC_SCRATCH_BYTES bytes per
 * GPU, until the process ends.  The call allocates no device, pinned or host
 * staging memory (control blocks are read back through a fixed host buffer of
 * the context) and creates no event.  Inputs and outputs are the caller's
 * device arrays, as for pins_solve_device, and the results are bitwise those
 * of pins_solve_device.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (from several contexts, threads or streams) race and
 * must be serialised by the caller.  The array keeps the last call's contents;
 * each call clears what must start at zero.  PINS_ENOMEM (nothing written)
 * when the problem's workspace (pins_workspace_bytes with count 1) exceeds
 * PINS_NOALLOC_SCRATCH_BYTES, e.g. a 128 x 128 grid; PINS_EINVAL for
 * p->profile != 0 (profiling creates events); other errors as
 * pins_solve_device. */
#define PINS_NOALLOC_SCRATCH_BYTES (64u << 20)
int pins_solve_device_noalloc(pins_ctx* ctx, const pins_problem* prob, const pins_params* p, pins_result* res,
                              void* stream);

/* ---- Checkpoint / resume of the outer loop ----
 * Under the implicit shift the k-th EPPA subproblem, eq. (eppa-sub), has the
 * exponent (F_i + G_j - (k+1) C_ij) / eta: the shifted cost C - eta log X^k
 * of Alg. 2 is carried by k and the accumulated row and column shifts A, B,
 * and the subproblem's dual iterate by (F, G).  After k completed outer
 * iterations the tuple (k, F, G, A, B) therefore fixes everything that
 * follows: it is a complete resume point.  All arrays are HOST arrays owned
 * by the caller. */
typedef struct {
    int32_t m, n;        /* sizes of the problem the state belongs to */
    int32_t outer_done;  /* k: outer iterations completed */
    int32_t flags;       /* bit1 of pins_result.flags so far (an earlier subproblem hit T2) */
    double* F;           /* m: row dual iterate of the last subproblem */
    double* G;           /* n: column dual iterate */
    double* A;           /* m: accumulated row shift */
    double* B;           /* n: accumulated column shift */
} pins_state;

/* pins_solve (HOST pointers, synchronous) over a range of outer iterations:
 * start after from->outer_done iterations (from = NULL: from the start, as
 * pins_solve), run up to `stop` completed iterations (0 = p->max_outer = K)
 * and, when save is non-NULL, write the state reached into save (its F, G, A,
 * B must point to m, n, m, n doubles; the call sets m, n, outer_done and
 * flags).  The subproblem tolerance follows the absolute iteration index
 * (final_tol only for iteration K-1), so a solve split at any stop and resumed
 * from the saved state gives bitwise the iterates and outputs of the unbroken
 * solve.  The outputs in *res describe the plan after `stop` iterations
 * (eps = eta/stop, outer_iters = stop); the iteration counters and kern_*
 * cover this call only.  Before iteration K-1 has run, a subproblem that hit
 * T2 shows as flags bit1, never as PINS_NOT_CONVERGED.  Needs the implicit
 * shift (else PINS_EUNSUPPORTED).  PINS_EINVAL when stop > K, when from does not match the problem's m and n,
 * when from->outer_done is not in [1, stop) or from has a NULL or non-finite
 * array, or when save has a NULL array; nothing is written then. */
int pins_solve_resume(pins_ctx* ctx, const pins_problem* prob, const pins_params* p, const pins_state* from,
                      int32_t stop, pins_state* save, pins_result* res);

/* Solve `count` independent problems in one batch (DEVICE pointers): every
 * kernel launch covers all instances still active, each instance keeps its
 * own iteration control, and each result equals the one its problem gets
 * alone.  All problems must share the cost kind (dense/points or grid).
 * Returns the worst status; res[i].status holds each instance's. */
int pins_solve_batch_device(pins_ctx* ctx, const pins_problem* probs, int count, const pins_params* p,
                            pins_result* res, void* stream);

/* Autotuner over the batch schedule and the tile shape.  Three choices of
 * pins_solve_batch_device are searched, each of whose best value depends on
 * the batch (how many instances, how uneven, how their Newton phases
 * overlap): the number of concurrent lanes (params.streams) and the graph
 * replay (params.graphs), which leave every result bitwise unchanged, and the
 * rows per tile of the dense passes (params.tile_rows), which changes the
 * summation order but keeps each result a function of its own instance.  The
 * search is greedy: lane counts 1 .. max_lanes (at most PINS_MAX_LANES and `count`)
 * with graphs off and the default tiles; then graphs on at the best count; then,
 * for each size class of m present in the batch, 8, 32 and 64 rows per tile.  Each
 * configuration is solved once untimed (workspace set-up) and then `reps`
 * times, timed with the host clock (each solve returns when it has finished),
 * and scored by its fastest rep.  *best receives *p with streams, graphs and
 * tile_rows set to the fastest configuration; trials (when non-NULL) receives
 * up to max_trials of the tried configurations in order, *ntrials (when
 * non-NULL) their number.  The outputs in res (DEVICE arrays, as for
 * pins_solve_batch_device) are those of the last solve.  Returns the batch's
 * worst status; PINS_EINVAL for max_lanes outside [1, PINS_MAX_LANES], reps < 1 or a NULL
 * best. */
typedef struct {
    int32_t streams, graphs;
    int32_t tile_rows[4];
    double ms; /* fastest of the reps */
} pins_tune_trial;
int pins_tune_batch_device(pins_ctx* ctx, const pins_problem* probs, int count, const pins_params* p,
                           int max_lanes, int reps, pins_result* res, void* stream, pins_params* best,
                           pins_tune_trial* trials, int max_trials, int32_t* ntrials);

/* ---- Measurement support ----
 * Issue rate of the hardware float exponential on HIP device `device`, the
 * ALU ceiling of a streamed warm-up sweep (one exponential per cost entry,
 * no cost bytes moved).  Launches `blocks` blocks of 256 threads, each thread
 * running 8 independent chains of `iters` exponentials (one multiply each),
 * timed with HIP events on the null stream; *exps_per_s receives the rate and
 * *ms (when non-NULL) the kernel time.  Allocates and frees its own small
 * buffer.  PINS_EINVAL for blocks or iters outside [1, 2^20] or a NULL
 * exps_per_s; PINS_EDEVICE / PINS_ENOMEM on runtime failure. */
int pins_probe_exp_rate(int device, int blocks, int iters, double* exps_per_s, double* ms);

/* The double exp of the FP64 dense passes (Tang's table-driven method, the
 * kernels' own code) applied on the device to x[0..n) into y[0..n) (DEVICE
 * arrays of n doubles, caller-owned), on `stream`, waiting for it.  For
 * checking the device evaluation against a reference.  PINS_EINVAL for NULL
 * arrays or n < 0; PINS_EDEVICE on runtime failure. */
int pins_probe_texp(const double* x, double* y, int n, void* stream);

/* ---- Serving (continuous batching) ----
 * A server owns `workers` (1..4) solver threads on HIP device `device`, each
 * with its own HIP stream and a live batch of up to max_batch requests whose
 * workspaces (and input/output staging) are carved from a device arena of
 * hbm_budget bytes (0 = 4 GiB) per worker.  A worker advances every request in
 * its batch by one outer iteration of Alg. 2 per round; between two rounds it
 * admits queued requests -- in arrival order, of the cost-kind family (grid,
 * or dense/points) of its batch, while a slot and arena room are free -- so
 * requests that arrive while others are on the GPU join them at the next
 * outer-iteration boundary, and each request leaves its batch as soon as its
 * own K outer iterations are done.  Batches of different workers overlap on
 * the device.  Each result is bitwise the one its problem gets alone with the
 * same parameters *p (p->streams, p->graphs and p->profile are ignored; the
 * implicit shift and hvp 0 or 1 are required, else PINS_EUNSUPPORTED).  A
 * request that does not fit into an empty batch's arena completes with
 * PINS_ENOMEM.  The server is used from any number of host threads. */
typedef struct pins_server pins_server;
int pins_server_create(int device, int workers, int max_batch, size_t hbm_budget, const pins_params* p,
                       pins_server** out);
/* Queue one problem given by HOST pointers (copied before the call returns);
 * *ticket identifies it.  PINS_EINVAL for an invalid problem (shape, kind,
 * marginals not positive, finite and summing to 1 within 1e-10, a dense cost
 * or point coordinates with a non-finite entry) or a stopping server, so that
 * no admitted request can fail the batch it joins. */
int pins_server_submit(pins_server* s, const pins_problem* prob, int64_t* ticket);
/* Block until the ticket's solve has finished; fill *res (scalars; alpha and
 * beta copied to res->alpha / res->beta when non-NULL, HOST arrays of m and n
 * doubles; X is not returned) and *latency_ms (submit to completion) when
 * non-NULL.  Returns the solve's status (or a negative error of its batch);
 * the ticket is released. */
int pins_server_wait(pins_server* s, int64_t ticket, pins_result* res, double* latency_ms);
/* Message of the last failed batch (valid while no other batch fails). */
const char* pins_server_last_error(const pins_server* s);
/* Finish every queued request, stop the workers and free the server. */
void pins_server_destroy(pins_server* s);

#ifdef __cplusplus
}
#endif
#endif
