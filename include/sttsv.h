/*
 * sttsv.h -- C ABI of the MI355X STTSV library.
 *
 * STTSV (sparse symmetric tensor times same vector, TTSV1 of Eq. (1)-(2))
 * on the order-r blowup adjacency tensor B of a non-uniform hypergraph
 * H = (V, E) (Sec. II), and the NQZ iteration for H-eigenvector centrality
 * that calls it on every step (Alg. 1).
 *
 *   B: for every edge e and every r-tuple i whose entry set is exactly e,
 *      B_i = w(e)/|beta(e)|, |beta(e)| = |e|! S(r,|e|), w(e) = |e| (Sec. II
 *      and its footnote), so that B 1^(r-1) = vertex degrees.
 *   y = B x^(r-1):  y_v = sum_{i2..ir} B_{v,i2..ir} x_{i2} ... x_{ir}  (Eq. (2)),
 *      evaluated per (edge, member) with the generating-function form of
 *      Alg. 2 (Sec. II-A), never enumerating the blowup entries.
 *
 * Conventions
 *   - Every call returns an int: STTSV_OK (0) or a negative STTSV_E* code.
 *     No exception crosses the ABI.  sttsv_strerror() names a code.
 *   - Vertex ids are 0-based int32 (the paper counts from 1); edge offsets are
 *     int64.  A hypergraph is passed as CSR: edge i is
 *     eidx[eptr[i] .. eptr[i+1]-1].
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory (e.g. from torch on a ROCm build).  Device work is
 *     ordered on the plan's stream (sttsv_opts.stream, default stream if
 *     NULL) and is asynchronous unless stated otherwise.
 *   - The library owns every buffer it allocates; callers own what they pass.
 */
#ifndef STTSV_H
#define STTSV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define STTSV_OK              0
#define STTSV_EINVAL         -1  /* invalid argument or malformed hypergraph        */
#define STTSV_ENOMEM         -2  /* host or device allocation failed                */
#define STTSV_EDISCONNECTED  -3  /* solver needs a connected hypergraph (Sec. II)   */
#define STTSV_ENOTCONV       -4  /* solver hit max_iter; partial result returned    */
#define STTSV_ENUMERIC       -5  /* NaN / Inf / non-positive value met in the solve */
#define STTSV_EHIP           -6  /* a HIP runtime call failed                       */
#define STTSV_ENOTSUP        -7  /* request outside the supported range             */

#define STTSV_MAX_ORDER      64  /* largest supported tensor order r                */

/* ---- precision of the series arithmetic ------------------------------- */
#define STTSV_PREC_FP64       0  /* series, weights, sums all in FP64               */
#define STTSV_PREC_FP32       1  /* series in FP32 (FMA), weights / products /      */
                                 /* per-vertex sums in FP64; an apply gathers x    */
                                 /* rounded to FP32 and stores each contribution   */
                                 /* as the upper 32 bits of its FP64 value (FP64   */
                                 /* range, 21 significant bits, rounded to nearest)*/
                                 /* which the reduction widens back exactly.  The  */
                                 /* solver's FP32 phase keeps FP64 x and terms.    */

typedef struct sttsv_plan_s* sttsv_plan_t;

/* Plan flags. */
#define STTSV_FLAG_GENERIC_ONLY 1  /* run every edge of size >= 4 through the generic */
                                   /* (runtime-size) kernel instead of the register-  */
                                   /* resident ones; results are bitwise identical    */
#define STTSV_FLAG_ONE_STREAM   2  /* launch every edge kernel on the plan's stream.  */
                                   /* By default the edge launches are spread over   */
                                   /* the plan's stream and two helper streams of    */
                                   /* default priority (event fork / join, so work   */
                                   /* stays ordered on the plan's stream); results   */
                                   /* are bitwise identical either way               */
#define STTSV_FLAG_PREFIX_REUSE 4  /* FP64 edges of size 4..7: one thread takes a run */
                                   /* of up to 4 consecutive canonical edges with the */
                                   /* same first two members and computes their      */
                                   /* shared prefix product phi_0 phi_1 once (the    */
                                   /* convolution memoisation of Sec. IV-B over the  */
                                   /* shared prefixes of Sec. III); results are      */
                                   /* bitwise identical                              */

/* Options for sttsv_plan.  Pass NULL for all defaults. */
typedef struct {
    int32_t precision;   /* STTSV_PREC_FP64 (default) or STTSV_PREC_FP32        */
    int32_t flags;       /* STTSV_FLAG_* bits (default 0)                        */
    void*   stream;      /* hipStream_t the plan's work is ordered on; NULL =   */
                         /* the default stream                                   */
    const double* edge_weights;  /* host, nullable: w(e) of every input edge   */
                         /* (double[m], finite and > 0) of the edge-weighted     */
                         /* hypergraph H = (V, E, w) of Sec. II; every blowup of */
                         /* e then holds w(e)/|beta(e)|.  NULL: w(e) = |e|, the  */
                         /* paper's choice (B 1^(r-1) = degrees).  Copied.       */
                         /* Must be NULL for sttsv_plan_batch (per-graph weights */
                         /* come with each sttsv_graph_desc).                    */
} sttsv_opts;

/*
 * sttsv_plan -- build an execution plan for the hypergraph (host CSR).
 *
 *   eptr  host, int64[m+1]: edge offsets, eptr[0] = 0, strictly increasing
 *         (every edge non-empty), eptr[m] = nnz.
 *   eidx  host, int32[nnz]: member vertex ids in [0, n); no vertex twice
 *         in one edge (E is a set system, Sec. II).  Member order and edge
 *         order are free; a repeated edge counts once per copy.
 *   m     number of edges (>= 1);  n  number of vertices (>= 1);
 *   r     tensor order, 2 <= r <= STTSV_MAX_ORDER, r >= max |e| (the blowup
 *         tensor may be of higher order than the rank of H).
 *   opts  host, nullable.
 *   out   host: receives the plan handle on success; untouched on error.
 *
 * The arrays are copied; the caller may free them on return.  The plan
 * holds all device buffers (member layout, per-incidence contributions,
 * node-major incidence lists, reduction schedule, weight table
 * w(e)/|beta(e)| (r-1)! per edge size, the degree-rank copy of x) and is
 * used by one host thread at a time.  Blocking (uploads are synchronous).
 * Errors: EINVAL (malformed input, or an edge weight that is not finite
 * and positive), ENOTSUP (r out of range, or m, n or nnz at or above 2^31),
 * ENOMEM, EHIP.
 */
int sttsv_plan(const int64_t* eptr, const int32_t* eidx, int64_t m, int32_t n,
               int32_t r, const sttsv_opts* opts, sttsv_plan_t* out);

/*
 * sttsv_apply -- y = B x^(r-1)  (TTSV1, Eq. (2); Alg. 2 per edge and member).
 *
 *   x  device, double[n], read only (any finite values; accuracy statements
 *      hold for x >= 0, where every term is non-negative).
 *   y  device, double[n], fully overwritten (isolated vertices get 0).
 *      Must not alias x.
 *
 * Uses the plan's precision and stream; asynchronous.  The result is
 * bitwise reproducible: each y_v is summed in a fixed order that depends only
 * on the hypergraph, never on launch timing (no floating-point atomics).
 * Errors: EINVAL (NULL arguments), EHIP (launch failure).
 */
int sttsv_apply(sttsv_plan_t plan, const double* x, double* y);

/* As sttsv_apply with an explicit precision (STTSV_PREC_*). */
int sttsv_apply_prec(sttsv_plan_t plan, const double* x, double* y, int32_t precision);

/*
 * sttsv_apply_timed -- sttsv_apply_prec, with every stage timed by a pair of
 * hipEvents recorded on the plan's stream (for measurement tools).
 *
 * Stage s is one of: the copy of x into degree-rank order that the edge
 * kernels gather from (kinds[s] = 3, sizes[s] = 0, counts[s] = n); the
 * edge-kernel launch of one size bucket
 * (kinds[s] = 0, sizes[s] = edge size k, counts[s] = edges in the bucket);
 * a fused launch of the generic kernel over several buckets whose suffix
 * stacks live in LDS (kinds[s] = 1, sizes[s] = window-range index, counts[s]
 * = edges covered), in global memory (kinds[s] = 5, as for kind 1), or that
 * keeps no suffix stacks and rebuilds each suffix series when it needs it
 * (kinds[s] = 6, as for kind 1; see STTSV_Q_BUCKET_STACK); a fused launch
 * of the lane-group kernel, where L lanes (a power of two >= |e|) share each
 * edge of buckets with few edges and long series chains (kinds[s] = 4, sizes
 * and counts as for kind 1); one level of
 * the node reduction (kinds[s] = 2, sizes[s] = level, counts[s] = chunks).
 * ms[s] = elapsed milliseconds of that stage.
 *   cap      capacity of the four host output arrays (entries)
 *   nstages  host: number of stages (set even when cap is too small, then
 *            EINVAL is returned and nothing is launched)
 * Synchronous (waits for the stream).  Same result as sttsv_apply_prec.
 */
int sttsv_apply_timed(sttsv_plan_t plan, const double* x, double* y, int32_t precision,
                      int32_t cap, int32_t* nstages, int32_t* kinds, int32_t* sizes,
                      int64_t* counts, float* ms);

/*
 * sttsv_apply_naive -- y = B x^(r-1) by the paper's NAIVE algorithm (Alg. 3,
 * complexity in Sec. IV): every (edge, member) pair multiplies out its own
 * generating function e^{x_v t} prod_{u != v}(e^{x_u t} - 1) with full-length
 * FP64 series (degrees 0..r-1), sharing nothing between members or edges:
 * |e|(|e|-1) truncated products per edge.  A comparison baseline for the
 * memoised kernels of sttsv_apply, not a faster path.
 *   x, y   device double[n], as for sttsv_apply (y fully overwritten; x != y).
 * Always FP64, whatever the plan's precision; the node reduction is the
 * plan's deterministic one, so the result is bitwise reproducible but not
 * bitwise equal to sttsv_apply's (the products round differently).
 * Asynchronous on the plan's stream; it shares the plan's contribution
 * buffer with sttsv_apply, so calls on one plan must not overlap.
 * Errors: EINVAL (NULL plan, x or y, or x == y), EHIP (launch failure).
 */
int sttsv_apply_naive(sttsv_plan_t plan, const double* x, double* y);

/*
 * sttsv_contract -- the full contraction B x^r = x . (B x^(r-1)) (the
 * quantity Sec. II's tensor defines on x^r; x^T y = B x^r).
 *   x    device double[n]
 *   y    device double[n], receives B x^(r-1) (FP64 series, as sttsv_apply_prec)
 *   out  host double: B x^r, summed by a fixed-shape tree (reproducible bit for bit)
 * Synchronous on the plan's stream; its reduction scratch lives in the plan
 * (allocated on the first call of this or zeigvec_sshopm, 2 n + ~1.6k
 * doubles, freed with the plan).  On a batched plan the contraction is over
 * the disjoint union.
 * Errors: EINVAL (NULL argument, x == y), ENOMEM, EHIP.
 */
int sttsv_contract(sttsv_plan_t plan, const double* x, double* y, double* out);

/*
 * sttsv_contract_noalloc -- sttsv_contract for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, hosts that
 * forbid allocation): same arguments, same kernels, same result bit for bit,
 * but its reduction scratch (1540 doubles, fixed: it does not grow with the
 * plan) lives in a static device array of the library, one per GPU, held
 * until the process ends; no allocator is called.  The plan's device must be
 * the current device (EINVAL otherwise).  Every call on one GPU uses that
 * GPU's array: calls that overlap on one GPU (other threads, other streams)
 * race and must be serialised by the caller.  Synchronous on the plan's
 * stream.  Errors: EINVAL (NULL argument, x == y, other device), EHIP.
 */
int sttsv_contract_noalloc(sttsv_plan_t plan, const double* x, double* y, double* out);

typedef struct {
    int32_t iterations;    /* updates of x performed                             */
    int32_t converged;     /* 1 when the stopping rule was met                   */
    double  lambda;        /* x . B x^(r-1) at the returned x                    */
    double  residual;      /* ||B x^(r-1) - lambda x||_2 at the returned x       */
} sttsv_zeig_info;

/*
 * zeigvec_sshopm -- a Z-eigenpair (B x^(r-1) = lambda x, ||x||_2 = 1) by the
 * shifted power method that Sec. I names as an STTSV consumer (Kolda and
 * Mayo's SS-HOPM, convex form): w = B x^(r-1) + alpha x, x <- w/||w||_2,
 * lambda = x . B x^(r-1), until |lambda_k - lambda_(k-1)| <= tol |lambda_k|.
 *   x0        device double[n] or NULL (all ones); normalised first; must not
 *             be zero.  May equal x_out.
 *   alpha     shift >= 0 (convex form)
 *   tol       >= 0 (0: run max_iter updates)
 *   max_iter  >= 0 updates of x
 *   x_out     device double[n]: the last iterate (unit 2-norm)
 *   info      host, nullable
 * On a batched plan the tensor is that of the disjoint union of its graphs.
 * FP64 series whatever the plan's precision.  Synchronous: waits for the
 * plan's stream (x0 may be produced there), iterates on a stream of its own
 * and returns when done.  lambda, the stopping test and the iteration count
 * stay on the device; 8 updates are one captured graph, replayed until the
 * device says stop, the host reading a small control block between replays.
 * Scratch (2 n + ~1.6k doubles) and the graph live in the plan from the first
 * call on (the graph is dropped when sttsv_plan_autotune changes the launch
 * sequence).  Errors: EINVAL (NULL plan or x_out, alpha < 0, tol < 0,
 * max_iter < 0), ENUMERIC (zero or non-finite norm; x_out untouched),
 * ENOTCONV (max_iter reached: x_out and info hold the last iterate), ENOMEM,
 * EHIP.
 */
int zeigvec_sshopm(sttsv_plan_t plan, const double* x0, double alpha, double tol, int32_t max_iter,
                   double* x_out, sttsv_zeig_info* info);

/*
 * sttsv_plan_autotune -- per size bucket and series type, time the kernel
 * variants that compute bitwise-identical contributions (register-resident
 * vs generic kernel for 4 <= |e| <= 7; for the generic kernel, suffix stack
 * in LDS, in global memory, or none with the suffix series rebuilt where
 * they are needed, the last for windows r - |e| + 1 >= 9 (FP64: <= 48)) on
 * the device and keep the fastest (a stack placement other than the
 * planner's default only when it is 3 % faster); then move the edge launches
 * between the stream lanes while whole applies get faster (samples of two
 * applies; the result kept only if it beats the starting assignment when
 * both are timed again in alternation).  Tuning never changes any bit of y.
 *   x           device, double[n]: a representative input (e.g. the start
 *               vector of a solve); only read.
 *   reps        >= 1 timed launches per candidate (median taken; at least 5
 *               two-apply samples for the lane search).
 *   cache_path  host string or NULL: text file of earlier choices, keyed by
 *               (series type, r, |e|, round(log2 edges)); choices found there
 *               are applied without timing, new ones are appended.
 *   tuned       host, nullable: number of (bucket, type) pairs decided.
 * Synchronous; drops the solver's captured hipGraph (rebuilt on next solve).
 */
int sttsv_plan_autotune(sttsv_plan_t plan, const double* x, int32_t reps, const char* cache_path,
                        int32_t* tuned);

/* ---- H-eigenvector centrality (Alg. 1) ------------------------------- */

/* Precision schedules of the solver. */
#define STTSV_SOLVE_FP64       0  /* every STTSV in FP64 series                       */
#define STTSV_SOLVE_FP32_FP64  1  /* FP32-series iterations until the criterion      */
                                  /* stops improving or falls below switch_tol, then */
                                  /* FP64-series iterations until it is < tol        */

typedef struct {
    int32_t max_iter;      /* default 500                                       */
    int32_t check_every;   /* iterations per graph replay between host checks  */
                           /* of the convergence flag (default 8)               */
    int32_t schedule;      /* STTSV_SOLVE_* (default FP64)                       */
    int32_t use_graph;     /* 1 (default): replay a captured hipGraph           */
    double  shift;         /* alpha >= 0: z <- z + alpha x^[r-1] (default 0)    */
    double  switch_tol;    /* FP32->FP64 switch threshold (default 1e-4)        */
} sttsv_solve_opts;

typedef struct {
    int32_t iterations;    /* repeat-loop passes of Alg. 1                      */
    int32_t iters_fp32;    /* of which with FP32 series                         */
    int32_t iters_fp64;    /* of which with FP64 series                         */
    int32_t converged;     /* 1 if criterion < tol                              */
    double  lambda_min;    /* min_v z_v / x_v^(r-1) at the returned x           */
    double  lambda_max;    /* max_v z_v / x_v^(r-1) at the returned x           */
    double  criterion;     /* (lambda_max - lambda_min) / lambda_min            */
} sttsv_solve_info;

/*
 * heigvec_solve -- NQZ iteration (Alg. 1) for the H-eigenvector centrality x:
 * positive x with B x^(r-1) = lambda x^[r-1] (Sec. II).
 *
 *   x0     device, double[n] or NULL.  NULL = the uniform start 1/n of
 *          Alg. 1; otherwise a warm start, entrywise > 0 and finite.
 *   tol    tau > 0: stop when (lambda_max - lambda_min)/lambda_min < tau.
 *   x_out  device, double[n]: the iterate whose TTSV1 met the test,
 *          normalised to ||x||_1 = 1 (Alg. 1).  May alias x0.
 *   info   host, nullable: iteration counts and the final eigenvalue bounds.
 *
 * Requires a connected hypergraph with no isolated vertex (the
 * Perron-Frobenius condition stated in Sec. II): else EDISCONNECTED.
 * ENOTCONV if max_iter passes did not meet tol (x_out and info then hold the
 * last iterate); ENUMERIC if a non-finite or non-positive value appears;
 * EINVAL for a bad x0 or tol.  Synchronises the plan's stream.
 */
int heigvec_solve(sttsv_plan_t plan, const double* x0, double tol, double* x_out,
                  sttsv_solve_info* info);

/* As heigvec_solve with options (opts host, nullable = defaults). */
int heigvec_solve_ex(sttsv_plan_t plan, const double* x0, double tol,
                     const sttsv_solve_opts* opts, double* x_out,
                     sttsv_solve_info* info);

/* ---- many hypergraphs in one plan -------------------------------------- */

/* One hypergraph of a batch (host CSR, same rules as sttsv_plan's arguments;
 * each graph has its own vertex count n and tensor order r). */
typedef struct {
    const int64_t* eptr;
    const int32_t* eidx;
    int64_t m;
    int32_t n;
    int32_t r;
    const double* w;     /* nullable: edge weights, as sttsv_opts.edge_weights */
} sttsv_graph_desc;

/*
 * sttsv_plan_batch -- one plan over G hypergraphs (their disjoint union).
 *
 * Graph g's vertices are numbered after those of graphs 0..g-1: vectors
 * passed to sttsv_apply / heigvec_solve_batch on a batch plan are the
 * concatenation of the per-graph vectors in graph order (offsets from
 * sttsv_plan_graph_info).  Edges of all graphs share the edge-kernel
 * launches (buckets keyed by (r, |e|)), and every graph's y is bitwise
 * identical to what a single-graph plan of it returns.
 *   G    >= 1;  gs  host, G descriptors (copied);  opts, out as sttsv_plan.
 * Errors: as sttsv_plan, for any graph.
 */
int sttsv_plan_batch(int32_t G, const sttsv_graph_desc* gs, const sttsv_opts* opts,
                     sttsv_plan_t* out);

/*
 * heigvec_solve_batch -- Alg. 1 for every graph of a plan at once, in one
 * captured hipGraph per check_every iterations; a graph that meets its test
 * is masked (its edges skipped, its x frozen) while the others go on.
 *   x0     device, concatenated double[n_total] warm starts, or NULL (uniform).
 *   x_out  device, concatenated double[n_total]; each graph's slice has l1 norm 1.
 *   infos  host, G entries (nullable).
 * Returns the worst per-graph status (EINVAL > ENUMERIC > ENOTCONV > OK);
 * EDISCONNECTED if any graph is not connected.  Synchronous.
 */
int heigvec_solve_batch(sttsv_plan_t plan, const double* x0, double tol,
                        const sttsv_solve_opts* opts, double* x_out,
                        sttsv_solve_info* infos);

/* Vertex offset, vertex count, edge count, order and connectivity of graph g. */
typedef struct {
    int64_t m;
    int32_t n, r, voff, connected;
} sttsv_graph_info;

int sttsv_plan_graph_info(sttsv_plan_t plan, int32_t g, sttsv_graph_info* info);

/* ---- learned warm start ------------------------------------------------ */
/*
 * A small hypergraph message-passing network predicts log x (up to a
 * constant) for the H-eigenvector centrality, to start Alg. 1 closer to its
 * fixed point.  Hidden width 64; features of vertex v: log(1+d_v), mean
 * log|e| over its edges, log(d_v)/(r-1), log(1 + sum over its edges of
 * (|e|-1)).  H0 = relu(F W0 + b0); two layers of {vertex->edge mean,
 * edge->vertex mean A, H = relu([H, A] W + b)}; score s = H2 w_out + b_out;
 * warm start x0 = exp(s - max s)/sum.  Dense products: BF16 inputs and
 * weights on the matrix cores, FP32 accumulation; FP32 master weights and
 * Adam.  Deterministic (fixed-order reductions).
 *
 * Parameters are one packed FP32 vector of STTSV_MPNN_NPARAM entries:
 * W0 (16 x 64, row-major, rows 4..15 unused = 0), b0 (64), W1 (128 x 64),
 * b1 (64), W2 (128 x 64), b2 (64), w_out (64), b_out (1).
 * All calls run on the default stream and are asynchronous unless stated.
 */
#define STTSV_MPNN_HIDDEN 64
#define STTSV_MPNN_NPARAM 17665

typedef struct sttsv_mpnn_graph_s* sttsv_mpnn_graph_t;
typedef struct sttsv_mpnn_s* sttsv_mpnn_t;

/* Device copy of a hypergraph for the network (host CSR as in sttsv_plan;
 * r >= 2 is only used by the features).  Synchronous.  EINVAL / ENOMEM. */
int sttsv_mpnn_graph(const int64_t* eptr, const int32_t* eidx, int64_t m, int32_t n, int32_t r,
                     sttsv_mpnn_graph_t* out);
int sttsv_mpnn_graph_destroy(sttsv_mpnn_graph_t g);

/* Network with initial parameters (host, STTSV_MPNN_NPARAM floats); Adam
 * moments start at 0.  Synchronous. */
int sttsv_mpnn_create(const float* params, sttsv_mpnn_t* out);
int sttsv_mpnn_destroy(sttsv_mpnn_t net);

/* Copy the current parameters and/or the last gradients to host memory
 * (either pointer nullable, STTSV_MPNN_NPARAM floats each).  Synchronous. */
int sttsv_mpnn_params(sttsv_mpnn_t net, float* params_out, float* grads_out);

/* Scores s (device float[n], nullable to keep them internal). */
int sttsv_mpnn_forward(sttsv_mpnn_t net, sttsv_mpnn_graph_t g, float* scores);

/* Forward + loss L = mean(u^2), u = (s - mean s) - (log x* - mean log x*),
 * + backward: gradients kept in the network.  x_star device double[n] > 0.
 * loss host, nullable (when given the call synchronises). */
int sttsv_mpnn_loss_grad(sttsv_mpnn_t net, sttsv_mpnn_graph_t g, const double* x_star, float* loss);

/* One Adam step with the stored gradients (bias-corrected). */
int sttsv_mpnn_adam(sttsv_mpnn_t net, float lr, float beta1, float beta2, float eps);

/* Warm start x0 = exp(s - max s) / sum (device double[n], > 0, l1 norm 1). */
int sttsv_mpnn_warm_start(sttsv_mpnn_t net, sttsv_mpnn_graph_t g, double* x0);

/*
 * sttsv_mpnn_query -- host copy (as FP32) of a value the last forward or
 * loss_grad call on graph g left in the network's workspace (for tests that
 * check each stage of the network against the FP64 oracle):
 *   STTSV_MQ_X0          n x 16  features (bf16 values, columns >= 4 zero)
 *   STTSV_MQ_Z0/Z1/Z2    n x 64  pre-activations of the three dense layers
 *   STTSV_MQ_X1/X2       n x 128 bf16 inputs [H, A] of dense layers 1 and 2
 *   STTSV_MQ_S, _DS      n       scores; dL/ds (after loss_grad)
 *   STTSV_MQ_DZ, _DH     n x 64  dL/dZ0 and dL/dH0 (after loss_grad)
 *   STTSV_MQ_DA          n x 64  dL/dA of layer 1 (after loss_grad)
 *   STTSV_MQ_DE          m x 64  dL/dEd of layer 1 (after loss_grad)
 * All row-major.  out host, count entries (EINVAL unless count is the size
 * above, or the workspace was never sized for g).  Synchronous.
 */
#define STTSV_MQ_Z0  0
#define STTSV_MQ_Z1  1
#define STTSV_MQ_Z2  2
#define STTSV_MQ_X1  3
#define STTSV_MQ_X2  4
#define STTSV_MQ_S   5
#define STTSV_MQ_DS  6
#define STTSV_MQ_DZ  7
#define STTSV_MQ_DA  8
#define STTSV_MQ_DE  9
#define STTSV_MQ_DH 10
#define STTSV_MQ_X0 11
int sttsv_mpnn_query(sttsv_mpnn_t net, sttsv_mpnn_graph_t g, int32_t what, float* out, int64_t count);

/* ---- the CCSS forest and the memoised STTSV over it (Alg. 4) ---------- */

typedef struct {
    int32_t levels;        /* depth of the forest (longest path)                 */
    int64_t nodes;         /* distinct path prefixes                             */
    int64_t roots;         /* level-1 nodes                                      */
    int64_t convolutions;  /* forest edges = nodes - roots: one truncated        */
                           /* series product each per STTSV                      */
    int64_t leaves;        /* special leaves: member slots of edges of size >= 2 */
    int64_t device_bytes;  /* device memory the forest and its workspaces hold   */
    double  build_ms;      /* host wall time of the construction                 */
} sttsv_ccss_info;

/*
 * sttsv_ccss_build -- build the Compound CSS forest of the plan's hypergraph
 * on the device (Sec. III): for every member u of every edge e of size >= 2
 * the path e \ {u}, members in the plan's degree-rank order, is a
 * root-to-level-(|e|-1) path; nodes are distinct prefixes, numbered per
 * level in (parent, vertex rank) order; (e, u) is a special leaf of the
 * node ending its path.  Built level by level with device radix sorts of
 * (parent, vertex) keys.  Replaces an earlier forest of the plan.
 *   info  host, nullable: sizes of the forest.
 * Synchronous.  Errors: EINVAL (NULL plan), ENOTSUP (batched plan: the
 * workspace windows follow one tensor order), ENOMEM, EHIP.
 */
int sttsv_ccss_build(sttsv_plan_t plan, sttsv_ccss_info* info);

/*
 * sttsv_apply_ccss -- y = B x^(r-1) by Alg. 4 over the forest (Sec. IV-B):
 * one truncated product per forest edge, each prefix's workspace computed
 * once and shared by every edge -- of any size -- whose member paths pass
 * through it; a special leaf (e, u) adds w(e)/|beta(e)| (r-1)! times the
 * coefficient of t^(r-1) in e^(x_u t) times its path's product.  FP64.
 * x, y device double[n] (x != y); the plan's node reduction sums the leaf
 * values, so y is bitwise reproducible (not bitwise equal to sttsv_apply's).
 * Asynchronous on the plan's stream; shares the plan's contribution buffer
 * with sttsv_apply.  Errors: EINVAL (NULL argument, x == y, no forest built),
 * EHIP.
 */
int sttsv_apply_ccss(sttsv_plan_t plan, const double* x, double* y);

/* ---- symmetric CP decomposition of the blowup tensor (Sec. I) -------- */

/* The model B ~ sum_l lambda_l a_l^(o r), l < R, fitted by least squares:
 *   f(lambda, A) = ||B||^2 - 2 sum_l lambda_l B a_l^r
 *                  + sum_{l,m} lambda_l lambda_m (a_l . a_m)^r,
 *   df/dlambda_l = -2 B a_l^r + 2 sum_m lambda_m (a_l . a_m)^r,
 *   df/da_l      = 2 r lambda_l (-B a_l^(r-1) + sum_m lambda_m (a_l . a_m)^(r-1) a_m).
 * Each evaluation takes R STTSVs (FP64 series), the step Sec. I names as the
 * bottleneck of this decomposition.  ||B||^2 sums W_S^2 / |beta(S)| over the
 * distinct vertex sets S, W_S the summed weight of the edges on S. */
#define STTSV_CP_MAX_R 32

typedef struct {
    int32_t iterations;   /* accepted steps                                  */
    int32_t halvings;     /* step halvings over all iterations               */
    double  f0;           /* objective at the start                          */
    double  f;            /* objective at the end                            */
    double  norm2;        /* ||B||^2                                         */
} sttsv_cp_info;

/*
 * sttsv_cp_objective_grad -- f, df/dA and df/dlambda at (A, lambda).
 *   R       1..STTSV_CP_MAX_R terms.
 *   A       device double[R * n]: column l (a_l) at A + l n, vertex order.
 *   lambda  device double[R].
 *   f       host double: the objective.
 *   dA      device double[R * n], same layout as A; dlambda device double[R].
 * Inner products are summed in a fixed tree, so results are bitwise
 * reproducible.  Synchronous (f is on the host on return); allocates a
 * workspace of (R + R^2 + 256 (R^2 + R)) doubles per call.  Errors: EINVAL
 * (NULL argument, R out of range), ENOTSUP (batched plan), ENOMEM, EHIP.
 */
int sttsv_cp_objective_grad(sttsv_plan_t plan, int32_t R, const double* A, const double* lambda, double* f,
                            double* dA, double* dlambda);

/*
 * sym_cp_descent -- gradient descent on (lambda, A) with Armijo
 * backtracking (the paper names the decomposition, not a method; this plain
 * one is taken): with g the gradient and t the trial step (first: step),
 * halve t until f(x - t g) <= f(x) - 1e-4 t ||g||^2 or 40 halvings were
 * taken, accept x - t g, and start the next iteration from 2 t.
 *   A, lambda  device, as above: the start on entry, the result on return.
 *   iters      iterations (>= 0); step > 0.
 *   info       host, nullable.
 * Synchronous.  Errors: EINVAL, ENOTSUP (batched plan), ENOMEM, EHIP.
 */
int sym_cp_descent(sttsv_plan_t plan, int32_t R, double* A, double* lambda, int32_t iters, double step,
                   sttsv_cp_info* info);

/* ---- plan introspection (host copies; used to check the layout) ------- */
#define STTSV_Q_PERM        0  /* int64[m]   input index of canonical edge c      */
#define STTSV_Q_MEM         1  /* int64[nnz] member slots (original vertex ids)   */
#define STTSV_Q_BUCKET_K    2  /* int64[nb]  edge size of each bucket (buckets are  */
                               /*            ordered by (r, k); see BUCKET_R)      */
#define STTSV_Q_BUCKET_M    3  /* int64[nb]  edge count of each bucket            */
#define STTSV_Q_TPTR        4  /* int64[n+1] node-major offsets                   */
#define STTSV_Q_TSLOT       5  /* int64[nnz] node-major slot lists                */
#define STTSV_Q_WEIGHTS     6  /* double[r+1] w/|beta| (r-1)! per size (index k)  */
#define STTSV_Q_SCALE_EXP   7  /* int64[r+1]  FP32 series scale exponent per size */
                               /*             (INT32_MIN: size runs in FP64), for */
                               /*             the first graph's order r           */
#define STTSV_Q_BUCKET_R    8  /* int64[nb]  tensor order of each bucket          */
#define STTSV_Q_CONTRIB    10  /* double[nnz] the per-incidence contributions of  */
                               /*            the last apply, in node-major order  */
                               /*            (an FP32 apply stores them as 32-bit */
                               /*            words: widened back exactly here;    */
                               /*            synchronises the plan's stream)      */
#define STTSV_Q_BUCKET_LANES 11 /* int64[nb] lanes per edge of each bucket's FP64 */
                               /*            kernel (0: one lane per edge; else a  */
                               /*            lane group, see sttsv_apply_timed)    */
#define STTSV_Q_BUCKET_STACK 16 /* int64[nb] where each bucket's generic-kernel   */
                               /*            suffix stacks live: bit 0 FP64, bit 1 */
                               /*            FP32 series (1 = LDS, 0 = global    */
                               /*            memory or no generic kernel); bit 2 */
                               /*            FP64, bit 3 FP32: 1 = no stack (the  */
                               /*            suffix series are recomputed; same  */
                               /*            bits of y)                          */
#define STTSV_Q_CCSS_LEVEL_N 12 /* int64[levels] nodes per level of the forest   */
#define STTSV_Q_CCSS_VERT   13  /* int64[nodes] vertex id of every node, level by  */
                                /*            level, in node order                 */
#define STTSV_Q_CCSS_PARENT 14  /* int64[nodes] parent's index in the level above  */
                                /*            (-1 on level 1)                      */
#define STTSV_Q_CCSS_LEAF   15  /* int64[nnz] node (index in its level) owning the */
                                /*            special leaf of every member slot    */
                                /*            (slot order as STTSV_Q_MEM; -1 for   */
                                /*            size-1 edges).  CCSS queries need a  */
                                /*            built forest (EINVAL otherwise)      */
#define STTSV_Q_BUCKET_RUNS 9  /* int64[nb]  FP64 prefix-reuse runs of each bucket */
                               /*            (0: the bucket does not reuse; else */
                               /*            m - runs edges take a shared prefix) */

/* Sizes of the plan: m, n, largest r, nnz, number of buckets, number of
 * graphs, connected flag (all graphs), and the number of streams the FP64
 * edge launches are spread over (1 with STTSV_FLAG_ONE_STREAM, and for plans
 * whose estimated edge work is too small to gain from the overlap). */
typedef struct {
    int64_t m, nnz;
    int32_t n, r, nbuckets, connected;
    int64_t device_bytes;  /* device memory held by the plan                     */
    int32_t graphs;
    int32_t lanes;
} sttsv_plan_info;

int sttsv_plan_get_info(sttsv_plan_t plan, sttsv_plan_info* info);

/* Copy one of the arrays above into host memory `out` of `count` elements
 * (EINVAL if count is not the array's length). */
int sttsv_plan_query(sttsv_plan_t plan, int32_t what, void* out, int64_t count);

/* Release a plan and all its device memory.  NULL is a no-op.  Waits for the
 * plan's stream first. */
int sttsv_plan_destroy(sttsv_plan_t plan);

/* Static string naming an error code. */
const char* sttsv_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* STTSV_H */
