/*
 * brt.h -- C ABI of the branching-random-tree solver for semilinear parabolic
 * PDEs on MI355X (gfx950).
 *
 * The library estimates u(x,t) for
 *
 *     u_t = a Lap(u) + f(u),   f(u) = sum_{j=0}^{7} c_j u^j,   u(x,0) = g(x),
 *
 * (problem statement of Sec. 1 of Acebron & Rodriguez-Rozas, "A new parallel
 * solver suited for arbitrary semilinear parabolic PDEs based on generalized
 * random trees", with L = a Lap and f a polynomial) at query points (x,t) by
 * Strategy A of Sec. 2.1: Monte Carlo over random branching trees whose value
 * is the product of vertex weights and of g at the leaves (eq. rep_strategyB),
 * binned by number of splits into the coefficients of a possibly divergent
 * series, which is then summed by a Pade approximant (end of Sec. 2.1 and
 * Sec. 2.4).  Every step runs in HIP kernels on one GPU.
 *
 * Conventions
 *  - Every call returns int: BRT_OK (0) or a negative BRT_E_* code.
 *    brt_last_error() returns a message for the calling thread's last error.
 *  - Structs start with struct_size = sizeof(struct); calls reject other sizes.
 *  - "host" pointers are read during the call only and never retained.
 *  - "device" pointers are caller-owned device memory (for example PyTorch
 *    tensors); the library writes them asynchronously on the given stream and
 *    never frees them.  Streams are hipStream_t passed as void* (NULL = the
 *    null stream).
 *  - The library never calls exit(); device faults surface as BRT_E_DEVICE.
 *    No C++ exception crosses the interface: a failed host allocation inside
 *    a call returns BRT_E_NOMEM.
 *
 * Randomness (the documented stream; any implementation of the method that
 * follows it walks the same trees): one Philox4x32-10 block (Salmon et al.,
 * SC'11) per tree node, key = (seed low 32 bits, seed high 32 bits), counter =
 * (node preorder index, tree index, point id, 0); word 0 is the clock uniform
 * U = (w0 + 0.5) 2^-32, word 1 the arity index floor(w1 K / 2^32), words 2-3
 * a Box-Muller pair u1 = (w2 + 0.5) 2^-32, u2 = w3 2^-32.  A node is a vertex
 * iff the FP64 product of U along its lineage (itself included) exceeds
 * theta = exp(-lambda t) computed on the host in FP64.  Strategy B (Sec. 2.2)
 * uses word 0 as the coin instead: with Q = floor(q 2^32) the node is a leaf
 * iff w0 < Q, and a vertex splits after the fraction S = (w0 - Q + 0.5) /
 * (2^32 - Q) of its time left.
 */
#ifndef BRT_H
#define BRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BRT_OK 0
#define BRT_E_ARG (-1)    /* invalid argument or struct_size */
#define BRT_E_DEVICE (-2) /* HIP runtime or kernel error */
#define BRT_E_NOMEM (-3)  /* device or host allocation failed */
#define BRT_E_BUSY (-4)   /* server admission queue full */
#define BRT_E_RANGE (-5)  /* a tree exceeded the kernel's stack depth (results of that point flagged) */
#define BRT_E_STATE (-6)  /* unknown ticket / object in the wrong state */

/* Initial data g (the u(x,0) families of the paper's examples).
 *  BRT_U0_CONST      params (g0)
 *  BRT_U0_LOGISTIC   params (A, s, x0, p, n0, n1): A (1 + exp(s (n.x - x0)))^(-p), p in {1,2,3,4}
 *                    (KPP data of Sec. 1, travelling waves of Example 3 and the Fisher wave)
 *  BRT_U0_GAUSS_SUM  u0_nterms terms (A, cx, cy, s): sum A exp(-|x - c|^2 / (2 s^2))
 *                    (heat-kernel data of Examples 1, 2 and 5)
 *  BRT_U0_COS2_BUMP  params (A, Ax, Ay): A cos^2(pi x / 2Ax) cos^2(pi y / 2Ay) for |x|<=Ax, |y|<=Ay,
 *                    else 0 (Example 4)
 * In 1-D the y parts are ignored. */
#define BRT_U0_CONST 0u
#define BRT_U0_LOGISTIC 1u
#define BRT_U0_GAUSS_SUM 2u
#define BRT_U0_COS2_BUMP 3u

/* The PDE (Sec. 1, eq. nonlinear_new with L = a Lap, constant polynomial coefficients). */
typedef struct brt_problem {
  uint32_t struct_size;
  uint32_t dim;          /* 1 or 2 */
  double diffusion;      /* a > 0; the paths are x + sqrt(2a) W (Feynman-Kac, eqs. green/SDE) */
  double coef[8];        /* c_0..c_7; c_1 is absorbed exactly into the exponential prefactor */
  uint32_t u0_kind;      /* BRT_U0_* */
  uint32_t u0_nterms;    /* BRT_U0_GAUSS_SUM: 1..8 */
  double u0_params[40];
  /* Variable coefficients (Sec. 2's c_j(x, t); Example 5): with coef_mod = BRT_COEF_MOD_GAUSS_TIME every
   * non-linear coefficient becomes c_j(x, t) = c_j exp(-beta_x x^2 - beta_y y^2) (t + t0)^(-coef_mod_pow),
   * evaluated where and when a tree splits (the split position and the PDE time left after the split).
   * The linear coefficient c_1 stays constant; BRT_COEF_MOD_GAUSS_TIME_ALL modulates c_1 too, and then c_1(x, t) u
   * is sampled as a branching with one child (it can no longer be absorbed into the prefactor e^{mu t}).
   * beta >= 0; coef_mod_pow is 0 or 1, and t0 > 0 when it is 1.  BRT_COEF_MOD_NONE (0) keeps every c_j
   * constant. */
  uint32_t coef_mod;
  uint32_t coef_mod_pow;
  double coef_mod_beta[2];
  double coef_mod_t0;
  /* Constant drift b of the operator L = a Lap + b . grad (Sec. 2.1's SDE with a constant drift term):
   * an edge of duration s moves its path by b s + sqrt(2a) W_s, exactly, with no time stepping.  Finite;
   * drift[1] must be 0 in 1-D.  {0, 0} is the paper's L = a Lap.  The domain-decomposition tail
   * (brt_pdd_*) takes drift-free problems only. */
  double drift[2];
  /* A general L (Sec. 2.1's SDE with state-dependent coefficients, integrated by the Euler scheme as in
   * Sec. 2.4): with sde = BRT_SDE_EULER every edge is integrated by Euler-Maruyama steps for the drift
   * b(x) = drift + drift_lin * x (componentwise) and the diffusion
   * sigma(x) = sqrt(2a) (1 + sigma_amp exp(-|x|^2 / (2 sigma_width^2))), i.e. the operator
   * L = sigma(x)^2/2 Lap + b(x) . grad.  An edge of duration s takes n = ceil(s / sde_dt) equal steps
   * (so the steps end at the branching times); step k of an edge draws its normals from the Philox block
   * (node, tree, point, k), step 0 from the node's own block.  sde_dt >= 1e-6; sigma_amp > -1; sigma_width
   * > 0 when sigma_amp != 0; drift_lin[1] = 0 in 1-D.  BRT_SDE_EXACT (0) takes one exact Gaussian increment
   * per edge and needs drift_lin = 0 and sigma_amp = 0.  The domain-decomposition tail takes
   * BRT_SDE_EXACT only.  The cost grows with the number of steps per edge, which is capped at 2^20 (longer
   * edges then take steps longer than sde_dt).  BRT_SDE_EULER needs FP64 paths (brt_mc.precision = 64):
   * the step count of an edge is a ceiling of its duration, which an FP32 path would round differently
   * at a step boundary; brt_problem_check returns BRT_E_ARG otherwise. */
  uint32_t sde;
  uint32_t sde_pad;
  double drift_lin[2];
  double sigma_amp;
  double sigma_width;
  double sde_dt;
} brt_problem;

#define BRT_SDE_EXACT 0u
#define BRT_SDE_EULER 1u

#define BRT_COEF_MOD_NONE 0u
#define BRT_COEF_MOD_GAUSS_TIME 1u
#define BRT_COEF_MOD_GAUSS_TIME_ALL 2u

/* Monte Carlo parameters shared by all points of one call. */
typedef struct brt_mc {
  uint32_t struct_size;
  uint32_t precision;    /* 32: paths, times and tree products in FP32 (clock product FP64, moments FP64);
                            64: everything in FP64 */
  uint64_t seed;         /* Philox key */
  double lambda;         /* clock rate > 0 (the paper's Strategy A is lambda = 1) */
  uint32_t max_order;    /* series order N_ord, 0..126: bins 0..N_ord and a tail bin */
  uint32_t prune;        /* 1: abandon a tree at its (N_ord+1)-th split (counted as overflow) */
  uint32_t node_cap;     /* abandon a tree when it would visit node number node_cap (1..2^21-1) */
  uint32_t pade_L;       /* Pade [L/M], L + M <= max_order */
  uint32_t pade_M;
  uint32_t strategy;     /* BRT_STRATEGY_A: exponential clock of rate lambda (Sec. 2.1);
                            BRT_STRATEGY_B: coin with P(leaf) = q and split after a uniform fraction of
                            the time left (Sec. 2.2) */
  double q;              /* Strategy B: leaf probability, 0 < q <= 1; without pruning the trees must be
                            subcritical, (1 - q) * mean arity < 1 */
} brt_mc;

#define BRT_STRATEGY_A 0u
#define BRT_STRATEGY_B 1u

/* Query points (host arrays, n entries each). */
typedef struct brt_points {
  uint32_t struct_size;
  uint32_t n;
  const double* x;          /* n*dim, row-major */
  const double* t;          /* n, t >= 0 */
  const uint64_t* n_trees;  /* n, 0..2^32-1 trees per point */
  const uint32_t* problem_id; /* n, index into the problem array; NULL = all 0 */
  const uint32_t* point_id;   /* n, Philox counter word 2; NULL = 0..n-1 */
  const uint32_t* tree_first; /* n, tree counter of each point's first tree (a later call continues a
                                 point's sample with fresh trees); NULL = 0 */
} brt_points;

/* The Pade step (end of Sec. 2.1; Sec. 2.4 on spurious poles and on judging an approximant across
 * numbers of coefficients).  For a requested [L/M] the degrees actually used come from the singular values
 * of the M x (M+1) linear conditions C[i][j] = a_{L+1+i-j} (i < M, j <= M; a_k = 0 for k < 0) that the
 * denominator q satisfies, C q = 0 (robust Pade of Gonnet, Guettel and Trefethen, SIAM Review 2013):
 * with s = ||a_0..a_{L+M}||_2, a singular value counts as zero when it is at most 1e-12 s; rank rho < M
 * lowers both degrees by M - rho and the test repeats; a full-rank C whose square block C[:, 1:] is rank
 * deficient (no denominator with q_0 = 1) moves to [L+1/M-1]; all-zero coefficients give [0/0].  q_0 = 1
 * and the square system (LU with partial pivoting) then give q, and u = P(1)/Q(1). */

/* Per-point flags (brt_out.flags). */
#define BRT_FLAG_POLE 1u       /* the approximant has a pole within 0.5 of the segment [0, 1] (counted by the
                                  argument principle along that contour): its value at 1 is unreliable */
#define BRT_FLAG_LOWERED 2u    /* the degrees used are below the requested [L/M] (rank test above) */
#define BRT_FLAG_OVERFLOW 4u   /* some trees were pruned */
#define BRT_FLAG_CAPPED 8u     /* some trees hit the node cap */
#define BRT_FLAG_DEPTH 16u     /* some trees exceeded the stack depth (their values are missing) */
#define BRT_FLAG_SENSITIVE 32u /* kappa = sum_k |du/da_k| |a_k| > 100: a relative error of 1e-5 in every
                                  coefficient (the accuracy of sums of FP32 paths) can move u by 1e-3 */

/* Columns of brt_out.pade_diag (doubles, BRT_PADE_DIAG per point). */
#define BRT_PADE_DIAG 6
#define BRT_DIAG_L 0           /* numerator degree used */
#define BRT_DIAG_M 1           /* denominator degree used */
#define BRT_DIAG_U_LM1 2       /* value of [L-1/M] (its own degree selection; NaN when L = 0) */
#define BRT_DIAG_U_MM1 3       /* value of [L/M-1] (NaN when M = 0) */
#define BRT_DIAG_KAPPA 4       /* sensitivity sum_k |du/da_k| |a_k| (exact gradient of the approximant) */
#define BRT_DIAG_MARGIN 5      /* how far the degree selection was from flipping: the smallest ratio of a
                                  deciding singular value to the threshold 1e-12 s, or its reciprocal
                                  (inf when no decision was needed); a lower bound of it when the full rank
                                  was settled by sigma_min(C[:, 1:]) >= 1/||C[:, 1:]^-1||_F */

/* Outputs.  All device pointers, caller-owned, each may be NULL.  B = max_order + 2. */
typedef struct brt_out {
  uint32_t struct_size;
  double* u;          /* n: Pade [L/M] value at z = 1 (u = e^{mu t} v applied) */
  double* se;         /* n: delta-method standard error of u */
  double* psum;       /* n: plain sum of all B coefficients */
  double* coef;       /* n*B: a_0..a_Nord, then the tail (Ne > N_ord, only without pruning) */
  double* coef_var;   /* n*B: variance of each coefficient estimate */
  uint64_t* hist;     /* n*(B+3): trees per bin, then overflow, capped, depth-exceeded counts */
  double* s1;         /* n*B: sum of tree values per bin (before the e^{mu t}/N scaling) */
  double* s2;         /* n*B: sum of squared tree values per bin */
  uint64_t* nodes;    /* n: tree nodes walked */
  uint32_t* flags;    /* n: BRT_FLAG_* */
  void* tree_f;       /* total trees, double: value of each tree (0 when abandoned); point i's trees
                         start at sum_{k<i} n_trees[k].  The running product is FP64 on both
                         precision paths (vertex weights reach e^{32} and overflow FP32). */
  uint32_t* tree_meta;/* total trees: bits 0-7 min(Ne,255), bit 8 overflow, bit 9 capped,
                         bit 10 depth exceeded, bits 11-31 nodes visited */
  double* pade_diag;  /* n*BRT_PADE_DIAG: degrees used, neighbour values, sensitivity, selection margin */
} brt_out;

typedef struct brt_ctx brt_ctx;
typedef struct brt_plan brt_plan;

/* Launch settings (defaults chosen by the library; brt_autotune picks them by measurement). */
typedef struct brt_launch {
  uint32_t struct_size;
  uint32_t waves_per_block;  /* 1..4 */
  uint32_t blocks_per_cu;    /* 0 = as many as fit */
  uint32_t chunk_trees;      /* trees handed to a wave at a time, multiple of 64 */
  uint32_t stack_depth;      /* LDS stack levels per lane; 0 = automatic */
} brt_launch;

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int brt_version(void);

/* Message of the calling thread's last error ("" if none). The pointer stays valid until the
 * thread's next brt_* call. */
const char* brt_last_error(void);

/* Create a context on HIP device `device`.  The context owns device scratch, cached graphs and
 * launch settings.  Errors: BRT_E_DEVICE, BRT_E_NOMEM. */
int brt_create(brt_ctx** out, int device);
void brt_destroy(brt_ctx* ctx);

/* Validate a problem and its Monte Carlo parameters (host only). */
int brt_problem_check(const brt_problem* problem, const brt_mc* mc);

/* Set / get the launch settings used by plans created afterwards. */
int brt_set_launch(brt_ctx* ctx, const brt_launch* launch);
int brt_get_launch(brt_ctx* ctx, brt_launch* launch);

/* Build a plan: normalise the problems (Strategy A change of variables of Sec. 2.1: u = v e^{mu t},
 * mu = c_1 + lambda, vertex weight K c_j / lambda e^{(j-1) mu tau}), upload the point records, cut
 * every point's trees into work chunks ordered by estimated cost, and reserve device scratch
 * (tree records unless the caller supplies brt_out.tree_f/tree_meta).  Host arrays are copied.
 * At most 64 problems per plan; all of one dim and u0_kind.  Problems that differ only in their
 * initial data (u0 parameters and term count) run as a family, their shared constants held once. */
int brt_plan_create(brt_ctx* ctx, uint32_t n_problems, const brt_problem* problems, const brt_mc* mc,
                    const brt_points* points, brt_plan** out);

/* Run a plan on `stream`: tree walk (persistent, work-stealing), per-bin moment reduction and the
 * FP64 finalize (coefficients, covariance, Pade, SE).  Asynchronous.  On a created stream (not NULL)
 * the first run with a given brt_out and stream is captured into a HIP graph (its kernels only: the
 * counters are cleared by a kernel, not a memset) and later runs with the same brt_out and stream
 * replay it; on the NULL stream, with graphs switched off (brt_plan_set_graph) or in timing mode the
 * kernels are enqueued one by one.  Both ways give bit-identical results. */
int brt_plan_execute(brt_plan* plan, const brt_out* out, void* stream);

/* Graph use of a plan: enable = 0 makes brt_plan_execute enqueue kernel by kernel on every stream
 * (default 1).  brt_plan_graph_stats reports (each pointer nullable) how many graphs the plan has
 * instantiated, how many graph launches and how many kernel-by-kernel runs it has made (host
 * counters; no synchronisation).  Errors: BRT_E_ARG (NULL plan). */
int brt_plan_set_graph(brt_plan* plan, int enable);
int brt_plan_graph_stats(const brt_plan* plan, uint64_t* captures, uint64_t* replays, uint64_t* direct);

/* Totals of a plan (host): number of points, trees, bins B, work chunks. */
int brt_plan_info(const brt_plan* plan, uint32_t* n_points, uint64_t* n_trees, uint32_t* n_bins,
                  uint32_t* n_chunks);

/* Device-side count of trees that exceeded the stack depth in the last run (synchronises). */
int brt_plan_depth_exceeded(brt_plan* plan, uint64_t* count);

/* Per-kernel timing mode (for measurement).  While enabled, brt_plan_execute enqueues the kernels
 * directly (no graph) and records HIP events on the launch stream around the walk, reduce and
 * finalize kernels of every run.  brt_plan_get_timing waits for the recorded runs, writes the summed
 * durations in milliseconds to ms[0] (walk), ms[1] (reduce), ms[2] (finalize), the number of runs to
 * *runs (nullable), and starts a new accumulation. */
int brt_plan_set_timing(brt_plan* plan, int enable);
int brt_plan_get_timing(brt_plan* plan, double* ms, uint64_t* runs);

void brt_plan_destroy(brt_plan* plan);

/* One-shot: plan_create + plan_execute + synchronise + plan_destroy.  Returns BRT_E_RANGE if any
 * tree exceeded the stack depth (other results are still written). */
int brt_solve(brt_ctx* ctx, uint32_t n_problems, const brt_problem* problems, const brt_mc* mc,
              const brt_points* points, const brt_out* out, void* stream);

/* brt_solve for callers that cannot allocate (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments and bit-identical results, with no device or
 * host allocation.  Every buffer brt_solve would allocate (problem table, point records, work chunks,
 * reduction partials, counters and, when out->tree_f / out->tree_meta are NULL, the tree records)
 * lives in one device array of the library, fixed in size, which each GPU the library runs on holds
 * until the process ends; the host tables live in fixed arrays.  Limits: at most
 * BRT_NOALLOC_MAX_POINTS points and BRT_NOALLOC_MAX_TREES trees in one call, pruning on and
 * 1 <= max_order <= BRT_NOALLOC_MAX_ORDER (the walker's stack is held in LDS only); beyond them it
 * returns BRT_E_ARG with a message and runs nothing.  All calls on one GPU share that array and
 * keep nothing from the previous call: calls that overlapped would race on it, so the library runs
 * them one at a time under a process-wide lock, and each call waits for its stream before it
 * returns.  The caller passes and owns the outputs as for brt_solve.  Returns BRT_E_RANGE if a tree
 * exceeded the stack depth. */
#define BRT_NOALLOC_MAX_POINTS 4096u
#define BRT_NOALLOC_MAX_TREES (1u << 22)
#define BRT_NOALLOC_MAX_ORDER 16u
int brt_solve_noalloc(brt_ctx* ctx, uint32_t n_problems, const brt_problem* problems, const brt_mc* mc,
                      const brt_points* points, const brt_out* out, void* stream);

/* Autotuner: time the tree walker for candidate launch settings (waves per block 1/2/4, LDS stack
 * levels 4..16, chunk sizes 256/1024/4096 trees) on the given points (subsampled to about 2^28 trees
 * when larger; fastest of three runs), set the fastest on the context (used by plans and servers
 * created afterwards) and write it to *best (nullable).  cache_path (nullable) is a JSON-lines file keyed by the GPU architecture and
 * the workload shape (precision, dim, initial-data family, arities, order, pruning): a cached entry
 * is applied without timing, a new result is appended.  Synchronises the device. */
int brt_autotune(brt_ctx* ctx, uint32_t n_problems, const brt_problem* problems, const brt_mc* mc,
                 const brt_points* points, const char* cache_path, brt_launch* best);

/* ------------------------------------------------------------------------------------------------
 * Serving: continuous batching of point-query requests (the data-parallel structure of the
 * probabilistic part of Sec. 3: independent points, each summed from independent trees).
 *
 * An engine thread runs ticks; each tick adds one round of `round_trees` trees to every unfinished
 * point of the admitted requests it covers, packing consecutive requests into shared launches (a
 * launch group closes once it holds 4096 unfinished points or 64 requests).  Requests whose problems
 * differ only in their initial data (u0 parameters and term count) share a group's walker constants;
 * a group with other differences keeps every problem's full record (slower, same results).  A point's
 * slot is freed as soon as the point finishes, not when its whole request does.
 * Admitted requests are split between two lanes with their own streams: while one lane's tick runs on
 * the device, the engine reads the other lane's results (copied back by its tick), admits requests and
 * enqueues that lane's next tick.  The reduction partials of every round stay on the device in the
 * point's slot; the finalize recomputes coefficients, Pade value and SE from them after every round.
 * A point finishes when its SE <= target_se or its trees reach max_trees; a request completes when
 * all its points finish.
 * Requests are admitted at tick boundaries while enough free slots (max_points, the memory bound)
 * remain; at most queue_cap requests wait, beyond that submit returns BRT_E_BUSY.  A point's trees
 * are addressed by (mc.seed, stream_id*1024 + point index, tree counter), so its results are
 * bit-identical whether it is served alone or in a mix.
 * ------------------------------------------------------------------------------------------------ */
typedef struct brt_server brt_server;

typedef struct brt_server_opts {
  uint32_t struct_size;
  uint32_t dim;                 /* problem family served: 1 or 2 */
  uint32_t u0_kind;             /* BRT_U0_* of every request */
  brt_mc mc;                    /* shared Monte Carlo parameters; mc.seed is the Philox key */
  uint32_t max_points;          /* device slots: points resident at once (1..2^20) */
  uint32_t round_trees;         /* trees per point per tick, a multiple of 8192 (<= 2^22) */
  uint32_t max_trees;           /* per-point cap, a multiple of round_trees (<= 2^26) */
  double target_se;             /* finish a point when its Pade SE <= target_se (0: always run to the cap) */
  uint32_t queue_cap;           /* requests waiting for admission (>= 1) */
  uint32_t max_active_requests; /* 0: no limit; 1: one request at a time (unbatched) */
} brt_server_opts;

typedef struct brt_request {
  uint32_t struct_size;
  uint32_t n;                   /* points, 1..min(1024, max_points) */
  const brt_problem* problem;   /* host; copied */
  const double* x;              /* host n*dim; copied */
  const double* t;              /* host n; copied */
  uint32_t stream_id;           /* < 2^22; the points' Philox ids are stream_id*1024 + i */
} brt_request;

typedef struct brt_result {     /* host buffers supplied by the caller, each nullable */
  uint32_t struct_size;
  double* u;                    /* n Pade values */
  double* se;                   /* n standard errors */
  double* coef;                 /* n*B coefficients (B = mc.max_order + 2) */
  uint64_t* trees;              /* n trees used per point */
  uint32_t* flags;              /* n BRT_FLAG_* */
  double latency_s;             /* written: submit to completion */
} brt_result;

typedef struct brt_server_stats {
  uint32_t struct_size;
  uint64_t submitted, completed, rejected, ticks, trees, nodes;
  double p50_latency_s, p99_latency_s, mean_latency_s;
  double busy_s;                /* device time of the ticks (HIP events around each tick, summed over lanes) */
  double span_s;                /* first submit to last completion */
  double trees_per_s;           /* trees / span_s */
} brt_server_stats;

/* Create a server on the context's device (allocates all device slots up front).  Errors:
 * BRT_E_ARG, BRT_E_NOMEM, BRT_E_DEVICE. */
int brt_server_create(brt_ctx* ctx, const brt_server_opts* opts, brt_server** out);
/* Queue a request (copies it).  BRT_E_BUSY if the admission queue is full. */
int brt_server_submit(brt_server* srv, const brt_request* req, uint64_t* ticket);
/* *done = 1 when the request is complete; then the results are written to `out` (nullable) and the
 * ticket is released.  BRT_E_STATE for an unknown ticket. */
int brt_server_poll(brt_server* srv, uint64_t ticket, brt_result* out, int* done);
/* Wait until every submitted request has completed (BRT_E_BUSY on timeout). */
int brt_server_drain(brt_server* srv, double timeout_s);
int brt_server_stats_get(brt_server* srv, brt_server_stats* out);
/* Stop the engine (requests in flight are abandoned) and free everything. */
void brt_server_destroy(brt_server* srv);

/* ------------------------------------------------------------------------------------------------
 * Domain decomposition tail (Sec. 3, the PDD algorithm): the Monte Carlo values at nodes on lines
 * of the space-time domain are interpolated into boundary data, which decouple the subdomains; each
 * subdomain is then solved by finite differences.
 *
 * Geometry.  The rectangle [x_lo, x_hi] x [y_lo, y_hi] is cut into px x py equal subdomains of
 * cx x cy fine cells (NX = px cx, NY = py cy; spacings hx = (x_hi - x_lo)/NX, hy likewise).  The cuts
 * and, with outer = BRT_PDD_OUTER_LINES, the four outer edges are lines.  Lines are numbered vertical
 * first (x = x_lo + k (x_hi - x_lo)/px, ascending k), then horizontal.  A vertical line carries ns_y
 * nodes uniform over [y_lo, y_hi], a horizontal line ns_x nodes uniform over [x_lo, x_hi], at the
 * times k T/nt (k = 1..nt); node values at t = 0 are u0.  With BRT_PDD_OUTER_ZERO the outer edges are
 * held at 0.
 *
 * Interpolation (Sec. 3, "Interpolation"): on each line the tensor product of not-a-knot cubic
 * splines over the uniform nodes, first along the line for every node time, then in time, evaluated
 * at every fine node of the line at every time level n T/n_steps.  A node on both a vertical and a
 * horizontal line takes the vertical line's value.
 *
 * Local solver (Sec. 3, "Local solver", Crank-Nicolson): the Peaceman-Rachford ADI form of
 * Crank-Nicolson for u_t = a (u_xx + u_yy) + sum_j c_j u^j on every subdomain, the reaction taken at
 * the extrapolated mid-step value (3 u^n - u^{n-1})/2 (u^{-1} = u^0):
 *     (I - rx/2 dxx) u*      = (I + ry/2 dyy) u^n + dt/2 F,
 *     (I - ry/2 dyy) u^{n+1} = (I + rx/2 dxx) u*  + dt/2 F,   rx = a dt/hx^2, ry = a dt/hy^2,
 * with u* on the vertical lines set to ((I + ry/2 dyy) g^n + (I - ry/2 dyy) g^{n+1})/2, which makes the
 * two half-steps exactly the factored Crank-Nicolson step.  All FP64.  The fields are row-major
 * (NY+1) x (NX+1) arrays of doubles, x fastest, node (i, j) at (x_lo + i hx, y_lo + j hy).
 * ------------------------------------------------------------------------------------------------ */
#define BRT_PDD_OUTER_LINES 0u
#define BRT_PDD_OUTER_ZERO 1u

typedef struct brt_pdd_grid {
  uint32_t struct_size;
  double x_lo, x_hi, y_lo, y_hi;
  uint32_t px, py;        /* subdomains per direction, 1..64 */
  uint32_t cx, cy;        /* fine cells per subdomain per direction, 2..1024 (16 lines of a subdomain stay in LDS) */
  double T;               /* final time > 0 */
  uint32_t n_steps;       /* time steps to T, 1..2^20 */
  uint32_t ns_x, ns_y;    /* nodes per horizontal / vertical line, 4..257 */
  uint32_t nt;            /* node time levels, 3..63 (with t = 0: at least 4 rows in time) */
  uint32_t outer;         /* BRT_PDD_OUTER_* */
} brt_pdd_grid;

typedef struct brt_pdd brt_pdd;

/* Create the tail for one 2-D problem on a grid: validates the grid, precomputes the tridiagonal
 * factors and allocates the device fields (three of (NY+1)(NX+1) doubles) and the boundary data
 * ((n_steps+1) x fine nodes per line, doubles).  Errors: BRT_E_ARG, BRT_E_NOMEM, BRT_E_DEVICE. */
int brt_pdd_create(brt_ctx* ctx, const brt_problem* problem, const brt_pdd_grid* grid, brt_pdd** out);
/* Node query points in line order, then time level k = 1..nt, then position along the line (host).
 * *n receives their number; xy (2n, x then y) and t (n) are written when not NULL. */
int brt_pdd_nodes(const brt_pdd* pdd, double* xy, double* t, uint64_t* n);
/* Number of lines and, per line (arrays of n_lines, each nullable): orientation (0 vertical,
 * 1 horizontal), its coordinate, and its number of fine nodes (NY+1 or NX+1). */
int brt_pdd_lines(const brt_pdd* pdd, uint32_t* n_lines, uint32_t* orient, double* coord, uint32_t* n_fine);
/* Interpolate node values (device, FP64, in the order of brt_pdd_nodes) into the boundary data of
 * every line at every time level (device, owned by pdd).  Asynchronous on `stream`. */
int brt_pdd_interpolate(brt_pdd* pdd, const double* node_values, void* stream);
/* Copy the boundary data of one line ((n_steps+1) x n_fine doubles, time level major) to dst
 * (device).  Asynchronous. */
int brt_pdd_boundary(const brt_pdd* pdd, uint32_t line, double* dst, void* stream);
/* Solve every subdomain from u0 at the grid nodes through `steps` time steps (1..n_steps) with the
 * current boundary data and write the field at step `steps` to `field` (device).  One persistent
 * cooperative launch; each phase's work items (32 lines of a subdomain, 16 for lines of more than 512
 * unknowns) are dealt statically to the blocks, and phases are separated by a barrier among the
 * blocks that own the same subdomains: one per subdomain or one per die when blocks and subdomains
 * split evenly (see brt_pdd_get_barrier), else one over the grid.  Asynchronous; BRT_E_DEVICE if a barrier timed out (reported
 * by the next brt_pdd_* call that synchronises: brt_pdd_get_timing). */
int brt_pdd_solve(brt_pdd* pdd, uint32_t steps, double* field, void* stream);
/* The whole tail: Monte Carlo at the nodes (a plan with `mc` and trees_per_node trees per node,
 * Pade values), interpolation, and the solve through n_steps.  node_u (device, nullable) receives the
 * node values.  Asynchronous. */
int brt_pdd_run(brt_pdd* pdd, const brt_mc* mc, uint64_t trees_per_node, double* node_u, double* field,
                void* stream);
/* Wait for the last run / solve and report its stage times in ms (events on its stream):
 * ms[0] Monte Carlo (0 after brt_pdd_solve), ms[1] interpolation, ms[2] subdomain solves; BRT_E_DEVICE
 * if the solver's grid barrier timed out. */
int brt_pdd_get_timing(brt_pdd* pdd, double* ms);
/* Barrier placement of the last solve (waits for it): *groups receives the number of barrier groups
 * (one per subdomain when the blocks split evenly over them and the subdomains over the dies, else 8
 * when blocks and subdomains split evenly over the dies, else 1; 0 before any solve) and
 * *die_local how many of them had all their blocks on one die.  Such a group synchronises through
 * its die's L2 alone (no L2 write-back at its barriers); the others use device-scope fences.  The
 * result does not depend on the placement.  Errors: BRT_E_ARG (NULL argument), BRT_E_DEVICE. */
int brt_pdd_get_barrier(brt_pdd* pdd, uint32_t* groups, uint32_t* die_local);
void brt_pdd_destroy(brt_pdd* pdd);

#ifdef __cplusplus
}
#endif
#endif /* BRT_H */
