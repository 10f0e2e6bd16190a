/*
 * pr.h -- C ABI of the componentwise PageRank library (libpr.so) for MI355X.
 *
 * Method: Engstrom & Silvestrov, "Graph partitioning and a componentwise
 * PageRank algorithm" (arXiv 1609.09068).  The library computes the
 * non-normalised PageRank R^(3) of Def. 3.5, i.e. the solution of
 *
 *        (I - c A^T) R = W                                          (Sec. 4.3)
 *
 * where A is the adjacency matrix of the input graph with every non-zero row
 * scaled to sum to one (Def. 3.4).  Self-loops are ignored by default, as in
 * the experiments (Sec. 5.2), or kept in A with the build option keep_loops
 * (the general definition); the partition never depends on them.  A
 * repeated edge counts with its multiplicity in A and in the out-degree, so
 * a weighted graph with integer weights (a Markov chain's transition
 * weights, a_uv = w_uv / sum_x w_ux) is passed exactly by repeating an edge
 * of weight k k times.
 *
 * Conventions for every entry point
 *  - A graph is CSR over out-edges: row_ptr[n+1] (int64, row_ptr[0] == 0,
 *    non-decreasing) and col_idx[m] (int32 in [0, n)), m = row_ptr[n].
 *    Host pointers; the caller keeps ownership and the library never keeps a
 *    caller pointer beyond the call.
 *  - Vertex ids are the caller's ids; every output that is indexed by vertex
 *    uses them.
 *  - Return value: PR_OK (0) on success, PR_NOT_CONVERGED (1) when an
 *    iteration limit was hit (outputs are still written), a negative PR_E*
 *    code on failure.  On failure nothing is written to outputs and
 *    pr_last_error() describes the cause.
 *  - Handles (pr_partition_t, pr_levels_t, pr_mlp_t) are owned by the library and
 *    released with pr_free().  A handle must not be used by two threads at
 *    the same time.
 *  - hip_stream is a hipStream_t (NULL = the null stream).  Device buffers
 *    passed in must be valid on the current HIP device.
 */
#ifndef PR_H_
#define PR_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define PR_OK 0
#define PR_NOT_CONVERGED 1
#define PR_EINVAL (-1)  /* bad argument: CSR, c outside (0,1), eps <= 0, W < 0 or not finite */
#define PR_ENOMEM (-2)  /* host or device allocation failed */
#define PR_EHIP (-3)    /* a HIP runtime call failed; the message carries its error string */
#define PR_EHANDLE (-4) /* NULL, unknown, freed, or wrong kind of handle */

typedef struct pr_partition_s pr_partition_t;
typedef struct pr_levels_s pr_levels_t;
typedef struct pr_mlp_s pr_mlp_t;

/* ------------------------------------------------------------- partition */

/*
 * pr_partition -- SCC/CAC partition of Sec. 4.1 (Theorem 3.1), on the host.
 *
 * Runs the modified Tarjan depth-first search of Sec. 4.1 (iterative, so a
 * path of 10^7 vertices is fine): strongly connected components are found as
 * in Tarjan's algorithm, levels are propagated during the search, and a
 * one-vertex component that points to CACs one level below it (and to no SCC
 * of two or more vertices on that level) is merged with all of them.
 * flags: must be 0.
 * Result (read with pr_partition_get) is the unique partition of
 * Theorem 3.1 in canonical form:
 *   comp[v]        component id, numbered in order of first appearance while
 *                  scanning v = 0..n-1 (Sec. 4.1, numbering pass)
 *   comp_level[k]  0-based level (Def. 3.3): a component with no edge to
 *                  another component has level 0
 *   comp_type[k]   1 = SCC of two or more vertices, 0 = CAC (one-vertex
 *                  components are CACs)
 *   comp_size[k]   number of vertices
 * Errors: PR_EINVAL for a malformed CSR or n outside [0, 2^31-2].
 */
int32_t pr_partition(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                     uint32_t flags, pr_partition_t** out);

/*
 * pr_partition_get -- copy the partition out.  Every pointer may be NULL to
 * skip that output; comp holds n entries, the per-component arrays hold
 * *n_comp entries (query n_comp first with the other pointers NULL).
 */
int32_t pr_partition_get(const pr_partition_t* p, int32_t* comp, int32_t* comp_level,
                         uint8_t* comp_type, int32_t* comp_size, int64_t* n_comp,
                         int32_t* n_levels);

/* ------------------------------------------------------------- the plan */

typedef struct pr_build_opts {
  /* SCCs with at most small_cutoff vertices (<= 256) are iterated by one
     wavefront each, their vector kept in LDS; 0 = default (64). */
  int32_t small_cutoff;
  /* SCCs with more than small_cutoff vertices and more internal edges than
     team_edges are iterated by every workgroup of the device in a gang
     phase (all such SCCs of one level together, one kernel launch per
     series term); the others by one workgroup each.  0 = default. */
  int32_t team_edges;
  /* wavefront lanes given to one row in the SCC product: rows_per_wave in
     {1, 4, 16, 64} rows share a 64-lane wavefront; 0 = default (16). */
  int32_t rows_per_wave;
  /* 1 = also keep the whole-graph pull CSR needed by method PLAIN. */
  int32_t build_plain;
  /* Autotuner of the launch shape: 0 = off (use the three fields above);
     2 = sweep rows_per_wave {1, 4, 16, 64} x small_cutoff {16, 64} x
     team_edges {16384, 65536}, timing solves of this plan on the device
     (W = 1, c = 0.85, eps 1e-6, mixed precision; method PLAIN too when
     build_plain), and keep the fastest; 1 = as 2 unless this graph was tuned
     before on this device: in this process, or in the text file named by
     the environment variable PR_AUTOTUNE_CACHE (read and appended to).
     The choice is reported by pr_levels_get_info. */
  int32_t autotune;
  /* 1 = keep self-loops in A (the general Def. 3.4: a loop counts in its
     vertex's out-degree; an SCC's series uses the diagonal; a one-vertex or
     CAC vertex's collected rank is divided by 1 - c a_vv, Sec. 4.3 and
     4.3.1).  0 (default) = ignore them, as in the paper's experiments.  The
     partition does not depend on loops. */
  int32_t keep_loops;
  /* workgroups per CU of the segment kernel with the tail estimate (FP32 or
     FP64 terms, no starting guess, unweighted, 16 or 64 rows per
     wavefront): 2 (more registers, no spills; best where a segment's chain
     of dependencies sets its time) or 3 (best where many SCC items are in
     flight at once).  0 (default) = 2, or the autotuner's choice when
     autotune is on (it times both on the chosen shape).  Other variants are
     unaffected. */
  int32_t seg_waves;
  int32_t reserved[5];
} pr_build_opts;

void pr_default_build_opts(pr_build_opts* o);

/*
 * pr_build_levels -- the intermediate step of Sec. 4.2, on the device.
 *
 * Copies the CSR to the device and builds, with HIP kernels, the solve
 * plan: components sorted by level (descending), type and size (descending),
 * ties by id (Sec. 4.2); vertices renumbered level-major and component-major
 * (topological order inside CACs); edges split into the pull CSR of edges
 * between components (used once, eq. PR:levels) and of edges inside
 * components; 1/outdeg; the work list of the persistent solve kernel.
 * p must come from pr_partition on the same graph (n and the CSR must match).
 * opts NULL = defaults.  The plan stays resident on the current device.
 * Errors: PR_EINVAL (mismatch, m >= 2^31), PR_ENOMEM, PR_EHIP.
 */
int32_t pr_build_levels(const pr_partition_t* p, int64_t n, const int64_t* row_ptr,
                        const int32_t* col_idx, const pr_build_opts* opts, void* hip_stream,
                        pr_levels_t** out);

/*
 * pr_build_levels_weighted -- the same plan for a weighted graph: a Markov
 * chain's transition weights (Def. 3.4, where A's non-zero rows are scaled
 * to sum to one; Sec. 4.3.1 uses the entries a_wu of that A).
 *
 * weight: host array of m doubles, one per edge in col_idx order; edge
 * u -> v gets a_uv = w_uv / s_u with s_u the total weight of u's out-edges
 * (self-loops only with keep_loops, repeated edges add up).  Weights must be
 * finite and non-negative; a zero weight leaves the edge in the partition
 * (the components and levels are those of the graph) but adds nothing to A,
 * and a vertex whose out-edges all weigh zero is dangling.  The array is
 * copied; the caller keeps ownership.  The partition is the unweighted one
 * (pr_partition on the same row_ptr / col_idx).
 *
 * Solves on a weighted plan run the same kernels with one multiply by the
 * edge weight in every gather (FP64 weights for x, W' and the residual, an
 * FP32 copy for FP32 series terms) and accept every option except
 * warm_start (PR_EINVAL: the network's features are those of unweighted
 * graphs).  The FP64 residual certificate uses the FP64 weights.
 * Errors: as pr_build_levels, and PR_EINVAL for a NULL, negative or
 * non-finite weight (the message names the first bad edge).
 */
int32_t pr_build_levels_weighted(const pr_partition_t* p, int64_t n, const int64_t* row_ptr,
                                 const int32_t* col_idx, const double* weight, const pr_build_opts* opts,
                                 void* hip_stream, pr_levels_t** out);

typedef struct pr_levels_info {
  int64_t n, m;             /* vertices, edges without self-loops */
  int64_t n_comp, n_levels;
  int64_t n_scc, n_cac, n_singleton;  /* components by kind */
  int64_t v_scc, v_cac, v_singleton;  /* vertices by kind of component */
  int64_t m_scc_internal;   /* edges inside SCCs (iterated) */
  int64_t m_cac_internal;   /* edges inside CACs, one-vertex components' kept loops included (used once) */
  int64_t m_between;        /* edges between components (used once) */
  int64_t n_items;          /* work items of the persistent segment kernels */
  int64_t n_gangs, n_gang_scc; /* gang phases, SCCs iterated in gang phases */
  int64_t v_gang;           /* vertices of the SCCs iterated in gang phases */
  int64_t m_gang_internal;  /* their internal edges (touched once per term) */
  int64_t m_gang_between;   /* edges entering them from higher levels */
  int64_t n_phases;         /* segment and gang phases of the componentwise solve */
  int64_t n_hubs;           /* rows summed in pieces (more than 2048 in-edges), all gangs */
  int32_t rows_per_wave, small_cutoff, team_edges, grid_wgs;
  int32_t seg_waves;        /* workgroups per CU of the tail-estimate segment kernel this plan runs
                               (2 or 3; 3 only when asked for and the plan is unweighted at 16 or 64
                               rows per wavefront) */
  int32_t reserved_i32;
} pr_levels_info;

int32_t pr_levels_get_info(const pr_levels_t* lv, pr_levels_info* info);

/* ------------------------------------------------------------- the solve */

#define PR_METHOD_COMPONENTWISE 0 /* level by level, Sec. 4.3 */
#define PR_METHOD_PLAIN 1         /* whole-graph power series, Sec. 4.3.2 / Sec. 5.2 method 1 */

#define PR_STOP_CERT_L1 0      /* per component: ||P_k||_1 <= eps (1-c) ||W'_C||_1 */
#define PR_STOP_PAPER_MAXABS 1 /* per component: max(P_k) < tol (listing of Sec. 4.3.2) */

#define PR_PREC_MIXED 0 /* series terms and SpMV in FP32; R, sums, norms, boundary mass in FP64 */
#define PR_PREC_FP64 1  /* everything in FP64 */
#define PR_PREC_AUTO 2  /* PR_PREC_MIXED when eps >= 2^-23 / (1 - c) (with PR_STOP_CERT_L1), else
                           PR_PREC_FP64: FP32 terms leave a relative error of about 2^-24 / (1 - c)
                           (the rounding of each term, carried through the series), so below that
                           target the refinement rounds would cost more than FP64 terms.
                           PR_STOP_PAPER_MAXABS: PR_PREC_MIXED.  pr_solve_stats.precision_used
                           reports the choice. */

typedef struct pr_solve_opts {
  int32_t method;    /* PR_METHOD_* */
  int32_t stop;      /* PR_STOP_* */
  int32_t precision; /* PR_PREC_* */
  int32_t use_graph; /* 1 = capture the launch sequence in a hipGraph and replay it */
  double eps;        /* PR_STOP_CERT_L1 target (relative 1-norm error bound); default 1e-6 */
  double tol;        /* PR_STOP_PAPER_MAXABS threshold; default 1e-9 */
  int64_t max_iter;  /* per-component iteration cap; default 100000 */
  pr_mlp_t* warm_start;/* NULL = start every SCC from P_0 = W' (Sec. 4.3.2) */
  int32_t trace;        /* 1 = record the item timeline (pr_levels_debug what = 4); slows the solve */
  int32_t kernel_timing;/* 1 = HIP events around every launch; per-family times land in the stats
                           (ignored with use_graph) */
  int32_t warm_scope;   /* with warm_start: 0 = only the SCCs iterated in gang phases (the large
                           ones, where the guess's two extra passes cost less than the terms it
                           saves), 1 = every SCC */
  int32_t small_direct; /* SCCs of at most this many vertices (0..80; default 0 = none) are solved
                           directly instead of iterated: (I - cA_CC^T)R_C = W'_C by FP64
                           Gauss-Jordan elimination in LDS without pivoting (the matrix is column
                           diagonally dominant), the paper's choice for small SCCs in the
                           per-component method dispatch of Sec. 4.3.  The matrix must fit the
                           LDS of the SCC's item: up to 24 vertices for an SCC run by one
                           wavefront (at most small_cutoff vertices), up to 80 for one run by a
                           workgroup; a plan built with small_cutoff <= 24 therefore solves every
                           SCC of up to small_direct vertices directly.  Either path gives the same
                           R bit for bit.  Such an SCC counts zero terms; its FP64 residual enters
                           the certificate. */
  int32_t tail_estimate;/* 1 = with PR_STOP_CERT_L1, every iterated SCC may also stop on a geometric
                           estimate of the rest of its series (Sec. 4.3.2 series, Sec. 4.4 error):
                           after term P_{k+1}, with rho = ||P_k||/||P_{k-1}|| < 1, it takes
                           R' = P_0 + ... + P_k + rho/(1-rho) P_k once ||P_{k+1} - rho P_k||_1 /
                           ((1-rho)(1-c)) <= eps ||W'_C||_1, which bounds ||R' - R*_C||_1 exactly as
                           the plain rule does (the residual of R' is (P_{k+1} - rho P_k)/(1-rho)).
                           The plain test is tried first.  After a kept starting guess the rule
                           runs on the residual series r_0, r_1, ... (rho from r_2 on).  With
                           PR_METHOD_PLAIN the rule runs on the whole graph's series.
                           Default 0. */
  int32_t refine;       /* FP64 residual certificate and refinement (Sec. 4.4): after the solve,
                           r = W - (I - c A^T) R is formed in FP64 over every edge and
                           cert_rel = ||r||_1 / ((1-c) ||R||_1), a bound that covers the rounding
                           of FP32 terms as well as the truncation of the series.  While it exceeds
                           eps (PR_STOP_CERT_L1 only), a correction solve (I - c A^T) d = r by the
                           same method, to the looser target 0.25 eps / cert_rel, and R += d.
                           0 (default) = at most 2 such rounds; k > 0 = at most k; -1 = no residual
                           pass (cert_rel is then the truncation bound alone). */
  int32_t cold;         /* 1 = launch every gang phase (large SCCs, or the whole graph for
                           PR_METHOD_PLAIN) for the worst-case term bound instead of the terms
                           earlier solves of this plan needed plus a margin: the launch cost of a
                           first solve.  Results do not depend on it.  Default 0. */
  int32_t gs_blocks;    /* 0 (default) = every SCC by the power series.  1..8 = the SCCs that one
                           workgroup iterates with their rows and slots in registers (above
                           small_cutoff, at most 1024 rows and 1024 slots, below team_edges) take
                           block Gauss-Seidel sweeps instead, the alternative Sec. 4.3.2 names:
                           the component's rows in plan order cut into gs_blocks blocks, each
                           block updated from the newest values of the blocks before it; the
                           component stops once ||R_new - R_old||_1 <= eps (1 - c) ||W'_C||_1
                           (the certificate adds c ||dR||_1 / (1 - c)).  One block is the Jacobi
                           iteration (the series, iterated on R).  Not with tail_estimate,
                           warm_start or a weighted plan (PR_EINVAL). */
} pr_solve_opts;

void pr_default_solve_opts(pr_solve_opts* o);

typedef struct pr_solve_stats {
  int64_t edge_iters;   /* edges touched: iterations x internal edges of each SCC, plus every other edge once */
  int64_t iters_max;    /* most iterations of any SCC (PLAIN: the iteration count) */
  int64_t iters_sum;    /* sum over SCCs of their iterations */
  int64_t n_iterated;   /* SCCs iterated */
  int64_t n_not_converged;
  int64_t ws_accepted, ws_rejected; /* warm start: per-SCC accept / fallback counts */
  double cert_abs;      /* bound on ||R* - R||_1: ||r||_1 / (1-c) from the FP64 residual r (refine >= 0),
                           else c/(1-c) * sum_C ||P_{K_C}||_1 (truncation only, see pr_solve) */
  double r_sum;         /* ||R||_1 */
  double cert_rel;      /* cert_abs / r_sum: bound on the relative 1-norm error */
  double time_ms;       /* host wall time of the pr_solve call, weight check included */
  int64_t vert_iters;   /* rows touched: iterations x vertices of each SCC, plus every other vertex once */
  double kernel_ms;     /* device time of the launches after the weight check (HIP events) */
  /* with kernel_timing = 1: device time and launch count per kernel family,
     [0] persistent segment kernel, [1] gang term kernel, [2] hub-row combine
     kernel, [3] final reductions; zero otherwise */
  double kt_ms[4];
  int64_t kt_count[4];
  int64_t gang_edge_iters; /* with kernel_timing = 1, COMPONENTWISE: the part of edge_iters */
  int64_t gang_vert_iters; /* and vert_iters done by gang launches */
  double cert_trunc_rel;   /* the truncation bound c/(1-c) sum_C ||P_{K_C}||_1 / ||R||_1 of the first
                              solve (rounding excluded) */
  double res_l1;           /* ||W - (I - c A^T) R||_1 of the returned R in FP64 (0 with refine = -1) */
  int32_t refine_rounds;   /* correction solves run (their terms and edges are included above) */
  int32_t precision_used;  /* PR_PREC_MIXED or PR_PREC_FP64 (the choice of PR_PREC_AUTO) */
  int32_t reserved[2];
} pr_solve_stats;

/*
 * pr_solve -- R^(3) for damping c and weights W (Def. 3.5), on the device.
 *
 * W_dev: n doubles (device), the weight vector in the caller's vertex order,
 *        non-negative and finite.
 * R_dev: n doubles (device), written with R in the caller's vertex order.
 * COMPONENTWISE follows Sec. 4.3: levels from the highest down, each vertex's
 * weight raised by the rank flowing in from higher levels (eq. PR:levels),
 * one-vertex components copied, CACs solved exactly in topological order
 * (Sec. 4.3.1), SCCs by the power series (Sec. 4.3.2) with the chosen stop
 * rule.  PLAIN runs the power series on the whole graph with the same rule.
 * With PR_STOP_CERT_L1 the relative 1-norm error of the series is below eps
 * in exact arithmetic (Sec. 4.4).  FP32 terms (PR_PREC_MIXED) add rounding
 * that the solve amplifies by up to 1/(1-c), which matters as c approaches 1
 * (at c = 0.99 it can exceed 1e-6 relative).  So by default (refine = 0)
 * the solve ends with an FP64 residual pass over every edge:
 * stats->cert_rel = ||W - (I - c A^T) R||_1 / ((1-c) ||R||_1) bounds the
 * relative 1-norm error of the returned R, rounding included (up to the
 * FP64 rounding of the residual itself, about 1e-16 relative), and while it
 * exceeds eps a correction solve refines R (see pr_solve_opts.refine).  When
 * the bound still exceeds eps after the allowed rounds the call returns
 * PR_NOT_CONVERGED.  After a refined solve, pr_levels_debug's per-solve
 * arrays (W', iterations) hold the last correction solve's values.
 * The call returns after the stream work has completed.
 * Errors: PR_EINVAL (c outside (0,1), eps <= 0, tol <= 0, W negative or not
 * finite, method PLAIN without build_plain), PR_EHIP.
 */
int32_t pr_solve(pr_levels_t* lv, double c, const void* W_dev, void* R_dev,
                 const pr_solve_opts* opts, void* hip_stream, pr_solve_stats* stats);

/*
 * pr_levels_debug -- copy an internal array of the last solve to the host
 * (for tests).  what: 0 = W' per vertex (double[n], caller's order; the
 * weight after eq. PR:levels), 1 = iterations per component (int32[n_comp],
 * component ids of the partition; 0 for non-SCC components), 2 = the plan's
 * vertex order (int32[n]: position -> caller's vertex id), 3 = per-workgroup
 * counters of the last solve (uint64[grid_wgs x 16]: edge and row
 * iterations, iteration max/sum, SCCs iterated, not converged, warm-start
 * accept/reject, then wall-clock ticks in vertex items, small-SCC items,
 * single-workgroup SCC items, gang launches, readiness waits, segment
 * kernels, the number
 * of gang launches and ticks in single-workgroup SCC iterations), 4 = the
 * item timeline of the last solve run with trace = 1 in its options
 * (uint64[n_items x 4]: workgroup | item kind << 32, tick when the item was
 * taken, tick when its rank inflow was complete, tick when it finished),
 * 5 = the plan's work items (int32[n_items x 4]: kind 0 vertex range
 * [a, b), 1 SCCs of ranks [a, b) one per wavefront, 2 the SCC of rank a on
 * one workgroup; c unused), 6 = first plan position of each component rank
 * (int32[n_comp + 1]), 7 = component id of each rank (int32[n_comp]).
 */
int32_t pr_levels_debug(const pr_levels_t* lv, int32_t what, void* host_out);

/* ------------------------------------------------------ starting guess
 *
 * The paper starts each SCC's power series from P_0 = W'_C (Sec. 4.3.2) and
 * names an earlier ranking as a possible initial rank (Sec. 7).  This part
 * learns a start: a network 4 -> 64 -> 64 -> 1 (GELU after both hidden
 * layers; BF16 operands on the matrix cores, FP32 accumulation) maps four
 * features of an SCC vertex v,
 *   f0 = log(1 + in-degree), f1 = log(1 + out-degree)   (loops ignored),
 *   f2 = log(1 + (W'_v - W_v) / s_C),  f3 = log(1 + R1_v / s_C),
 *   s_C = ||W'_C||_1 / |C|,  R1 = W'_C + c A_CC^T W'_C   (one series step),
 * to y_v, and R_0,v = s_C exp(y_v).  With pr_solve_opts.warm_start set, each
 * SCC forms r_0 = W'_C + c A_CC^T R_0 - R_0 (FP64) and keeps the guess when
 * ||r_0||_1 < ||c A_CC^T W'_C||_1: its series then runs on r_0 and
 * R_C = R_0 + sum_k (c A_CC^T)^k r_0, which is the same R_C (Def. 3.5).
 * Otherwise it starts from W'_C as without a guess.
 *
 * Parameters: one flat float vector of 4545 values, in this order:
 * W1 [64 x 4] row-major, b1 [64], W2 [64 x 64] row-major, b2 [64],
 * W3 [64], b3 [1].  Training: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the
 * mean squared error over a batch; FP32 master weights, BF16 copies.
 * All calls return PR_EHANDLE for a handle that is not a live pr_mlp_t and
 * PR_EINVAL when the device current now is not the one the network was made
 * on.  Device buffers are the caller's and are not kept past the call.
 */
#define PR_MLP_PARAMS 4545

/* New network on the current device, weights uniform in
 * (-1/sqrt(fan_in), 1/sqrt(fan_in)) from a counter-based stream of `seed`. */
int32_t pr_mlp_create(uint64_t seed, pr_mlp_t** out);
/* Replace the weights (host float[4545]); resets the Adam state.
 * PR_EINVAL if a value is not finite. */
int32_t pr_mlp_set_params(pr_mlp_t* mlp, const float* host_params);
/* Copy the FP32 weights to host float[4545]. */
int32_t pr_mlp_get_params(const pr_mlp_t* mlp, float* host_out);
/* y_dev[i] = network(X_dev[4i .. 4i+3]) for i < n (device floats, row-major
 * features); returns after the stream work completes. */
int32_t pr_mlp_predict(const pr_mlp_t* mlp, int64_t n, const float* X_dev, float* y_dev, void* hip_stream);
/* Gradient of the mean squared error (1/n) sum_i (y_i - t_i)^2 over the n
 * rows (X_dev float[n x 4], t_dev float[n], device) without a step:
 * grad_host float[4545] (nullable), *loss = the mean squared error. */
int32_t pr_mlp_grad(pr_mlp_t* mlp, int64_t n, const float* X_dev, const float* t_dev, float* grad_host,
                    double* loss, void* hip_stream);
/* pr_mlp_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result, bit for bit, but the
 * per-wavefront partial gradients live in a static device array of the
 * library (at most 1024 partial vectors, 17.8 MiB, which covers every batch
 * size: the gradient kernel runs at most 256 workgroups), not in a buffer the
 * network allocates on first use.  The call allocates nothing; grad_host and
 * loss are written as by pr_mlp_grad.  Every call on a device shares that
 * device's array, so calls that overlap on one GPU (other threads, other
 * streams) race; each call writes every partial it reads, so no clearing is
 * needed.  PR_EINVAL if a batch needed more partials than the array holds. */
int32_t pr_mlp_grad_noalloc(pr_mlp_t* mlp, int64_t n, const float* X_dev, const float* t_dev, float* grad_host,
                            double* loss, void* hip_stream);
/* One Adam step with learning rate lr on the batch; *loss (nullable) = the
 * batch's mean squared error before the step.  PR_EINVAL for n <= 0 or a
 * learning rate that is not positive and finite. */
int32_t pr_mlp_train_step(pr_mlp_t* mlp, int64_t n, const float* X_dev, const float* t_dev, float lr,
                          double* loss, void* hip_stream);
/* Weights and Adam state to / from a file ("PRMLP001", int32 4545, int64
 * step, float[3 x 4545]: weights, first and second moments).  pr_mlp_load
 * returns PR_EINVAL for a file that is not in this format. */
int32_t pr_mlp_save(const pr_mlp_t* mlp, const char* path);
int32_t pr_mlp_load(const char* path, pr_mlp_t** out);
/* Features of every SCC vertex from the weights W' of the last pr_solve on
 * this plan (training data): F_dev float[n x 4] (the features above,
 * caller's vertex order), s_dev float[n] (s_C), mask_dev uint8[n] (1 for a
 * vertex of an SCC, else 0 and zero features).  W_dev: the W of that solve. */
int32_t pr_warm_features(const pr_levels_t* lv, double c, const void* W_dev, float* F_dev, float* s_dev,
                         uint8_t* mask_dev, void* hip_stream);

/* --------------------------------------------------------------- common */

/* Release any handle; NULL, unknown and already-released handles are ignored. */
void pr_free(void* handle);

/* Thread-local description of the last failure on this thread. */
const char* pr_last_error(void);

/* Measurement: the achievable read bandwidth of the current device, the
 * ceiling the gather-bound kernels are reported against.  Reads the device
 * buffer buf_dev (bytes long, 16-byte aligned) reps times with 16-byte loads
 * from a grid of 8 workgroups per compute unit and writes the average
 * milliseconds per pass to *ms_out (so bytes / ms is the rate).  A buffer far
 * larger than the 256 MB last-level cache measures HBM; a smaller one, after
 * the untimed warm-up passes, the cache.  Returns after the work completes. */
int32_t pr_bandwidth_probe(const void* buf_dev, int64_t bytes, int32_t reps, void* hip_stream, double* ms_out);

/* Library version string. */
const char* pr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PR_H_ */
