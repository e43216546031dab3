/*
 * qap_rlt2 -- level-2 RLT dual-ascent lower bound for the Quadratic
 * Assignment Problem on one AMD Instinct MI355X (gfx950).
 *
 * Method: Goncalves, Pessoa, Drummond, Bentes, Farias, "Solving the Quadratic
 * Assignment Problem on heterogeneous environment (CPUs and GPUs) with the
 * application of Level 2 Reformulation and Linearization Technique",
 * arXiv 1510.02065.  Problem statement: Section 2, equations (1)-(4).  Dual
 * state and reduced-cost matrices B, C, D: Section 3.  Dual ascent:
 * Section 4, Algorithm 1; cost concentration Section 4.1, spreading
 * Section 4.2, complementary transfer Section 4.3.
 *
 * Conventions for every call
 * --------------------------
 *  - Every function returns a qap_status; nothing throws or aborts across the
 *    ABI.  On a non-OK status qap_last_error() returns a thread-local message.
 *  - Matrices are row-major, 0-based.  F[i*N+k] is the flow from facility i
 *    to facility k; D[j*N+n] the distance from location j to location n.
 *  - Inputs are copied; the caller keeps ownership of every buffer it passes.
 *  - Handles are not thread-safe: use one handle from one thread at a time.
 *  - Sizes: 3 <= N <= QAP_RLT2_MAX_N.  The reduced-cost array D has
 *    N^2 (N-1)^2 (N-2)^2 entries (8 bytes each in FP64 mode, 4 in FP32 mode);
 *    the device holds one block of each complementary pair, half of them,
 *    unless the option `complementary` is 0.  Creation fails with
 *    QAP_ENOMEM if it does not fit in free device memory.
 *
 * Compact layouts used by qap_rlt2_read_state and qap_rlt2_lap_values
 * --------------------------------------------------------------------
 *  B: N x N, index i*N + j.
 *  C: N^2 blocks C_ij of (N-1)^2 entries; block (i,j) starts at
 *     (i*N+j)*(N-1)^2 and holds rows k != i, columns n != j in ascending
 *     original index: entry (k', n') at k'*(N-1) + n', k' = k - [k > i],
 *     n' = n - [n > j].  The position of c_ijkn in C is written beta(ijkn).
 *  D: N^2 (N-1)^2 blocks D_ijkn of (N-2)^2 entries; block D_ijkn is the
 *     beta(ijkn)-th block and holds rows p not in {i,k} and columns q not in
 *     {j,n} in ascending original index (Section 4.1).
 */
#ifndef QAP_RLT2_H
#define QAP_RLT2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QAP_RLT2_MAX_N 64

typedef enum {
    QAP_OK = 0,
    QAP_EINVAL = -1,   /* bad argument (size, NULL pointer, non-finite input) */
    QAP_ENOMEM = -2,   /* device or host allocation failed                    */
    QAP_EDEVICE = -3,  /* a HIP call failed; the message names it             */
    QAP_ESTATE = -4    /* handle unusable after an earlier device failure     */
} qap_status;

typedef enum {
    QAP_FP64 = 0,            /* all reduced costs and transfers in FP64         */
    QAP_FP32_CERTIFIED = 1,  /* FP32 reduced costs, every receiving write
                                at or below its exact value (rounded toward
                                -inf, or computed in FP64 and lowered by a
                                proven bound on its rounding error), FP64
                                bound and FP64 certification (see
                                qap_rlt2_certify): the stored state never
                                represents more than the true objective, so
                                the bound is proven valid; the trajectory
                                drifts below FP64 by about one FP32 ulp per
                                write                                         */
    QAP_FP32_NEAREST = 2     /* FP32 reduced costs, every receiving write
                                computed in FP64 and rounded to nearest once,
                                FP64 bound and FP64 certification: follows the
                                FP64 trajectory without a systematic drift;
                                the certification removes any negative stored
                                entry, and the state's represented objective
                                differs from the true one only by accumulated
                                FP32 roundings                                */
} qap_precision;

/* Assignment solver of every cost concentration (Section 4.1). */
typedef enum {
    QAP_LAP_SOLVER_CANONICAL = 0, /* Hungarian method (shortest augmenting
                                     paths), then the canonical optimal dual:
                                     the mean of the column- and row-canonical
                                     points, which does not depend on the
                                     solver's path (the oracle's choice)     */
    QAP_LAP_SOLVER_AUCTION = 1    /* auction algorithm with eps-scaling (the
                                     solver of the paper's GPU code, Section
                                     6), dual from the final prices: feasible,
                                     within n * eps of optimal, so the bound is
                                     valid, but the trajectory is its own     */
} qap_lap_solver;

typedef struct {
    int precision;    /* qap_precision                                        */
    int device;       /* HIP device ordinal; -1 = the calling thread's current */
    void* stream;     /* hipStream_t to run on; NULL = a stream the handle owns */
    int trace_level;  /* 0: bound only; 1: per-iteration LB and LB' (default);
                         2: also the value moved by every concentration of the
                         most recent iteration (qap_rlt2_lap_values)           */
    int use_graph;    /* 1 (default): qap_rlt2_ascend replays one captured HIP
                         graph per iteration; 0: plain launches                */
    int autotune;     /* 1 (default): during the first qap_rlt2_ascend, time the
                         concentration kernels of every family and size class
                         over the lanes per problem (8, 16, 32 or 64, with as
                         many columns per lane as the size needs) on a
                         restored copy of the live data, and keep the fastest;
                         the algorithm's decisions do not depend on the
                         choice, only the rounding of its final sums.  0: the
                         configuration with the most problems per wave that
                         fits in LDS                                          */
    const char* tune_cache; /* nullable path of a text file that stores the
                         tuned choices and is read back by later handles     */
    int complementary; /* 1 (default): store one block of each pair of
                         complementary D blocks D_ijkn, D_knij (Section 6) and
                         concentrate it once, S going to both c_ijkn and
                         c_knij.  The six-way transfer leaves the two blocks
                         equal and a concentration keeps them so, so the state
                         is bit for bit that of 0, which stores and
                         concentrates every block, with half the memory     */
    double K;          /* stop rule of Algorithm 1: an instance stops once
                         LB' / UB < K (progress below K), 0 = never on progress */
    double UB;         /* upper bound of the stop rule: an instance stops once
                         LB >= UB; UB <= 0 turns the whole rule off (default) */
    int level;         /* 2 (default): the level-2 RLT dual (B, C, D);
                         1: the level-1 dual (B and C only, no D: an iteration
                         is steps 1, 5, 6, 7 and 8), the dual of the strong
                         branching of Section 6                              */
    int lap_solver;    /* qap_lap_solver of the concentrations (default 0)    */
    int overlap;       /* 1 (default): in a batch of instances of several
                         sizes, qap_rlt2_ascend runs the sweep of each size
                         and then its D->C concentration on a second stream,
                         beside the next size's sweep (both streams at the
                         default priority; the same results bit for bit);
                         0: one step after the other                         */
} qap_rlt2_opts;

typedef struct qap_rlt2 qap_rlt2;

/* Fill *opts with the defaults (FP64, current device, own stream,
 * trace_level 1, use_graph 1, autotune 1, no tune cache, complementary 1,
 * no stop rule, level 2). */
qap_status qap_rlt2_default_opts(qap_rlt2_opts* opts);

/* Create a dual-ascent state for the QAP of equation (1) with flows F and
 * distances D (both N x N host arrays, FP64) and run iteration 0.
 *
 * Initial dual (the lines of Algorithm 1 before its loop): LB = 0,
 * b_ij = f_ii d_jj, c_ijkn = f_ik d_jn, d = 0.  Iteration 0 then concentrates
 * every C_ij into b_ij and B into LB, which makes LB the Gilmore-Lawler
 * bound.  Equivalent to qap_rlt2_create_ex(N, F, D, NULL, 0.0, NULL, out). */
qap_status qap_rlt2_create(int N, const double* F, const double* D, qap_rlt2** out);

/* As qap_rlt2_create, with optional linear costs B0 (N x N host array added
 * to b_ij, or NULL), a constant added to LB (for a branch-and-bound node whose
 * fixed assignments contribute a known cost) and options (NULL = defaults). */
qap_status qap_rlt2_create_ex(int N, const double* F, const double* D,
                              const double* B0, double constant,
                              const qap_rlt2_opts* opts, qap_rlt2** out);

/* Run `iters` >= 0 iterations of the Algorithm 1 loop body (at most: an
 * instance whose stop rule has fired runs no further iteration and keeps its
 * state, and the call returns early once every instance has stopped):
 *   1. spread B -> C: c_ijkn += b_ij / (N-1), then b = 0        (Section 4.2)
 *   2. spread C -> D: d_ijknpq += c_ijkn / (N-2), then c = 0     (Section 4.2)
 *   3. transfer among the six complementary D coefficients of equation (11):
 *      each becomes their mean                                    (Section 4.3)
 *   4. concentrate every D_ijkn into c_ijkn by an assignment solve (4.1)
 *   5. transfer between the complementary pair c_ijkn, c_knij of
 *      equation (10): both become their mean                    (Section 4.3)
 *   6. concentrate every C_ij into b_ij                           (4.1)
 *   7. concentrate B into LB'                                      (4.1)
 *   8. LB += LB'
 * Concentration of an n x n block M solves the assignment problem over M,
 * adds its value S to the parent coefficient and replaces M by the residual
 * under the canonical optimal dual: the mean of the residuals under the
 * column-canonical and row-canonical optimal dual points (the greatest dual
 * vector <= 0 on the optimal dual face, for columns and for rows).
 * *bound (nullable) receives LB after the last iteration (FP64 mode) or the
 * certified bound of qap_rlt2_certify (FP32 mode).  Blocks until done. */
qap_status qap_rlt2_ascend(qap_rlt2* h, int iters, double* bound);

/* Run a single step of the loop body above, for inspection.  Steps 1-3 run
 * as one fused pass: step must be 3 (steps 1-3), 4, 5, 6 or 7 (steps 7-8).
 * Every step only enqueues its kernels on the handle's stream and returns;
 * step 7 counts the iteration, whose trace entry reaches the host at the
 * next call that reads the trace or runs qap_rlt2_ascend.  A fault in an
 * enqueued kernel surfaces at the next blocking call. */
qap_status qap_rlt2_step(qap_rlt2* h, int step);

/* Certified bound, FP64: with m(beta) the minimum of block D_beta,
 * c~ = c + (N-2) min(0, m); with m'(ij) the minimum of C~_ij,
 * b~ = b + (N-1) min(0, m'); LB_cert = LB + N min(0, min b~).  LB_cert is a
 * lower bound on every permutation's objective as represented by the stored
 * state, whatever the signs of the stored reduced costs. */
qap_status qap_rlt2_certify(qap_rlt2* h, double* certified);

/* Bound after the most recent iteration and the number of loop iterations
 * instance 0 has run (iteration 0 counts as 0; each loop iteration adds 1). */
qap_status qap_rlt2_bound(qap_rlt2* h, double* lb, int64_t* iterations);

/* Per-iteration trace (trace_level >= 1): entries t = 0 .. *count-1 hold LB
 * and LB' after iteration t (t = 0 is iteration 0).  At most `capacity`
 * entries are written; *count receives the number available.  lb and
 * lbprime may be NULL. */
qap_status qap_rlt2_trace(qap_rlt2* h, int64_t capacity, int64_t* count,
                          double* lb, double* lbprime);

/* Values S moved by the concentrations of the most recent iteration (needs
 * trace_level 2): sD[beta(ijkn)] for D_ijkn -> c_ijkn (N^2 (N-1)^2 entries),
 * sC[i*N+j] for C_ij -> b_ij (N^2 entries), *sB for B -> LB'.  Each pointer
 * may be NULL. */
qap_status qap_rlt2_lap_values(qap_rlt2* h, double* sD, double* sC, double* sB);

/* Copy the current dual state to host FP64 arrays in the compact layouts
 * above (FP32 state is widened exactly; with one stored block per
 * complementary pair, both blocks of the pair receive it).  Each pointer may
 * be NULL. */
qap_status qap_rlt2_read_state(qap_rlt2* h, double* lb, double* B, double* C, double* D);

/* Release the handle and all of its device memory.  NULL-safe. */
void qap_rlt2_destroy(qap_rlt2* h);

/* ---- many instances in one handle (branch-and-bound nodes) ------------------
 * Section 6 of the paper runs the dual ascent at every node of a
 * branch-and-bound tree; a node is a smaller QAP with linear costs and a
 * constant (see qap_subproblem).  A batch handle holds `count` independent
 * instances of possibly different sizes and advances all of them together:
 * every step of an iteration is one launch over all instances (one per
 * segment-size class for the concentration steps), and qap_rlt2_ascend
 * replays one HIP graph per iteration.  Every call above applies to all
 * instances; the calls that return one instance's data (bound, trace,
 * lap_values, read_state) return instance 0's.
 *
 * qap_rlt2_batch_create: N[k], F[k], D[k] as for qap_rlt2_create_ex; B0
 * (nullable, or with nullable entries) and constant (nullable: all 0) per
 * instance.  Each instance runs its own iteration 0. */
qap_status qap_rlt2_batch_create(int count, const int32_t* N, const double* const* F,
                                 const double* const* D, const double* const* B0,
                                 const double* constant, const qap_rlt2_opts* opts,
                                 qap_rlt2** out);

/* Number of instances in the handle. */
qap_status qap_rlt2_count(qap_rlt2* h, int* count);

/* Per-instance LB (count entries, nullable) and certified bound (nullable;
 * the FP64 cascade of qap_rlt2_certify, per instance). */
qap_status qap_rlt2_batch_bounds(qap_rlt2* h, double* lb, double* certified);

/* Instance k's versions of qap_rlt2_trace, qap_rlt2_lap_values and
 * qap_rlt2_read_state (sizes follow instance k's N). */
qap_status qap_rlt2_instance_trace(qap_rlt2* h, int k, int64_t capacity, int64_t* count,
                                   double* lb, double* lbprime);
qap_status qap_rlt2_instance_lap_values(qap_rlt2* h, int k, double* sD, double* sC, double* sB);
qap_status qap_rlt2_instance_state(qap_rlt2* h, int k, double* lb, double* B, double* C, double* D);

/* Branch-and-bound node of a QAP (Section 6): fix facility fac[t] at location
 * loc[t] for t < m (distinct facilities, distinct locations).  The remaining
 * free facilities and locations, in ascending order, form a QAP of size
 * M = N - m with flows Fsub (M x M), distances Dsub (M x M), linear costs
 *   B0sub[a][b] = sum_t f(i, fac_t) d(j, loc_t) + f(fac_t, i) d(loc_t, j)
 * for free facility i = a-th and free location j = b-th, and
 *   *constant = sum_{t,u} f(fac_t, fac_u) d(loc_t, loc_u),
 * so that the parent's objective of any completion equals *constant plus the
 * node's objective with linear costs B0sub.  Host memory, FP64; the caller
 * owns all buffers.  Errors: QAP_EINVAL for bad indices or NULL pointers. */
qap_status qap_subproblem(int N, const double* F, const double* D, int m, const int32_t* fac,
                          const int32_t* loc, double* Fsub, double* Dsub, double* B0sub,
                          double* constant);

/* Batched linear assignment with canonical dual (Section 4.1, the operation
 * behind every cost concentration).
 *
 * batch   number of problems (>= 0).
 * n       n[b] in [0, 64]: size of problem b.
 * mat_off problem b's n[b] x n[b] row-major matrix starts at element
 *         mat_off[b] of `cost`.  Matrices must not overlap.
 * vec_off problem b's vectors start at element vec_off[b] of `assign` and at
 *         element 4*vec_off[b] of `duals`; ranges must not overlap.
 * cost    matrices, FP64 (dtype QAP_FP64) or FP32 (QAP_FP32_CERTIFIED, with
 *         every residual and value rounded toward -inf; QAP_FP32_NEAREST,
 *         rounded to nearest).  With QAP_LAP_RESIDUAL each matrix is
 *         overwritten by its residual.
 * value   value[b] receives S, the optimal assignment value reached through
 *         the canonical dual (FP64).
 * duals   nullable; same dtype as cost: [uc | vc | ur | vr], 4 n[b] values:
 *         column-canonical point (uc, vc) and row-canonical point (ur, vr).
 * assign  nullable; assign[r] = column given to row r by an optimal
 *         assignment (not unique when there are ties).
 * flags   QAP_LAP_DEVICE: every pointer above is device memory (of the
 *         calling thread's current device) and the call is asynchronous on
 *         `stream`; a device pass sorts the problems by size into a
 *         workspace of 16 bytes per problem taken from the stream-ordered
 *         allocator (hipMallocAsync) and released the same way.  Sizes
 *         outside [0, 64] are not checked on the host: such a problem's
 *         value is NaN and nothing else of it is written.  Otherwise all
 *         pointers are host memory, sizes are checked (QAP_EINVAL) and the
 *         call is synchronous.  QAP_LAP_RESIDUAL: write residuals in place.
 *         Problems of size n run in segments of the narrowest of 8, 16, 32
 *         or 64 lanes that holds n, several problems per wave.
 *         QAP_LAP_AUCTION: solve by the auction algorithm
 *         (QAP_LAP_SOLVER_AUCTION); value is then the dual value of the final
 *         prices (<= the optimum, within n * 2^-38 max|M| of it in FP64,
 *         n * 2^-20 max|M| in FP32), duals are that point completed as for
 *         the canonical one, and assign the auction's assignment.
 * stream  hipStream_t or NULL (the null stream). */
#define QAP_LAP_DEVICE 1
#define QAP_LAP_RESIDUAL 2
#define QAP_LAP_AUCTION 4
qap_status qap_lap_solve(int batch, const int32_t* n, const int64_t* mat_off,
                         const int64_t* vec_off, void* cost, int dtype,
                         double* value, void* duals, int32_t* assign,
                         int flags, void* stream);

/* qap_lap_solve with device pointers, allocating nothing: for callers that
 * cannot call hipMalloc or the stream-ordered allocator (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments and results as qap_lap_solve with QAP_LAP_DEVICE (every pointer
 * is device memory of the calling thread's current device; asynchronous on
 * `stream`).  The size bucketing uses a static device array of the library
 * (16 MiB, one per device, held until the process ends) instead of a
 * workspace.  Errors: QAP_EINVAL when flags lack QAP_LAP_DEVICE or when
 * batch > QAP_LAP_NOALLOC_MAX_BATCH; QAP_EDEVICE for HIP errors.  Every call
 * on a device shares that device's array (each call clears what it needs on
 * its stream first): calls that overlap on one device, on different streams
 * or threads without ordering between them, race and give wrong results. */
#define QAP_LAP_NOALLOC_MAX_BATCH 1048576
qap_status qap_lap_solve_noalloc(int batch, const int32_t* n, const int64_t* mat_off,
                                 const int64_t* vec_off, void* cost, int dtype,
                                 double* value, void* duals, int32_t* assign,
                                 int flags, void* stream);

/* ---- stop rule, state I/O, snapshots ---------------------------------------- */

/* Stop rule of Algorithm 1 (the loop runs while LB' / UB >= K and LB < UB):
 * set K and UB for every instance of the handle (UB <= 0 turns the rule off).
 * Takes effect from the next iteration; an instance that has already stopped
 * stays stopped. */
qap_status qap_rlt2_set_stop(qap_rlt2* h, double K, double UB);

/* Per-instance status: active[k] = 1 while instance k's dual ascent runs, 0
 * once its stop rule has fired; iterations[k] = loop iterations it has run.
 * Either pointer may be NULL; each holds qap_rlt2_count entries. */
qap_status qap_rlt2_batch_status(qap_rlt2* h, int* active, int64_t* iterations);

/* Assignment found by the most recent concentration of instance k's B into
 * LB' (step 7): perm[i] = location of facility i, a permutation of the
 * instance (its objective is an upper bound on the instance's optimum;
 * Algorithm 1's UB).  N entries. */
qap_status qap_rlt2_instance_assignment(qap_rlt2* h, int k, int32_t* perm);

/* Inverse of qap_rlt2_instance_state: overwrite instance k's LB and reduced
 * costs from host FP64 arrays in the compact layouts above (each pointer
 * nullable: that part is left as it is).  FP32 modes round each entry once
 * (toward -inf in QAP_FP32_CERTIFIED, to nearest in QAP_FP32_NEAREST).  With
 * one stored block per complementary pair, block D_ijkn with i < k is read and
 * its complement's values are ignored.  A level-1 handle ignores D. */
qap_status qap_rlt2_load_state(qap_rlt2* h, int k, const double* lb, const double* B, const double* C,
                               const double* D);

/* Snapshot of the whole handle (every instance's LB, B, C, D, stop flags,
 * iteration counts, traces and tuned kernel choices) into host memory, for
 * checkpointing a long run (Section 7).  *size receives the bytes needed;
 * with buf NULL or capacity < *size nothing else is written (and QAP_OK is
 * returned when buf is NULL, QAP_EINVAL otherwise). */
qap_status qap_rlt2_snapshot(qap_rlt2* h, void* buf, uint64_t capacity, uint64_t* size);

/* Restore a snapshot into a handle created with the same instances and
 * options (QAP_EINVAL if the sizes, precision, level or storage differ).
 * Iterations after the restore produce the same bits as iterations of the
 * handle the snapshot was taken from. */
qap_status qap_rlt2_restore(qap_rlt2* h, const void* buf, uint64_t size);

/* ---- branch and bound (Section 6) --------------------------------------------- */

/* Children of instance k of handle h: child c fixes facility fac[c] at
 * location loc[c] (indices of instance k, which must be free: 0..N-1).  The
 * new handle holds `count` instances of size N-1 whose facilities and
 * locations are instance k's others in ascending order, and whose dual state
 * is inherited from instance k's current reduced costs:
 *   LB' = LB + b_ab,  b'_ij = b_ij + c_ijab + c_abij,
 *   c'_ijkn = c_ijkn + d_abijkn + d_ijabkn + d_ijknab,  d' = d restricted,
 * a valid dual of the child at least as strong as the parent's LB.  level 2
 * keeps D; level 1 makes level-1 children (no D; the terms above move into
 * C all the same).  Options are instance k's handle's (stop rule included).
 * Call between iterations (not inside a qap_rlt2_step sequence).  Needs
 * N - 1 >= 3. */
qap_status qap_rlt2_children(qap_rlt2* h, int k, int count, const int32_t* fac, const int32_t* loc, int level,
                             qap_rlt2** out);

/* Strong branching of Section 6 at instance k: every child (a -> b) of the
 * instance is evaluated with the level-1 dual ascent (inherited from the
 * instance's reduced costs, `iters` level-1 iterations), bounds[a*N + b]
 * receives its bound (the certified bound in FP32 modes).  The chosen branch
 * is the facility (kind 0, row a) or location (kind 1, column b) whose
 * children's smallest bound is the largest, i.e. the branch that raises the
 * node's bound the most; ties go to the larger sum of bounds, then rows
 * before columns, then the lower index.  kind, index and bounds nullable. */
qap_status qap_rlt2_strong_branch(qap_rlt2* h, int k, int iters, double* bounds, int* kind, int* index);

/* QAP objective of permutation perm (perm[i] = location of facility i) with
 * linear costs B0 (nullable) and a constant: sum_{i,k} f_ik d_perm(i)perm(k)
 * + sum_i B0[i][perm(i)] + constant.  Host FP64. */
qap_status qap_objective(int N, const double* F, const double* D, const double* B0, double constant,
                         const int32_t* perm, double* value);

/* Upper-bound heuristic of Algorithm 1 (UB): pairwise-exchange descent from
 * perm (in: a permutation, out: a local optimum where no exchange of two
 * facilities' locations lowers the objective); *value its objective.  Host. */
qap_status qap_ub_local_search(int N, const double* F, const double* D, const double* B0, double constant,
                               int32_t* perm, double* value);

typedef struct {
    int precision;          /* qap_precision of every node's dual ascent          */
    int device;             /* HIP device; -1 = current                           */
    void* stream;           /* hipStream_t or NULL                                */
    int root_iters;         /* dual-ascent iterations at the root                 */
    int iters;              /* dual-ascent iterations at every other node         */
    double K;               /* progress limit of the stop rule (0: none)          */
    double UB;              /* initial upper bound; <= 0: from the heuristic      */
    int strong_iters;       /* level-1 iterations of the strong-branching
                               evaluation; < 0: no strong branching (branch on
                               the lowest free facility)                          */
    int leaf_size;          /* nodes with at most this many free facilities are
                               enumerated on the host (3..9)                       */
    int64_t max_nodes;      /* stop after this many dual-ascent nodes (0: none)  */
    const char* checkpoint; /* nullable: checkpoint file (written atomically)     */
    int64_t checkpoint_every; /* dual-ascent nodes between checkpoints (>= 1)     */
    int resume;             /* 1: continue the run saved in `checkpoint`          */
} qap_bnb_params;

typedef struct {
    double value;                 /* best objective found                        */
    int32_t perm[QAP_RLT2_MAX_N]; /* its permutation (facility -> location)       */
    double root_bound;            /* bound of the root node                       */
    int64_t nodes;                /* nodes whose dual ascent ran (resumed runs
                                     included)                                    */
    int64_t pruned;               /* nodes discarded by their bound               */
    int64_t leaves;               /* nodes enumerated on the host                 */
    int complete;                 /* 1: the tree is exhausted, value is optimal   */
} qap_bnb_result;

qap_status qap_bnb_default_params(qap_bnb_params* p);

/* Branch and bound of Section 6 on one GPU: a depth-first search whose every
 * node runs the level-2 dual ascent (this library's), with the children of a
 * node created together in one batch handle that inherits the node's reduced
 * costs (qap_rlt2_children), strong branching (qap_rlt2_strong_branch), the
 * stop rule against the incumbent, incumbents from the heuristic and from the
 * B-level assignments of every node, and checkpoints of the open nodes (their
 * fixed assignments) with the incumbent and counters.  Resumed nodes restart
 * their dual ascent from their subproblem.  Host arrays F and D (N x N),
 * 3 <= N <= QAP_RLT2_MAX_N. */
qap_status qap_bnb_solve(int N, const double* F, const double* D, const qap_bnb_params* p,
                         qap_bnb_result* result);

/* Thread-local description of the most recent failure ("" if none). */
const char* qap_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QAP_RLT2_H */
