/*
 * qap_swarm.h -- C ABI of the MI355X (gfx950) implementation of the
 * multi-swarm discrete particle swarm optimisation for the Quadratic
 * Assignment Problem of Szwed & Chmiel (arXiv:1504.05158).
 *
 * Problem (Sec. 2.1, eq. qap): n facilities, n locations, flow matrix F and
 * distance matrix D (both n x n, row-major int32).  A solution is a
 * permutation p with p[i] = location of facility i (0-based); its cost is
 *     C(p) = sum_{i,j} F[i][j] * D[p[i]][p[j]]
 * (diagonal terms included: the installation cost of Sec. 2.1).
 *
 * Method (Sec. 3.1-3.2): every particle holds a solution X (a permutation
 * matrix, rows = locations, columns = facilities) and a real n x n velocity V.
 * One iteration per particle:
 *   X(t+1) = S_x(X(t) + V(t))                 S_x = SecondTarget (Alg. 1)
 *   V(t+1) = S_v(c1 V + c2 r2 (P^L - X) + c3 r3 (P^G - X))   (eq. velocity)
 * then the goal of X(t+1), up to `local_search` best-improvement pair
 * exchanges (local improvement; 0 = none), the particle best P^L, the swarm
 * best P^G, and in migration mode Alg. 2 every `migration_period` iterations.
 *
 * Conventions shared by every entry point:
 *  - Return value: QAP_OK (0) or a negative QAP_ERR_* code.  No C++
 *    exception crosses the ABI.  A device error is sticky: once it has been
 *    seen, every later call on the handle returns QAP_ERR_DEVICE.
 *  - Host pointers only, caller-owned; the library copies what it needs.
 *    Device memory is owned by the handle and freed by qap_swarm_destroy.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Random numbers come from a Philox4x32-10 counter-based stream keyed by
 *    the seed, so a run is a deterministic function of (instance, params).
 */
#ifndef QAP_SWARM_H
#define QAP_SWARM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    QAP_OK = 0,
    QAP_ERR_INVALID_ARG = -1, /* NULL pointer or a parameter outside its range */
    QAP_ERR_RANGE = -2,       /* F, D values too wide for the requested / any exact path */
    QAP_ERR_NOMEM = -3,       /* device or host allocation failed */
    QAP_ERR_DEVICE = -4,      /* HIP runtime error (sticky) */
    QAP_ERR_UNSUPPORTED = -5  /* valid request this build does not provide */
};

enum { QAP_SV_RAW = 0, QAP_SV_NORM = 1 };          /* S_v of Sec. 3.1 */
enum { QAP_INDEPENDENT = 0, QAP_MIGRATION = 1 };   /* swarm modes (Sec. 3.2) */
enum { QAP_PATH_AUTO = 0, QAP_PATH_INT8_MFMA = 1, QAP_PATH_INT32 = 2, QAP_PATH_SPLIT_MFMA = 3 }; /* swap-delta contraction */
enum { QAP_MAX_EXCHANGES = 65535 }; /* largest local_search */
enum { QAP_SX_SECOND_TARGET = 0, QAP_SX_PICK_COLUMN = 1 }; /* S_x procedures */
enum { QAP_ENGINE_FUSED = 0, QAP_ENGINE_PLAIN = 1 }; /* one fused kernel per step vs per-stage kernels */

typedef struct qap_swarm qap_swarm; /* opaque handle */

/* A QAP instance (Sec. 2.1): F and D are n x n row-major, 2 <= n <= 256. */
typedef struct {
    int32_t n;
    const int32_t* F;
    const int32_t* D;
} qap_instance;

/* Run parameters (the columns of Table 1 plus the readings this library fixes).
 *  num_swarms m >= 1, particles_per_swarm S >= 1 (particle index g*S + s).
 *  c1, c2, c3 in [0, 1]: inertia, self-recognition, social factor (Sec. 2.2).
 *  vmax > 0: bound of S_v (Sec. 3.1).  velocity_kernel: QAP_SV_RAW / QAP_SV_NORM.
 *  st_depth in [0, n-1]: SecondTarget depth d (Alg. 1, d < n).
 *  mode, migration_factor, migration_period: Alg. 2 with depth
 *    floor(migration_factor * m), which must be < m/2; the period is >= 1.
 *  local_search: best-improvement pair exchanges per particle-iteration, 0 to
 *    QAP_MAX_EXCHANGES: each exchange takes the pair with the smallest delta
 *    (ties to the smallest a, then b) and is made only if it lowers the goal;
 *    the first non-improving pair ends the search (a local optimum of the
 *    pair-exchange neighbourhood; a large value runs to one).
 *  delta_path: contraction used for the pair-exchange deltas, all exact.
 *    INT8_MFMA: every F, D entry in [-128, 127].  SPLIT_MFMA: F and D
 *    symmetric, every entry in [-16384, 16383] and
 *    8 (n + 3) max|F| max|D| < 2^31; each matrix outside the int8 range is
 *    split into a low plane (M mod 128) and a high plane (floor(M / 128)) and
 *    the plane products are int8 MFMAs combined in int32.  INT32: any instance
 *    with n max|F| max|D| < 2^31, on VALU.  A requested MFMA path that the
 *    instance does not meet fails with QAP_ERR_RANGE.  AUTO picks int8, else
 *    byte-split, else int32.  The MFMA paths need the fused engine, n <= 160
 *    and SecondTarget; otherwise the instance runs on the int32 path, which
 *    qap_swarm_path reports.
 *  engine: QAP_ENGINE_FUSED (one kernel per step for int8 and byte-split
 *    instances, per-stage kernels otherwise; steps replay a HIP graph) or QAP_ENGINE_PLAIN (one
 *    kernel per stage, int32 contraction).
 *  seed: key of the random stream.  stream: hipStream_t to run on (NULL = the
 *    library's own stream).
 *  sx_procedure: QAP_SX_SECOND_TARGET (Alg. 1 with st_depth; st_depth = 0 is the
 *    paper's GlobalMax) or QAP_SX_PICK_COLUMN (columns visited in a random
 *    order, each taking its largest key over the rows left; runs on the
 *    per-stage kernels, whatever the engine).
 *  stream_groups: 0 = automatic (swarms on the fused kernel are stepped as up
 *    to 3 concurrent groups of swarms, see qap_swarm_step and qap_plan), or
 *    1-QAP_MAX_CHAINS to set the number of groups of this instance (results
 *    are the same for every choice). */
typedef struct {
    int32_t num_swarms;
    int32_t particles_per_swarm;
    float c1, c2, c3;
    float vmax;
    int32_t velocity_kernel;
    int32_t st_depth;
    int32_t mode;
    float migration_factor;
    int32_t migration_period;
    int32_t local_search;
    int32_t delta_path;
    int32_t engine;
    uint64_t seed;
    void* stream;
    int32_t stream_groups;
    int32_t sx_procedure;
} qap_params;

/* Host-side copy of one instance's state (checkpoint / inspection).  Every
 * pointer is caller-owned and may be NULL to skip that member.  P = m*S.
 *   V       float  [P][n][n]  row = location, column = facility
 *   X, PL   int32  [P][n]     current solution and particle best (p[i] = location)
 *   goal, goalPL  int64 [P]
 *   PG      int32  [m][n],  goalPG int64 [m]   swarm bests
 *   best_*  best solution ever seen, the iteration, swarm and member it came from
 *   iteration: number of completed iterations (0 after init). */
typedef struct {
    float* V;
    int32_t* X;
    int32_t* PL;
    int64_t* goal;
    int64_t* goalPL;
    int32_t* PG;
    int64_t* goalPG;
    int32_t* best_perm;
    int64_t best_goal;
    int32_t best_iter, best_swarm, best_particle;
    int32_t iteration;
} qap_state;

/* Create a handle for one instance and run the initialisation, iteration 0
 * (Sec. 3.3: particles start from random solutions; Table 2 counts a solution
 * found at initialisation as iteration 0): random permutations by
 * Fisher-Yates, random velocities vmax (2u - 1) passed through S_v (Sec. 3.1),
 * their goals (eq. qap), P^L = X, the swarm bests P^G and the best-ever record.
 * Errors: QAP_ERR_INVALID_ARG (NULL, n outside [2,256], a parameter outside
 * the ranges above), QAP_ERR_RANGE (an MFMA path requested that the data do
 * not meet, or
 * n * max|F| * max|D| >= 2^31 so no exact int32 contraction exists),
 * QAP_ERR_NOMEM, QAP_ERR_DEVICE.  On error *out is NULL. */
int qap_swarm_init(const qap_instance* inst, const qap_params* prm, qap_swarm** out);

/* Same for `count` independent instances that step together (each with its
 * own params and seed; the engine and stream of prms[0] apply to all).  Each
 * instance is the method of Sec. 3.1-3.2 on its own data; the batching is the
 * library's: one launch per kernel class serves every instance of the class
 * (where the paper launches separate kernels per iteration, Sec. 3.3).
 * Instance k is addressed by index k in the calls below.  Errors as for
 * qap_swarm_init; prms[k].engine must equal prms[0].engine. */
int qap_swarm_init_batch(const qap_instance* insts, const qap_params* prms, int32_t count,
                         qap_swarm** out);

/* Enqueue `iterations` >= 0 iterations on the handle's stream and return
 * without waiting.  One iteration of every particle: r2, r3 (Sec. 3.1),
 * X(t+1) = S_x(X(t) + V(t)) (eq. position, Alg. 1 SecondTarget), V(t+1) by
 * eq. velocity with S_v, the goal (eq. qap) and the local-improvement pair
 * exchanges, P^L; then per swarm P^G and the best-ever record, and Alg. 2
 * (migration, Sec. 3.2) every migration_period iterations.
 * Device errors surface here or on a later call.
 * Independent swarms on the fused kernel are stepped as up to 3 groups of
 * swarms, each on a stream of the library's own: the groups start after the
 * work already on the handle's stream and the handle's stream continues after
 * all of them, so results and ordering are as on one stream (and bit-identical
 * to stepping the swarms as one group).  One iteration of a group is one launch
 * per fused-kernel class (instances with the same padded size and symmetry
 * share a launch), the per-stage kernels of instances outside the int8 path,
 * and one batched launch each for the swarm bests and the finish step.  The
 * first call captures each group's iteration into a HIP graph, replayed once
 * per iteration; a stream that cannot be captured keeps eager launches. */
int qap_swarm_step(qap_swarm* h, int32_t iterations);

/* Launch plans and the autotuner (runtime; no passage of the paper: the
 * paper launches separate kernels per iteration from its host, Sec. 3.3).
 * A plan says how the iterations of a handle are launched; results are
 * bit-identical under every plan.
 *   stream_chains: concurrent chains of launches, each on its own stream
 *     (1..QAP_MAX_CHAINS).  Chain 0 runs on the handle's stream.  A process's
 *     streams share the HIP runtime's hardware queues (GPU_MAX_HW_QUEUES, 4
 *     by default) and kernels of two streams on one queue run one after the
 *     other: k chains overlap fully with k + 1 queues or more.
 *   split: QAP_SPLIT_SWARMS -- every instance's swarms are spread over the
 *     chains (an instance whose stream_groups parameter is set keeps that many
 *     groups at most); QAP_SPLIT_INSTANCES -- whole instances, the heaviest
 *     (particles x n^2) first onto the least loaded chain; QAP_SPLIT_CLASSES --
 *     whole kernel classes (instances sharing a launch: padded size,
 *     contraction kind, symmetry and diagonals; the instances on per-stage
 *     kernels form one more), the heaviest first onto the least loaded chain.
 *   iters_per_graph: 0 = eager kernel launches; k >= 1 (at most 64) =
 *     iterations replayed from graphs of k iterations (single-iteration graphs
 *     for the rest of a step and around migrations).
 *   ms_per_iteration: filled by qap_swarm_tune (the chosen plan's time).
 * A handle starts on the plan cached for its workload (see qap_swarm_tune),
 * else on 3 chains (or the instances' stream_groups), split by swarms, graphs
 * of 8 iterations.  qap_swarm_set_plan may be called between any two steps
 * (QAP_ERR_INVALID_ARG for a plan outside the ranges above).
 * qap_swarm_tune times every plan (chains 1..c x split x {eager, 1, 8}
 * iterations per graph, where c = GPU_MAX_HW_QUEUES - 1 (4 queues when the
 * variable is unset), at most QAP_MAX_CHAINS; the instance and class splits
 * only for several instances) on the handle's own work, each from iteration 0 -- 10
 * iterations of warm-up, then trial_iterations (1..4096) between events --
 * then times the 4 fastest again on 2 x trial_iterations, keeps the fastest
 * of that round, and returns the handle to iteration 0 (the state init made,
 * re-created from the seed).  It must be called before the first step
 * (QAP_ERR_INVALID_ARG otherwise).  If the environment variable
 * QAP_SWARM_TUNE_CACHE names a file, the choice is appended to it under a
 * signature of the device and the workload, and later handles with the same
 * signature start on it without timing. */
enum { QAP_MAX_CHAINS = 4, QAP_SPLIT_SWARMS = 0, QAP_SPLIT_INSTANCES = 1, QAP_SPLIT_CLASSES = 2 };
typedef struct {
    int32_t stream_chains;
    int32_t split;
    int32_t iters_per_graph;
    float ms_per_iteration;
} qap_plan;
int qap_swarm_get_plan(qap_swarm* h, qap_plan* plan);
int qap_swarm_set_plan(qap_swarm* h, const qap_plan* plan);
int qap_swarm_tune(qap_swarm* h, int32_t trial_iterations, qap_plan* chosen);

/* Runtime introspection (no passage of the paper).
 * *active (may be NULL) = 1 if qap_swarm_step replays captured graphs (0:
 * eager launches, before the first step, or while profiling); *streams (may be
 * NULL) = number of stream groups, i.e. concurrent launches of each stage per
 * iteration. */
int qap_swarm_graph(qap_swarm* h, int32_t* active, int32_t* streams);

/* Wait for the handle's stream (runtime; no passage of the paper). */
int qap_swarm_sync(qap_swarm* h);

/* Best solution ever seen by an instance (waits first).  Kept apart from the
 * swarm bests because Alg. 2 may replace a swarm's P^G by a worse solution
 * (Sec. 3.2); the iteration it was found at is Table 2's "Iter".  perm: n
 * entries, may be NULL; goal / iter_found may be NULL. */
int qap_swarm_best(qap_swarm* h, int32_t instance, int64_t* goal, int32_t* perm, int32_t* iter_found);

/* Current swarm-best goals (m entries, the goals of P^G of Sec. 3.2) of an
 * instance (waits first). */
int qap_swarm_swarm_bests(qap_swarm* h, int32_t instance, int64_t* goals);

/* Copy an instance's state -- each particle's X, V, P^L (Sec. 3.1) and each
 * swarm's P^G (Sec. 3.2) -- to / from host buffers (waits first).  set_state
 * validates every permutation and returns QAP_ERR_INVALID_ARG on a bad one;
 * it requires V, X, PL, goal, goalPL, PG, goalPG and best_perm. */
int qap_swarm_get_state(qap_swarm* h, int32_t instance, qap_state* st);
int qap_swarm_set_state(qap_swarm* h, int32_t instance, const qap_state* st);

/* Evaluate `count` permutations (host, [count][n]) of an instance with the
 * handle's device contraction path: goals [count] (eq. qap) and, if deltas is
 * not NULL, the full pair-exchange delta matrices [count][n][n] (delta(a,b) =
 * C(p with a, b exchanged) - C(p), zero diagonal: the pair-exchange
 * neighbourhood of Sec. 2.1).  Every permutation is validated
 * (QAP_ERR_INVALID_ARG).  Waits for the result. */
int qap_swarm_eval(qap_swarm* h, int32_t instance, const int32_t* perms, int32_t count,
                   int64_t* goals, int64_t* deltas);

/* The pair-exchange delta matrix (delta(a,b) = C(p with a, b exchanged) -
 * C(p), Sec. 2.1, eq. qap) of the solution that particle `particle` of an
 * instance took from S_x (eq. position, Alg. 1) in the last step, before its
 * local-improvement exchanges: out [n][n] (caller-owned host memory, zero
 * diagonal), and that permutation in perm [n] (may be NULL).  The selection is
 * recomputed by the step's own S_x code from the buffers of the previous
 * state, which the last step only read, and the deltas come from the
 * instance's contraction path.  Errors: QAP_ERR_INVALID_ARG for a NULL out, a
 * particle outside [0, m*S), or no step since init or set_state.  Waits. */
int qap_swarm_deltas(qap_swarm* h, int32_t instance, int32_t particle, int64_t* out, int32_t* perm);

/* Runtime introspection (no passage of the paper).
 * Path actually used by an instance: QAP_PATH_INT8_MFMA, QAP_PATH_SPLIT_MFMA
 * or QAP_PATH_INT32 in *delta_path, and 1 in *symmetric if F and D are both
 * symmetric. */
int qap_swarm_path(qap_swarm* h, int32_t instance, int32_t* delta_path, int32_t* symmetric);

/* Population statistics of the current goals of an instance (the percentile
 * ranks and probability mass functions of Sec. 4.2), computed on the device;
 * waits.  For each of nq (0..QAP_STATS_MAX_RANKS) ranks q_ppm[j] in parts per
 * million (1..10^6): the nearest-rank value, i.e. the value at position
 * ceil(q N / 10^6) (at least 1) of the N goals in ascending order, per swarm
 * into swarm_q [m][nq] (N = particles per swarm) and over all particles into
 * pop_q [nq].  For bins (0..QAP_STATS_MAX_BINS) > 0 with lo < hi and
 * (hi - lo) * bins < 2^62: the number of goals g with lo <= g < hi in bin
 * floor((g - lo) * bins / (hi - lo)), per swarm into swarm_hist [m][bins] and
 * over all particles into pop_hist [bins].  Every output may be NULL. */
enum { QAP_STATS_MAX_RANKS = 64, QAP_STATS_MAX_BINS = 4096 };
int qap_swarm_stats(qap_swarm* h, int32_t instance, int32_t nq, const int32_t* q_ppm, int64_t* swarm_q,
                    int64_t* pop_q, int32_t bins, int64_t lo, int64_t hi, int64_t* swarm_hist, int64_t* pop_hist);

/* Per-iteration statistics: the percentile ranks and PMFs of Sec. 4.2 (Figs.
 * 4-7 follow them iteration by iteration), recorded on the device after
 * every iteration of qap_swarm_step into a ring of `capacity` records
 * (1..QAP_HISTORY_MAX_RECORDS) per instance, with the definitions of
 * qap_swarm_stats (nq ranks q_ppm, bins over [lo, hi); at least one of nq,
 * bins > 0).  Recording adds, after every iteration, one launch on the
 * handle's stream once every stream chain has finished the iteration, and no
 * host synchronisation; steps then replay single-iteration graphs.
 * qap_swarm_history_start (re)starts recording (earlier records are
 * dropped), qap_swarm_history_stop ends it and frees the ring.
 * qap_swarm_history_read (waits) gives the latest min(max_records, records
 * kept) iterations, oldest first: *count of them, their iteration numbers
 * iters [count], swarm_q [count][m][nq], pop_q [count][nq],
 * swarm_hist [count][m][bins], pop_hist [count][bins] (each may be NULL);
 * QAP_ERR_INVALID_ARG if the instance is not recording. */
enum { QAP_HISTORY_MAX_RECORDS = 1 << 20 };
int qap_swarm_history_start(qap_swarm* h, int32_t instance, int32_t capacity, int32_t nq, const int32_t* q_ppm,
                            int32_t bins, int64_t lo, int64_t hi);
int qap_swarm_history_stop(qap_swarm* h, int32_t instance);
int qap_swarm_history_read(qap_swarm* h, int32_t instance, int32_t max_records, int32_t* count, int32_t* iters,
                           int64_t* swarm_q, int64_t* pop_q, int64_t* swarm_hist, int64_t* pop_hist);

/* qap_swarm_stats for callers that cannot allocate memory (code under graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments and results, computed without any device or host allocation.
 * Its scratch (segment offsets, ranks, selected values, bin counts) lives in
 * a fixed device array of QAP_STATS_SCRATCH_BYTES, one per GPU, set up at the
 * first init on that GPU and held until the process ends.  A request needing
 * more -- 4 (m + 3) + 16 (m + 1) max(nq, 1) + 8 (m + 1) max(bins, 1) bytes,
 * each of the four parts rounded up to 256 -- returns QAP_ERR_UNSUPPORTED
 * (qap_swarm_stats has no such limit).  Every call on one GPU uses the same
 * array, which keeps the last call's contents: calls that overlap in time on
 * one GPU (from other threads or on other handles' streams) race, and the
 * library does not serialise them.  Waits for the result. */
enum { QAP_STATS_SCRATCH_BYTES = 4194304 };
int qap_swarm_stats_noalloc(qap_swarm* h, int32_t instance, int32_t nq, const int32_t* q_ppm, int64_t* swarm_q,
                            int64_t* pop_q, int32_t bins, int64_t lo, int64_t hi, int64_t* swarm_hist,
                            int64_t* pop_hist);

/* Kernel timing for measurement (runtime; no passage of the paper).
 * enable = 1 switches the handle to
 * profiled stepping: every later qap_swarm_step launches its kernels one by
 * one (no graph) with HIP events recorded around each stage on the stream it
 * runs on, and the counters restart from zero; enable = 0 switches back.
 * stage_ms (QAP_NUM_STAGES doubles, may be NULL) receives the summed kernel
 * time per stage -- summed over the stream groups, whose launches overlap in
 * time (qap_swarm_graph gives their number) -- and *launches the number of
 * iterations profiled (waits first).  Stages: QAP_STAGE_SX (S_x), QAP_STAGE_VELOCITY,
 * QAP_STAGE_GOAL_DELTA (goal, deltas, exchange, P^L), QAP_STAGE_FUSED (the
 * whole particle iteration in one kernel), QAP_STAGE_BESTS (swarm bests,
 * best-ever, migration). */
enum { QAP_STAGE_SX = 0, QAP_STAGE_VELOCITY = 1, QAP_STAGE_GOAL_DELTA = 2, QAP_STAGE_FUSED = 3,
       QAP_STAGE_BESTS = 4, QAP_NUM_STAGES = 5 };
int qap_swarm_profile(qap_swarm* h, int32_t enable, double* stage_ms, int64_t* launches);

/* Release every device and host resource of the handle (NULL is a no-op). */
void qap_swarm_destroy(qap_swarm* h);

/* Test hooks for the failure paths (no passage of the paper).
 * qap_swarm_fail_alloc(k), k >= 1: the k-th device allocation the library
 * makes from now on (in any call, process-wide) fails as if the device were
 * out of memory, once; k = 0 cancels.  The call that meets it returns
 * QAP_ERR_NOMEM having released what it had allocated (an init leaves no
 * handle; any other call leaves the handle usable).
 * qap_swarm_live_allocations: the number of device allocations the library
 * currently holds. */
int qap_swarm_fail_alloc(int32_t nth);
int64_t qap_swarm_live_allocations(void);

/* Static text for a return code. */
const char* qap_swarm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* QAP_SWARM_H */
