/*
 * dgs.h -- Deep Greedy Switching (DGS) for the Linear Sum Assignment
 * Problem on AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Method: Roverso, Naiem, El-Beltagy, El-Ansary, "GPU-Based Heuristic
 * Solver for Linear Sum Assignment Problems Under Real-time Constraints"
 * (arXiv:1106.5694).
 *
 * Problem (Section 3): n agents, n jobs, integer benefit a_ij of giving job
 * j to agent i; find a permutation tau (tau[i] = job of agent i) with a
 * large total benefit f = sum_i a[i][tau[i]].  The benefit matrix is
 * row-major int32: benefit[i * n + j] = a_ij.
 *
 * What every solve computes (Sections 3.1-3.3, Algorithms 1 and 2):
 *   1. greedy start: agents 0..n-1 in order, each takes its best free job
 *      (lowest job index on ties);
 *   2. repeat: every agent finds its best 2-exchange (ADE: agent i takes job
 *      j, the owner of j takes i's old job; gain = change of f, lowest j on
 *      ties), the best exchange over all agents is applied (largest gain,
 *      lowest agent on ties) if its gain is > 0, and the agents are
 *      re-evaluated; stop when no exchange improves f.
 *   The result (tau, f, number of switches) is a deterministic function of
 *   the input; it is bit-identical to a plain CPU implementation of the
 *   same steps.
 *
 * Value range: every |a_ij| must be <= DGS_MAX_ABS_BENEFIT (2^29 - 1), so
 * that every exchange gain (a sum of four entries) fits in int32.  Larger
 * values are rejected with DGS_E_RANGE.
 *
 * Errors: every entry point returns a dgs_status.  On any error the output
 * buffers are left untouched and dgs_last_error() describes the failure
 * (thread-local).  No entry point aborts the process.
 *
 * Memory: the caller owns every buffer it passes.  Inputs are only read for
 * the duration of the call (server: until the request completes).  The
 * library owns its device memory and streams.  A solve holds the transpose
 * of the benefit matrix (4 n*m bytes) and, for a host matrix, a device copy
 * of it; the default steepest-ascent solve of a square instance also holds
 * a copy permuted by the start assignment (4 n^2 bytes), which is left out
 * (same results, slower switching) when it does not fit and for server
 * requests.
 */
#ifndef DGS_H
#define DGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dgs_status {
    DGS_OK = 0,
    DGS_E_INVAL = 1,  /* NULL pointer, n < 1, n > max, bad permutation, bad ticket */
    DGS_E_RANGE = 2,  /* some |a_ij| > DGS_MAX_ABS_BENEFIT */
    DGS_E_NOMEM = 3,  /* device allocation failed or request exceeds the budget */
    DGS_E_DEVICE = 4, /* HIP runtime error or no usable GPU */
    DGS_E_AGAIN = 5   /* server: request not finished yet */
} dgs_status;

#define DGS_MAX_ABS_BENEFIT 536870911 /* 2^29 - 1 */
/* Largest n of any call.  The default (steepest-ascent) solve, the batched
 * solve and dgs_solve_rect's m take n <= DGS_MAX_N_SWITCH; DGS_LAZY takes
 * n <= 16384; DGS_PARALLEL takes n <= DGS_MAX_N.  Larger n: DGS_E_INVAL. */
#define DGS_MAX_N 262144
#define DGS_MAX_N_SWITCH 65535

/* dgs_options.flags */
#define DGS_DEVICE_PTRS 0x1u /* benefit, assign_out, init_assign are device pointers */
#define DGS_PROFILE 0x2u     /* also time each phase with HIP events (dgs_result.phase_ms) */
#define DGS_AUTOTUNE 0x4u    /* batch plans: pick the solver's workgroup size by timing it */
/* dgs_solve_ex: Parallel DGS (Algorithm 3 with Check Conflicts, Algorithm 4)
 * instead of the steepest-ascent switching loop.  Each round evaluates every
 * agent (best exchange, lowest job on ties) and every job (best agent to
 * take it, its owner taking that agent's job; lowest agent on ties) afresh.
 * Check Conflicts then looks at the agents with a positive best in index
 * order, then at the jobs with a positive best in index order; each such
 * exchange involves two agents (agent i and the current owner of its best
 * job; job j's best agent and j's current owner) and is kept unless one of
 * them was claimed by an exchange kept before it (a kept exchange claims
 * both).  All kept exchanges are applied at once.  It stops when no
 * exchange improves f; max_switches then bounds the number of ROUNDS (< 0:
 * no bound).  Ends at a 2-exchange local optimum like the default mode, by
 * another trajectory.  n <= DGS_MAX_N.  In this mode and in DGS_LAZY the
 * switching phase of phase_ms holds every round's (pass's) evaluation,
 * rescans and stalls stay 0, and device_ms also spans the host's read of
 * each round's (pass's) count. */
#define DGS_PARALLEL 0x8u
/* dgs_solve_ex: lazy DGS, Algorithm 1 with stale stored bests.  Each pass evaluates every
 * agent (best job, lowest job on ties) and every job (best agent to take it,
 * lowest agent on ties) and stores the positive improvements; then, while a
 * stored improvement is positive, it follows the agent's stored exchange if
 * the largest stored agent value is strictly larger than the largest stored
 * job value, else the job's (lowest index on ties), zeroes the value it
 * followed, applies the exchange only if it raises f and then re-evaluates
 * only the two agents and two jobs involved (the other stored values stay
 * stale).  Passes repeat until one applies nothing.  Ends at a 2-exchange
 * local optimum by the paper's own trajectory.  dgs_result.rounds = passes,
 * dgs_result.attempts = exchanges tried.  n <= 16384; not combinable with
 * DGS_PARALLEL. */
#define DGS_LAZY 0x10u
/* dgs_solve_ex and dgs_solve_rect: start from the global greedy assignment
 * instead of the agent-order greedy one (Section 3.1 asks for a greedy start
 * that takes the benefits into account; this is its variant that looks at
 * all of them at once): while an agent is free, the largest entry a_ij over
 * free agents and free jobs is taken (the lowest agent, then the lowest job,
 * among equal entries).  Computed on the device in rounds of pairs that are
 * the largest entry of both their row and their column among the free ones
 * (all of them are taken by the one-at-a-time rule before anything that
 * could block them); the rounds stop when every agent holds a job.  Ignored
 * when init_assign is given; rejected by dgs_solve_batched and
 * dgs_solve_noalloc (DGS_E_INVAL). */
#define DGS_GLOBAL_GREEDY 0x20u

/* dgs_result.phase_ms indices (filled only with DGS_PROFILE) */
#define DGS_PHASE_RANGE 0  /* value-range check of the benefit matrix */
#define DGS_PHASE_INIT 1   /* greedy start (Section 3.1), or loading init_assign */
#define DGS_PHASE_LAYOUT 2 /* transpose + assignment-ordered working matrix */
#define DGS_PHASE_SCAN 3   /* difference evaluation of every agent (Algorithm 2) */
#define DGS_PHASE_SWITCH 4 /* switching phase until no improving switch is left */
#define DGS_NUM_PHASES 5

typedef struct dgs_options {
    /* Stop after this many switches (< 0: run to the end).  The paper's
     * anytime property (Section 3): DGS always holds a full assignment, so
     * stopping early returns the assignment reached so far. */
    int64_t max_switches;
    /* NULL: greedy start.  Else a permutation of 0..n-1 used as the start
     * (the paper's random start, Section 3.1, or a resumed state).  A
     * non-permutation is rejected with DGS_E_INVAL. */
    const int32_t *init_assign;
    uint32_t flags;
    /* hipStream_t to run on (NULL: the library's own stream).  The call is
     * synchronous either way: it returns when the result is written. */
    void *stream;
} dgs_options;

typedef struct dgs_result {
    int64_t initial_benefit; /* f of the start assignment */
    int64_t total_benefit;   /* f of the returned assignment */
    int64_t switches;        /* number of 2-exchanges applied */
    int64_t rescans;         /* full re-evaluations of agents during switching */
    int64_t stalls;          /* switching rounds that applied no switch (waited for a re-evaluation) */
    float device_ms;         /* device time of the solve (HIP events) */
    float phase_ms[DGS_NUM_PHASES]; /* per-phase device time (DGS_PROFILE only, else 0) */
    int64_t rounds;          /* DGS_PARALLEL: rounds that applied at least one exchange; DGS_LAZY: passes (else 0) */
    int64_t attempts;        /* DGS_LAZY: exchanges tried, applied or not (else 0) */
} dgs_result;

/* Solve one instance with default options (greedy start, run to the end).
 * benefit: host pointer, n*n int32, row-major.  assign_out: host pointer,
 * n int32; on success assign_out[i] = job of agent i. */
dgs_status dgs_solve(const int32_t *benefit, int32_t n, int32_t *assign_out);

/* As dgs_solve with options (may be NULL) and an optional result record
 * (res may be NULL). */
dgs_status dgs_solve_ex(const int32_t *benefit, int32_t n, int32_t *assign_out,
                        const dgs_options *opt, dgs_result *res);

/* Rectangular instance: n agents, m >= n jobs (the paper's motivating n
 * providers and m receivers, Section 1).  benefit is n*m int32, row-major;
 * assign_out has n entries (distinct jobs in [0, m)); jobs nobody holds are
 * unassigned.  Steepest-ascent DGS over two kinds of change: agent i takes
 * job j from its owner k, who takes i's job (a 2-exchange), or agent i moves
 * to an unassigned job j, leaving its old job unassigned (gain
 * a[i][j] - a[i][tau(i)]).  Each agent's best is the lowest job among its
 * largest gains; the best agent (lowest index on ties) is applied while its
 * gain is > 0.  The greedy start lets agents 0..n-1 take their best free job
 * in turn (DGS_GLOBAL_GREEDY: the global greedy start).  The solver treats
 * each unassigned job as held by a virtual agent of benefit 0 (a move is the
 * 2-exchange with it) whose row is never stored: device memory is the n*m
 * matrix (copied in unless DGS_DEVICE_PTRS), its m*n transpose and O(m)
 * vectors, and the evaluation reads the 2*n*m real entries.  m <=
 * DGS_MAX_N_SWITCH.  opt may be NULL; init_assign (n distinct jobs),
 * max_switches, DGS_DEVICE_PTRS, DGS_PROFILE, DGS_GLOBAL_GREEDY and stream
 * apply; DGS_PARALLEL and DGS_LAZY are rejected (DGS_E_INVAL), as are m < n
 * and a non-injective init_assign. */
dgs_status dgs_solve_rect(const int32_t *benefit, int32_t n, int32_t m, int32_t *assign_out,
                          const dgs_options *opt, dgs_result *res);

/* Solve `count` independent instances of possibly different sizes in one
 * device pass (one persistent launch; small instances run one per
 * workgroup).  benefits[b] / assign_outs[b] / ns[b] describe instance b
 * (host pointers, or device pointers with DGS_DEVICE_PTRS).  results may be
 * NULL, else it has `count` entries.  opt may be NULL; its max_switches
 * applies to every instance; init_assign must be NULL.  Every instance's
 * result is identical to dgs_solve_ex on that instance alone. */
dgs_status dgs_solve_batched(int32_t count, const int32_t *const *benefits, const int32_t *ns,
                             int32_t *const *assign_outs, dgs_result *results,
                             const dgs_options *opt);

/* ---- Batch plans: the same batch shape solved again and again ----------
 * A plan fixes `count` instance sizes ns[b] (1 <= n <= 2048 each) and owns
 * device buffers for every instance's benefit matrix and assignment.  A run
 * solves all instances (each result identical to dgs_solve_ex on that
 * instance alone) with one persistent launch, one workgroup per instance,
 * largest first.  The device work of a run (queue reset, the launch, the
 * readback of the per-instance results) is captured once in a HIP graph and
 * replayed by later runs.
 * Tuning: with DGS_AUTOTUNE in opt->flags, the first run times each
 * workgroup size of the batched solver (256 or 512 threads, i.e. 8 or 4
 * agents per thread) on the plan's inputs and keeps the fastest; results do
 * not depend on the choice.  The choice is kept per size class for the
 * process, and in the text file named by the environment variable
 * DGS_TUNE_CACHE when it is set (read by the first plan creation that sees
 * the variable name that file, its entries overriding earlier choices;
 * appended after every new tuning).  opt may be NULL; only max_switches and flags are
 * used (DGS_DEVICE_PTRS is ignored: the plan's buffers are device memory). */
typedef struct dgs_batch_plan dgs_batch_plan;

dgs_status dgs_batch_plan_create(int32_t count, const int32_t *ns, const dgs_options *opt,
                                 dgs_batch_plan **out);

/* Device address of instance b's benefit buffer (n*n int32, row-major) and
 * of its assignment (n int32), valid until the plan is destroyed; NULL for
 * a bad plan or index. */
int32_t *dgs_batch_plan_benefit(dgs_batch_plan *p, int32_t b);
int32_t *dgs_batch_plan_assign(dgs_batch_plan *p, int32_t b);

/* One run.  benefits: NULL (the matrices already sit in the plan's device
 * buffers) or `count` host pointers copied in first.  assign_outs: NULL
 * (assignments stay in the plan's device buffers) or `count` host pointers.
 * results: NULL or `count` records; device_ms is the time of the graph.
 * Runs of one plan must not overlap (the plan is not thread-safe). */
dgs_status dgs_batch_plan_run(dgs_batch_plan *p, const int32_t *const *benefits,
                              int32_t *const *assign_outs, dgs_result *results);

/* Workgroup size and grid the plan launches with (after tuning, if any). */
dgs_status dgs_batch_plan_config(dgs_batch_plan *p, int32_t *block, int32_t *grid);

void dgs_batch_plan_destroy(dgs_batch_plan *p);

/* Difference evaluation (Section 3.2, Algorithm 2) of every agent for a
 * given assignment: for each agent i, the best 2-exchange gain over all
 * jobs j != assign[i] and the job reaching it (lowest j on ties).  The
 * best is reported even when it is <= 0.  For n == 1 agent 0 has no
 * exchange: gain_out[0] = INT64_MIN, job_out[0] = -1.
 * assign: n int32 permutation.  gain_out: n int64.  job_out: n int32.
 * Pointers are host pointers unless opt->flags has DGS_DEVICE_PTRS (then
 * benefit, assign, gain_out and job_out are all device pointers).  opt may
 * be NULL; only flags and stream are used.  res may be NULL; its device_ms
 * is the time of the evaluation kernels. */
dgs_status dgs_diff_eval(const int32_t *benefit, int32_t n, const int32_t *assign,
                         int64_t *gain_out, int32_t *job_out, const dgs_options *opt,
                         dgs_result *res);

/* ---- Serving: continuous batching of periodic LSAP requests ---------- *
 * A stream of independent instances (the periodic re-assignment setting of
 * Section 1) solved as they arrive.  Requests with n <= 2048 that are waiting
 * when the batch worker is free are solved together in one batched launch
 * (as dgs_solve_batched); larger requests run concurrently on their own
 * streams, each admitted when its footprint fits the memory budget and its
 * switching loop fits the compute units left free by the running ones.
 * Every result equals dgs_solve on the same instance. */

typedef struct dgs_server dgs_server;

typedef struct dgs_server_config {
    /* Device bytes the server may hold for requests (0: 64 GiB).  Every
     * buffer of a request comes from a memory pool the server owns and goes
     * back to it when the request completes; the pool keeps freed memory for
     * reuse up to this many bytes. */
    uint64_t hbm_budget_bytes;
    int32_t max_slots;         /* requests resident on the device at once (0: 64) */
    int32_t max_n;             /* largest accepted n (0: 16384) */
} dgs_server_config;

typedef struct dgs_server_stats {
    int64_t submitted;
    int64_t completed;
    int64_t queued;      /* admitted to the queue, not yet on the device */
    int64_t resident;    /* on the device now */
    double inst_per_s;   /* completed / (last completion - first submit) */
    double p50_us;       /* submit -> result ready, over completed requests */
    double p99_us;
} dgs_server_stats;

/* Footprint of one request of size n on the device, in bytes. */
uint64_t dgs_server_footprint(int32_t n);

dgs_status dgs_server_create(const dgs_server_config *cfg, dgs_server **out);

/* Queue one request.  benefit: host pointer, n*n int32, row-major; it must
 * stay valid until the ticket completes.  Never waits for the GPU.
 * DGS_E_NOMEM if the request can never fit the budget; DGS_E_INVAL for
 * n < 1 or n > max_n. */
dgs_status dgs_server_submit(dgs_server *s, const int32_t *benefit, int32_t n,
                             uint64_t *ticket_out);

/* DGS_E_AGAIN while pending; DGS_OK once done (assign_out, n int32, is
 * written and the ticket is consumed).  res may be NULL. */
dgs_status dgs_server_poll(dgs_server *s, uint64_t ticket, int32_t *assign_out,
                           dgs_result *res);

/* As poll, waiting up to timeout_us (< 0: forever). */
dgs_status dgs_server_wait(dgs_server *s, uint64_t ticket, int32_t *assign_out,
                           dgs_result *res, int64_t timeout_us);

/* Statistics so far (the statistics call of the boundary; named _get since
 * the record's typedef already takes the name dgs_server_stats). */
dgs_status dgs_server_stats_get(dgs_server *s, dgs_server_stats *out);

/* Waits for every queued request, then frees everything. */
void dgs_server_destroy(dgs_server *s);

/* ---- Solving without allocating ------------------------------------------
 * For callers that cannot allocate device memory: code running while a HIP
 * graph is being captured, tight serving loops, harnesses that forbid
 * hipMalloc.  Same computation and result as dgs_solve_ex with
 * DGS_DEVICE_PTRS: benefit (n*n int32, row-major), assign_out (n int32) and
 * opt->init_assign (if any, n int32) are device pointers on the calling
 * thread's current device.  Every device buffer of the solve lives in one
 * fixed array of DGS_NOALLOC_BYTES inside the library, one per GPU, held
 * from the library's load until the process ends; hence n <=
 * DGS_NOALLOC_MAX_N (larger n: DGS_E_INVAL).  The call allocates nothing: no
 * hipMalloc, hipFree, pool or pinned host memory (results come back into a
 * static host block).  Its first call on a device only looks up that GPU's
 * array address and creates the timing events.  opt may be NULL;
 * max_switches, init_assign, DGS_PROFILE and stream (NULL: the library's
 * stream on the device the library first used, else the null stream) apply;
 * DGS_PARALLEL and DGS_LAZY are rejected (DGS_E_INVAL).  The array keeps the
 * last call's contents and every buffer is re-initialised by each call.
 * Calls on one GPU share its array: the library serializes them with a
 * lock, but work the caller enqueues itself that reads or overlaps a running
 * call's buffers races with it.  Synchronous: returns once assign_out and
 * res are written. */
#define DGS_NOALLOC_MAX_N 4096
#define DGS_NOALLOC_BYTES (72ull << 20) /* 4n^2 transpose + vectors at n = 4096 */
dgs_status dgs_solve_noalloc(const int32_t *benefit, int32_t n, int32_t *assign_out,
                             const dgs_options *opt, dgs_result *res);

/* ---- Misc --------------------------------------------------------------- */

const char *dgs_status_string(dgs_status st);

/* Message of the last error raised on the calling thread ("" if none). */
const char *dgs_last_error(void);

/* Library version string. */
const char *dgs_version(void);

/* Free the device and pinned host memory and the events the library caches
 * between calls (workspaces of finished solves, the batched solver's
 * staging).  Safe to call at any time; solves in progress keep their own
 * workspaces.  Later calls allocate again as needed.  It also runs at
 * process exit, before the HIP runtime's own teardown. */
void dgs_release_cached(void);

#ifdef __cplusplus
}
#endif

#endif /* DGS_H */
