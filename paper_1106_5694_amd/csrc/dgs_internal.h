// Internal interface between the C ABI (dgs_api.cpp) and the gfx950
// kernels (dgs_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/dgs.h"

namespace dgs {

typedef unsigned long long u64;

// Device state of one single-instance solve.  Layout (all row-major int32,
// n x n, 64-bit element offsets):
//   A   the caller's benefit matrix a_ij (read-only)
//   AT  its transpose: AT[j][i] = a_ij (read-only after the build).  Row
//       tau(c) of AT is column c of the assignment-ordered matrix
//       W[r][c] = a[r][tau(c)] (the benefit agent r would get from agent c's
//       current job), which the evaluation reads this way; W itself is
//       never built.
// Vectors (n entries): tau (job of agent), sigma (agent of job), d (current
// benefit of agent c, d[c] = a[c][tau(c)]).
// Per-agent best record: bk = packed key of the best exchange (gain, job),
// bb = bound key (every other exchange of the agent is <= bb), bc = the
// partner agent of the best exchange.
// Length of the candidate lists the full evaluation hands to the switching loop.
constexpr int kScanListLen = 8;

// Rectangular instances (nr agents, n >= nr jobs) run as n agents: agents
// nr..n-1 are virtual agents of benefit 0 for every job, each holding one
// job nobody really holds, so an exchange with one of them is a real
// agent's move to an unassigned job.  Their rows are never stored: A is
// nr x n (row stride n) and AT is n x nr (row stride nr); every read of a
// virtual agent's benefit is 0.  Square instances have nr = n.
struct Instance {
    int32_t n = 0;
    int32_t nr = 0;  // real agents (rows of A); n for a square instance
    const int32_t *A = nullptr;
    int32_t *AT = nullptr;
    int32_t *tau = nullptr;
    int32_t *sigma = nullptr;
    int32_t *d = nullptr;
    u64 *bk = nullptr;
    u64 *bb = nullptr;
    int32_t *bc = nullptr;
    // scratch for the switch loop and small reductions
    int64_t *stats = nullptr;    // [0] switches, [1] gain sum, [2] f0, [3] re-evaluations, [4] stalls,
                                 // [5] accepted in the last parallel round, [6] scratch sum
    int32_t *flags = nullptr;    // [0] range error, [1] permutation error, [2] wait timed out
    void *words = nullptr;       // exchange words of the switching loop
    void *greedy = nullptr;      // scratch of the greedy start
    void *glob = nullptr;        // scratch of the global greedy start
    void *scan = nullptr;        // scratch of the difference evaluation (per-block top-2)
    u64 *lists = nullptr;        // [n][kScanListLen] initial candidate lists (keys, 0 = empty)
    int32_t *W = nullptr;        // n x n, W[r][c] = a[r][tau0(c)] for the start assignment tau0, read by
                                 // the steepest-ascent loop of a square instance, or null: that loop then
                                 // reads A
    int32_t *par = nullptr;      // [n] Parallel DGS: partner of each accepted agent, else -1
};

// Host-side helpers of the C ABI (dgs_api.cpp).
void set_error(const char *fmt, ...);  // thread-local message for dgs_last_error
dgs_status ensure_context();            // device, stream and switch-loop grid, once

// Return DGS_E_DEVICE (with a message) from the enclosing function when a HIP call fails.
#define DGS_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            ::dgs::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            return DGS_E_DEVICE;                                                            \
        }                                                                                   \
    } while (0)

hipError_t launch_range_check(const int32_t *A, int64_t count, int32_t *flag, hipStream_t s);
// Greedy start (dgs_greedy.hip); scratch of greedy_scratch_bytes(n).
size_t greedy_scratch_bytes(int n);
// rows agents (0..rows-1) over cols jobs; agents rows..cols-1 then take the
// jobs left free in increasing order.
// persistent: one cooperative launch that holds the whole device (callers that
// do not share the device), else rounds of two launches.
hipError_t launch_greedy_rounds(const int32_t *A, int32_t rows, int32_t cols, int32_t *tau, int32_t *sigma,
                                void *scratch, int32_t *err, bool persistent, hipStream_t s);
// Virtual agents rows..n-1 take the jobs with sigma = -1 in increasing order.
hipError_t launch_fill_virtual(int32_t *tau, int32_t *sigma, int32_t rows, int32_t n, hipStream_t s);
// Global greedy start (largest remaining entry first, lowest agent, then
// lowest job, on ties) of rows agents over cols jobs, by rounds of locally
// dominant pairs; AT is the cols x rows transpose; scratch of
// global_greedy_scratch_bytes(rows, cols); the host reads the matched count
// every few rounds into *host_count (pinned).  Agents rows..cols-1 then take
// the jobs left free in increasing order.
size_t global_greedy_scratch_bytes(int rows, int cols);
hipError_t run_global_greedy(const int32_t *A, const int32_t *AT, int32_t rows, int32_t cols, int32_t *tau,
                             int32_t *sigma, void *scratch, int64_t *host_count, int64_t *rounds_out,
                             hipStream_t s);
// p[0..n) = v (a kernel, so that it can sit in a captured graph)
hipError_t launch_fill(int32_t *p, int32_t n, int32_t v, hipStream_t s);
hipError_t launch_invert_checked(const int32_t *tau, int32_t n, int32_t *sigma, int32_t *flag,
                                 hipStream_t s);
// AT (cols x rows) = transpose of A (rows x cols).
hipError_t launch_transpose(const int32_t *A, int32_t *AT, int32_t rows, int32_t cols, hipStream_t s);
// W[r][c] = a[r][tau(c)] for the rows r < rows of A (rows x n; tau: n agents; W: rows x n, device).
hipError_t launch_permuted(const int32_t *A, const int32_t *tau, int32_t rows, int32_t n, int32_t *W,
                           hipStream_t s);
// d[r] = a[r][tau(r)] (0 for virtual agents r >= nr) and the objective sum.
hipError_t launch_benefits(const int32_t *A, const int32_t *tau, int32_t n, int32_t nr, int32_t *d, int64_t *f,
                           hipStream_t s);
// Symmetric tile-pair difference evaluation from A^T through tau
// (dgs_scan.hip): each agent's best exchange into I.bk / I.bc, its candidate
// list into I.lists and the list's bound into I.bb.
size_t scan_pairs_scratch_bytes(int n);
hipError_t launch_scan_pairs(const Instance &I, void *scratch, hipStream_t s);
// The same evaluation, in one pass writing each agent's best keyed by job
// into by_job (its partner
// sigma(job) into partner, if not null: the agent side, ADE) and its best
// keyed by partner agent into by_agent (the best agent to take the agent's
// job, lowest agent on ties: the job side, JDE, of job tau(agent)).
hipError_t launch_scan_best_transposed(const Instance &I, void *scratch, hipStream_t s, u64 *by_job,
                                       int32_t *partner, u64 *by_agent);
// Largest n of the switching loop with cooperative re-evaluation (16-bit agent
// and job fields): the largest n of the steepest-ascent solve.
constexpr int kSwitchExMaxN = 65535;
// Switching loop with cooperative re-evaluation (dgs_switch3.hip), for 2 <= n <= kSwitchExMaxN:
// grid of switch_v3_grid(n) workgroups, exchange words of switch_v3_word_bytes(n) (set to 0xFF first).
int switch_v3_grid(int n);
size_t switch_v3_word_bytes(int n);
hipError_t launch_switch_v3(const Instance &I, int64_t max_switches, void *words, int32_t *err, bool coop,
                            hipStream_t s);
// Workgroups the switching loop of an n-agent solve keeps resident.
int switch_loop_grid(int n);

// Host staging (pinned), timing events and, for calls without a memory
// pool, a cached device block of the batched solver.  The library keeps one
// for its own calls; the server's small-request worker owns another.
struct BatchArena {
    std::mutex mu;
    char *dev = nullptr;
    size_t bytes = 0;
    char *host = nullptr;  // pinned staging for items / order / results
    size_t host_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};
// Frees what the arena holds (device block, pinned staging, events).
void batch_arena_clear(BatchArena &A);

// Internal entry points used by the server (dgs_api.cpp).  With a memory
// pool, every device buffer of the call comes from it (stream-ordered on s)
// and goes back to it before the call returns.
dgs_status solve_internal(const int32_t *benefit, int32_t n, int32_t *assign_out, int64_t max_switches, bool dev,
                          bool coop, hipStream_t s, dgs_result *res, hipMemPool_t pool);
dgs_status solve_batch_internal(int32_t count, const int32_t *const *benefits, const int32_t *ns,
                                int32_t *const *outs, dgs_result *results, int64_t max_switches, int grid_cap,
                                hipStream_t s, hipMemPool_t pool, BatchArena *arena);
int device_cus();

// Batched single-workgroup solver (dgs_batch.hip) for instances with n <= kBatchMaxN.
constexpr int kBatchMaxN = 2048;
struct BatchItem {
    const int32_t *A;  // n x n benefits (device)
    int32_t *tau;      // n outputs (device)
    int32_t *AT;       // n x n scratch
    u64 *lists;        // 2n scratch
    int64_t *res;      // [0] f0 [1] f [2] switches [3] re-evaluations [4] status
    u64 *part;  // batch_part_bytes(n) scratch: the evaluation's per (agent, block) partials
    int n;
    int tile0;   // first of the instance's batch_tiles(n) transpose tiles (running count in table order)
    int pair0;   // first of its batch_pairs(n) evaluation tile pairs (likewise)
    int pad;
};
// Running totals of a batch's item table.
struct BatchTotals {
    int64_t tiles = 0, pairs = 0;
};
// The batched solve: the greedy starts (one workgroup per instance; then the same
// workgroups transpose every instance), every instance's difference evaluation over the
// whole device, then the switching (one workgroup per instance).  queue: three words,
// cleared.
hipError_t launch_batch(const BatchItem *items, const int32_t *order, int count, int32_t *queue,
                        int64_t max_switches, const BatchTotals &tot, int block, int grid, hipStream_t s);
// Transpose tiles, evaluation tile pairs and partials bytes of an instance of size n.
inline int64_t batch_tiles(int n) {
    const int64_t nt = (n + 63) / 64;
    return nt * nt;
}
inline int64_t batch_pairs(int n) {
    const int64_t nt = (n + 63) / 64;
    return nt * (nt + 1) / 2;
}
inline size_t batch_part_bytes(int n) { return (size_t)n * (size_t)((n + 63) / 64) * 2 * sizeof(u64); }
// Fills a batch item's offsets from the running totals and advances them.
inline void batch_place(BatchItem &it, BatchTotals &tot) {
    it.tile0 = (int)tot.tiles;
    it.pair0 = (int)tot.pairs;
    it.pad = 0;
    tot.tiles += batch_tiles(it.n);
    tot.pairs += batch_pairs(it.n);
}
int batch_grid_limit(int block);

// Parallel DGS (dgs_parallel.hip): one round of Check Conflicts over the
// fresh agent bests in I.bk / I.bc and job bests in I.bb (per owner agent),
// the kept exchanges per agent into acc, then the swaps (stats[0] and [1]
// advanced, stats[5] = kept count).
int parallel_max_agents();
hipError_t launch_parallel_round(const Instance &I, int32_t *acc, hipStream_t s);

// Lazy DGS (dgs_lazy.hip): the switching phase of one pass of Algorithm 1
// with stale stored bests as one cooperative launch of lazy_grid(n)
// workgroups, for n <= kLazyMaxN.  Reads the pass's evaluation (agent side
// in I.bk, job side per owner agent in jde); exchange words of
// lazy_word_bytes(n) (set to 0xFF first); keeps tau, sigma and d; advances
// stats[0], [1] and [7] (attempts) and sets stats[5] to the switches of the
// pass.
constexpr int kLazyMaxN = 16384;
int lazy_grid(int n);
size_t lazy_word_bytes(int n);
hipError_t launch_lazy_pass(const Instance &I, const u64 *jde, void *words, int64_t max_switches, hipStream_t s);

hipError_t launch_export_best(const Instance &I, int64_t *gain_out, int32_t *job_out,
                              hipStream_t s);

}  // namespace dgs
