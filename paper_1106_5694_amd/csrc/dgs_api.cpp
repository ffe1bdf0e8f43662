// C ABI of the DGS library (declared in include/dgs.h).
//
// Host side only: argument checks, device workspaces, stream handling and
// the order of kernel launches.  Every step of the method itself runs in
// the kernels of dgs_kernels.hip; there is no CPU fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dgs.h"
#include "dgs_internal.h"

namespace dgs {

thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

// ---- device context ---------------------------------------------------------------

struct Context {
    std::once_flag once;
    int device = -1;
    hipStream_t stream = nullptr;
    dgs_status init_status = DGS_OK;
    std::string init_error;
    // Cooperative switch loops need every workgroup resident; one at a time.
    std::mutex loop_mu;
};

Context g_ctx;

void teardown_at_exit();

dgs_status ensure_context() {
    std::call_once(g_ctx.once, [] {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess || count < 1) {
            g_ctx.init_status = DGS_E_DEVICE;
            g_ctx.init_error = std::string("no HIP device: ") + hipGetErrorString(e);
            return;
        }
        if (hipGetDevice(&g_ctx.device) != hipSuccess) g_ctx.device = 0;
        if (hipStreamCreateWithFlags(&g_ctx.stream, hipStreamNonBlocking) != hipSuccess) {
            g_ctx.init_status = DGS_E_DEVICE;
            g_ctx.init_error = "hipStreamCreate failed";
            return;
        }
        // Registered after the HIP runtime is up, so it runs before the
        // runtime's own teardown (and before that of tools attached to it).
        std::atexit(teardown_at_exit);
    });
    if (g_ctx.init_status != DGS_OK) set_error("%s", g_ctx.init_error.c_str());
    return g_ctx.init_status;
}

namespace {

// ---- workspaces -----------------------------------------------------------------------
// One workspace holds the device buffers of one instance of size <= cap.
// By default workspaces are cached (released ones are reused by later calls
// of a size they fit) so repeated solves do not pay for allocation.  A call
// that brings a memory pool (the server) takes its buffers from that pool,
// stream-ordered, and returns them at the end of the call: the pool, not the
// cache, then bounds the device memory it holds.

struct Workspace {
    int32_t cap = 0;       // largest n of the vectors
    size_t mat_bytes = 0;  // capacity of the transpose (and of the benefit copy)
    bool has_acopy = false;
    int32_t *acopy = nullptr;  // device copy of a host benefit matrix
    int32_t *at = nullptr;
    int32_t *wperm = nullptr;  // W[r][c] = a[r][tau0(c)] of a square steepest-ascent solve (or null)
    char *vec = nullptr;  // vectors + scratch
    size_t vec_bytes = 0;
    hipMemPool_t pool = nullptr;  // buffers from this pool (freed on `stream`), else from hipMalloc
    hipStream_t stream = nullptr;
};

std::mutex g_ws_mu;
std::multimap<int32_t, Workspace *> g_ws_free;

// Host-side resources of a call: a pinned block for the results read back
// and the timing events.  Cached on their own (freeing pinned memory waits
// for the whole device), also for calls whose buffers come from a pool.
struct HostRes {
    int64_t *stats = nullptr;  // pinned, 16 int64: stats[8], flags[4] (as int64), per-mode scratch
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ph[DGS_NUM_PHASES + 1] = {};  // phase boundaries (DGS_PROFILE)
};

std::mutex g_host_mu;
std::vector<HostRes *> g_host_free;

void destroy_host(HostRes *h) {
    if (!h) return;
    if (h->stats) (void)hipHostFree(h->stats);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    for (auto &e : h->ph)
        if (e) (void)hipEventDestroy(e);
    delete h;
}

dgs_status acquire_host(HostRes **out) {
    {
        std::lock_guard<std::mutex> lk(g_host_mu);
        if (!g_host_free.empty()) {
            *out = g_host_free.back();
            g_host_free.pop_back();
            return DGS_OK;
        }
    }
    HostRes *h = new HostRes();
    bool ok = hipHostMalloc((void **)&h->stats, 16 * sizeof(int64_t), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipEventCreate(&h->ev0) == hipSuccess && hipEventCreate(&h->ev1) == hipSuccess;
    for (auto &e : h->ph) ok = ok && hipEventCreate(&e) == hipSuccess;
    if (!ok) {
        set_error("pinned allocation or hipEventCreate failed");
        destroy_host(h);
        return DGS_E_DEVICE;
    }
    *out = h;
    return DGS_OK;
}

void release_host(HostRes *h) {
    std::lock_guard<std::mutex> lk(g_host_mu);
    g_host_free.push_back(h);
}

// Byte layout of the vector block of a workspace.  Every piece starts on a
// 256-byte boundary; vec_layout() is the single source of the offsets used
// both to size the allocation and to carve it.
struct VecLayout {
    size_t tau, sigma, d, bc, bk, bb, lists, stats, flags, words, greedy, glob, scan, par, total;
};

VecLayout vec_layout(int32_t n) {
    VecLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    };
    L.tau = take((size_t)n * 4);
    L.sigma = take((size_t)n * 4);
    L.d = take((size_t)n * 4);
    L.bc = take((size_t)n * 4);
    L.bk = take((size_t)n * 8);
    L.bb = take((size_t)n * 8);
    L.lists = take((size_t)n * 8 * kScanListLen);
    L.stats = take(8 * sizeof(int64_t));
    L.flags = take(4 * sizeof(int32_t));
    const bool ex = n >= 2 && n <= kSwitchExMaxN;
    L.words = take(ex ? switch_v3_word_bytes(n) : 0);
    L.greedy = take(greedy_scratch_bytes(n));
    L.glob = take(global_greedy_scratch_bytes(n, n));
    L.scan = take(scan_pairs_scratch_bytes(n));
    L.par = take((size_t)n * 4);
    L.total = off;
    return L;
}

void free_ws(Workspace *w) {
    if (!w) return;
    for (void *p : {(void *)w->acopy, (void *)w->at, (void *)w->wperm, (void *)w->vec}) {
        if (!p) continue;
        if (w->pool)
            (void)hipFreeAsync(p, w->stream);
        else
            (void)hipFree(p);
    }
    delete w;
}

// Device buffers for an instance of n agents (nr of them real: matrices of
// nr x n entries): from the cache (pool == NULL) or from `pool`, ordered on
// `stream`.  need_w: also the n x n matrix W of the steepest-ascent loop (left out, not an
// error, when it does not fit).
dgs_status alloc_ws(int32_t n, int32_t nr, bool need_acopy, bool need_w, hipMemPool_t pool, hipStream_t stream,
                    Workspace **out) {
    const size_t mat = (size_t)nr * (size_t)n * sizeof(int32_t);
    if (!pool) {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        for (auto it = g_ws_free.lower_bound(n); it != g_ws_free.end(); ++it) {
            // do not hand a huge workspace to a tiny problem
            if (it->first > 2 * n + 1024) break;
            if (need_acopy && !it->second->has_acopy) continue;
            if (need_w && !it->second->wperm) continue;
            if (it->second->mat_bytes < mat) continue;
            *out = it->second;
            g_ws_free.erase(it);
            return DGS_OK;
        }
    }
    Workspace *w = new Workspace();
    w->cap = n;
    w->mat_bytes = mat;
    w->pool = pool;
    w->stream = stream;
    auto dev = [&](void **p, size_t bytes) {
        return (pool ? hipMallocFromPoolAsync(p, bytes, pool, stream) : hipMalloc(p, bytes)) == hipSuccess;
    };
    auto fail = [&](const char *what) {
        set_error("device allocation of %s for n=%d failed", what, n);
        free_ws(w);
        return DGS_E_NOMEM;
    };
    if (need_acopy) {
        if (!dev((void **)&w->acopy, mat)) return fail("benefit copy");
        w->has_acopy = true;
    }
    if (!dev((void **)&w->at, mat)) return fail("transpose");
    if (need_w && !dev((void **)&w->wperm, mat)) {
        // W only speeds the switching loop up: without it the loop reads A (same results)
        w->wperm = nullptr;
        (void)hipGetLastError();  // the failed allocation must not surface at a later launch check
    }
    w->vec_bytes = vec_layout(n).total;
    if (!dev((void **)&w->vec, w->vec_bytes)) return fail("vectors");
    *out = w;
    return DGS_OK;
}

// Back to the cache, or (pool buffers) back to the pool.
void release_ws(Workspace *w) {
    if (w->pool) {
        free_ws(w);
        return;
    }
    std::lock_guard<std::mutex> lk(g_ws_mu);
    g_ws_free.emplace(w->cap, w);
}

// Carve an Instance out of a workspace (n <= w->cap).
Instance carve(Workspace *w, const int32_t *A, int32_t n, int32_t nr) {
    Instance I;
    I.n = n;
    I.nr = nr;
    I.A = A;
    I.AT = w->at;
    const VecLayout L = vec_layout(n);
    char *p = w->vec;
    I.tau = (int32_t *)(p + L.tau);
    I.sigma = (int32_t *)(p + L.sigma);
    I.d = (int32_t *)(p + L.d);
    I.bc = (int32_t *)(p + L.bc);
    I.bk = (u64 *)(p + L.bk);
    I.bb = (u64 *)(p + L.bb);
    I.lists = (u64 *)(p + L.lists);
    I.stats = (int64_t *)(p + L.stats);
    I.flags = (int32_t *)(p + L.flags);
    I.words = p + L.words;
    I.greedy = p + L.greedy;
    I.scan = p + L.scan;
    I.par = (int32_t *)(p + L.par);
    I.glob = p + L.glob;
    return I;
}

bool is_perm_host(const int32_t *p, int32_t n) {
    std::vector<char> seen((size_t)n, 0);
    for (int32_t i = 0; i < n; ++i) {
        if (p[i] < 0 || p[i] >= n || seen[(size_t)p[i]]) return false;
        seen[(size_t)p[i]] = 1;
    }
    return true;
}

// Reads an init assignment (host or device) and checks it on the host.
dgs_status check_init(const int32_t *init, int32_t n, bool dev, hipStream_t s) {
    std::vector<int32_t> h;
    const int32_t *p = init;
    if (dev) {
        h.resize((size_t)n);
        DGS_HIP(hipMemcpyAsync(h.data(), init, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        DGS_HIP(hipStreamSynchronize(s));
        p = h.data();
    }
    if (!is_perm_host(p, n)) {
        set_error("init_assign is not a permutation of 0..n-1");
        return DGS_E_INVAL;
    }
    return DGS_OK;
}

enum class Mode { Solve, DiffEval };

struct Call {
    const int32_t *benefit;
    int32_t n;
    const int32_t *assign_in;  // start (solve) or the assignment to evaluate
    int64_t max_switches;
    int32_t nr = 0;            // real agents of a rectangular instance (benefit is nr x n); 0: square
    bool init_host = false;    // assign_in is a host pointer even when dev is set
    bool global_greedy = false;  // start from the global greedy (largest remaining entry first)
    bool dev;
    bool profile;
    bool coop = true;  // cooperative switching launch (else the caller owns co-residency)
    bool parallel = false;  // Parallel DGS rounds instead of the switching loop (max_switches = max rounds)
    bool lazy = false;      // lazy DGS passes (Algorithm 1 with stale stored bests) instead of the switching loop
    bool permuted = true;   // a square steepest-ascent solve builds W for its switching loop (+4n^2 bytes)
    hipMemPool_t pool = nullptr;  // device buffers from this pool (stream-ordered) instead of the cache
    Workspace *ws = nullptr;      // a workspace the caller holds (not taken from or returned to the cache)
    HostRes *host = nullptr;      // host resources the caller holds (likewise)
    hipStream_t stream;
};

// Parallel DGS (Algorithm 3): rounds of Check Conflicts + apply, each
// followed by a fresh difference evaluation of every agent and every job,
// until a round keeps nothing.  Expects the evaluation of the start
// assignment in I.bk / I.bc (agents) and I.bb (jobs, per owner agent).  The
// evaluations read A^T through tau, so W is never built.
dgs_status parallel_rounds(const Instance &I, HostRes *h, int64_t max_rounds, int64_t *rounds_out, hipStream_t s) {
    int64_t rounds = 0;
    int64_t *accepted = h->stats + 12;
    while (max_rounds < 0 || rounds < max_rounds) {
        DGS_HIP(launch_parallel_round(I, I.par, s));
        DGS_HIP(hipMemcpyAsync(accepted, I.stats + 5, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        DGS_HIP(hipStreamSynchronize(s));
        if (*accepted == 0) break;
        ++rounds;
        if (max_rounds >= 0 && rounds >= max_rounds) break;
        // fresh d and evaluation; stats[6] takes the objective sum (f0 stays the start's)
        DGS_HIP(launch_benefits(I.A, I.tau, I.n, I.nr, I.d, I.stats + 6, s));
        DGS_HIP(launch_scan_best_transposed(I, I.scan, s, I.bk, I.bc, I.bb));
    }
    *rounds_out = rounds;
    return DGS_OK;
}

// Lazy DGS (Algorithm 1 with stale stored bests): passes of a full
// evaluation of agents (into I.bk) and jobs (per owner agent, into I.bb,
// free in this mode) followed by the switching phase of the pass (one
// cooperative launch), until a pass applies nothing or max_switches is
// reached.  d must be current; the passes keep tau, sigma and d.
dgs_status lazy_passes(const Instance &I, HostRes *h, int64_t max_switches, bool coop, int64_t *passes_out,
                       hipStream_t s) {
    int64_t passes = 0, S = 0;
    int64_t *hs = h->stats + 10;  // [0..5] = stats[0..5]
    if (lazy_word_bytes(I.n) > switch_v3_word_bytes(I.n)) {
        set_error("internal: lazy exchange words do not fit");
        return DGS_E_DEVICE;
    }
    while (I.n >= 2 && (max_switches < 0 || S < max_switches)) {
        DGS_HIP(launch_scan_best_transposed(I, I.scan, s, I.bk, nullptr, I.bb));
        ++passes;
        DGS_HIP(launch_fill((int32_t *)I.words, (int32_t)(lazy_word_bytes(I.n) / 4), -1, s));
        {
            // the cooperative pass holds the whole device
            std::unique_lock<std::mutex> lk(g_ctx.loop_mu, std::defer_lock);
            if (coop) lk.lock();
            DGS_HIP(launch_lazy_pass(I, I.bb, I.words, max_switches, s));
            int32_t *err = (int32_t *)(h->stats + 9);  // rewritten by the final flags copy
            DGS_HIP(hipMemcpyAsync(hs, I.stats, 6 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            DGS_HIP(hipMemcpyAsync(err, I.flags + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            DGS_HIP(hipStreamSynchronize(s));
            S = hs[0];
            if (hs[5] == 0 || *err != 0) break;  // a broken invariant is reported by the caller
        }
    }
    if (I.n < 2) passes = 1;  // one pass that finds nothing to store
    *passes_out = passes;
    return DGS_OK;
}

// The whole device pipeline of one instance.
dgs_status run_instance(const Call &c, Mode mode, int32_t *assign_out, int64_t *gain_out, int32_t *job_out,
                        dgs_result *res) {
    const int32_t n = c.n;
    const int32_t nr = c.nr > 0 ? c.nr : n;  // real agents (rows of the benefit matrix)
    hipStream_t s = c.stream;
    if (nr != n && (c.parallel || c.lazy || mode != Mode::Solve)) {
        set_error("internal: rectangular instances run the steepest-ascent solve only");
        return DGS_E_INVAL;
    }
    if (c.parallel && n > parallel_max_agents()) {
        set_error("parallel mode supports n <= %d", parallel_max_agents());
        return DGS_E_INVAL;
    }
    if (!c.parallel && !c.lazy && mode == Mode::Solve && n > kSwitchExMaxN) {
        set_error("the steepest-ascent solve supports n <= %d (DGS_PARALLEL: n <= %d)", kSwitchExMaxN,
                  parallel_max_agents());
        return DGS_E_INVAL;
    }
    if (c.lazy && (c.parallel || n > kLazyMaxN)) {
        set_error(c.parallel ? "DGS_LAZY and DGS_PARALLEL exclude each other" : "lazy mode supports n <= %d",
                  kLazyMaxN);
        return DGS_E_INVAL;
    }
    const bool init_dev = c.dev && !c.init_host;
    if (c.assign_in && !c.ws) {  // (a caller-held workspace comes with its own host-side check)
        dgs_status st = check_init(c.assign_in, n, init_dev, s);
        if (st != DGS_OK) return st;
    }
    HostRes *h = c.host;
    dgs_status st = h ? DGS_OK : acquire_host(&h);
    if (st != DGS_OK) return st;
    Workspace *w = c.ws;
    // the steepest-ascent loop of a square instance reads W (a caller-held workspace has none)
    const bool steepest = mode == Mode::Solve && !c.parallel && !c.lazy && n >= 2;
    // (rectangular instances read A: measured no better; a call without switches needs no W)
    const bool use_w = steepest && nr == n && c.permuted && c.max_switches != 0;
    st = w ? DGS_OK : alloc_ws(n, nr, !c.dev, use_w, c.pool, s, &w);
    if (st != DGS_OK) {
        if (!c.host) release_host(h);
        return st;
    }
    struct Guard {
        Workspace *w;
        HostRes *h;
        ~Guard() {
            if (w) release_ws(w);
            if (h) release_host(h);
        }
    } guard{c.ws ? nullptr : w, c.host ? nullptr : h};

    const size_t mat = (size_t)nr * (size_t)n * sizeof(int32_t);
    if (vec_layout(n).total > w->vec_bytes || mat > w->mat_bytes) {
        set_error("internal: workspace too small for n=%d", n);
        return DGS_E_NOMEM;
    }
    const int32_t *A = c.dev ? c.benefit : w->acopy;
    Instance I = carve(w, A, n, nr);
    I.W = use_w ? w->wperm : nullptr;
    if (!c.dev) DGS_HIP(hipMemcpyAsync(w->acopy, c.benefit, mat, hipMemcpyHostToDevice, s));

    DGS_HIP(hipEventRecord(h->ev0, s));
    auto mark = [&](int i) { return c.profile ? hipEventRecord(h->ph[i], s) : hipSuccess; };
    // cleared by kernels (no memset nodes if a caller captures the stream)
    DGS_HIP(launch_fill((int32_t *)I.stats, 16, 0, s));
    DGS_HIP(launch_fill(I.flags, 4, 0, s));
    DGS_HIP(mark(DGS_PHASE_RANGE));
    DGS_HIP(launch_range_check(A, (int64_t)nr * n, I.flags, s));
    DGS_HIP(mark(DGS_PHASE_INIT));
    const bool gg = c.global_greedy && !c.assign_in;
    if (c.assign_in) {
        DGS_HIP(hipMemcpyAsync(I.tau, c.assign_in, (size_t)n * 4,
                               init_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        DGS_HIP(launch_invert_checked(I.tau, n, I.sigma, I.flags + 1, s));
    } else if (gg) {
        // the global greedy start reads columns too: the transpose comes first
        DGS_HIP(launch_transpose(A, I.AT, nr, n, s));
        int64_t gg_rounds = 0;
        DGS_HIP(run_global_greedy(A, I.AT, nr, n, I.tau, I.sigma, I.glob, h->stats + 12, &gg_rounds, s));
    } else {
        // the persistent greedy holds the whole device, like the switching loop
        std::unique_lock<std::mutex> lk(g_ctx.loop_mu, std::defer_lock);
        if (c.coop) lk.lock();
        DGS_HIP(launch_greedy_rounds(A, nr, n, I.tau, I.sigma, I.greedy, I.flags + 2, c.coop, s));
        if (c.coop) {  // finished before another solve may take the device; a failed start stops here
            int32_t *gerr = (int32_t *)(h->stats + 12);
            DGS_HIP(hipMemcpyAsync(gerr, I.flags + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            DGS_HIP(hipStreamSynchronize(s));
            if (*gerr) {
                set_error("internal device check failed in the greedy start (code %d)", *gerr);
                return DGS_E_DEVICE;
            }
        }
    }
    DGS_HIP(mark(DGS_PHASE_LAYOUT));
    if (!gg) DGS_HIP(launch_transpose(A, I.AT, nr, n, s));
    if (I.W) DGS_HIP(launch_permuted(A, I.tau, nr, n, I.W, s));
    DGS_HIP(launch_benefits(A, I.tau, n, nr, I.d, I.stats + 2, s));
    DGS_HIP(mark(DGS_PHASE_SCAN));
    if (c.parallel && mode == Mode::Solve)
        DGS_HIP(launch_scan_best_transposed(I, I.scan, s, I.bk, I.bc, I.bb));
    else if (!c.lazy || mode != Mode::Solve)
        DGS_HIP(launch_scan_pairs(I, I.scan, s));  // (lazy passes evaluate at their start)
    DGS_HIP(mark(DGS_PHASE_SWITCH));
    int64_t rounds = 0;
    if (mode == Mode::Solve && c.parallel) {
        st = parallel_rounds(I, h, c.max_switches, &rounds, s);
        if (st != DGS_OK) return st;
    } else if (mode == Mode::Solve && c.lazy) {
        st = lazy_passes(I, h, c.max_switches, c.coop, &rounds, s);
        if (st != DGS_OK) return st;
    } else if (mode == Mode::Solve) {
        // The loops exit at once when the range check failed.  n = 1 has no
        // exchange at all.  Cooperative switching loops of concurrent calls
        // run one at a time (each needs its whole grid resident).
        std::unique_lock<std::mutex> lk(g_ctx.loop_mu, std::defer_lock);
        if (c.coop) lk.lock();
        if (n >= 2) {
            // stale round tags must not match rounds 0 and 1
            DGS_HIP(launch_fill((int32_t *)I.words, (int32_t)(switch_v3_word_bytes(n) / 4), -1, s));
            DGS_HIP(launch_switch_v3(I, c.max_switches, I.words, I.flags + 2, c.coop, s));
        }
        if (c.coop) {
            DGS_HIP(hipEventRecord(h->ev1, s));
            DGS_HIP(hipEventSynchronize(h->ev1));
        }
    } else {
        DGS_HIP(launch_export_best(I, gain_out, job_out, s));
    }
    DGS_HIP(mark(DGS_NUM_PHASES));
    DGS_HIP(hipEventRecord(h->ev1, s));
    DGS_HIP(hipMemcpyAsync(h->stats, I.stats, 8 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DGS_HIP(hipMemcpyAsync(h->stats + 8, I.flags, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DGS_HIP(hipStreamSynchronize(s));
    const int32_t *flags = (const int32_t *)(h->stats + 8);
    if (flags[0]) {
        set_error("benefit entry outside [-(2^29-1), 2^29-1]");
        return DGS_E_RANGE;
    }
    if (flags[1]) {
        set_error("init_assign is not a permutation of 0..n-1");
        return DGS_E_INVAL;
    }
    if (flags[2]) {
        set_error("internal device check failed (code %d)", flags[2]);
        return DGS_E_DEVICE;
    }
    if (mode == Mode::Solve) {  // the real agents' jobs
        DGS_HIP(hipMemcpyAsync(assign_out, I.tau, (size_t)nr * 4,
                               c.dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
        DGS_HIP(hipStreamSynchronize(s));
    }
    if (res) {
        float ms = 0.f;
        DGS_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        const int64_t *hs = h->stats;
        res->initial_benefit = hs[2];
        res->total_benefit = hs[2] + hs[1];
        res->switches = hs[0];
        res->rescans = hs[3];
        res->stalls = hs[4];
        res->rounds = rounds;
        res->attempts = c.lazy ? hs[7] : 0;
        res->device_ms = ms;
        for (int i = 0; i < DGS_NUM_PHASES; ++i) {
            float pm = 0.f;
            if (c.profile) DGS_HIP(hipEventElapsedTime(&pm, h->ph[i], h->ph[i + 1]));
            res->phase_ms[i] = pm;
        }
    }
    return DGS_OK;
}

// ---- batched solves ------------------------------------------------------------------
// Instances with n <= kBatchMaxN run in one persistent launch (one workgroup
// per instance, largest first); larger ones run one after another through
// the single-instance path.  The device arena is cached between calls.

struct BatchCall {
    int32_t count;
    const int32_t *const *benefits;
    const int32_t *ns;
    int32_t *const *outs;
    dgs_result *results;
    int64_t max_switches;
    bool dev;
    bool profile;
    int grid_cap = 0;  // > 0: at most this many workgroups (the server reserves the rest)
    hipMemPool_t pool = nullptr;  // device buffers from this pool per call (else the arena's cached block)
    BatchArena *arena = nullptr;  // host staging and events (else the library's own arena)
    hipStream_t stream;
};

BatchArena g_batch;

int g_batch_block = 256;  // workgroup size of the batched solver (autotuned)

// Host staging and events of the arena; its cached device block too unless
// the call brings a pool.
dgs_status batch_reserve(BatchArena &A, size_t dev_bytes, size_t host_bytes, bool cache_dev) {
    if (cache_dev && dev_bytes > A.bytes) {
        if (A.dev) (void)hipFree(A.dev);
        A.dev = nullptr;
        A.bytes = 0;
        if (hipMalloc((void **)&A.dev, dev_bytes) != hipSuccess) {
            set_error("device allocation of %zu bytes for a batch failed", dev_bytes);
            return DGS_E_NOMEM;
        }
        A.bytes = dev_bytes;
    }
    if (host_bytes > A.host_bytes) {
        if (A.host) (void)hipHostFree(A.host);
        A.host = nullptr;
        A.host_bytes = 0;
        if (hipHostMalloc((void **)&A.host, host_bytes, hipHostMallocDefault) != hipSuccess) {
            set_error("pinned allocation of %zu bytes for a batch failed", host_bytes);
            return DGS_E_NOMEM;
        }
        A.host_bytes = host_bytes;
    }
    if (!A.ev0) {
        if (hipEventCreate(&A.ev0) != hipSuccess || hipEventCreate(&A.ev1) != hipSuccess) {
            set_error("hipEventCreate failed");
            return DGS_E_DEVICE;
        }
    }
    return DGS_OK;
}

dgs_status run_batch(const BatchCall &c) {
    hipStream_t s = c.stream;
    std::vector<int32_t> small, large;
    for (int32_t b = 0; b < c.count; ++b) (c.ns[b] <= kBatchMaxN ? small : large).push_back(b);
    // largest first: the longest instances start first (LPT order)
    std::stable_sort(small.begin(), small.end(), [&](int32_t x, int32_t y) { return c.ns[x] > c.ns[y]; });
    const size_t m = small.size();
    if (m) {
        BatchArena &arena = c.arena ? *c.arena : g_batch;
        std::lock_guard<std::mutex> lk(arena.mu);
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        size_t mat = 0, vec = 0;
        for (int32_t b : small) {
            mat += al((size_t)c.ns[b] * c.ns[b] * 4);
            vec += al((size_t)c.ns[b] * 4);
        }
        size_t lists = 0, parts = 0;
        for (int32_t b : small) lists += al((size_t)c.ns[b] * 16);
        for (int32_t b : small) parts += al(batch_part_bytes(c.ns[b]));
        const size_t items_b = al(m * sizeof(BatchItem)), order_b = al(m * 4), res_b = al(m * 5 * 8);
        const size_t dev_bytes =
            (c.dev ? 0 : mat) + mat + lists + parts + (c.dev ? 0 : vec) + items_b + order_b + res_b + 256;
        const size_t host_bytes = items_b + order_b + res_b;
        dgs_status st = batch_reserve(arena, dev_bytes, host_bytes, !c.pool);
        if (st != DGS_OK) return st;
        char *block = arena.dev;
        if (c.pool && hipMallocFromPoolAsync((void **)&block, dev_bytes, c.pool, s) != hipSuccess) {
            set_error("device allocation of %zu bytes for a batch failed", dev_bytes);
            return DGS_E_NOMEM;
        }
        struct PoolBlock {
            char *p;
            hipStream_t s;
            bool pooled;
            ~PoolBlock() {
                if (pooled) (void)hipFreeAsync(p, s);
            }
        } pool_block{block, s, c.pool != nullptr};
        char *p = block;
        char *acopy = nullptr, *tauo = nullptr;
        if (!c.dev) {
            acopy = p;
            p += mat;
        }
        char *at = p;
        p += mat;
        char *lst = p;
        p += lists;
        char *prt = p;
        p += parts;
        if (!c.dev) {
            tauo = p;
            p += vec;
        }
        BatchItem *d_items = (BatchItem *)p;
        p += items_b;
        int32_t *d_order = (int32_t *)p;
        p += order_b;
        int64_t *d_res = (int64_t *)p;
        p += res_b;
        int32_t *d_queue = (int32_t *)p;
        BatchItem *h_items = (BatchItem *)arena.host;
        int32_t *h_order = (int32_t *)(arena.host + items_b);
        int64_t *h_res = (int64_t *)(arena.host + items_b + order_b);
        size_t om = 0, ov = 0, ol = 0, op = 0;
        BatchTotals tot;
        for (size_t x = 0; x < m; ++x) {
            const int32_t b = small[x];
            const int32_t n = c.ns[b];
            BatchItem &it = h_items[x];
            if (c.dev) {
                it.A = c.benefits[b];
                it.tau = c.outs[b];
            } else {
                DGS_HIP(hipMemcpyAsync(acopy + om, c.benefits[b], (size_t)n * n * 4, hipMemcpyHostToDevice, s));
                it.A = (const int32_t *)(acopy + om);
                it.tau = (int32_t *)(tauo + ov);
                ov += al((size_t)n * 4);
            }
            it.AT = (int32_t *)(at + om);
            it.lists = (u64 *)(lst + ol);
            it.res = d_res + 5 * x;
            it.n = n;
            it.part = (u64 *)(prt + op);
            op += al(batch_part_bytes(n));
            batch_place(it, tot);
            om += al((size_t)n * n * 4);
            ol += al((size_t)n * 16);
            h_order[x] = (int32_t)x;
        }
        DGS_HIP(hipMemcpyAsync(d_items, h_items, m * sizeof(BatchItem), hipMemcpyHostToDevice, s));
        DGS_HIP(hipMemcpyAsync(d_order, h_order, m * 4, hipMemcpyHostToDevice, s));
        DGS_HIP(launch_fill(d_queue, 3, 0, s));
        const int limit = batch_grid_limit(g_batch_block);
        if (limit < 1) {
            set_error("cannot size the batched solver's grid");
            return DGS_E_DEVICE;
        }
        int grid = (int)std::min<size_t>(m, (size_t)limit);
        if (c.grid_cap > 0) grid = std::min(grid, c.grid_cap);
        DGS_HIP(hipEventRecord(arena.ev0, s));
        DGS_HIP(launch_batch(d_items, d_order, (int)m, d_queue, c.max_switches, tot, g_batch_block, grid, s));
        DGS_HIP(hipEventRecord(arena.ev1, s));
        DGS_HIP(hipMemcpyAsync(h_res, d_res, m * 5 * 8, hipMemcpyDeviceToHost, s));
        DGS_HIP(hipStreamSynchronize(s));
        for (size_t x = 0; x < m; ++x) {
            if (h_res[5 * x + 4] != DGS_OK) {
                set_error("batch instance %d: benefit entry outside [-(2^29-1), 2^29-1]", small[x]);
                return (dgs_status)h_res[5 * x + 4];
            }
        }
        float ms = 0.f;
        DGS_HIP(hipEventElapsedTime(&ms, arena.ev0, arena.ev1));
        if (!c.dev) {
            size_t ov2 = 0;
            for (size_t x = 0; x < m; ++x) {
                const int32_t b = small[x];
                DGS_HIP(hipMemcpyAsync(c.outs[b], tauo + ov2, (size_t)c.ns[b] * 4, hipMemcpyDeviceToHost, s));
                ov2 += al((size_t)c.ns[b] * 4);
            }
            DGS_HIP(hipStreamSynchronize(s));
        }
        if (c.results) {
            for (size_t x = 0; x < m; ++x) {
                dgs_result &r = c.results[small[x]];
                std::memset(&r, 0, sizeof r);
                r.initial_benefit = h_res[5 * x];
                r.total_benefit = h_res[5 * x + 1];
                r.switches = h_res[5 * x + 2];
                r.rescans = h_res[5 * x + 3];
                r.device_ms = ms;  // the whole batched launch
            }
        }
    }
    for (int32_t b : large) {
        Call one;
        one.benefit = c.benefits[b];
        one.n = c.ns[b];
        one.assign_in = nullptr;
        one.max_switches = c.max_switches;
        one.dev = c.dev;
        one.profile = c.profile;
        one.pool = c.pool;
        one.stream = s;
        dgs_status st = run_instance(one, Mode::Solve, c.outs[b], nullptr, nullptr,
                                     c.results ? &c.results[b] : nullptr);
        if (st != DGS_OK) return st;
    }
    return DGS_OK;
}

dgs_status check_common(const int32_t *benefit, int32_t n, const void *out) {
    if (!benefit || !out) {
        set_error("NULL pointer argument");
        return DGS_E_INVAL;
    }
    if (n < 1 || n > DGS_MAX_N) {
        set_error("n=%d outside [1, %d]", n, DGS_MAX_N);
        return DGS_E_INVAL;
    }
    return DGS_OK;
}

}  // namespace

void batch_arena_clear(BatchArena &A) {
    if (A.dev) (void)hipFree(A.dev);
    if (A.host) (void)hipHostFree(A.host);
    if (A.ev0) (void)hipEventDestroy(A.ev0);
    if (A.ev1) (void)hipEventDestroy(A.ev1);
    A.dev = A.host = nullptr;
    A.bytes = A.host_bytes = 0;
    A.ev0 = A.ev1 = nullptr;
}

int switch_loop_grid(int n) {
    if (n < 2) return 0;
    return switch_v3_grid(std::min(n, kSwitchExMaxN));
}

int device_cus() {
    int cus = 0;
    if (ensure_context() != DGS_OK) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g_ctx.device) != hipSuccess) return 0;
    return cus;
}

dgs_status solve_internal(const int32_t *benefit, int32_t n, int32_t *assign_out, int64_t max_switches, bool dev,
                          bool coop, hipStream_t s, dgs_result *res, hipMemPool_t pool) {
    dgs_status st = check_common(benefit, n, assign_out);
    if (st != DGS_OK) return st;
    if ((st = ensure_context()) != DGS_OK) return st;
    Call c;
    c.benefit = benefit;
    c.n = n;
    c.assign_in = nullptr;
    c.max_switches = max_switches;
    c.dev = dev;
    c.profile = false;
    c.coop = coop;
    c.pool = pool;
    c.permuted = false;  // the server's requests keep their footprint at two matrices
    c.stream = s ? s : g_ctx.stream;
    return run_instance(c, Mode::Solve, assign_out, nullptr, nullptr, res);
}

dgs_status solve_batch_internal(int32_t count, const int32_t *const *benefits, const int32_t *ns,
                                int32_t *const *outs, dgs_result *results, int64_t max_switches, int grid_cap,
                                hipStream_t s, hipMemPool_t pool, BatchArena *arena) {
    dgs_status st = ensure_context();
    if (st != DGS_OK) return st;
    BatchCall c;
    c.count = count;
    c.benefits = benefits;
    c.ns = ns;
    c.outs = outs;
    c.results = results;
    c.max_switches = max_switches;
    c.dev = false;
    c.profile = false;
    c.grid_cap = grid_cap;
    c.pool = pool;
    c.arena = arena;
    c.stream = s ? s : g_ctx.stream;
    return run_batch(c);
}

// At process exit: give back everything the library still holds (cached
// workspaces, host resources, the batch arena) and its stream, while the HIP
// runtime is still up.  Batch plans and servers belong to the caller, who
// destroys them.
void noalloc_release_events();

void teardown_at_exit() {
    dgs_release_cached();
    noalloc_release_events();
    if (g_ctx.stream) {
        (void)hipStreamSynchronize(g_ctx.stream);
        (void)hipStreamDestroy(g_ctx.stream);
        g_ctx.stream = nullptr;
    }
    g_ctx.init_status = DGS_E_DEVICE;
    g_ctx.init_error = "the library has been shut down (process exit)";
}

// ---- solving without allocating ------------------------------------------------------
// dgs_solve_noalloc's device workspace is this fixed array: each GPU that
// loads the library's code object holds its own copy until the process ends.
// In host code the name `scratch` is only a host-side stand-in; the device
// address of a GPU's copy comes from hipGetSymbolAddress, looked up once per
// device with that device current, and only that address is ever handed to
// kernels or copies.
constexpr int32_t kNoAllocMaxN = DGS_NOALLOC_MAX_N;
constexpr size_t kNoAllocBytes = (size_t)DGS_NOALLOC_BYTES;
__device__ __align__(256) char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;

struct NoAllocDevice {
    std::once_flag once;
    dgs_status status = DGS_OK;
    std::string error;
    char *ptr = nullptr;   // device address of this GPU's `scratch`
    HostRes host;          // timing events made at set-up; stats -> stats_buf
    int64_t stats_buf[16] = {};
    std::mutex mu;         // calls on one GPU run one at a time
};

NoAllocDevice g_noalloc[kMaxDevices];

// Once per device, with that device current: the array's device address and
// the call's timing events.  Nothing is allocated after this.
dgs_status noalloc_setup(int device, NoAllocDevice **out) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device %d outside the %d devices dgs_solve_noalloc supports", device, kMaxDevices);
        return DGS_E_DEVICE;
    }
    NoAllocDevice &D = g_noalloc[device];
    std::call_once(D.once, [&D] {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            D.status = DGS_E_DEVICE;
            D.error = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
            return;
        }
        D.ptr = (char *)p;
        bool ok = hipEventCreate(&D.host.ev0) == hipSuccess && hipEventCreate(&D.host.ev1) == hipSuccess;
        for (auto &ev : D.host.ph) ok = ok && hipEventCreate(&ev) == hipSuccess;
        if (!ok) {
            D.status = DGS_E_DEVICE;
            D.error = "hipEventCreate failed";
            return;
        }
        D.host.stats = D.stats_buf;  // results are read back into this (pageable) block
    });
    if (D.status != DGS_OK) {
        set_error("%s", D.error.c_str());
        return D.status;
    }
    *out = &D;
    return DGS_OK;
}

}  // namespace

// At process exit (the arrays themselves go with the code object).
void noalloc_release_events() {
    for (NoAllocDevice &D : g_noalloc) {
        if (!D.ptr) continue;
        for (hipEvent_t *e : {&D.host.ev0, &D.host.ev1}) {
            if (*e) (void)hipEventDestroy(*e);
            *e = nullptr;
        }
        for (auto &e : D.host.ph) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
    }
}

}  // namespace dgs

using namespace dgs;

extern "C" {

const char *dgs_status_string(dgs_status st) {
    switch (st) {
        case DGS_OK: return "ok";
        case DGS_E_INVAL: return "invalid argument";
        case DGS_E_RANGE: return "benefit out of range";
        case DGS_E_NOMEM: return "out of device memory or budget";
        case DGS_E_DEVICE: return "device error";
        case DGS_E_AGAIN: return "not finished";
    }
    return "unknown status";
}

const char *dgs_last_error(void) { return g_last_error.c_str(); }

const char *dgs_version(void) { return "dgs-gfx950 0.1"; }

void dgs_release_cached(void) {
    std::multimap<int32_t, Workspace *> drop;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        drop.swap(g_ws_free);
    }
    for (auto &kv : drop) free_ws(kv.second);
    std::vector<HostRes *> hosts;
    {
        std::lock_guard<std::mutex> lk(g_host_mu);
        hosts.swap(g_host_free);
    }
    for (HostRes *h : hosts) destroy_host(h);
    std::lock_guard<std::mutex> lk(g_batch.mu);
    batch_arena_clear(g_batch);
}

dgs_status dgs_solve_ex(const int32_t *benefit, int32_t n, int32_t *assign_out, const dgs_options *opt,
                        dgs_result *res) {
    g_last_error.clear();
    dgs_status st = check_common(benefit, n, assign_out);
    if (st != DGS_OK) return st;
    if ((st = ensure_context()) != DGS_OK) return st;
    Call c;
    c.benefit = benefit;
    c.n = n;
    c.assign_in = opt ? opt->init_assign : nullptr;
    c.max_switches = opt ? opt->max_switches : -1;
    c.dev = opt && (opt->flags & DGS_DEVICE_PTRS);
    c.profile = opt && (opt->flags & DGS_PROFILE);
    c.parallel = opt && (opt->flags & DGS_PARALLEL);
    c.lazy = opt && (opt->flags & DGS_LAZY);
    c.global_greedy = opt && (opt->flags & DGS_GLOBAL_GREEDY);
    c.stream = (opt && opt->stream) ? (hipStream_t)opt->stream : g_ctx.stream;
    return run_instance(c, Mode::Solve, assign_out, nullptr, nullptr, res);
}

dgs_status dgs_solve_noalloc(const int32_t *benefit, int32_t n, int32_t *assign_out, const dgs_options *opt,
                             dgs_result *res) {
    g_last_error.clear();
    if (!benefit || !assign_out) {
        set_error("NULL pointer argument");
        return DGS_E_INVAL;
    }
    if (n < 1 || n > kNoAllocMaxN) {
        set_error("n=%d outside [1, %d] (the fixed workspace of dgs_solve_noalloc)", n, kNoAllocMaxN);
        return DGS_E_INVAL;
    }
    if (opt && (opt->flags & (DGS_PARALLEL | DGS_LAZY | DGS_GLOBAL_GREEDY))) {
        set_error("dgs_solve_noalloc runs the steepest-ascent mode from the agent-order greedy start only");
        return DGS_E_INVAL;
    }
    dgs_status st = ensure_context();
    if (st != DGS_OK) return st;
    int device = 0;
    DGS_HIP(hipGetDevice(&device));
    NoAllocDevice *D = nullptr;
    if ((st = noalloc_setup(device, &D)) != DGS_OK) return st;
    std::lock_guard<std::mutex> lk(D->mu);
    hipStream_t s = (opt && opt->stream) ? (hipStream_t)opt->stream
                                         : (device == g_ctx.device ? g_ctx.stream : (hipStream_t)0);
    const int32_t *init = opt ? opt->init_assign : nullptr;
    if (init) {  // checked on the host without heap memory (n <= kNoAllocMaxN)
        int32_t h[kNoAllocMaxN];
        uint32_t seen[(kNoAllocMaxN + 31) / 32] = {};
        DGS_HIP(hipMemcpyAsync(h, init, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        DGS_HIP(hipStreamSynchronize(s));
        for (int32_t i = 0; i < n; ++i) {
            const int32_t j = h[i];
            if (j < 0 || j >= n || ((seen[j >> 5] >> (j & 31)) & 1u)) {
                set_error("init_assign is not a permutation of 0..n-1");
                return DGS_E_INVAL;
            }
            seen[j >> 5] |= 1u << (j & 31);
        }
    }
    // the transpose first, then the vectors, all inside this GPU's array
    const size_t mat = ((size_t)n * (size_t)n * 4 + 255) & ~(size_t)255;
    Workspace w;
    w.cap = n;
    w.mat_bytes = mat;
    w.at = (int32_t *)D->ptr;
    w.vec = D->ptr + mat;
    w.vec_bytes = kNoAllocBytes - mat;
    Call c;
    c.benefit = benefit;
    c.n = n;
    c.assign_in = init;
    c.max_switches = opt ? opt->max_switches : -1;
    c.dev = true;
    c.profile = opt && (opt->flags & DGS_PROFILE);
    c.ws = &w;
    c.host = &D->host;
    c.stream = s;
    return run_instance(c, Mode::Solve, assign_out, nullptr, nullptr, res);
}

dgs_status dgs_solve(const int32_t *benefit, int32_t n, int32_t *assign_out) {
    return dgs_solve_ex(benefit, n, assign_out, nullptr, nullptr);
}

dgs_status dgs_solve_rect(const int32_t *benefit, int32_t n, int32_t m, int32_t *assign_out,
                          const dgs_options *opt, dgs_result *res) {
    g_last_error.clear();
    dgs_status st = check_common(benefit, m, assign_out);
    if (st != DGS_OK) return st;
    if (n < 1 || n > m) {
        set_error("rectangular instance needs 1 <= n <= m (n=%d, m=%d)", n, m);
        return DGS_E_INVAL;
    }
    if (opt && (opt->flags & (DGS_PARALLEL | DGS_LAZY))) {
        set_error("rectangular instances use the steepest-ascent mode only");
        return DGS_E_INVAL;
    }
    if ((st = ensure_context()) != DGS_OK) return st;
    const bool dev = opt && (opt->flags & DGS_DEVICE_PTRS);
    hipStream_t s = (opt && opt->stream) ? (hipStream_t)opt->stream : g_ctx.stream;
    // a caller's start: its n jobs, then the unused jobs in increasing order
    // for the virtual agents n..m-1 (host memory)
    std::vector<int32_t> init;
    if (opt && opt->init_assign) {
        init.resize((size_t)n);
        if (dev) {
            DGS_HIP(hipMemcpyAsync(init.data(), opt->init_assign, (size_t)n * 4, hipMemcpyDeviceToHost, s));
            DGS_HIP(hipStreamSynchronize(s));
        } else {
            std::copy(opt->init_assign, opt->init_assign + n, init.begin());
        }
        std::vector<char> used((size_t)m, 0);
        for (int32_t i = 0; i < n; ++i) {
            if (init[i] < 0 || init[i] >= m || used[(size_t)init[i]]) {
                set_error("init_assign is not n distinct jobs of 0..m-1");
                return DGS_E_INVAL;
            }
            used[(size_t)init[i]] = 1;
        }
        for (int32_t j = 0; j < m; ++j)
            if (!used[(size_t)j]) init.push_back(j);
    }
    Call c;
    c.benefit = benefit;
    c.n = m;
    c.nr = n;
    c.assign_in = init.empty() ? nullptr : init.data();
    c.init_host = true;
    c.global_greedy = opt && (opt->flags & DGS_GLOBAL_GREEDY);
    c.max_switches = opt ? opt->max_switches : -1;
    c.dev = dev;
    c.profile = opt && (opt->flags & DGS_PROFILE);
    c.stream = s;
    return run_instance(c, Mode::Solve, assign_out, nullptr, nullptr, res);
}

dgs_status dgs_diff_eval(const int32_t *benefit, int32_t n, const int32_t *assign, int64_t *gain_out,
                         int32_t *job_out, const dgs_options *opt, dgs_result *res) {
    g_last_error.clear();
    dgs_status st = check_common(benefit, n, gain_out);
    if (st != DGS_OK) return st;
    if (!assign || !job_out) {
        set_error("NULL pointer argument");
        return DGS_E_INVAL;
    }
    if ((st = ensure_context()) != DGS_OK) return st;
    Call c;
    c.benefit = benefit;
    c.n = n;
    c.assign_in = assign;
    c.max_switches = 0;
    c.dev = opt && (opt->flags & DGS_DEVICE_PTRS);
    c.profile = opt && (opt->flags & DGS_PROFILE);
    c.stream = (opt && opt->stream) ? (hipStream_t)opt->stream : g_ctx.stream;
    if (c.dev) return run_instance(c, Mode::DiffEval, nullptr, gain_out, job_out, res);
    // host outputs: evaluate into device buffers, then copy
    int64_t *dg = nullptr;
    int32_t *dj = nullptr;
    if (hipMalloc((void **)&dg, (size_t)n * 8) != hipSuccess || hipMalloc((void **)&dj, (size_t)n * 4) != hipSuccess) {
        if (dg) (void)hipFree(dg);
        set_error("device allocation failed");
        return DGS_E_NOMEM;
    }
    st = run_instance(c, Mode::DiffEval, nullptr, dg, dj, res);
    if (st == DGS_OK) {
        if (hipMemcpy(gain_out, dg, (size_t)n * 8, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(job_out, dj, (size_t)n * 4, hipMemcpyDeviceToHost) != hipSuccess) {
            set_error("copy of evaluation results failed");
            st = DGS_E_DEVICE;
        }
    }
    (void)hipFree(dg);
    (void)hipFree(dj);
    return st;
}

dgs_status dgs_solve_batched(int32_t count, const int32_t *const *benefits, const int32_t *ns,
                             int32_t *const *assign_outs, dgs_result *results, const dgs_options *opt) {
    g_last_error.clear();
    if (count < 0 || (count > 0 && (!benefits || !ns || !assign_outs))) {
        set_error("bad batch arguments");
        return DGS_E_INVAL;
    }
    if (opt && opt->init_assign) {
        set_error("init_assign is not supported for batches");
        return DGS_E_INVAL;
    }
    if (opt && (opt->flags & (DGS_PARALLEL | DGS_LAZY | DGS_GLOBAL_GREEDY))) {
        set_error("batches run the steepest-ascent mode from the agent-order greedy start only");
        return DGS_E_INVAL;
    }
    for (int32_t b = 0; b < count; ++b) {
        dgs_status st = check_common(benefits[b], ns[b], assign_outs[b]);
        if (st != DGS_OK) return st;
    }
    if (count == 0) return DGS_OK;
    dgs_status st = ensure_context();
    if (st != DGS_OK) return st;
    BatchCall c;
    c.count = count;
    c.benefits = benefits;
    c.ns = ns;
    c.outs = assign_outs;
    c.results = results;
    c.max_switches = opt ? opt->max_switches : -1;
    c.dev = opt && (opt->flags & DGS_DEVICE_PTRS);
    c.profile = opt && (opt->flags & DGS_PROFILE);
    c.stream = (opt && opt->stream) ? (hipStream_t)opt->stream : g_ctx.stream;
    return run_batch(c);
}

}  // extern "C"
