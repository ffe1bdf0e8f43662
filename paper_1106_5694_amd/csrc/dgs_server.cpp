// dgs_server_*: a request loop for periodic LSAP instances with continuous
// batching (include/dgs.h).
//
// Requests wait in arrival order.  Two kinds of workers take them:
//   * the small-request worker: every time it is free it takes *all* waiting
//     requests with n <= kBatchMaxN that fit the device-memory budget and
//     solves them in one batched launch (one workgroup per instance), so
//     requests that arrive while a batch runs join the next one;
//   * large-request workers (one stream each): a waiting large request starts
//     as soon as its device footprint fits the memory budget and its
//     switching loop fits the compute units left over by the requests
//     already running, and its kernels overlap theirs on the device.
// The switching loops run as plain launches: the server admits them only
// while the workgroups of all running loops fit the device together, which
// is what a cooperative launch would otherwise guarantee for a single one.
// Every result is identical to dgs_solve on the same input.
//
// Device memory: every buffer of a request comes from a memory pool the
// server owns (stream-ordered allocations on the worker's stream) and goes
// back to it when the request completes; the pool keeps at most the budget
// once its streams synchronize.  Admission keeps the footprints of the
// requests on the device within the budget, so the memory the server holds
// stays within the budget too (the library's own caches are not used).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dgs.h"
#include "dgs_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket;
    const int32_t *benefit;
    int32_t n;
    uint64_t bytes;
    Clock::time_point submitted;
};

struct Done {
    std::vector<int32_t> tau;
    dgs_result res;
    dgs_status st;
    Clock::time_point finished;
};

constexpr int kLargeWorkers = 4;

// Workgroups the switching loop of an n-agent request keeps resident.
int loop_wgs(int32_t n) {
    if (n <= dgs::kBatchMaxN) return 0;
    return dgs::switch_loop_grid(n);
}

}  // namespace

struct dgs_server {
    dgs_server_config cfg;
    int cus = 0;
    std::mutex mu;
    std::condition_variable cv_work;  // workers wait for requests / capacity
    std::condition_variable cv_done;  // waiters wait for results
    std::deque<Request> queue;
    std::unordered_map<uint64_t, Done> done;
    std::unordered_map<uint64_t, int32_t> pending_n;
    uint64_t next_ticket = 1;
    uint64_t bytes_in_use = 0;
    int32_t resident = 0;
    int wgs_in_use = 0;       // resident switching-loop workgroups of large requests
    bool small_running = false;
    bool stopping = false;
    std::vector<std::thread> workers;
    std::vector<double> lat_us;
    int64_t submitted = 0, completed = 0;
    hipMemPool_t pool = nullptr;  // every device buffer of the server's requests
    dgs::BatchArena arena;        // host staging and events of the small-request worker
    Clock::time_point first_submit, last_finish;
    bool any_submit = false;
};

namespace {

void finish(dgs_server *s, const Request &r, Done &&d) {
    s->lat_us.push_back(std::chrono::duration<double, std::micro>(d.finished - r.submitted).count());
    s->completed += 1;
    s->last_finish = d.finished;
    s->pending_n.erase(r.ticket);
    s->done.emplace(r.ticket, std::move(d));
}

void small_worker(dgs_server *s) {
    hipStream_t stream = nullptr;
    (void)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    for (;;) {
        std::vector<Request> batch;
        int grid_cap = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            auto has_small = [&] {
                for (const Request &r : s->queue)
                    if (r.n <= dgs::kBatchMaxN) return true;
                return false;
            };
            s->cv_work.wait(lk, [&] { return has_small() || (s->stopping && s->queue.empty()); });
            if (!has_small()) break;
            // every waiting small request that fits the budget and the slots joins
            for (auto it = s->queue.begin(); it != s->queue.end();) {
                if (it->n <= dgs::kBatchMaxN && s->resident < s->cfg.max_slots &&
                    s->bytes_in_use + it->bytes <= s->cfg.hbm_budget_bytes) {
                    s->bytes_in_use += it->bytes;
                    s->resident += 1;
                    batch.push_back(*it);
                    it = s->queue.erase(it);
                } else {
                    ++it;
                }
            }
            if (batch.empty()) {
                // capacity is held by running requests: wait for a completion
                s->cv_work.wait(lk);
                continue;
            }
            s->small_running = true;
            grid_cap = std::max(1, s->cus - s->wgs_in_use);
        }
        std::vector<const int32_t *> bens;
        std::vector<int32_t> ns;
        std::vector<Done> outs(batch.size());
        std::vector<int32_t *> optr;
        std::vector<dgs_result> res(batch.size());
        for (size_t i = 0; i < batch.size(); ++i) {
            bens.push_back(batch[i].benefit);
            ns.push_back(batch[i].n);
            outs[i].tau.resize((size_t)batch[i].n);
            optr.push_back(outs[i].tau.data());
        }
        const dgs_status st = dgs::solve_batch_internal((int32_t)batch.size(), bens.data(), ns.data(),
                                                        optr.data(), res.data(), -1, grid_cap, stream, s->pool,
                                                        &s->arena);
        const auto now = Clock::now();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (size_t i = 0; i < batch.size(); ++i) {
                outs[i].res = res[i];
                outs[i].st = st;
                outs[i].finished = now;
                s->bytes_in_use -= batch[i].bytes;
                s->resident -= 1;
                finish(s, batch[i], std::move(outs[i]));
            }
            s->small_running = false;
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
    if (stream) (void)hipStreamDestroy(stream);
}

void large_worker(dgs_server *s) {
    hipStream_t stream = nullptr;
    (void)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    for (;;) {
        Request r;
        int wgs = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            auto pick = [&]() -> std::deque<Request>::iterator {
                // the oldest large request that fits memory, slots and compute units
                for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
                    if (it->n <= dgs::kBatchMaxN) continue;
                    const int need = loop_wgs(it->n);
                    if (s->resident < s->cfg.max_slots && s->bytes_in_use + it->bytes <= s->cfg.hbm_budget_bytes &&
                        s->wgs_in_use + need <= s->cus)
                        return it;
                    return s->queue.end();  // keep arrival order among large requests
                }
                return s->queue.end();
            };
            auto has_large = [&] {
                for (const Request &q : s->queue)
                    if (q.n > dgs::kBatchMaxN) return true;
                return false;
            };
            s->cv_work.wait(lk, [&] { return pick() != s->queue.end() || (s->stopping && !has_large()); });
            auto it = pick();
            if (it == s->queue.end()) break;
            r = *it;
            s->queue.erase(it);
            wgs = loop_wgs(r.n);
            s->bytes_in_use += r.bytes;
            s->resident += 1;
            s->wgs_in_use += wgs;
        }
        Done d;
        d.tau.resize((size_t)r.n);
        std::memset(&d.res, 0, sizeof d.res);
        d.st = dgs::solve_internal(r.benefit, r.n, d.tau.data(), -1, false, /*coop=*/false, stream, &d.res,
                                   s->pool);
        d.finished = Clock::now();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->bytes_in_use -= r.bytes;
            s->resident -= 1;
            s->wgs_in_use -= wgs;
            finish(s, r, std::move(d));
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
    if (stream) (void)hipStreamDestroy(stream);
}

double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    double pos = p * (double)(v.size() - 1);
    size_t lo = (size_t)pos;
    size_t hi = std::min(lo + 1, v.size() - 1);
    double f = pos - (double)lo;
    return v[lo] * (1.0 - f) + v[hi] * f;
}

}  // namespace

extern "C" {

uint64_t dgs_server_footprint(int32_t n) {
    const uint64_t nn = (uint64_t)n * (uint64_t)n;
    if (n <= dgs::kBatchMaxN) return 2 * 4 * nn + 32 * (uint64_t)n + 4096;  // copy + transpose
    // device copy + transpose (no permuted copy W: the switching loop reads A), evaluation partials,
    // vectors and lists
    return 2 * 4 * nn + 2 * 16 * (uint64_t)n * (((uint64_t)n + 63) / 64) + 256 * (uint64_t)n + (1u << 20);
}

dgs_status dgs_server_create(const dgs_server_config *cfg, dgs_server **out) {
    if (!out) return DGS_E_INVAL;
    const int cus = dgs::device_cus();
    if (cus < 1) return DGS_E_DEVICE;
    dgs_server *s = new dgs_server();
    s->cus = cus;
    s->cfg.hbm_budget_bytes = (cfg && cfg->hbm_budget_bytes) ? cfg->hbm_budget_bytes : (64ull << 30);
    int device = 0;
    bool ok = hipGetDevice(&device) == hipSuccess;
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    uint64_t keep = s->cfg.hbm_budget_bytes;  // freed blocks kept for reuse up to the budget
    ok = ok && hipMemPoolCreate(&s->pool, &props) == hipSuccess;
    ok = ok && hipMemPoolSetAttribute(s->pool, hipMemPoolAttrReleaseThreshold, &keep) == hipSuccess;
    if (!ok) {
        if (s->pool) (void)hipMemPoolDestroy(s->pool);
        delete s;
        return DGS_E_DEVICE;
    }
    s->cfg.max_slots = (cfg && cfg->max_slots > 0) ? cfg->max_slots : 64;
    s->cfg.max_n = (cfg && cfg->max_n > 0) ? cfg->max_n : 16384;
    if (s->cfg.max_n > dgs::kSwitchExMaxN) s->cfg.max_n = dgs::kSwitchExMaxN;
    s->workers.emplace_back(small_worker, s);
    for (int i = 0; i < kLargeWorkers; ++i) s->workers.emplace_back(large_worker, s);
    *out = s;
    return DGS_OK;
}

dgs_status dgs_server_submit(dgs_server *s, const int32_t *benefit, int32_t n, uint64_t *ticket_out) {
    if (!s || !benefit || !ticket_out) return DGS_E_INVAL;
    if (n < 1 || n > s->cfg.max_n) return DGS_E_INVAL;
    const uint64_t bytes = dgs_server_footprint(n);
    if (bytes > s->cfg.hbm_budget_bytes) return DGS_E_NOMEM;
    if (loop_wgs(n) > s->cus) return DGS_E_NOMEM;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return DGS_E_INVAL;
        Request r;
        r.ticket = s->next_ticket++;
        r.benefit = benefit;
        r.n = n;
        r.bytes = bytes;
        r.submitted = Clock::now();
        if (!s->any_submit) {
            s->any_submit = true;
            s->first_submit = r.submitted;
        }
        s->submitted += 1;
        s->pending_n.emplace(r.ticket, n);
        s->queue.push_back(r);
        *ticket_out = r.ticket;
    }
    s->cv_work.notify_all();
    return DGS_OK;
}

static dgs_status take_done(dgs_server *s, uint64_t ticket, int32_t *assign_out, dgs_result *res) {
    auto it = s->done.find(ticket);
    if (it == s->done.end()) return s->pending_n.count(ticket) ? DGS_E_AGAIN : DGS_E_INVAL;
    dgs_status st = it->second.st;
    if (st == DGS_OK) {
        if (assign_out) std::memcpy(assign_out, it->second.tau.data(), it->second.tau.size() * sizeof(int32_t));
        if (res) *res = it->second.res;
    }
    s->done.erase(it);
    return st;
}

dgs_status dgs_server_poll(dgs_server *s, uint64_t ticket, int32_t *assign_out, dgs_result *res) {
    if (!s) return DGS_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    return take_done(s, ticket, assign_out, res);
}

dgs_status dgs_server_wait(dgs_server *s, uint64_t ticket, int32_t *assign_out, dgs_result *res,
                           int64_t timeout_us) {
    if (!s) return DGS_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] { return s->done.count(ticket) || !s->pending_n.count(ticket); };
    if (timeout_us < 0) {
        s->cv_done.wait(lk, ready);
    } else {
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    }
    return take_done(s, ticket, assign_out, res);
}

dgs_status dgs_server_stats_get(dgs_server *s, dgs_server_stats *out) {
    if (!s || !out) return DGS_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->queued = (int64_t)s->queue.size();
    out->resident = s->resident;
    double span = s->completed ? std::chrono::duration<double>(s->last_finish - s->first_submit).count() : 0.0;
    out->inst_per_s = span > 0 ? (double)s->completed / span : 0.0;
    out->p50_us = percentile(s->lat_us, 0.50);
    out->p99_us = percentile(s->lat_us, 0.99);
    return DGS_OK;
}

void dgs_server_destroy(dgs_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();  // each worker synchronized and destroyed its stream
    dgs::batch_arena_clear(s->arena);
    (void)hipMemPoolDestroy(s->pool);
    delete s;
}

}  // extern "C"
