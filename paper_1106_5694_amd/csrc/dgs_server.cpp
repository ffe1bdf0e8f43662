// dgs_server_*: a request loop for periodic LSAP instances (include/dgs.h).
//
// Requests are admitted against a device-memory budget and a slot count,
// solved on the device by worker threads (each with its own stream, so the
// copy of one request overlaps the solve of another), and handed back
// through tickets.  Results are identical to dgs_solve_ex on the same input.
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

}  // namespace

struct dgs_server {
    dgs_server_config cfg;
    std::mutex mu;
    std::condition_variable cv_work;  // workers wait for requests / memory
    std::condition_variable cv_done;  // waiters wait for results
    std::deque<Request> queue;
    std::unordered_map<uint64_t, Done> done;
    std::unordered_map<uint64_t, int32_t> pending_n;
    uint64_t next_ticket = 1;
    uint64_t bytes_in_use = 0;
    int32_t resident = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
    std::vector<double> lat_us;
    int64_t submitted = 0, completed = 0;
    Clock::time_point first_submit, last_finish;
    bool any_submit = false;
};

namespace {

void worker_main(dgs_server *s) {
    hipStream_t stream = nullptr;
    (void)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    for (;;) {
        Request r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            // FIFO admission: the head waits until its footprint fits.
            s->cv_work.wait(lk, [&] {
                if (s->queue.empty()) return s->stopping;
                const Request &h = s->queue.front();
                return s->resident < s->cfg.max_slots && s->bytes_in_use + h.bytes <= s->cfg.hbm_budget_bytes;
            });
            if (s->queue.empty() && s->stopping) break;
            r = s->queue.front();
            s->queue.pop_front();
            s->bytes_in_use += r.bytes;
            s->resident += 1;
        }
        Done d;
        d.tau.resize((size_t)r.n);
        dgs_options opt;
        opt.max_switches = -1;
        opt.init_assign = nullptr;
        opt.flags = 0;
        opt.stream = stream;
        std::memset(&d.res, 0, sizeof d.res);
        d.st = dgs_solve_ex(r.benefit, r.n, d.tau.data(), &opt, &d.res);
        d.finished = Clock::now();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->bytes_in_use -= r.bytes;
            s->resident -= 1;
            s->lat_us.push_back(std::chrono::duration<double, std::micro>(d.finished - r.submitted).count());
            s->completed += 1;
            s->last_finish = d.finished;
            s->pending_n.erase(r.ticket);
            s->done.emplace(r.ticket, std::move(d));
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
    return 3 * 4 * nn + 48 * (uint64_t)n + (1u << 20);
}

dgs_status dgs_server_create(const dgs_server_config *cfg, dgs_server **out) {
    if (!out) return DGS_E_INVAL;
    dgs_server *s = new dgs_server();
    s->cfg.hbm_budget_bytes = (cfg && cfg->hbm_budget_bytes) ? cfg->hbm_budget_bytes : (64ull << 30);
    s->cfg.max_slots = (cfg && cfg->max_slots > 0) ? cfg->max_slots : 64;
    s->cfg.max_n = (cfg && cfg->max_n > 0) ? cfg->max_n : 16384;
    const int nworkers = std::max(1, std::min(4, (int)s->cfg.max_slots));
    for (int i = 0; i < nworkers; ++i) s->workers.emplace_back(worker_main, s);
    *out = s;
    return DGS_OK;
}

dgs_status dgs_server_submit(dgs_server *s, const int32_t *benefit, int32_t n, uint64_t *ticket_out) {
    if (!s || !benefit || !ticket_out) return DGS_E_INVAL;
    if (n < 1 || n > s->cfg.max_n) return DGS_E_INVAL;
    const uint64_t bytes = dgs_server_footprint(n);
    if (bytes > s->cfg.hbm_budget_bytes) return DGS_E_NOMEM;
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
    s->cv_work.notify_one();
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
    for (auto &t : s->workers) t.join();
    delete s;
}

}  // extern "C"
