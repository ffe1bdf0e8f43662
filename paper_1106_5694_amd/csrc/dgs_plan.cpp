// dgs_batch_plan_*: a fixed batch shape solved repeatedly (include/dgs.h).
//
// The plan owns every device buffer of its instances, so the launch of the
// batched solver has fixed arguments; its device work (queue reset, the
// persistent launch, the readback of the per-instance results) is captured
// once in a HIP graph and replayed by every later run.  The queue reset is
// a fill kernel, not a memset node.
//
// Tuning: the batched solver comes in two workgroup sizes (256 or 512
// threads, i.e. 8 or 4 agents per thread); both give the same results.
// With DGS_AUTOTUNE the first run times both on the plan's inputs and keeps
// the faster.  Choices are kept per size class (count, largest n rounded up
// to a power of two, log2 of the total number of entries) for the process,
// and in the DGS_TUNE_CACHE text file ("<class> <block>" per line), read
// again whenever the variable names another file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dgs.h"
#include "dgs_internal.h"

namespace dgs {
namespace {

constexpr int kPlanBlocks[2] = {256, 512};

std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
std::string g_tune_file;  // the DGS_TUNE_CACHE file read last

std::string size_class(const std::vector<int32_t> &ns) {
    int64_t entries = 0;
    int largest = 0;
    for (int32_t n : ns) {
        entries += (int64_t)n * n;
        largest = std::max(largest, (int)n);
    }
    int p2 = 1;
    while (p2 < largest) p2 <<= 1;
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= entries) ++lg;
    char buf[64];
    snprintf(buf, sizeof buf, "c%zu_n%d_e%d", ns.size(), p2, lg);
    return buf;
}

// Reads the DGS_TUNE_CACHE file when the variable names a file not read yet;
// its entries override the choices held so far.
void tune_load_locked() {
    const char *path = getenv("DGS_TUNE_CACHE");
    if (!path || !*path || g_tune_file == path) return;
    g_tune_file = path;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char key[128];
    int block = 0;
    while (fscanf(f, "%127s %d", key, &block) == 2)
        if (block == kPlanBlocks[0] || block == kPlanBlocks[1]) g_tune[key] = block;
    fclose(f);
}

void tune_store_locked(const std::string &key, int block) {
    g_tune[key] = block;
    const char *path = getenv("DGS_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d\n", key.c_str(), block);
    fclose(f);
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace dgs

struct dgs_batch_plan {
    int32_t count = 0;
    std::vector<int32_t> ns;
    std::vector<int32_t> slot_of;  // instance -> launch slot (largest first)
    std::vector<int32_t> inst_of;  // launch slot -> instance
    int64_t max_switches = -1;
    bool autotune = false;
    bool tuned = false;
    std::string key;
    int block = 256;
    int grid = 1;
    hipStream_t stream = nullptr;
    char *dev = nullptr;
    std::vector<int32_t *> A, tau;  // per instance
    dgs::BatchItem *d_items = nullptr;
    dgs::BatchTotals tot;  // tiles, pairs and agents of all instances
    int32_t *d_order = nullptr;
    int64_t *d_res = nullptr;  // 5 per launch slot
    int32_t *d_queue = nullptr;
    int64_t *h_res = nullptr;  // pinned copy of d_res
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

using dgs::set_error;

int grid_for(const dgs_batch_plan *p, int block) {
    const int limit = dgs::batch_grid_limit(block);
    return limit < 1 ? 0 : std::min(p->count, limit);
}

void drop_graph(dgs_batch_plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

void free_plan(dgs_batch_plan *p) {
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    drop_graph(p);
    if (p->dev) (void)hipFree(p->dev);
    if (p->h_res) (void)hipHostFree(p->h_res);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    if (p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

dgs_status check_results(const dgs_batch_plan *p) {
    for (int32_t x = 0; x < p->count; ++x) {
        const int64_t st = p->h_res[5 * x + 4];
        if (st == DGS_E_RANGE) {
            set_error("batch instance %d: benefit entry outside [-(2^29-1), 2^29-1]", p->inst_of[x]);
            return DGS_E_RANGE;
        }
        if (st != DGS_OK) {
            set_error("batch instance %d: solver status %lld", p->inst_of[x], (long long)st);
            return DGS_E_DEVICE;
        }
    }
    return DGS_OK;
}

// One run outside a graph with the given workgroup size; *ms = kernel time.
dgs_status run_eager(dgs_batch_plan *p, int block, float *ms) {
    const int grid = grid_for(p, block);
    if (grid < 1) {
        set_error("cannot size the batched solver's grid");
        return DGS_E_DEVICE;
    }
    hipStream_t s = p->stream;
    DGS_HIP(dgs::launch_fill(p->d_queue, 3, 0, s));
    DGS_HIP(hipEventRecord(p->ev0, s));
    DGS_HIP(dgs::launch_batch(p->d_items, p->d_order, p->count, p->d_queue, p->max_switches, p->tot, block, grid, s));
    DGS_HIP(hipEventRecord(p->ev1, s));
    DGS_HIP(hipMemcpyAsync(p->h_res, p->d_res, (size_t)p->count * 5 * 8, hipMemcpyDeviceToHost, s));
    DGS_HIP(hipStreamSynchronize(s));
    DGS_HIP(hipEventElapsedTime(ms, p->ev0, p->ev1));
    return check_results(p);
}

dgs_status capture(dgs_batch_plan *p) {
    hipStream_t s = p->stream;
    DGS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = dgs::launch_fill(p->d_queue, 3, 0, s);
    if (e == hipSuccess)
        e = dgs::launch_batch(p->d_items, p->d_order, p->count, p->d_queue, p->max_switches, p->tot, p->block,
                              p->grid, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_res, p->d_res, (size_t)p->count * 5 * 8, hipMemcpyDeviceToHost, s);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        set_error("graph capture of the batched solver failed: %s",
                  hipGetErrorString(e != hipSuccess ? e : e2));
        return DGS_E_DEVICE;
    }
    p->graph = g;
    DGS_HIP(hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0));
    return DGS_OK;
}

dgs_status tune(dgs_batch_plan *p) {
    float best_ms = 0.f;
    int best = p->block;
    for (int b = 0; b < 2; ++b) {
        float ms = 0.f;
        dgs_status st = run_eager(p, dgs::kPlanBlocks[b], &ms);
        if (st != DGS_OK) return st;
        if (b == 0 || ms < best_ms) {
            best_ms = ms;
            best = dgs::kPlanBlocks[b];
        }
    }
    {
        std::lock_guard<std::mutex> lk(dgs::g_tune_mu);
        dgs::tune_store_locked(p->key, best);
    }
    if (best != p->block) drop_graph(p);
    p->block = best;
    p->grid = grid_for(p, best);
    p->tuned = true;
    return DGS_OK;
}

}  // namespace

extern "C" {

dgs_status dgs_batch_plan_create(int32_t count, const int32_t *ns, const dgs_options *opt, dgs_batch_plan **out) {
    if (!out || !ns || count < 1) {
        set_error("dgs_batch_plan_create: NULL argument or count < 1");
        return DGS_E_INVAL;
    }
    for (int32_t b = 0; b < count; ++b) {
        if (ns[b] < 1 || ns[b] > dgs::kBatchMaxN) {
            set_error("batch plan instance %d: n=%d outside [1, %d]", b, ns[b], dgs::kBatchMaxN);
            return DGS_E_INVAL;
        }
    }
    dgs_status st = dgs::ensure_context();
    if (st != DGS_OK) return st;
    dgs_batch_plan *p = new dgs_batch_plan();
    p->count = count;
    p->ns.assign(ns, ns + count);
    p->max_switches = opt ? opt->max_switches : -1;
    p->autotune = opt && (opt->flags & DGS_AUTOTUNE);
    p->key = dgs::size_class(p->ns);
    {
        std::lock_guard<std::mutex> lk(dgs::g_tune_mu);
        dgs::tune_load_locked();
        auto it = dgs::g_tune.find(p->key);
        if (it != dgs::g_tune.end()) {
            p->block = it->second;
            p->tuned = true;
        }
    }
    p->grid = grid_for(p, p->block);
    auto fail = [&](dgs_status code, const char *what) {
        set_error("dgs_batch_plan_create: %s", what);
        free_plan(p);
        return code;
    };
    if (p->grid < 1) return fail(DGS_E_DEVICE, "cannot size the batched solver's grid");

    // launch order: largest first (LPT), ties in instance order
    p->inst_of.resize((size_t)count);
    for (int32_t b = 0; b < count; ++b) p->inst_of[b] = b;
    std::stable_sort(p->inst_of.begin(), p->inst_of.end(),
                     [&](int32_t x, int32_t y) { return p->ns[x] > p->ns[y]; });
    p->slot_of.resize((size_t)count);
    for (int32_t x = 0; x < count; ++x) p->slot_of[p->inst_of[x]] = x;

    size_t mat = 0, lists = 0, vec = 0, parts = 0;
    for (int32_t n : p->ns) {
        mat += dgs::al256((size_t)n * n * 4);
        lists += dgs::al256((size_t)n * 16);
        vec += dgs::al256((size_t)n * 4);
        parts += dgs::al256(dgs::batch_part_bytes(n));
    }
    const size_t items_b = dgs::al256((size_t)count * sizeof(dgs::BatchItem));
    const size_t order_b = dgs::al256((size_t)count * 4);
    const size_t res_b = dgs::al256((size_t)count * 5 * 8);
    const size_t total = 2 * mat + lists + parts + vec + items_b + order_b + res_b + 256;
    if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess)
        return fail(DGS_E_DEVICE, "hipStreamCreate failed");
    if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess)
        return fail(DGS_E_DEVICE, "hipEventCreate failed");
    if (hipMalloc((void **)&p->dev, total) != hipSuccess) return fail(DGS_E_NOMEM, "device allocation failed");
    if (hipHostMalloc((void **)&p->h_res, (size_t)count * 5 * 8, hipHostMallocDefault) != hipSuccess)
        return fail(DGS_E_NOMEM, "pinned allocation failed");

    char *q = p->dev;
    char *a_base = q;
    q += mat;
    char *at_base = q;
    q += mat;
    char *l_base = q;
    q += lists;
    char *p_base = q;
    q += parts;
    char *t_base = q;
    q += vec;
    p->d_items = (dgs::BatchItem *)q;
    q += items_b;
    p->d_order = (int32_t *)q;
    q += order_b;
    p->d_res = (int64_t *)q;
    q += res_b;
    p->d_queue = (int32_t *)q;

    p->A.assign((size_t)count, nullptr);
    p->tau.assign((size_t)count, nullptr);
    std::vector<dgs::BatchItem> items((size_t)count);
    std::vector<int32_t> order((size_t)count);
    size_t om = 0, ol = 0, ov = 0, op = 0;
    for (int32_t x = 0; x < count; ++x) {
        const int32_t b = p->inst_of[x];
        const int32_t n = p->ns[b];
        p->A[b] = (int32_t *)(a_base + om);
        p->tau[b] = (int32_t *)(t_base + ov);
        dgs::BatchItem &it = items[x];
        it.A = p->A[b];
        it.tau = p->tau[b];
        it.AT = (int32_t *)(at_base + om);
        it.lists = (dgs::u64 *)(l_base + ol);
        it.res = p->d_res + 5 * x;
        it.n = n;
        it.part = (dgs::u64 *)(p_base + op);
        op += dgs::al256(dgs::batch_part_bytes(n));
        dgs::batch_place(it, p->tot);
        order[x] = x;
        om += dgs::al256((size_t)n * n * 4);
        ol += dgs::al256((size_t)n * 16);
        ov += dgs::al256((size_t)n * 4);
    }
    if (hipMemcpyAsync(p->d_items, items.data(), (size_t)count * sizeof(dgs::BatchItem), hipMemcpyHostToDevice,
                       p->stream) != hipSuccess ||
        hipMemcpyAsync(p->d_order, order.data(), (size_t)count * 4, hipMemcpyHostToDevice, p->stream) !=
            hipSuccess ||
        hipStreamSynchronize(p->stream) != hipSuccess)
        return fail(DGS_E_DEVICE, "upload of the instance table failed");
    *out = p;
    return DGS_OK;
}

int32_t *dgs_batch_plan_benefit(dgs_batch_plan *p, int32_t b) {
    return (p && b >= 0 && b < p->count) ? p->A[b] : nullptr;
}

int32_t *dgs_batch_plan_assign(dgs_batch_plan *p, int32_t b) {
    return (p && b >= 0 && b < p->count) ? p->tau[b] : nullptr;
}

dgs_status dgs_batch_plan_run(dgs_batch_plan *p, const int32_t *const *benefits, int32_t *const *assign_outs,
                              dgs_result *results) {
    if (!p) {
        set_error("dgs_batch_plan_run: NULL plan");
        return DGS_E_INVAL;
    }
    hipStream_t s = p->stream;
    if (benefits) {
        for (int32_t b = 0; b < p->count; ++b) {
            if (!benefits[b]) {
                set_error("dgs_batch_plan_run: benefits[%d] is NULL", b);
                return DGS_E_INVAL;
            }
        }
        for (int32_t b = 0; b < p->count; ++b)
            DGS_HIP(hipMemcpyAsync(p->A[b], benefits[b], (size_t)p->ns[b] * p->ns[b] * 4, hipMemcpyHostToDevice, s));
    }
    if (assign_outs) {
        for (int32_t b = 0; b < p->count; ++b) {
            if (!assign_outs[b]) {
                set_error("dgs_batch_plan_run: assign_outs[%d] is NULL", b);
                return DGS_E_INVAL;
            }
        }
    }
    if (p->autotune && !p->tuned) {
        dgs_status st = tune(p);
        if (st != DGS_OK) return st;
    }
    if (!p->exec) {
        dgs_status st = capture(p);
        if (st != DGS_OK) return st;
    }
    DGS_HIP(hipEventRecord(p->ev0, s));
    DGS_HIP(hipGraphLaunch(p->exec, s));
    DGS_HIP(hipEventRecord(p->ev1, s));
    DGS_HIP(hipStreamSynchronize(s));
    dgs_status st = check_results(p);
    if (st != DGS_OK) return st;
    float ms = 0.f;
    DGS_HIP(hipEventElapsedTime(&ms, p->ev0, p->ev1));
    if (assign_outs) {
        for (int32_t b = 0; b < p->count; ++b)
            DGS_HIP(hipMemcpyAsync(assign_outs[b], p->tau[b], (size_t)p->ns[b] * 4, hipMemcpyDeviceToHost, s));
        DGS_HIP(hipStreamSynchronize(s));
    }
    if (results) {
        for (int32_t b = 0; b < p->count; ++b) {
            const int64_t *r = p->h_res + 5 * (size_t)p->slot_of[b];
            dgs_result &o = results[b];
            std::memset(&o, 0, sizeof o);
            o.initial_benefit = r[0];
            o.total_benefit = r[1];
            o.switches = r[2];
            o.rescans = r[3];
            o.device_ms = ms;
        }
    }
    return DGS_OK;
}

dgs_status dgs_batch_plan_config(dgs_batch_plan *p, int32_t *block, int32_t *grid) {
    if (!p) {
        set_error("dgs_batch_plan_config: NULL plan");
        return DGS_E_INVAL;
    }
    if (block) *block = p->block;
    if (grid) *grid = p->grid;
    return DGS_OK;
}

void dgs_batch_plan_destroy(dgs_batch_plan *p) {
    if (p) free_plan(p);
}

}  // extern "C"
