// Greedy start of DGS on gfx950 (Section 3.1): agents 0..n-1 in order, each
// takes its free job of largest benefit, lowest job index on ties.
//
// The sequential dependency is kept exactly, in rounds of kRound agents:
//   1. k_greedy_topk: one workgroup per agent of the round; each of its
//      kTopkWaves waves keeps the kRound best keys (benefit, job) of its share
//      of the columns among the jobs free at the start of the round (wave64
//      bitonic sort / merge in registers), then the wave lists are merged
//      pairwise in LDS into the agent's list;
//   2. k_greedy_resolve: one wave walks the round's agents in order; an
//      agent takes the first key of its list whose job is still free.  At
//      most kRound - 1 jobs are taken inside a round, so the list of kRound
//      keys never runs out: its first free entry is the agent's greedy choice.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgs_device.h"
#include "dgs_internal.h"

namespace dgs {
namespace {

using namespace dev;

constexpr int kRound = 64;       // agents per round = list length = wave size
constexpr int kTopkWaves = 16;   // waves per agent
constexpr int kTopkBlock = 64 * kTopkWaves;

__device__ __forceinline__ u64 kmax(u64 a, u64 b) { return a > b ? a : b; }
__device__ __forceinline__ u64 kmin(u64 a, u64 b) { return a < b ? a : b; }

// Sort one key per lane, descending across the wave (bitonic network).
__device__ __forceinline__ u64 wave_sort_desc(u64 v, int lane) {
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const u64 o = shfl_xor64(v, j);
            const bool desc_block = (lane & k) == 0 || k == 64;
            const bool lower = (lane & j) == 0;
            v = (desc_block == lower) ? kmax(v, o) : kmin(v, o);
        }
    }
    return v;
}

// A bitonic sequence across the wave -> sorted descending.
__device__ __forceinline__ u64 wave_bitonic_desc(u64 v, int lane) {
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) {
        const u64 o = shfl_xor64(v, j);
        v = ((lane & j) == 0) ? kmax(v, o) : kmin(v, o);
    }
    return v;
}

// Top kRound of the union of two descending lists (one key per lane each).
__device__ __forceinline__ u64 wave_merge_top(u64 a, u64 b, int lane) {
    return wave_bitonic_desc(kmax(a, reverse_lanes64(b)), lane);
}

// The kRound best keys (benefit, job) of the free columns [c0, c1) of row Ar,
// c1 - c0 <= 64 * kSel, sorted descending across the wave.  Every lane holds
// its columns' keys in registers; a binary search on the benefit (the high
// word of the key) finds the largest threshold T with at least kRound keys at
// or above it: those keys contain the best kRound.  When they number at most
// 2 kRound they are compacted into `buf` (this wave's 2 x 64 LDS slots) and
// sorted; otherwise (many equal benefits at T) the keys are merged in batches.
constexpr int kSel = 16;  // keys per lane

__device__ __forceinline__ int count_at_least(const uint32_t (&h)[kSel], uint32_t T) {
    int c = 0;
#pragma unroll
    for (int u = 0; u < kSel; ++u) c += __popcll(__ballot(h[u] >= T));
    return c;
}

__device__ u64 wave_top_select(const int32_t *Ar, const uint32_t *taken, int c0, int c1, int lane, u64 *buf) {
    u64 key[kSel];
    uint32_t h[kSel];  // benefit part of each key (0: none)
#pragma unroll
    for (int u = 0; u < kSel; ++u) {
        const int c = c0 + u * 64 + lane;
        bool ok = false;
        int v = 0;
        if (c < c1) {
            ok = !((taken[c >> 5] >> (c & 31)) & 1u);
            v = Ar[c];
        }
        key[u] = ok ? mk_key(v, c) : 0;
        h[u] = (uint32_t)(key[u] >> 32);
    }
    // threshold: the largest T with count(h >= T) >= kRound (T = 1 takes every key)
    uint32_t T = 1;
    if (count_at_least(h, 1) > kRound) {
        uint32_t lo = 0xFFFFFFFFu, hi = 0;
#pragma unroll
        for (int u = 0; u < kSel; ++u) {
            if (h[u]) lo = min(lo, h[u]);
            hi = max(hi, h[u]);
        }
        // wave-wide min of lo and max of hi
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            lo = min(lo, (uint32_t)__shfl_xor((int)lo, m, 64));
            hi = max(hi, (uint32_t)__shfl_xor((int)hi, m, 64));
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        hi = __builtin_amdgcn_readfirstlane(hi);
        // invariant: count(h >= lo) >= kRound; the answer lies in [lo, hi]
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo + 1) / 2;
            if (count_at_least(h, mid) >= kRound)
                lo = mid;
            else
                hi = mid - 1;
        }
        T = lo;
    }
    const int C = count_at_least(h, T);
    if (C <= 2 * kRound) {
        int base = 0;
#pragma unroll
        for (int u = 0; u < kSel; ++u) {
            const bool sel = h[u] >= T;
            const unsigned long long m = __ballot(sel);
            if (sel) buf[base + __popcll(m & ((1ull << lane) - 1))] = key[u];
            base += __popcll(m);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        const u64 a = lane < C ? buf[lane] : 0;
        const u64 b = lane + 64 < C ? buf[lane + 64] : 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // buf may be reused by the caller
        return wave_merge_top(wave_sort_desc(a, lane), wave_sort_desc(b, lane), lane);
    }
    u64 list = 0;
#pragma unroll
    for (int u = 0; u < kSel; ++u) {
        const u64 k = h[u] >= T ? key[u] : 0;
        if (__ballot(k != 0)) list = wave_merge_top(list, wave_sort_desc(k, lane), lane);
    }
    return list;
}

struct TopkParams {
    const int32_t *A;
    const uint32_t *taken;  // bitmap of jobs taken before this round
    u64 *lists;             // [kRound][64]
    int n;     // jobs (columns, the row stride of A)
    int row0;  // first agent of the round
};

__global__ __launch_bounds__(kTopkBlock) void k_greedy_topk(TopkParams P) {
    __shared__ u64 wl[kTopkWaves][64];
    __shared__ u64 cand[kTopkWaves][2 * 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row = P.row0 + blockIdx.x;
    const int32_t *Ar = P.A + (int64_t)row * P.n;
    // the row's columns, split evenly over the waves in whole batches of 64
    const int sub = ((P.n + kTopkWaves * 64 - 1) / (kTopkWaves * 64)) * 64;  // columns per wave
    const int c0 = w * sub;
    const int c1 = min(P.n, c0 + sub);
    u64 list = 0;
    if (sub <= 64 * kSel) {
        list = wave_top_select(Ar, P.taken, c0, c1, lane, cand[w]);
    } else {
        // streaming: batches of 64 keys, sorted and merged when many pass the running bound
        u64 lmin = 0;
        constexpr int U = 8;  // batches loaded ahead
        for (int g0 = c0; g0 < c1; g0 += 64 * U) {
            int val[U];
            bool ok[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = g0 + u * 64 + lane;
                ok[u] = false;
                val[u] = 0;
                if (c < c1) {
                    ok[u] = !((P.taken[c >> 5] >> (c & 31)) & 1u);
                    val[u] = Ar[c];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = g0 + u * 64 + lane;
                u64 key = ok[u] ? mk_key(val[u], c) : 0;
                if (key <= lmin) key = 0;
                const unsigned long long m = __ballot(key != 0);
                if (m == 0) continue;
                if (__popcll(m) > 8) {
                    list = wave_merge_top(list, wave_sort_desc(key, lane), lane);
                } else {
                    unsigned long long mm = m;
                    while (mm) {
                        const int src = __ffsll((long long)mm) - 1;
                        mm &= mm - 1;
                        const u64 k = readlane64(key, src);
                        // insert k into the descending list: lanes below k shift down by one
                        const u64 up = ((u64)(uint32_t)__shfl_up((int)(uint32_t)(list >> 32), 1, 64) << 32) |
                                       (u64)(uint32_t)__shfl_up((int)(uint32_t)list, 1, 64);
                        if (list < k) list = (lane == 0 || up > k) ? k : up;
                    }
                }
                lmin = readlane64(list, 63);
            }
        }
    }
    // pairwise merges of the wave lists: after the step of span s, wave w (w % 2s == 0)
    // holds the top kRound of waves w .. w + 2s - 1
    wl[w][lane] = list;
#pragma unroll
    for (int span = 1; span < kTopkWaves; span *= 2) {
        __syncthreads();
        if (w % (2 * span) == 0) {
            list = wave_merge_top(list, wl[w + span][lane], lane);
            wl[w][lane] = list;
        }
    }
    if (w == 0) P.lists[(size_t)blockIdx.x * 64 + lane] = list;
}

struct ResolveParams {
    const u64 *lists;
    uint32_t *taken;
    int32_t *tau;
    int32_t *sigma;
    int32_t *err;
    int n;  // jobs
    int row0;
    int rows;
};

// One workgroup: stage the round's lists and the taken bitmap in LDS, then
// wave 0 resolves the agents in order; the choices are written out at the end.
__global__ __launch_bounds__(256) void k_greedy_resolve(ResolveParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int pick[kRound];
    u64 *L = (u64 *)smem;                                      // rows * 64
    uint32_t *tk = (uint32_t *)(smem + (size_t)P.rows * 64 * 8);  // n / 32 words
    const int words = (P.n + 31) >> 5;
    // stage the lists (16-byte loads, all in flight: rows * 32 <= 8 * 256) and the bitmap
    {
        const int total4 = P.rows * 32;
        const int4 *src = (const int4 *)P.lists;
        int4 *dst = (int4 *)L;
        int4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[min((int)threadIdx.x + u * 256, total4 - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = threadIdx.x + u * 256;
            if (i < total4) dst[i] = v[u];
        }
    }
    for (int i = threadIdx.x; i < words; i += blockDim.x) tk[i] = P.taken[i];
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        // agent ri + 1's list is read while agent ri is resolved
        u64 nxt = L[lane];
        int my_pick = -1;  // lane ri keeps agent ri's choice
        for (int ri = 0; ri < P.rows; ++ri) {
            const u64 cur = nxt;
            if (ri + 1 < P.rows) nxt = L[(size_t)(ri + 1) * 64 + lane];
            const int c = cur ? key_index(cur) : 0;
            const bool fr = cur != 0 && !((tk[c >> 5] >> (c & 31)) & 1u);
            const unsigned long long m = __ballot(fr);
            if (m == 0) {  // cannot happen (see above); never index with it
                if (lane == 0) atomicOr(P.err, 4);
                continue;
            }
            const int pc = key_index(readlane64(cur, __ffsll((long long)m) - 1));
            if (lane == 0) atomicOr(&tk[pc >> 5], 1u << (pc & 31));
            if (lane == ri) my_pick = pc;
        }
        pick[lane] = my_pick;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < words; i += blockDim.x) P.taken[i] = tk[i];
    if (threadIdx.x < P.rows) {
        const int c = pick[threadIdx.x];
        if (c >= 0) {
            P.tau[P.row0 + threadIdx.x] = c;
            P.sigma[c] = P.row0 + threadIdx.x;
        }
    }
}

// The virtual agents rows..n-1 of a rectangular instance take the jobs that
// no real agent holds (sigma = -1), in increasing job order.  One workgroup:
// each thread counts the free jobs of its stretch, an exclusive scan in LDS
// gives its first virtual agent.
constexpr int kFillBlock = 1024;

__global__ __launch_bounds__(kFillBlock) void k_fill_virtual(int32_t *tau, int32_t *sigma, int rows, int n) {
    __shared__ int cnt[kFillBlock];
    const int t = threadIdx.x;
    const int per = (n + kFillBlock - 1) / kFillBlock;
    const int j0 = t * per, j1 = min(n, j0 + per);
    int c = 0;
    for (int j = j0; j < j1; ++j) c += sigma[j] < 0;
    cnt[t] = c;
    __syncthreads();
    for (int off = 1; off < kFillBlock; off <<= 1) {  // inclusive scan (Hillis-Steele)
        const int v = t >= off ? cnt[t - off] : 0;
        __syncthreads();
        cnt[t] += v;
        __syncthreads();
    }
    int agent = rows + cnt[t] - c;
    for (int j = j0; j < j1; ++j) {
        if (sigma[j] >= 0) continue;
        if (agent < n) {  // (exactly n - rows jobs are free)
            tau[agent] = j;
            sigma[j] = agent;
        }
        ++agent;
    }
}

// ---- global greedy start ------------------------------------------------------------
// While an agent is free, the largest entry a_ij over free agents i and free
// jobs j is taken (the lowest agent, then the lowest job, among equal
// entries: a strict order of the entries, the key (a_ij, -i, -j)).  Built
// in rounds: a pair (i, j) whose entry is the largest of agent i's entries
// over free jobs (the head of i) and of job j's entries over free agents (the
// column best of j) is taken by the one-at-a-time rule before any other
// entry of i or of j (every such entry left later is smaller), so all such
// pairs of a round are taken together; every round takes at least the
// largest remaining entry.  A head stays valid while its job is free and a
// column best while its agent is free (the free sets only shrink), so only
// invalidated ones are searched again.

struct GGState {
    const int32_t *A;   // rows x cols
    const int32_t *AT;  // cols x rows
    int32_t *tau;       // [rows] job of agent, -1 free
    int32_t *sigma;     // [cols] agent of job, -1 free
    int32_t *head;      // [rows] best free job of a free agent (-1 unknown)
    int32_t *colbest;   // [cols] best free agent of a job (-1 unknown)
    int32_t *want;      // [cols] last round in which some head pointed at the job
    unsigned long long *count;  // agents matched so far
    int rows, cols;
};

// One wave per free agent: its head (largest entry over free jobs, lowest job
// on ties); marks the head's job as wanted in this round.
__global__ __launch_bounds__(256) void k_gg_heads(GGState P, int round) {
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= P.rows || P.tau[i] >= 0) return;
    int h = P.head[i];
    if (h < 0 || P.sigma[h] >= 0) {
        const int32_t *row = P.A + (int64_t)i * P.cols;
        u64 best = 0;
        int j = lane;
        for (; j + 192 < P.cols; j += 256) {  // four requests in flight per lane
            const int v0 = row[j], v1 = row[j + 64], v2 = row[j + 128], v3 = row[j + 192];
            const int s0 = P.sigma[j], s1 = P.sigma[j + 64], s2 = P.sigma[j + 128], s3 = P.sigma[j + 192];
            if (s0 < 0) best = umax64(best, mk_key(v0, j));
            if (s1 < 0) best = umax64(best, mk_key(v1, j + 64));
            if (s2 < 0) best = umax64(best, mk_key(v2, j + 128));
            if (s3 < 0) best = umax64(best, mk_key(v3, j + 192));
        }
        for (; j < P.cols; j += 64)
            if (P.sigma[j] < 0) best = umax64(best, mk_key(row[j], j));
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) best = umax64(best, shfl_xor64(best, m));
        h = best ? key_index(best) : -1;  // rows <= cols: a free job always exists
        if (lane == 0) P.head[i] = h;
    }
    if (lane == 0 && h >= 0) P.want[h] = round;
}

// One wave per wanted job: its column best (largest entry over free agents,
// lowest agent on ties), searched again only when its agent was taken.
__global__ __launch_bounds__(256) void k_gg_cols(GGState P, int round) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= P.cols || P.want[j] != round) return;
    const int c = P.colbest[j];
    if (c >= 0 && P.tau[c] < 0) return;
    const int32_t *col = P.AT + (int64_t)j * P.rows;
    u64 best = 0;
    for (int i = lane; i < P.rows; i += 64)
        if (P.tau[i] < 0) best = umax64(best, mk_key(col[i], i));
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) best = umax64(best, shfl_xor64(best, m));
    if (lane == 0) P.colbest[j] = best ? key_index(best) : -1;
}

// A free agent whose head's column best is itself takes its head.
__global__ __launch_bounds__(256) void k_gg_match(GGState P) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= P.rows || P.tau[i] >= 0) return;
    const int h = P.head[i];
    if (h >= 0 && P.colbest[h] == i) {
        P.tau[i] = h;
        P.sigma[h] = i;
        atomicAdd(P.count, 1ull);
    }
}

}  // namespace

size_t global_greedy_scratch_bytes(int rows, int cols) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return al((size_t)rows * 4) + 2 * al((size_t)cols * 4) + 256;
}

hipError_t run_global_greedy(const int32_t *A, const int32_t *AT, int32_t rows, int32_t cols, int32_t *tau,
                             int32_t *sigma, void *scratch, int64_t *host_count, int64_t *rounds_out,
                             hipStream_t s) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char *p = (char *)scratch;
    GGState P;
    P.A = A;
    P.AT = AT;
    P.tau = tau;
    P.sigma = sigma;
    P.head = (int32_t *)p;
    P.colbest = (int32_t *)(p + al((size_t)rows * 4));
    P.want = (int32_t *)(p + al((size_t)rows * 4) + al((size_t)cols * 4));
    P.count = (unsigned long long *)(p + al((size_t)rows * 4) + 2 * al((size_t)cols * 4));
    P.rows = rows;
    P.cols = cols;
    hipError_t e;
    if ((e = launch_fill(tau, rows, -1, s)) != hipSuccess || (e = launch_fill(sigma, cols, -1, s)) != hipSuccess ||
        (e = launch_fill(P.head, rows, -1, s)) != hipSuccess ||
        (e = launch_fill(P.colbest, cols, -1, s)) != hipSuccess ||
        (e = launch_fill(P.want, cols, -1, s)) != hipSuccess || (e = launch_fill((int32_t *)P.count, 2, 0, s)) != hipSuccess)
        return e;
    const unsigned gh = (unsigned)((rows + 3) / 4), gc = (unsigned)((cols + 3) / 4), gm = (unsigned)((rows + 255) / 256);
    constexpr int kPerCheck = 8;  // rounds between reads of the matched count (extra rounds are empty)
    int round = 0;
    for (;;) {
        for (int k = 0; k < kPerCheck; ++k, ++round) {
            hipLaunchKernelGGL(k_gg_heads, dim3(gh), dim3(256), 0, s, P, round);
            hipLaunchKernelGGL(k_gg_cols, dim3(gc), dim3(256), 0, s, P, round);
            hipLaunchKernelGGL(k_gg_match, dim3(gm), dim3(256), 0, s, P);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(host_count, P.count, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (*host_count >= rows) break;
        if (round > rows + kPerCheck) return hipErrorUnknown;  // every round takes a pair: cannot happen
    }
    *rounds_out = round;
    return launch_fill_virtual(tau, sigma, rows, cols, s);
}

hipError_t launch_fill_virtual(int32_t *tau, int32_t *sigma, int32_t rows, int32_t n, hipStream_t s) {
    if (rows >= n) return hipSuccess;
    hipLaunchKernelGGL(k_fill_virtual, dim3(1), dim3(kFillBlock), 0, s, tau, sigma, rows, n);
    return hipGetLastError();
}

size_t greedy_scratch_bytes(int n) {
    return (size_t)kRound * 64 * sizeof(u64) + (((size_t)n + 31) / 32) * 4 + 256;
}

hipError_t launch_greedy_rounds(const int32_t *A, int32_t rows, int32_t n, int32_t *tau, int32_t *sigma,
                                void *scratch, int32_t *err, hipStream_t s) {
    u64 *lists = (u64 *)scratch;
    uint32_t *taken = (uint32_t *)((char *)scratch + (size_t)kRound * 64 * sizeof(u64));
    const int words = (n + 31) / 32;
    hipError_t e = launch_fill((int32_t *)taken, words, 0, s);
    if (e != hipSuccess) return e;
    if (rows < n && (e = launch_fill(sigma, n, -1, s)) != hipSuccess) return e;
    const size_t rshm = (size_t)kRound * 64 * sizeof(u64) + (size_t)words * 4;
    e = hipFuncSetAttribute((const void *)k_greedy_resolve, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rshm);
    if (e != hipSuccess) return e;
    for (int row0 = 0; row0 < rows; row0 += kRound) {
        const int cnt = rows - row0 < kRound ? rows - row0 : kRound;
        TopkParams T{A, taken, lists, n, row0};
        hipLaunchKernelGGL(k_greedy_topk, dim3((unsigned)cnt), dim3(kTopkBlock), 0, s, T);
        ResolveParams R{lists, taken, tau, sigma, err, n, row0, cnt};
        const size_t shm = (size_t)cnt * 64 * sizeof(u64) + (size_t)words * 4;
        hipLaunchKernelGGL(k_greedy_resolve, dim3(1), dim3(256), shm, s, R);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_fill_virtual(tau, sigma, rows, n, s);
}

}  // namespace dgs
