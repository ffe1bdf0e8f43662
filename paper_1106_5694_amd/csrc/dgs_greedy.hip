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
// The single-instance solve runs the same rule as one persistent launch
// (k_greedy_pipe: lists of agent i from the jobs free once agents < i - 63
// have picked, computed while earlier agents resolve); the rounds remain for
// callers that share the device (the batched solver, the server) and for
// n > 32768.
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

// Bitonic network over the wave, one key per lane.  The block size K and the
// lane distance J are template arguments, so every exchange is a VALU lane
// permute (a distance known only at run time would go through the LDS).
// Stages J, J / 2, ..., 1 of blocks of K lanes; blocks with (lane & K) == 0,
// and all lanes when K = 64, are ordered descending.
template <int K, int J>
__device__ __forceinline__ u64 bitonic_pass(u64 v, int lane) {
    const u64 o = xor_lanes64<J>(v);
    const bool desc_block = (lane & K) == 0 || K == 64;
    const bool lower = (lane & J) == 0;
    v = (desc_block == lower) ? kmax(v, o) : kmin(v, o);
    if constexpr (J > 1) return bitonic_pass<K, J / 2>(v, lane);
    return v;
}

// Sort one key per lane, descending across the wave (blocks of 2, 4, ..., 64).
template <int K = 2>
__device__ __forceinline__ u64 wave_sort_desc(u64 v, int lane) {
    v = bitonic_pass<K, K / 2>(v, lane);
    if constexpr (K < 64) return wave_sort_desc<K * 2>(v, lane);
    return v;
}

// A bitonic sequence across the wave -> sorted descending.
__device__ __forceinline__ u64 wave_bitonic_desc(u64 v, int lane) { return bitonic_pass<64, 32>(v, lane); }

// Top kRound of the union of two descending lists (one key per lane each).
__device__ __forceinline__ u64 wave_merge_top(u64 a, u64 b, int lane) {
    return wave_bitonic_desc(kmax(a, reverse_lanes64(b)), lane);
}

// The kRound best keys (benefit, job) of the free columns [c0, c1) of a row,
// c1 - c0 <= 64 * kSel, sorted descending across the wave.  Every lane holds
// its columns' keys in registers; a binary search on the benefit (the high
// word of the key) finds the largest threshold T with at least kRound keys at
// or above it.  The best kRound are then the keys above T (fewer than kRound)
// and, of the keys at T, those of the lowest columns: the first ones in column
// order c0 + u * 64 + lane, u outer.  They are compacted into `buf` (this
// wave's 64 LDS slots) and sorted once.
constexpr int kSel = 16;  // keys per lane

// Wave minimum / maximum (every lane active).
__device__ __forceinline__ uint32_t wave_min32(uint32_t v) {
    v = min(v, xor_lanes<32>(v));
    v = min(v, xor_lanes<16>(v));
    v = min(v, xor_lanes<8>(v));
    v = min(v, xor_lanes<4>(v));
    v = min(v, xor_lanes<2>(v));
    return min(v, xor_lanes<1>(v));
}
__device__ __forceinline__ uint32_t wave_max32(uint32_t v) {
    v = max(v, xor_lanes<32>(v));
    v = max(v, xor_lanes<16>(v));
    v = max(v, xor_lanes<8>(v));
    v = max(v, xor_lanes<4>(v));
    v = max(v, xor_lanes<2>(v));
    return max(v, xor_lanes<1>(v));
}

__device__ __forceinline__ int count_at_least(const uint32_t (&h)[kSel], uint32_t T) {
    int c = 0;
#pragma unroll
    for (int u = 0; u < kSel; ++u) c += __popcll(__ballot(h[u] >= T));
    return c;
}

// The entries Ar[c0 + u * 64 + lane], u < kSel, of the columns below c1 (0 past c1).
__device__ __forceinline__ void row_part_load(const int32_t *Ar, int c0, int c1, int lane, int (&v)[kSel]) {
#pragma unroll
    for (int u = 0; u < kSel; ++u) {
        const int c = c0 + u * 64 + lane;
        v[u] = c < c1 ? Ar[c] : 0;
    }
}

__device__ u64 wave_top_select(const int (&v)[kSel], const uint32_t *taken, int c0, int c1, int lane, u64 *buf) {
    u64 key[kSel];
    uint32_t h[kSel];  // benefit part of each key (0: none)
#pragma unroll
    for (int u = 0; u < kSel; ++u) {
        const int c = c0 + u * 64 + lane;
        const bool ok = c < c1 && !((taken[c >> 5] >> (c & 31)) & 1u);
        key[u] = ok ? mk_key(v[u], c) : 0;
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
        lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_min32(lo));
        hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_max32(hi));
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
    // keys above T all go; of the keys at T, the first `room` in column order
    const int room = kRound - (T == 0xFFFFFFFFu ? 0 : count_at_least(h, T + 1));
    const unsigned long long below = (1ull << lane) - 1;
    int base = 0, ties = 0;
#pragma unroll
    for (int u = 0; u < kSel; ++u) {
        const bool at = h[u] == T && h[u] != 0;
        const unsigned long long tm = __ballot(at);
        const bool sel = h[u] > T || (at && ties + __popcll(tm & below) < room);
        const unsigned long long m = __ballot(sel);
        if (sel) buf[base + __popcll(m & below)] = key[u];
        base += __popcll(m);
        ties += __popcll(tm);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const u64 a = lane < base ? buf[lane] : 0;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // buf may be reused by the caller
    return wave_sort_desc(a, lane);
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
        int vals[kSel];
        row_part_load(Ar, c0, c1, lane, vals);
        list = wave_top_select(vals, P.taken, c0, c1, lane, cand[w]);
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

// ---- the greedy start as one persistent launch ---------------------------------------
// Producers and one resolver workgroup run at the same time (a cooperative
// launch, so all are resident).  Work item (i, q), one producer workgroup:
// the kRound best keys of agent i over part q of the columns (kPart columns)
// among the jobs free once agents 0 .. i - kRound have picked; the row's
// entries are loaded before the picks are awaited.  At most kRound - 1 more
// jobs are taken before agent i picks, so the list holds agent i's best free
// job of that part.  In the resolver workgroup, staging waves load the part
// lists, merge an agent's parts into one sorted list of kRound keys and put
// it into an LDS ring; the resolver wave walks the agents in order and takes
// the best key of the agent's list whose job is still free.  Producers learn
// the picks from the resolver's pick words (throttled by its progress word)
// and the staging waves read the lists, both with relaxed agent-scope
// atomics; every word carries its agent (plus one) as a 16-bit tag and the
// buffers are cleared first, so a word is current exactly when its tag
// matches and no fence is needed.  n <= kPipeMaxN (16-bit jobs and tags; at
// most kMaxParts parts).
constexpr int kPW = 8;                     // waves per workgroup
constexpr int kPipeT = 64 * kPW;           // threads per workgroup
constexpr int kPart = kPW * 64 * kSel;     // columns per part (8192)
constexpr int kRingA = 2 * kRound;         // list slots in device memory (agents in flight <= kRound)
constexpr int kRingL = kRound;             // agents staged in the resolver's LDS (one merged list each)
// spin limits (each well above a second): LDS polls, polls of device memory
constexpr long long kPipeSpin = 1ll << 24, kPipeSpinG = 1ll << 20;
constexpr int kPipeMaxN = 32768;
constexpr int kMaxParts = (kPipeMaxN + kPart - 1) / kPart;  // 4
constexpr int kStage = 8;  // lists in flight per staging wave

struct PipeParams {
    const int32_t *A;   // rows x n
    u64 *lists;         // [kRingA][Q][kRound] tagged keys
    uint32_t *picks;    // [-2 .. rows) (agent + 1) << 16 | job (picks[-2], picks[-1]: spare); tau, sigma are written from them
    int *progress;      // agents resolved so far; -1 once the resolver has given up
    int32_t *err;
    int rows, n, Q;
    int A_per;          // agents per batch of a staging wave (A_per * Q <= kStage)
};

// key (benefit, job) of mk_key -> the same order with the tag in bits 31..16
// and 0xFFFF - job below (0: none, with the tag).
__device__ __forceinline__ u64 tag_key(u64 k, uint32_t tag) {
    if (!k) return (u64)(tag << 16);
    return (k & 0xFFFFFFFF00000000ull) | (u64)(tag << 16) | (u64)(0xFFFFu - (uint32_t)key_index(k));
}
__device__ __forceinline__ uint32_t key_tag(u64 k) { return ((uint32_t)k >> 16) & 0xFFFFu; }
__device__ __forceinline__ int tkey_job(u64 k) { return (int)(0xFFFFu - ((uint32_t)k & 0xFFFFu)); }

// Stop the pipeline: flag the error; producers learn it from the progress word, the
// resolver's other waves from `fail`.
__device__ __forceinline__ void pipe_give_up(const PipeParams &P, int *fail) {
    atomicOr(P.err, 16);
    __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (blockIdx.x == 0) __hip_atomic_store(P.progress, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The resolver wave: agents in order, each takes the first job of its staged list that
// is free.  The list holds the jobs of the agent's best keys in decreasing key order
// (0xFFFF: no key), so the first free job is the lowest free lane: one ballot.  Agents go
// in pairs (a, a + 1) whose two chains run side by side: a + 1 takes its lowest free
// lane unless that lane holds a's job, else its next free lane (a list's jobs are
// distinct).  The LDS reads of the next pair's taken words and of the pair after it's
// jobs go out before the current pair chooses, so no LDS round trip is on the per-pair
// path.  The jobs are read right after their ready flags, without waiting: this wave's
// LDS accesses complete in order, so when a flag read sees the staged value the job read
// sees the staged jobs (otherwise it is read again once the flag is set).  A pair's
// picks are published at the top of the next step, before the taken-word reads of the
// pair after it, which then miss only the previous pair's two jobs (excluded by
// comparison).  Every lane runs the stores (the same value to one address, or to a
// lane's own spare word), so the loop has no branch.
constexpr int kTkWords = (kPipeMaxN + 31) / 32;  // taken bitmap words; 64 spare words follow

__device__ __forceinline__ void pipe_resolve(const PipeParams &P, uint32_t *tk, uint32_t (*ring)[64], int *rdy,
                                             int *done, int *fail, int lane) {
    static_assert((kRingL & (kRingL - 1)) == 0, "ring slots by mask");
    static_assert(kPipeMaxN / 32 == kTkWords, "the first spare word holds job kPipeMaxN");
    auto word = [&](uint32_t j) { return tk[(j & (kPipeMaxN - 1)) >> 5]; };
    auto flag = [&](int k) {
        return __hip_atomic_load(&rdy[k & (kRingL - 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    // (an atomic load, so the compiler issues it where it stands, ahead of the choice)
    auto jobs = [&](int k) {
        return __hip_atomic_load(&ring[k & (kRingL - 1)][lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    auto wait = [&](int k) -> bool {  // bounded wait until agent k's list is staged
        long long spins = 0;
        while (flag(k) != k + 1) {
            if (++spins > kPipeSpin || __hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                if (lane == 0) pipe_give_up(P, fail);
                return false;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        return true;
    };
    // agent k's job is published at the top of the next step (and after the loop).  k < 0
    // publishes nothing: its job kPipeMaxN sets a bit in lane 0's spare word, and its pick
    // word is one of the spare slots picks[-2], picks[-1].
    auto publish = [&](int k, int j) {
        // lane 0 sets the job's bit; the other lanes or 0 into their spare words
        atomicOr(&tk[lane == 0 ? (j >> 5) : kTkWords + lane], lane == 0 ? 1u << (j & 31) : 0u);
        __hip_atomic_store(&P.picks[k], ((uint32_t)(k + 1) << 16) | (uint32_t)j, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    };
    auto progress = [&](int nd) {
        __hip_atomic_store(P.progress, nd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // relaxed: the published agents' jobs were consumed (used) before this store
        __hip_atomic_store(&done[lane], nd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    const int R = P.rows;
    uint32_t jr[4];  // jobs of agents 0..3 (0xFFFF past the last agent)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        jr[k] = 0xFFFFu;
        if (k < R) {
            if (!wait(k)) return;
            jr[k] = jobs(k);
        }
    }
    uint32_t ja = jr[0], jb = jr[1], jna = jr[2], jnb = jr[3];  // the pair, the next pair
    uint32_t wa = word(ja), wb = word(jb);  // their taken words, missing the previous pair's jobs
    int j2 = kPipeMaxN, j1 = kPipeMaxN;      // the previous pair's jobs (none: no list holds them)
    for (int a = 0; a < R; a += 2) {
        publish(a - 2, j2);
        publish(a - 1, j1);
        progress(a);
        const uint32_t wna = word(jna), wnb = word(jnb);
        const int f4 = flag(a + 4), f5 = flag(a + 5);  // (slots past the last agent: ignored)
        __atomic_signal_fence(__ATOMIC_SEQ_CST);      // the job reads stay after the flag reads
        uint32_t j4 = jobs(a + 4), j5 = jobs(a + 5);
        auto is_free = [&](uint32_t j, uint32_t w) {
            return (j < (uint32_t)kPipeMaxN) & (((w >> (j & 31)) & 1u) == 0u) & ((int)j != j2) & ((int)j != j1);
        };
        const unsigned long long ma = __ballot(is_free(ja, wa));
        const unsigned long long mb = __ballot(is_free(jb, wb));
        const unsigned long long mb2 = mb & (mb - 1);  // without its lowest lane
        const int pa = __builtin_amdgcn_readlane((int)ja, (int)__builtin_ctzll(ma | (1ull << 63)));
        const int pb1 = __builtin_amdgcn_readlane((int)jb, (int)__builtin_ctzll(mb | (1ull << 63)));
        const int pb2 = __builtin_amdgcn_readlane((int)jb, (int)__builtin_ctzll(mb2 | (1ull << 63)));
        const bool b_real = a + 1 < R;
        const bool ok_b = mb2 != 0 || (mb != 0 && pb1 != pa);
        if (ma == 0 || (b_real && !ok_b)) {  // cannot happen (a list never runs dry); never index with it
            if (lane == 0) pipe_give_up(P, fail);
            return;
        }
        j2 = pa;
        j1 = b_real ? (pb1 != pa ? pb1 : pb2) : kPipeMaxN;
        ja = jna;
        jb = jnb;
        wa = wna;
        wb = wnb;
        if (a + 4 < R && f4 != a + 5) {
            if (!wait(a + 4)) return;
            j4 = jobs(a + 4);
        }
        if (a + 5 < R && f5 != a + 6) {
            if (!wait(a + 5)) return;
            j5 = jobs(a + 5);
        }
        jna = a + 4 < R ? j4 : 0xFFFFu;
        jnb = a + 5 < R ? j5 : 0xFFFFu;
    }
    // the last pair (its second agent only when it exists)
    const int last = (R - 1) & ~1;
    if (R > 0) {
        publish(last, j2);
        publish(last + 1 < R ? last + 1 : -1, j1);
        progress(R);
    }
}

__global__ __launch_bounds__(kPipeT) void k_greedy_pipe(PipeParams P) {
    __shared__ uint32_t tk[kTkWords + 64];          // taken jobs (producer: picks absorbed; resolver: all)
    __shared__ u64 wl[kPW][64];
    __shared__ u64 cand[kPW][2 * 64];
    __shared__ uint32_t ring[kRingL][64];           // resolver: the jobs of one merged list per staged agent
    __shared__ u64 stg[kPW - 1][kStage][64];        // resolver: a staging wave's part lists
    __shared__ int rdy[kRingL];
    __shared__ int done[64], fail;  // done[0]: agents resolved (every lane writes its own word)
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int words = (P.n + 31) >> 5;
    for (int x = t; x < words; x += kPipeT) tk[x] = 0;
    if (t < kRingL) rdy[t] = 0;
    if (t < 64) done[t] = 0;
    if (t == 0) fail = 0;
    __syncthreads();
    auto give_up = [&]() { pipe_give_up(P, &fail); };

    if (blockIdx.x == 0) {  // ---- the resolver ----
        if (w == 0) {
            pipe_resolve(P, tk, ring, rdy, done, &fail, lane);
        } else {
            // waves 1..kPW-1 stage the lists of batches of A_per consecutive agents: load them
            // (A_per * Q <= kStage lists in flight per wave) as soon as they are produced, then
            // copy them into their slots once the consumer is past the slots' previous agents
            const int Aper = P.A_per;
            const int nb = (P.rows + Aper - 1) / Aper;
            for (int b = w - 1; b < nb; b += kPW - 1) {
                const int k0 = b * Aper, cnt = min(Aper, P.rows - k0);
                // list e = agent k0 + e / Q, part e % Q
                const int ne = cnt * P.Q;
                u64 v[kStage];
#pragma unroll
                for (int e = 0; e < kStage; ++e) {
                    const int k = k0 + e / P.Q, qq = e % P.Q;
                    v[e] = e < ne ? __hip_atomic_load(&P.lists[((size_t)(k % kRingA) * P.Q + qq) * kRound + lane],
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                  : 0;
                }
                long long spins = 0;
                for (;;) {
                    bool ok = true;
#pragma unroll
                    for (int e = 0; e < kStage; ++e)
                        ok &= e >= ne || key_tag(v[e]) == ((uint32_t)(k0 + e / P.Q + 1) & 0xFFFFu);
                    if (__all(ok)) break;
                    if (++spins > kPipeSpinG || __hip_atomic_load(&fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                        if (lane == 0) give_up();
                        return;
                    }
                    __builtin_amdgcn_s_sleep(1);
#pragma unroll
                    for (int e = 0; e < kStage; ++e) {
                        const int k = k0 + e / P.Q, qq = e % P.Q;
                        if (e < ne && key_tag(v[e]) != ((uint32_t)(k + 1) & 0xFFFFu))
                            v[e] = __hip_atomic_load(&P.lists[((size_t)(k % kRingA) * P.Q + qq) * kRound + lane],
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                // one list per agent, the top kRound keys over its parts (an agent's keys share
                // their tag, so tagged keys order as (benefit, -job)), merged in this wave's
                // LDS area: agent a's list replaces entry a, whose part list is merged by then
                u64(*sv)[64] = stg[w - 1];
#pragma unroll
                for (int e = 0; e < kStage; ++e)
                    if (e < ne) sv[e][lane] = v[e];
                if (P.Q > 1) {
                    for (int a = 0; a < cnt; ++a) {
                        u64 list = sv[a * P.Q][lane];
#pragma unroll
                        for (int f = 1; f < kMaxParts; ++f)  // compile-time stages: lane exchanges on the VALU
                            if (f < P.Q) list = wave_merge_top(list, sv[a * P.Q + f][lane], lane);
                        sv[a][lane] = list;
                    }
                }
                spins = 0;
                while (__hip_atomic_load(&done[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) <= k0 + cnt - 1 - kRingL) {
                    if (++spins > kPipeSpin || __hip_atomic_load(&fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                        if (lane == 0) give_up();
                        return;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                for (int a = 0; a < cnt; ++a) ring[(k0 + a) % kRingL][lane] = (uint32_t)tkey_job(sv[a][lane]);
                if (lane == 0)
                    for (int k = k0; k < k0 + cnt; ++k)
                        // relaxed: this wave's LDS writes of the slot come first, in order
                        __hip_atomic_store(&rdy[k % kRingL], k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        return;
    }

    // ---- a producer: items blockIdx.x - 1, + (gridDim.x - 1), ... in order ----
    const long long items = (long long)P.rows * P.Q, stride = gridDim.x - 1;
    int absorbed = 0;  // picks of agents < absorbed are in tk
    for (long long it = blockIdx.x - 1; it < items; it += stride) {
        const int i = (int)(it / P.Q), q = (int)(it % P.Q);
        const int need = i - (kRound - 1);  // picks of agents < need must be in tk
        // the row's entries do not depend on the picks: their loads go out first
        const int c0 = q * kPart + w * 64 * kSel, c1 = min(P.n, c0 + 64 * kSel);
        int vals[kSel];
        row_part_load(P.A + (int64_t)i * P.n, c0, c1, lane, vals);
        if (need > absorbed) {
            // one lane waits for the resolver to pass need - 1, napping about 0.2 us per agent
            // still to resolve (few polls of one word from producers far ahead)
            if (t == 0) {
                long long spins = 0;
                for (;;) {
                    const int p = __hip_atomic_load(P.progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (p >= need) break;
                    if (p < 0 || ++spins > kPipeSpinG) {
                        give_up();
                        break;
                    }
                    const int naps = min(need - p, 16);
                    for (int z = 0; z < naps; ++z) __builtin_amdgcn_s_sleep(8);
                }
            }
            __syncthreads();
            if (fail) return;
        }
        for (int k = absorbed + t; k < need; k += kPipeT) {
            long long spins = 0;
            uint32_t v = __hip_atomic_load(&P.picks[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while ((v >> 16) != ((uint32_t)(k + 1) & 0xFFFFu)) {
                if (++spins > kPipeSpinG) {
                    give_up();
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
                v = __hip_atomic_load(&P.picks[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            const int j = (int)(v & 0xFFFFu);
            if (j < P.n) atomicOr(&tk[j >> 5], 1u << (j & 31));
        }
        if (need > absorbed) absorbed = need;
        __syncthreads();
        if (fail) return;
        u64 list = c0 < c1 ? wave_top_select(vals, tk, c0, c1, lane, cand[w]) : 0;
        wl[w][lane] = list;
#pragma unroll
        for (int span = 1; span < kPW; span *= 2) {
            __syncthreads();
            if (w % (2 * span) == 0) {
                list = wave_merge_top(list, wl[w + span][lane], lane);
                wl[w][lane] = list;
            }
        }
        if (w == 0) {
            u64 *dst = P.lists + ((size_t)(i % kRingA) * P.Q + q) * kRound;
            __hip_atomic_store(&dst[lane], tag_key(list, (uint32_t)(i + 1) & 0xFFFFu), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();  // wl, cand and tk are reused by the next item
    }
}

// tau and sigma of the real agents from the pick words (after the persistent launch).
__global__ __launch_bounds__(256) void k_picks_to_tau(const uint32_t *picks, int32_t *tau, int32_t *sigma, int rows) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= rows) return;
    const int j = (int)(picks[i] & 0xFFFFu);
    tau[i] = j;
    sigma[j] = i;
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
        best = wave_max64(best);
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
    best = wave_max64(best);
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

static int pipe_parts(int n) { return (n + kPart - 1) / kPart; }

size_t greedy_scratch_bytes(int n) {
    const size_t rounds = (size_t)kRound * 64 * sizeof(u64) + (((size_t)n + 31) / 32) * 4 + 256;
    const size_t pipe = (size_t)kRingA * pipe_parts(n) * kRound * sizeof(u64) + (size_t)n * 4 + 512;
    return rounds > pipe ? rounds : pipe;
}

// The greedy start as one persistent launch (rows <= n <= kPipeMaxN); false when
// the device cannot hold the grid (the caller then runs the rounds).
static bool launch_greedy_pipe(const int32_t *A, int32_t rows, int32_t n, int32_t *tau, int32_t *sigma,
                               void *scratch, int32_t *err, hipStream_t s, hipError_t *e) {
    static int cap = -1;
    if (cap < 0) {
        int dev = 0, cus = 0, per = 0;
        cap = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_greedy_pipe, kPipeT, 0) == hipSuccess)
            cap = cus * per;
    }
    const int Q = pipe_parts(n);
    const long long items = (long long)rows * Q;
    if (cap < 2 || n > kPipeMaxN) return false;
    PipeParams P;
    P.A = A;
    P.lists = (u64 *)scratch;
    uint32_t *pick_words = (uint32_t *)((char *)scratch + (size_t)kRingA * Q * kRound * sizeof(u64));
    P.picks = pick_words + 2;  // picks[-2], picks[-1] are spare slots
    P.progress = (int *)((char *)pick_words + (((size_t)rows * 4 + 8 + 255) & ~(size_t)255));  // within n * 4 + 512
    P.err = err;
    P.rows = rows;
    P.n = n;
    P.Q = Q;
    // a batch is a quarter of the ring at most, so staging runs ahead of the consumer
    P.A_per = kStage / Q < kRingL / 4 ? kStage / Q : kRingL / 4;
    if (P.A_per < 1) P.A_per = 1;
    // tags start at 1: cleared words never match
    if ((*e = launch_fill((int32_t *)P.lists, kRingA * Q * kRound * 2, 0, s)) != hipSuccess) return true;
    if ((*e = launch_fill((int32_t *)pick_words, rows + 2, 0, s)) != hipSuccess) return true;
    if ((*e = launch_fill(P.progress, 1, 0, s)) != hipSuccess) return true;
    if (rows < n && (*e = launch_fill(sigma, n, -1, s)) != hipSuccess) return true;
    const long long grid = 1 + (items < cap - 1 ? items : cap - 1);
    void *args[] = {&P};
    *e = hipLaunchCooperativeKernel((const void *)k_greedy_pipe, dim3((unsigned)grid), dim3(kPipeT), args, 0, s);
    if (*e != hipSuccess) return true;
    hipLaunchKernelGGL(k_picks_to_tau, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, P.picks, tau, sigma, rows);
    if ((*e = hipGetLastError()) == hipSuccess) *e = launch_fill_virtual(tau, sigma, rows, n, s);
    return true;
}

hipError_t launch_greedy_rounds(const int32_t *A, int32_t rows, int32_t n, int32_t *tau, int32_t *sigma,
                                void *scratch, int32_t *err, bool persistent, hipStream_t s) {
    hipError_t pe = hipSuccess;
    if (persistent && launch_greedy_pipe(A, rows, n, tau, sigma, scratch, err, s, &pe)) return pe;
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
