// Greedy start of DGS on gfx950 (Section 3.1): agents 0..n-1 in order, each
// takes its free job of largest benefit, lowest job index on ties.
//
// The sequential dependency is kept exactly, in rounds of kRound agents:
//   1. k_greedy_topk: for every agent of the round and every chunk of
//      columns, the kRound best keys (benefit, job) among the jobs free at
//      the start of the round (wave64 bitonic sort / merge in registers);
//   2. k_greedy_resolve: one wave walks the round's agents in order; an
//      agent takes, over its chunk lists, the best key whose job is still
//      free.  At most kRound - 1 jobs are taken inside a round, so no chunk
//      list of kRound keys runs out of free entries: the first free entry of
//      a chunk list is the chunk's best free job, and the best over chunks is
//      the agent's greedy choice.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgs_device.h"
#include "dgs_internal.h"

namespace dgs {
namespace {

using namespace dev;

constexpr int kRound = 64;    // agents per round = list length = wave size
constexpr int kTopkBlock = 256;  // 4 waves per (agent, chunk)
constexpr int kMaxChunks = 4;

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

struct TopkParams {
    const int32_t *A;
    const uint32_t *taken;  // bitmap of jobs taken before this round
    u64 *lists;             // [kRound][chunks][64]
    int n;
    int row0;      // first agent of the round
    int rows;      // agents in this round (<= kRound)
    int chunk;     // columns per chunk (multiple of 256)
    int chunks;
};

__global__ __launch_bounds__(kTopkBlock) void k_greedy_topk(TopkParams P) {
    __shared__ u64 wl[kTopkBlock / 64][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = blockIdx.x, ri = blockIdx.y;
    const int row = P.row0 + ri;
    const int32_t *Ar = P.A + (int64_t)row * P.n;
    // columns of this chunk, split evenly over the 4 waves in whole batches of 64
    const int cbeg = p * P.chunk;
    const int ccnt = min(P.chunk, P.n - cbeg);
    const int sub = ((ccnt + 4 * 64 - 1) / (4 * 64)) * 64;  // columns per wave
    const int c0 = cbeg + w * sub;
    const int c1 = min(cbeg + ccnt, c0 + sub);
    u64 list = 0, lmin = 0;
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
    wl[w][lane] = list;
    __syncthreads();
    if (w == 0) {
        u64 v = wl[0][lane];
#pragma unroll
        for (int x = 1; x < kTopkBlock / 64; ++x) v = wave_merge_top(v, wl[x][lane], lane);
        P.lists[((size_t)ri * P.chunks + p) * 64 + lane] = v;
    }
}

struct ResolveParams {
    const u64 *lists;
    uint32_t *taken;
    int32_t *tau;
    int32_t *sigma;
    int32_t *err;
    int n;
    int row0;
    int rows;
    int chunks;
};

// One workgroup: stage the round's lists and the taken bitmap in LDS, then
// wave 0 resolves the agents in order; the choices are written out at the end.
__global__ __launch_bounds__(256) void k_greedy_resolve(ResolveParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int pick[kRound];
    u64 *L = (u64 *)smem;                                                   // rows * chunks * 64
    uint32_t *tk = (uint32_t *)(smem + (size_t)P.rows * P.chunks * 64 * 8);  // n / 32 words
    const int words = (P.n + 31) >> 5;
    const int total = P.rows * P.chunks * 64;
    // stage the lists: 16-byte loads, eight in flight per thread (total is a multiple of 64)
    {
        const int4 *src = (const int4 *)P.lists;
        int4 *dst = (int4 *)L;
        const int total4 = total / 2;
        for (int base = threadIdx.x; base < total4; base += 8 * blockDim.x) {
            int4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = base + u * blockDim.x;
                if (i < total4) v[u] = src[i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = base + u * blockDim.x;
                if (i < total4) dst[i] = v[u];
            }
        }
    }
    for (int i = threadIdx.x; i < words; i += blockDim.x) tk[i] = P.taken[i];
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int chunks = P.chunks;
        // the lists of agent ri + 1 are read while agent ri is resolved
        u64 nxt[kMaxChunks];
#pragma unroll
        for (int p = 0; p < kMaxChunks; ++p) nxt[p] = p < chunks ? L[(size_t)p * 64 + lane] : 0;
        int my_pick = -1;  // lane ri keeps agent ri's choice
        for (int ri = 0; ri < P.rows; ++ri) {
            u64 cur[kMaxChunks];
#pragma unroll
            for (int p = 0; p < kMaxChunks; ++p) cur[p] = nxt[p];
            if (ri + 1 < P.rows) {
#pragma unroll
                for (int p = 0; p < kMaxChunks; ++p)
                    nxt[p] = p < chunks ? L[((size_t)(ri + 1) * chunks + p) * 64 + lane] : 0;
            }
            uint32_t word[kMaxChunks];
#pragma unroll
            for (int p = 0; p < kMaxChunks; ++p) {
                const int c = cur[p] ? key_index(cur[p]) : 0;
                word[p] = tk[c >> 5];
            }
            u64 best = 0;
#pragma unroll
            for (int p = 0; p < kMaxChunks; ++p) {
                const int c = cur[p] ? key_index(cur[p]) : 0;
                const bool fr = cur[p] != 0 && !((word[p] >> (c & 31)) & 1u);
                const unsigned long long m = __ballot(fr);
                if (m) best = kmax(best, readlane64(cur[p], __ffsll((long long)m) - 1));
            }
            if (best == 0) {  // cannot happen (see above); never index with it
                if (lane == 0) atomicOr(P.err, 4);
                continue;
            }
            const int c = key_index(best);
            if (lane == 0) atomicOr(&tk[c >> 5], 1u << (c & 31));
            if (lane == ri) my_pick = c;
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

}  // namespace

size_t greedy_chunk_cols(int n) {
    // at most kMaxChunks chunks; each chunk a multiple of the workgroup's 256 columns
    size_t c = 4096;
    while ((size_t)kMaxChunks * c < (size_t)n) c *= 2;
    return c;
}

size_t greedy_scratch_bytes(int n) {
    const size_t chunks = ((size_t)n + greedy_chunk_cols(n) - 1) / greedy_chunk_cols(n);
    return (size_t)kRound * chunks * 64 * sizeof(u64) + (((size_t)n + 31) / 32) * 4 + 256;
}

hipError_t launch_greedy_rounds(const int32_t *A, int32_t n, int32_t *tau, int32_t *sigma, void *scratch,
                                int32_t *err, hipStream_t s) {
    const int chunk = (int)greedy_chunk_cols(n);
    const int chunks = (n + chunk - 1) / chunk;
    u64 *lists = (u64 *)scratch;
    uint32_t *taken = (uint32_t *)((char *)scratch + (size_t)kRound * chunks * 64 * sizeof(u64));
    const int words = (n + 31) / 32;
    hipError_t e = hipMemsetAsync(taken, 0, (size_t)words * 4, s);
    if (e != hipSuccess) return e;
    const size_t rshm = (size_t)kRound * chunks * 64 * sizeof(u64) + (size_t)words * 4;
    e = hipFuncSetAttribute((const void *)k_greedy_resolve, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rshm);
    if (e != hipSuccess) return e;
    for (int row0 = 0; row0 < n; row0 += kRound) {
        const int rows = n - row0 < kRound ? n - row0 : kRound;
        TopkParams T{A, taken, lists, n, row0, rows, chunk, chunks};
        hipLaunchKernelGGL(k_greedy_topk, dim3((unsigned)chunks, (unsigned)rows), dim3(kTopkBlock), 0, s, T);
        ResolveParams R{lists, taken, tau, sigma, err, n, row0, rows, chunks};
        const size_t shm = (size_t)rows * chunks * 64 * sizeof(u64) + (size_t)words * 4;
        hipLaunchKernelGGL(k_greedy_resolve, dim3(1), dim3(256), shm, s, R);
    }
    return hipGetLastError();
}

}  // namespace dgs
