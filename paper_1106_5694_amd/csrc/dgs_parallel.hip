// Parallel DGS (Algorithm 3) on gfx950: each round takes the fresh per-agent
// bests of the difference evaluation, keeps the exchanges that Check
// Conflicts (Algorithm 4) accepts and applies all of them at once.
//
// Check Conflicts is a walk over the agents in index order in which agent i
// (with a positive best, job j_i held by agent i' = sigma(j_i)) is accepted
// unless i or i' was claimed by an agent accepted before it; an accepted
// agent claims both.  The walk is inherently ordered, so it runs in one
// wave: 64 agents at a time out of an LDS stage that the whole workgroup
// fills, the claims of earlier chunks read from an LDS bitmap and the
// conflicts inside a chunk resolved lane by lane with ballots (the lowest
// open candidate is accepted, every later lane that touches its pair drops
// out).  The accepted pairs are disjoint, so the apply kernel swaps them
// without any ordering and each gain is exact.
#include "dgs_device.h"

namespace dgs {
namespace {

using dev::key_gain;

// Agents the claim bitmap covers (32 KiB of LDS).
constexpr int kParMaxAgents = 1 << 18;
constexpr int kClaimThreads = 1024;
// Agents staged in LDS per pass (32 KiB): the whole workgroup loads their
// partners with every load in flight, then one wave walks them.
constexpr int kStage = 8192;
constexpr int kStagePer = kStage / kClaimThreads;

// acc[i] = partner of accepted agent i, else -1; stats[5] = accepted count.
// Nothing is accepted after a range error (flags[0]).
__global__ __launch_bounds__(kClaimThreads) void k_par_claims(const u64 *__restrict__ bk,
                                                              const int32_t *__restrict__ bc, int n,
                                                              int32_t *__restrict__ acc, int64_t *stats,
                                                              const int32_t *flags) {
    __shared__ uint32_t claimed[kParMaxAgents / 32];
    __shared__ int32_t cand[kStage];
    const int t = threadIdx.x, lane = t & 63;
    const int words = (n + 31) >> 5;
    for (int w = t; w < words; w += kClaimThreads) claimed[w] = 0;
    const bool bad = flags[0] != 0;
    auto is_claimed = [&](int x) { return (claimed[x >> 5] >> (x & 31)) & 1u; };
    long long count = 0;
    for (int s0 = 0; s0 < n; s0 += kStage) {
        const int m = min(kStage, n - s0);
        u64 k[kStagePer];
        int32_t c[kStagePer];
#pragma unroll
        for (int u = 0; u < kStagePer; ++u) {
            const int x = t + u * kClaimThreads;
            const int i = x < m ? s0 + x : s0;  // clamped: every load issued, none out of bounds
            k[u] = bk[i];
            c[u] = bc[i];
        }
#pragma unroll
        for (int u = 0; u < kStagePer; ++u) {
            const int x = t + u * kClaimThreads;
            const bool pos = x < m && !bad && k[u] != 0 && key_gain(k[u]) > 0;
            cand[x] = pos ? c[u] : -1;
        }
        __syncthreads();
        if (t < 64) {
            for (int b = 0; b < m; b += 64) {
                const int x = b + lane, i = s0 + x;
                const int p = x < m ? cand[x] : -1;
                if (__ballot(p >= 0) == 0) continue;
                const bool open0 = p >= 0 && !is_claimed(i) && !is_claimed(p);
                u64 open = __ballot(open0);
                bool ok = false;
                while (open) {
                    const int L = __builtin_ctzll(open);
                    const int iL = s0 + b + L;
                    const int pL = __builtin_amdgcn_readlane(p, L);  // L is wave-uniform
                    ok |= lane == L;
                    const bool hit = i == pL || p == iL || p == pL;
                    open &= ~(__ballot(hit) | (1ull << L));
                }
                if (ok) {
                    atomicOr(&claimed[i >> 5], 1u << (i & 31));
                    atomicOr(&claimed[p >> 5], 1u << (p & 31));
                }
                if (x < m) cand[x] = ok ? p : -1;
                count += __popcll(__ballot(ok));
                __threadfence_block();  // this chunk's claims land before the next chunk reads them
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kStagePer; ++u) {
            const int x = t + u * kClaimThreads;
            if (x < m) acc[s0 + x] = cand[x];
        }
        __syncthreads();  // the stage is rewritten by the next pass
    }
    if (t == 0) stats[5] = count;
}

// Check Conflicts for n <= kSmallN, all in LDS and in parallel, with the
// same result as the ordered walk.  A node is an agent; candidate x (an
// agent with a positive best) touches nodes x and p_x.  Each iteration:
// (1) every node takes the lowest undecided candidate touching it; (2) a
// candidate that is the lowest on both of its nodes is accepted and claims
// them -- every earlier candidate touching them is decided and none of
// those was accepted (x would have been rejected), which is exactly the
// walk's condition; (3) an undecided candidate touching a claimed node is
// rejected -- the claimer is earlier, as it was the lowest undecided there.
// The lowest undecided candidate always passes (2), so each iteration
// decides at least one candidate and the loop ends.
constexpr int kSmallN = 16384;
constexpr int kSmallPer = kSmallN / kClaimThreads;

__global__ __launch_bounds__(kClaimThreads) void k_par_claims_small(const u64 *__restrict__ bk,
                                                                    const int32_t *__restrict__ bc, int n,
                                                                    int32_t *__restrict__ acc, int64_t *stats,
                                                                    const int32_t *flags) {
    __shared__ int32_t pv[kSmallN];     // partner of an undecided or accepted candidate, else -1
    __shared__ int32_t first[kSmallN];  // lowest undecided candidate touching the node
    __shared__ uint32_t claimed[kSmallN / 32];
    __shared__ uint32_t accepted[kSmallN / 32];
    __shared__ int s_open[2];  // iteration it reads s_open[it & 1] and clears the other
    const int t = threadIdx.x;
    const bool bad = flags[0] != 0;
    {
        u64 k[kSmallPer];
        int32_t c[kSmallPer];
#pragma unroll
        for (int u = 0; u < kSmallPer; ++u) {
            const int x = t + u * kClaimThreads;
            const int i = x < n ? x : 0;  // clamped: every load issued, none out of bounds
            k[u] = bk[i];
            c[u] = bc[i];
        }
#pragma unroll
        for (int u = 0; u < kSmallPer; ++u) {
            const int x = t + u * kClaimThreads;
            pv[x] = (x < n && !bad && k[u] != 0 && key_gain(k[u]) > 0) ? c[u] : -1;
        }
    }
    for (int w = t; w < kSmallN / 32; w += kClaimThreads) claimed[w] = accepted[w] = 0;
    if (t == 0) s_open[0] = 0;
    auto bit = [](const uint32_t *m, int x) { return (m[x >> 5] >> (x & 31)) & 1u; };
    for (int it = 0; it <= n; ++it) {
#pragma unroll
        for (int u = 0; u < kSmallPer; ++u) first[t + u * kClaimThreads] = 0x7fffffff;
        __syncthreads();
        // every thread has read the flag of the previous iteration
        if (t == 0) s_open[(it + 1) & 1] = 0;
#pragma unroll
        for (int u = 0; u < kSmallPer; ++u) {
            const int x = t + u * kClaimThreads;
            const int p = pv[x];
            if (p >= 0 && !bit(accepted, x)) {
                atomicMin(&first[x], x);
                atomicMin(&first[p], x);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kSmallPer; ++u) {
            const int x = t + u * kClaimThreads;
            const int p = pv[x];
            if (p >= 0 && !bit(accepted, x) && first[x] == x && first[p] == x) {
                atomicOr(&accepted[x >> 5], 1u << (x & 31));
                atomicOr(&claimed[x >> 5], 1u << (x & 31));
                atomicOr(&claimed[p >> 5], 1u << (p & 31));
            }
        }
        __syncthreads();
        int open = 0;
#pragma unroll
        for (int u = 0; u < kSmallPer; ++u) {
            const int x = t + u * kClaimThreads;
            const int p = pv[x];
            if (p >= 0 && !bit(accepted, x)) {
                if (bit(claimed, x) || bit(claimed, p))
                    pv[x] = -1;
                else
                    open = 1;
            }
        }
        if (open) s_open[it & 1] = 1;
        __syncthreads();
        if (s_open[it & 1] == 0) break;
    }
    long long count = 0;
#pragma unroll
    for (int u = 0; u < kSmallPer; ++u) {
        const int x = t + u * kClaimThreads;
        if (x < n) {
            const bool ok = pv[x] >= 0 && bit(accepted, x);
            acc[x] = ok ? pv[x] : -1;
            count += ok;
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) count += __shfl_xor(count, m, 64);
    __syncthreads();
    if ((t & 63) == 0) first[t >> 6] = (int)count;
    __syncthreads();
    if (t == 0) {
        long long total = 0;
        for (int w = 0; w < kClaimThreads / 64; ++w) total += first[w];
        stats[5] = total;
    }
}

// Swap the jobs of every accepted pair (disjoint pairs: no ordering
// needed); stats[0] += accepted, stats[1] += their gains.
__global__ __launch_bounds__(256) void k_par_apply(const int32_t *__restrict__ acc, const u64 *__restrict__ bk, int n,
                                                   int32_t *tau, int32_t *sigma, int64_t *stats) {
    __shared__ long long part[4][2];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int p = i < n ? acc[i] : -1;
    long long g = 0, c = 0;
    if (p >= 0) {
        const int ti = tau[i], tp = tau[p];
        tau[i] = tp;
        tau[p] = ti;
        sigma[tp] = i;
        sigma[ti] = p;
        g = key_gain(bk[i]);
        c = 1;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        g += __shfl_xor(g, m, 64);
        c += __shfl_xor(c, m, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        part[threadIdx.x >> 6][0] = c;
        part[threadIdx.x >> 6][1] = g;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long cs = part[0][0] + part[1][0] + part[2][0] + part[3][0];
        if (cs) {
            atomicAdd((unsigned long long *)&stats[0], (unsigned long long)cs);
            atomicAdd((unsigned long long *)&stats[1],
                      (unsigned long long)(part[0][1] + part[1][1] + part[2][1] + part[3][1]));
        }
    }
}

}  // namespace

int parallel_max_agents() { return kParMaxAgents; }

hipError_t launch_parallel_round(const Instance &I, int32_t *acc, hipStream_t s) {
    if (I.n <= kSmallN)
        hipLaunchKernelGGL(k_par_claims_small, dim3(1), dim3(kClaimThreads), 0, s, (const u64 *)I.bk,
                           (const int32_t *)I.bc, I.n, acc, I.stats, (const int32_t *)I.flags);
    else
        hipLaunchKernelGGL(k_par_claims, dim3(1), dim3(kClaimThreads), 0, s, (const u64 *)I.bk,
                           (const int32_t *)I.bc, I.n, acc, I.stats, (const int32_t *)I.flags);
    hipLaunchKernelGGL(k_par_apply, dim3((unsigned)((I.n + 255) / 256)), dim3(256), 0, s, (const int32_t *)acc,
                       (const u64 *)I.bk, I.n, I.tau, I.sigma, I.stats);
    return hipGetLastError();
}

}  // namespace dgs
