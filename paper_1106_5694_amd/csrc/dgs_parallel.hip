// Parallel DGS (Algorithm 3) on gfx950: each round takes the fresh
// evaluation of every agent (best exchange keyed by job, ADE) and of every
// job (best agent to take it, JDE), keeps the exchanges that Check Conflicts
// (Algorithm 4) lets through and applies all of them at once.
//
// Check Conflicts walks the agents with a positive best in index order, then
// the jobs with a positive best in index order.  Every exchange involves two
// agents: agent i and the owner sigma(j_i) of i's best job, or for job j its
// best agent i_j and its owner sigma(j).  An exchange is kept unless one of
// its two agents was claimed by an exchange kept before it; a kept exchange
// claims both.  The kept exchanges are disjoint, so the apply kernel swaps
// them without any ordering and each gain is exact.
//
// The result of a round is encoded per agent in acc: -1 (nothing), p (agent
// exchange of this agent with partner p; gain from its ADE key) or
// p | kJobFlag (this agent takes the job of owner p; gain from the JDE key
// stored for p, the job's owner).
#include "dgs_device.h"

namespace dgs {
namespace {

using dev::key_gain;
using dev::key_index;

// Agents the claim bitmap covers (32 KiB of LDS).
constexpr int kParMaxAgents = 1 << 18;
constexpr int kJobFlag = 1 << 30;
constexpr int kClaimThreads = 1024;
// Candidates staged in LDS per pass (two 32 KiB arrays): the whole
// workgroup loads their nodes with every load in flight, then one wave
// walks them.
constexpr int kStage = 8192;
constexpr int kStagePer = kStage / kClaimThreads;

__device__ __forceinline__ bool positive(u64 k) { return k != 0 && key_gain(k) > 0; }

// The ordered walk for n > kSmallN.  Lane x of the walking wave holds
// candidate (u, v) (u < 0: none); the lowest open lane is kept, every later
// lane that touches u or v of it drops out.  Returns the lanes kept.
__device__ __forceinline__ bool walk_chunk(uint32_t *claimed, int u, int v, int lane) {
    auto is_claimed = [&](int x) { return (claimed[x >> 5] >> (x & 31)) & 1u; };
    const bool open0 = u >= 0 && !is_claimed(u) && !is_claimed(v);
    u64 open = __ballot(open0);
    bool ok = false;
    while (open) {
        const int L = __builtin_ctzll(open);
        const int uL = __builtin_amdgcn_readlane(u, L);  // L is wave-uniform
        const int vL = __builtin_amdgcn_readlane(v, L);
        ok |= lane == L;
        const bool hit = u == uL || u == vL || v == uL || v == vL;
        open &= ~(__ballot(hit) | (1ull << L));
    }
    if (ok) {
        atomicOr(&claimed[u >> 5], 1u << (u & 31));
        atomicOr(&claimed[v >> 5], 1u << (v & 31));
    }
    __threadfence_block();  // this chunk's claims land before the next chunk reads them
    return ok;
}

// Nothing is kept after a range error (flags[0]).
__global__ __launch_bounds__(kClaimThreads) void k_par_claims(const u64 *__restrict__ bk,
                                                              const int32_t *__restrict__ bc,
                                                              const u64 *__restrict__ jde,
                                                              const int32_t *__restrict__ sigma, int n,
                                                              int32_t *__restrict__ acc, int64_t *stats,
                                                              const int32_t *flags) {
    __shared__ uint32_t claimed[kParMaxAgents / 32];
    __shared__ int32_t cu[kStage], cv[kStage];
    const int t = threadIdx.x, lane = t & 63;
    const int words = (n + 31) >> 5;
    for (int w = t; w < words; w += kClaimThreads) claimed[w] = 0;
    const bool bad = flags[0] != 0;
    long long count = 0;
    // phase 0: agents in index order (u = i, v = sigma(j_i)); phase 1: jobs in
    // index order (u = sigma(j), v = i_j)
#pragma unroll 1
    for (int phase = 0; phase < 2; ++phase) {
        for (int s0 = 0; s0 < n; s0 += kStage) {
            const int m = min(kStage, n - s0);
            if (phase == 0) {
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
                    const bool pos = x < m && !bad && positive(k[u]);
                    cu[x] = pos ? s0 + x : -1;
                    cv[x] = pos ? c[u] : -1;
                }
            } else {
                int32_t o[kStagePer];
                u64 k[kStagePer];
#pragma unroll
                for (int u = 0; u < kStagePer; ++u) {
                    const int x = t + u * kClaimThreads;
                    o[u] = sigma[x < m ? s0 + x : s0];
                }
#pragma unroll
                for (int u = 0; u < kStagePer; ++u) k[u] = jde[o[u]];
#pragma unroll
                for (int u = 0; u < kStagePer; ++u) {
                    const int x = t + u * kClaimThreads;
                    const bool pos = x < m && !bad && positive(k[u]);
                    cu[x] = pos ? o[u] : -1;
                    cv[x] = pos ? key_index(k[u]) : -1;
                }
            }
            __syncthreads();
            if (t < 64) {
                for (int b = 0; b < m; b += 64) {
                    const int x = b + lane;
                    const int u = x < m ? cu[x] : -1, v = x < m ? cv[x] : -1;
                    if (__ballot(u >= 0) == 0) continue;
                    const bool ok = walk_chunk(claimed, u, v, lane);
                    if (x < m) cu[x] = ok ? u : -1;
                    count += __popcll(__ballot(ok));
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kStagePer; ++u) {
                const int x = t + u * kClaimThreads;
                if (x < m) {
                    if (phase == 0)
                        acc[s0 + x] = cu[x] >= 0 ? cv[x] : -1;
                    else if (cu[x] >= 0)
                        acc[cv[x]] = cu[x] | kJobFlag;  // this agent was free: no agent exchange wrote it
                }
            }
            __syncthreads();  // the stage is rewritten by the next pass; phase 1 writes after phase 0
        }
    }
    if (t == 0) stats[5] = count;
}

// Check Conflicts for n <= kSmallN, all in LDS and in parallel, with the
// same result as the ordered walk, one phase at a time (agents, then jobs).
// Candidate c of a phase touches two nodes (agents) u_c and v_c.  Each
// iteration: (1) an undecided candidate touching a claimed node is rejected;
// (2) every node takes the lowest undecided candidate touching it; (3) a
// candidate that is the lowest on both of its nodes is kept and claims them.
// A candidate kept in (3) has every earlier candidate touching its nodes
// decided and none of those kept (it would have been rejected in (1)), which
// is exactly the walk's condition; a rejection in (1) comes from a kept
// candidate that is earlier (it was the lowest undecided on that node), or
// from the agent phase.  The lowest undecided candidate always passes (3),
// so each iteration decides at least one candidate and the loop ends.
constexpr int kSmallN = 16384;
constexpr int kSmallPer = kSmallN / kClaimThreads;

__global__ __launch_bounds__(kClaimThreads) void k_par_claims_small(const u64 *__restrict__ bk,
                                                                    const int32_t *__restrict__ bc,
                                                                    const u64 *__restrict__ jde,
                                                                    const int32_t *__restrict__ sigma, int n,
                                                                    int32_t *__restrict__ acc, int64_t *stats,
                                                                    const int32_t *flags) {
    // candidate c: nodes (u, v) packed as u | v << 16 (n <= 2^14), -1 when
    // none or rejected
    __shared__ int32_t pv[kSmallN];
    __shared__ int32_t first[kSmallN];  // lowest undecided candidate touching the node
    __shared__ uint32_t claimed[kSmallN / 32];
    __shared__ uint32_t kept[kSmallN / 32];
    __shared__ int s_open[2];  // iteration it reads s_open[it & 1] and clears the other
    __shared__ long long s_count[kClaimThreads / 64];
    const int t = threadIdx.x;
    const bool bad = flags[0] != 0;
    auto bit = [](const uint32_t *m, int x) { return (m[x >> 5] >> (x & 31)) & 1u; };
    for (int w = t; w < kSmallN / 32; w += kClaimThreads) claimed[w] = 0;
    long long count = 0;
#pragma unroll 1
    for (int phase = 0; phase < 2; ++phase) {
        // stage the phase's candidates, half of a thread's entries at a time
        // (every load of a half in flight at once)
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            constexpr int H = kSmallPer / 2;
            u64 k[H];
            int32_t c[H];
            if (phase == 0) {
#pragma unroll
                for (int u = 0; u < H; ++u) {
                    const int x = t + (h * H + u) * kClaimThreads;
                    const int i = x < n ? x : 0;  // clamped: every load issued, none out of bounds
                    k[u] = bk[i];
                    c[u] = bc[i];
                }
#pragma unroll
                for (int u = 0; u < H; ++u) {
                    const int x = t + (h * H + u) * kClaimThreads;
                    pv[x] = (x < n && !bad && positive(k[u])) ? (x | c[u] << 16) : -1;
                }
            } else {
#pragma unroll
                for (int u = 0; u < H; ++u) {
                    const int x = t + (h * H + u) * kClaimThreads;
                    c[u] = sigma[x < n ? x : 0];
                }
#pragma unroll
                for (int u = 0; u < H; ++u) k[u] = jde[c[u]];
#pragma unroll
                for (int u = 0; u < H; ++u) {
                    const int x = t + (h * H + u) * kClaimThreads;
                    pv[x] = (x < n && !bad && positive(k[u])) ? (c[u] | key_index(k[u]) << 16) : -1;
                }
            }
        }
        for (int w = t; w < kSmallN / 32; w += kClaimThreads) kept[w] = 0;
        if (t == 0) s_open[0] = 0;
        __syncthreads();
#pragma unroll 1
        for (int it = 0; it <= n; ++it) {
            // (1) reject what touches a claimed node
            int open = 0;
#pragma unroll
            for (int u = 0; u < kSmallPer; ++u) {
                const int x = t + u * kClaimThreads;
                const int p = pv[x];
                if (p >= 0 && !bit(kept, x)) {
                    if (bit(claimed, p & 0xFFFF) || bit(claimed, p >> 16))
                        pv[x] = -1;
                    else
                        open = 1;
                }
                first[x] = 0x7fffffff;
            }
            if (open) s_open[it & 1] = 1;
            __syncthreads();
            if (s_open[it & 1] == 0) break;
            // every thread has read the flag of this iteration
            if (t == 0) s_open[(it + 1) & 1] = 0;
            // (2) lowest undecided candidate per node
#pragma unroll
            for (int u = 0; u < kSmallPer; ++u) {
                const int x = t + u * kClaimThreads;
                const int p = pv[x];
                if (p >= 0 && !bit(kept, x)) {
                    atomicMin(&first[p & 0xFFFF], x);
                    atomicMin(&first[p >> 16], x);
                }
            }
            __syncthreads();
            // (3) keep the candidates lowest on both nodes
#pragma unroll
            for (int u = 0; u < kSmallPer; ++u) {
                const int x = t + u * kClaimThreads;
                const int p = pv[x];
                if (p >= 0 && !bit(kept, x) && first[p & 0xFFFF] == x && first[p >> 16] == x) {
                    atomicOr(&kept[x >> 5], 1u << (x & 31));
                    atomicOr(&claimed[(p & 0xFFFF) >> 5], 1u << (p & 31));
                    atomicOr(&claimed[(p >> 16) >> 5], 1u << ((p >> 16) & 31));
                }
            }
            __syncthreads();
        }
        // outputs of the phase (phase 1 writes only agents no exchange of phase 0 holds)
#pragma unroll
        for (int u = 0; u < kSmallPer; ++u) {
            const int x = t + u * kClaimThreads;
            if (x < n) {
                const int p = pv[x];
                const bool ok = p >= 0 && bit(kept, x);
                if (phase == 0)
                    acc[x] = ok ? p >> 16 : -1;
                else if (ok)
                    acc[p >> 16] = (p & 0xFFFF) | kJobFlag;
                count += ok;
            }
        }
        __syncthreads();  // pv, kept and first are rewritten by the next phase
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) count += __shfl_xor(count, m, 64);
    if ((t & 63) == 0) s_count[t >> 6] = count;
    __syncthreads();
    if (t == 0) {
        long long total = 0;
        for (int w = 0; w < kClaimThreads / 64; ++w) total += s_count[w];
        stats[5] = total;
    }
}

// Swap the jobs of every kept pair (disjoint pairs: no ordering needed);
// stats[0] += kept, stats[1] += their gains.
__global__ __launch_bounds__(256) void k_par_apply(const int32_t *__restrict__ acc, const u64 *__restrict__ bk,
                                                   const u64 *__restrict__ jde, int n, int32_t *tau, int32_t *sigma,
                                                   int64_t *stats) {
    __shared__ long long part[4][2];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int a = i < n ? acc[i] : -1;
    long long g = 0, c = 0;
    if (a >= 0) {
        const int p = a & (kJobFlag - 1);
        const int ti = tau[i], tp = tau[p];
        tau[i] = tp;
        tau[p] = ti;
        sigma[tp] = i;
        sigma[ti] = p;
        g = key_gain((a & kJobFlag) ? jde[p] : bk[i]);
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
                           (const int32_t *)I.bc, (const u64 *)I.bb, (const int32_t *)I.sigma, I.n, acc, I.stats,
                           (const int32_t *)I.flags);
    else
        hipLaunchKernelGGL(k_par_claims, dim3(1), dim3(kClaimThreads), 0, s, (const u64 *)I.bk,
                           (const int32_t *)I.bc, (const u64 *)I.bb, (const int32_t *)I.sigma, I.n, acc, I.stats,
                           (const int32_t *)I.flags);
    hipLaunchKernelGGL(k_par_apply, dim3((unsigned)((I.n + 255) / 256)), dim3(256), 0, s, (const int32_t *)acc,
                       (const u64 *)I.bk, (const u64 *)I.bb, I.n, I.tau, I.sigma, I.stats);
    return hipGetLastError();
}

}  // namespace dgs
