// Parallel DGS (Algorithm 3) on gfx950: each round takes the fresh per-agent
// bests of the difference evaluation, keeps the exchanges that Check
// Conflicts (Algorithm 4) accepts and applies all of them at once.
//
// Check Conflicts is a walk over the agents in index order in which agent i
// (with a positive best, job j_i held by agent i' = sigma(j_i)) is accepted
// unless i or i' was claimed by an agent accepted before it; an accepted
// agent claims both.  The walk is inherently ordered, so it runs in one
// wave: 64 agents at a time, the claims of earlier chunks read from an LDS
// bitmap and the conflicts inside a chunk resolved lane by lane with
// ballots (the lowest open candidate is accepted, every later lane that
// touches its pair drops out).  The accepted pairs are disjoint, so the
// apply kernel swaps them without any ordering and each gain is exact.
#include "dgs_device.h"

namespace dgs {
namespace {

using dev::key_gain;

// Agents the claim bitmap covers (32 KiB of LDS).
constexpr int kParMaxAgents = 1 << 18;

// acc[i] = partner of accepted agent i, else -1.  stats[0] += accepted,
// stats[1] += their gains, stats[5] = accepted.  Nothing is accepted after
// a range error (flags[0]).
__global__ __launch_bounds__(64) void k_par_claims(const u64 *__restrict__ bk, const int32_t *__restrict__ bc, int n,
                                                   int32_t *__restrict__ acc, int64_t *stats,
                                                   const int32_t *flags) {
    __shared__ uint32_t claimed[kParMaxAgents / 32];
    const int lane = threadIdx.x;
    const int words = (n + 31) >> 5;
    for (int w = lane; w < words; w += 64) claimed[w] = 0;
    __syncthreads();
    const bool bad = flags[0] != 0;
    auto is_claimed = [&](int x) { return (claimed[x >> 5] >> (x & 31)) & 1u; };
    long long count = 0, gains = 0;
    for (int base = 0; base < n; base += 64) {
        const int i = base + lane;
        int p = -1;
        long long g = 0;
        if (i < n && !bad) {
            const u64 k = bk[i];
            if (k != 0 && key_gain(k) > 0) {
                p = bc[i];
                g = key_gain(k);
            }
        }
        const bool cand = p >= 0 && !is_claimed(i) && !is_claimed(p);
        u64 open = __ballot(cand);
        bool ok = false;
        while (open) {
            const int L = __builtin_ctzll(open);
            const int iL = base + L;
            const int pL = __shfl(p, L, 64);
            ok |= lane == L;
            const bool hit = i == pL || p == iL || p == pL;
            open &= ~(__ballot(hit) | (1ull << L));
        }
        if (ok) {
            atomicOr(&claimed[i >> 5], 1u << (i & 31));
            atomicOr(&claimed[p >> 5], 1u << (p & 31));
        }
        if (i < n) acc[i] = ok ? p : -1;
        const u64 okm = __ballot(ok);
        count += __popcll(okm);
        long long s = ok ? g : 0;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
        gains += s;
        __syncthreads();  // the claims of this chunk before the next chunk reads them
    }
    if (lane == 0) {
        stats[0] += count;
        stats[1] += gains;
        stats[5] = count;
    }
}

// Swap the jobs of every accepted pair (disjoint pairs: no ordering needed).
__global__ __launch_bounds__(256) void k_par_apply(const int32_t *__restrict__ acc, int n, int32_t *tau,
                                                   int32_t *sigma) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int p = acc[i];
    if (p < 0) return;
    const int ti = tau[i], tp = tau[p];
    tau[i] = tp;
    tau[p] = ti;
    sigma[tp] = i;
    sigma[ti] = p;
}

}  // namespace

int parallel_max_agents() { return kParMaxAgents; }

hipError_t launch_parallel_round(const Instance &I, int32_t *acc, hipStream_t s) {
    hipLaunchKernelGGL(k_par_claims, dim3(1), dim3(64), 0, s, (const u64 *)I.bk, (const int32_t *)I.bc, I.n, acc,
                       I.stats, (const int32_t *)I.flags);
    hipLaunchKernelGGL(k_par_apply, dim3((unsigned)((I.n + 255) / 256)), dim3(256), 0, s, (const int32_t *)acc,
                       I.n, I.tau, I.sigma);
    return hipGetLastError();
}

}  // namespace dgs
