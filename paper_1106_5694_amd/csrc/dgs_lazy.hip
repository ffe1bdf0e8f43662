// Lazy DGS, Algorithm 1 as printed, on gfx950: the switching phase of one
// pass in one workgroup.
//
// The pass starts from a full evaluation of every agent (ADE: best job,
// lowest job on ties) and every job (JDE: best agent to take it, lowest
// agent on ties), computed by the tile-pair evaluation.  Only positive
// improvements are stored.  Then, while a stored improvement is positive:
// the agent i* and the job j* with the largest stored values (lowest index
// on ties) are found; i*'s stored exchange is followed if its value is
// strictly larger than j*'s, else j*'s; the value followed is zeroed; the
// exchange is applied only if it raises f, and then the two agents and the
// two jobs it involves are evaluated afresh.  Other stored values stay as
// they were (stale).
//
// Layout: one workgroup of 1024 threads.  The stored improvements of all
// agents and jobs sit in LDS (2 x 64 KiB for n <= 16384), where one thread
// can update any entry; the stored partners (a job for an agent, an agent
// for a job) sit in global memory, read once per attempt.  An applied
// exchange (agent i takes job j from agent c, c takes i's old job t0) is
// re-evaluated in one pass over every partner e: after the switch the four
// scans share their terms, g_i(e) = a[i][tau(e)] + a[e][j] - d(i) - d(e)
// serves agent i (keyed by job tau(e)) and job j (owner i, keyed by agent
// e), and g_c(e) likewise serves agent c and job t0.  All waves of the
// workgroup share one CU and its L1, so global writes are visible to the
// workgroup after a barrier.
#include "dgs_device.h"

namespace dgs {
namespace {

using namespace dev;

constexpr int kLazyThreads = 1024;
constexpr int kLazyWaves = kLazyThreads / 64;
constexpr int kLazyPer = 16;  // stored entries per thread and side
static_assert(kLazyThreads * kLazyPer == kLazyMaxN, "lazy layout");

struct LazyParams {
    const int32_t *A;
    const int32_t *AT;
    int32_t *tau;
    int32_t *sigma;
    int32_t *d;
    const u64 *ade;  // per agent: best key (gain, job) of the pass's evaluation
    const u64 *jde;  // per agent c: best key (gain, agent) over agents taking c's job
    int64_t *stats;  // [0] switches, [1] gain sum, [5] switches of this pass, [7] attempts
    int32_t *ja;     // stored job of each agent
    int32_t *ij;     // stored agent of each job
    const int32_t *flags;
    int32_t *err;
    int n;
    int64_t max_switches;
};

__device__ __forceinline__ u64 wave_max64(u64 v) {
    v = umax64(v, xor_lanes64<32>(v));
    v = umax64(v, xor_lanes64<16>(v));
    v = umax64(v, xor_lanes64<8>(v));
    v = umax64(v, xor_lanes64<4>(v));
    v = umax64(v, xor_lanes64<2>(v));
    return umax64(v, xor_lanes64<1>(v));
}

// Partners of one re-evaluation loaded together.
constexpr int kEvalChunk = 8;
static_assert(kLazyPer % kEvalChunk == 0, "chunks");
// A row of A is staged in LDS in stretches of kStageInts entries (32 KiB,
// the LDS left beside the stored values), so that the re-evaluation's reads
// a[i][tau(e)] gather from LDS instead of sending one request per entry.
constexpr int kStageInts = 8192;
constexpr int kStagePer = kStageInts / kLazyThreads;
static_assert(6 * kLazyWaves * 8 <= kStageInts * 4, "maxima fit in the stage");

__global__ __launch_bounds__(kLazyThreads) void k_lazy_pass(LazyParams P) {
    __shared__ int32_t ga[kLazyMaxN];  // stored improvement of each agent (0: none)
    __shared__ int32_t gj[kLazyMaxN];  // stored improvement of each job (0: none)
    // a stretch of a row of A for the re-evaluation's gathered reads; the
    // argmax's and the re-evaluation's per-wave maxima share its first bytes
    // (never in use at the same time: barriers separate the phases)
    __shared__ __align__(16) int32_t stage[kStageInts];
    u64(*wk)[kLazyWaves] = (u64(*)[kLazyWaves])stage;        // [2][waves]: stored agent / job keys
    u64(*rk)[kLazyWaves] = (u64(*)[kLazyWaves])stage + 2;    // [4][waves]: the four re-evaluations
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int n = P.n;
    const bool bad = P.flags[0] != 0;
    for (int x = t; x < kLazyMaxN; x += kLazyThreads) {
        int g1 = 0, g2 = 0;
        if (x < n && !bad) {
            const u64 k = P.ade[x];
            if (k != 0 && key_gain(k) > 0) {
                g1 = key_gain(k);
                P.ja[x] = key_index(k);
            }
            const u64 q = P.jde[P.sigma[x]];
            if (q != 0 && key_gain(q) > 0) {
                g2 = key_gain(q);
                P.ij[x] = key_index(q);
            }
        }
        ga[x] = g1;
        gj[x] = g2;
    }
    __syncthreads();
    const long long s0 = P.stats[0];
    long long applied = 0, attempts = 0, gains = 0;
    for (;;) {
        if (P.max_switches >= 0 && s0 + applied >= P.max_switches) break;
        // every attempt zeroes one positive value and an applied switch sets at
        // most four: more attempts than this means a broken invariant
        if (attempts > 2LL * n + 4 * applied + 16) {
            if (t == 0) *P.err = 3;
            break;
        }
        u64 ka = 0, kj = 0;
#pragma unroll 4
        for (int s = 0; s < kLazyPer; ++s) {
            const int x = t + s * kLazyThreads;
            const int a = ga[x], b = gj[x];
            if (a > 0) ka = umax64(ka, mk_key(a, x));
            if (b > 0) kj = umax64(kj, mk_key(b, x));
        }
        ka = wave_max64(ka);
        kj = wave_max64(kj);
        if (lane == 0) {
            wk[0][w] = ka;
            wk[1][w] = kj;
        }
        __syncthreads();
        u64 KA = 0, KJ = 0;
#pragma unroll
        for (int v = 0; v < kLazyWaves; ++v) {
            KA = umax64(KA, wk[0][v]);
            KJ = umax64(KJ, wk[1][v]);
        }
        if (KA == 0 && KJ == 0) break;  // no positive stored value left
        const bool by_agent = (KA ? key_gain(KA) : 0) > (KJ ? key_gain(KJ) : 0);
        const int e = key_index(by_agent ? KA : KJ);
        const int i = by_agent ? e : P.ij[e];
        const int j = by_agent ? P.ja[e] : e;
        ++attempts;
        const int c = P.sigma[j], t0 = P.tau[i];
        const int ai = P.A[(size_t)i * n + j], ac = P.A[(size_t)c * n + t0];
        const int gain = c != i ? (ai + ac) - (P.d[i] + P.d[c]) : 0;
        __syncthreads();  // every thread has read wk, tau, sigma and d
        if (t == 0) {
            if (by_agent)
                ga[e] = 0;
            else
                gj[e] = 0;
        }
        if (gain <= 0) {  // the guard: f would not rise
            __syncthreads();
            continue;
        }
        if (t == 0) {
            P.tau[i] = j;
            P.tau[c] = t0;
            P.sigma[j] = i;
            P.sigma[t0] = c;
            P.d[i] = ai;
            P.d[c] = ac;
        }
        ++applied;
        gains += gain;
        __syncthreads();  // the switch is visible to the workgroup
        u64 kai = 0, kac = 0, kjj = 0, kjt = 0;
        // partners e = t + 1024 s, in two halves of kEvalChunk per thread
#pragma nounroll
        for (int s0c = 0; s0c < kLazyPer; s0c += kEvalChunk) {
            int te[kEvalChunk];  // jobs after the switch
#pragma unroll
            for (int u = 0; u < kEvalChunk; ++u) {
                const int x = t + (s0c + u) * kLazyThreads;
                te[u] = P.tau[x < n ? x : 0];  // clamped: every load issued, none out of bounds
            }
#pragma nounroll
            for (int side = 0; side < 2; ++side) {
                const int r = side == 0 ? i : c;  // row of A read through tau
                int va[kEvalChunk];                // a[r][tau(e)], gathered from LDS stretch by stretch
#pragma unroll
                for (int u = 0; u < kEvalChunk; ++u) va[u] = 0;
#pragma nounroll
                for (int h0 = 0; h0 < n; h0 += kStageInts) {
                    const int len = min(kStageInts, n - h0);
                    int v[kStagePer];
#pragma unroll
                    for (int u = 0; u < kStagePer; ++u) {
                        const int q = t + u * kLazyThreads;
                        v[u] = P.A[(size_t)r * n + h0 + (q < len ? q : 0)];
                    }
                    __syncthreads();  // the previous stretch (or the maxima) is no longer read
#pragma unroll
                    for (int u = 0; u < kStagePer; ++u) {
                        const int q = t + u * kLazyThreads;
                        if (q < len) stage[q] = v[u];
                    }
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < kEvalChunk; ++u) {
                        const int q = te[u] - h0;
                        if (q >= 0 && q < len) va[u] = stage[q];
                    }
                }
                // agent r's candidates (keyed by job) and those of its new job
                // (keyed by agent) share g(e) = a[r][tau(e)] + a[e][job] - d(r) - d(e)
                const int jr = side == 0 ? j : t0;
                const int dr = side == 0 ? ai : ac;
                u64 ka = 0, kj = 0;
#pragma unroll
                for (int u = 0; u < kEvalChunk; ++u) {
                    const int x = t + (s0c + u) * kLazyThreads;
                    const int xx = x < n ? x : 0;
                    const int g = (va[u] + P.AT[(size_t)jr * n + xx]) - (dr + P.d[xx]);
                    if (x < n && x != r) {
                        ka = umax64(ka, mk_key(g, te[u]));
                        kj = umax64(kj, mk_key(g, x));
                    }
                }
                if (side == 0) {
                    kai = umax64(kai, ka);
                    kjj = umax64(kjj, kj);
                } else {
                    kac = umax64(kac, ka);
                    kjt = umax64(kjt, kj);
                }
            }
        }
        __syncthreads();  // the last stretch is no longer read: the maxima reuse its bytes
        kai = wave_max64(kai);
        kac = wave_max64(kac);
        kjj = wave_max64(kjj);
        kjt = wave_max64(kjt);
        if (lane == 0) {
            rk[0][w] = kai;
            rk[1][w] = kac;
            rk[2][w] = kjj;
            rk[3][w] = kjt;
        }
        __syncthreads();
        if (t < 4) {
            u64 k = 0;
            for (int v = 0; v < kLazyWaves; ++v) k = umax64(k, rk[t][v]);
            const bool pos = k != 0 && key_gain(k) > 0;
            const int g = pos ? key_gain(k) : 0;
            const int x = t == 0 ? i : t == 1 ? c : t == 2 ? j : t0;
            if (t < 2) {
                ga[x] = g;
                if (pos) P.ja[x] = key_index(k);
            } else {
                gj[x] = g;
                if (pos) P.ij[x] = key_index(k);
            }
        }
        __syncthreads();  // the new stored values are visible
    }
    if (t == 0) {
        P.stats[0] += applied;
        P.stats[1] += gains;
        P.stats[5] = applied;
        P.stats[7] += attempts;
    }
}

}  // namespace

hipError_t launch_lazy_pass(const Instance &I, const u64 *jde, int64_t max_switches, hipStream_t s) {
    LazyParams P{I.A, I.AT, I.tau, I.sigma, I.d, I.bk, jde, I.stats, I.bc, I.par, I.flags, I.flags + 2, I.n,
                 max_switches};
    hipLaunchKernelGGL(k_lazy_pass, dim3(1), dim3(kLazyThreads), 0, s, P);
    return hipGetLastError();
}

}  // namespace dgs
