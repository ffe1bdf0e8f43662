// Switching phase of DGS on gfx950 (Section 3.3, Algorithm 1 read as
// steepest ascent: every round applies the best 2-exchange over all agents,
// until none improves the objective), with cooperative re-evaluation.
//
// Grid: G = ceil(n / 256) workgroups of 256 threads.  Thread t of workgroup
// q owns agent r = 256 q + t and keeps in registers its job tau(r), its
// benefit d(r) = a[r][tau(r)] and its candidate list: up to kM exact
// candidates (gain, job, partner agent) and a bound that no candidate
// outside the list exceeds, so a non-empty list's maximum is the agent's
// exact best exchange.  The benefit matrix and its transpose are read-only;
// everything a workgroup learns about other agents comes through the
// per-round exchange of words.
//
// Exchange: per round every workgroup writes kW 64-bit words and reads all
// workgroups' words.  Each word carries the round number in its low 8 bits
// and is written and read with relaxed agent-scope atomics; the words are
// double-buffered by round parity, so a word is current exactly when its tag
// matches and no fences are needed.
//
// A workgroup's words: its best exchange (over its agents' lists, with the
// job, partner and own job of that exchange), its two most promising
// pending agents (agents whose list ran empty while their bound still
// promises a positive gain) with their jobs and benefits, and its top-2
// "shares" for each target of the round.  The share for target x is the best two of
// g(r, x) over the workgroup's agents r.  Because g(r, x) = g(x, r), the
// shares of all workgroups together are x's full re-evaluation: x's new list
// holds the workgroup bests above the largest workgroup second, and that
// second bounds everything else.  Targets are the two agents switched in
// the previous round (their candidates all change) and up to kD pending
// agents chosen in the previous round, largest bound first; only the active
// targets' words are exchanged.  No agent is ever re-evaluated by one
// workgroup alone, and an owner rebuilds its targets' lists while the
// round's loads are in flight.
//
// Decision (identical in every workgroup, computed from the words alone):
// the best exchange among the workgroup bests and the targets' new bests.
// If a pending agent's bound beats it, the round applies nothing (a stall);
// that agent is a target of this round and exact in the next one.
// Otherwise the switch (i*, j*) with partner k = sigma(j*) is applied and
// every other agent r receives its two changed candidates exactly:
// g(r, i*) for job j* and g(r, k) for job tau(i*).
//
// Loads: g(r, x) = a[r][tau(x)] + a[x][tau(r)] - d(r) - d(x).  The first term
// is row tau(x) of AT at column r, read coalesced.  The second is, for an
// agent r that has not switched in this loop, row x of the matrix
// W[x][c] = a[x][tau0(c)] (tau0: the start assignment; built once for square
// instances) at column r: coalesced too, where a[x][tau(r)] from A costs one
// cache line per agent.  Agents that have switched read A.  W is never written
// here.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgs_device.h"
#include "dgs_internal.h"

namespace dgs {
namespace {

using namespace dev;

constexpr int kT = 256;                       // threads = agents per workgroup
constexpr int kM = 8;                         // candidate list length
constexpr int kD = 8;                         // pending agents re-evaluated per round
constexpr int kTargets = 2 + kD;              // share target slots: i*, k, then the chosen pending agents
// words of a workgroup in a round: best exchange, its payload, two pending agents and their
// (benefit, job), then two share words per active target
constexpr int kWBest = 0, kWPay = 1, kWPend = 2, kWInfo = 4, kWShare = 6;
constexpr int kW = kWShare + 2 * kTargets;    // most words per workgroup per round
constexpr int kMaxG = 256;                    // n <= 65535
constexpr int kGatherPer = (kMaxG * kW + kT - 1) / kT;
constexpr long long kSpinLimit = 1ll << 27;

// ---- keys ------------------------------------------------------------------------------
// List entry: gain^bias:32 | 0xFFFF-job:16 | partner agent:16.  Agent key:
// gain^bias:32 | 0xFFFF-agent:16 | 0:16.  In both, unsigned order of the
// upper 48 bits is (gain ascending, index descending); 0 = none.
__device__ __forceinline__ u64 gbias(int g) { return (u64)((uint32_t)g ^ 0x80000000u) << 32; }
__device__ __forceinline__ u64 le_key(int g, int job, int partner) {
    return gbias(g) | ((u64)(0xFFFFu - (uint32_t)job) << 16) | (u64)(uint32_t)partner;
}
__device__ __forceinline__ u64 ak_key(int g, int agent) {
    return gbias(g) | ((u64)(0xFFFFu - (uint32_t)agent) << 16);
}
__device__ __forceinline__ int kgain(u64 k) { return (int)((uint32_t)(k >> 32) ^ 0x80000000u); }
__device__ __forceinline__ int kidx(u64 k) { return (int)(0xFFFFu - (uint32_t)((k >> 16) & 0xFFFFu)); }
__device__ __forceinline__ int kpartner(u64 k) { return (int)(k & 0xFFFFu); }
__device__ __forceinline__ u64 hi48(u64 k) { return k & ~(u64)0xFFFF; }

// ---- wave64 reductions on the DPP path -----------------------------------------------
// 32-bit max in four steps (quad_perm xor 1, quad_perm xor 2, reversal within
// 8 lanes, reversal within 16 lanes: each pairs disjoint groups of lanes that
// already agree), each folded into one v_max_u32_dpp, then the four 16-lane
// rows through readlane.  A 64-bit key takes two such passes: the high words,
// then the low words of the lanes that hold the high maximum.  Call with all
// 64 lanes active; the result is uniform.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ uint32_t dppu(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t umax32(uint32_t a, uint32_t b) { return a > b ? a : b; }

// The four DPP steps: afterwards every 16-lane row holds its maximum.
__device__ __forceinline__ uint32_t row_fold(uint32_t v) {
    v = umax32(v, dppu<kDppXor1>(v));
    v = umax32(v, dppu<kDppXor2>(v));
    v = umax32(v, dppu<kDppHalfMirror>(v));
    v = umax32(v, dppu<kDppMirror>(v));
    return v;
}
__device__ __forceinline__ uint32_t rows_max(uint32_t v) {
    const uint32_t a = umax32((uint32_t)__builtin_amdgcn_readlane((int)v, 0), (uint32_t)__builtin_amdgcn_readlane((int)v, 16));
    const uint32_t b = umax32((uint32_t)__builtin_amdgcn_readlane((int)v, 32), (uint32_t)__builtin_amdgcn_readlane((int)v, 48));
    return umax32(a, b);
}
__device__ __forceinline__ uint32_t wave_max32(uint32_t v) { return rows_max(row_fold(v)); }

__device__ __forceinline__ u64 wave_max(u64 v) {
    const uint32_t hi = wave_max32((uint32_t)(v >> 32));
    const uint32_t lo = wave_max32((uint32_t)(v >> 32) == hi ? (uint32_t)v : 0u);
    return ((u64)hi << 32) | lo;
}

// Two independent 64-bit maxima, their steps interleaved (the DPP steps of one
// fill the other's wait states).
__device__ __forceinline__ void wave_max_pair(u64 &a, u64 &b) {
    const uint32_t ah = (uint32_t)(a >> 32), bh = (uint32_t)(b >> 32);
    uint32_t x = ah, y = bh;
    x = umax32(x, dppu<kDppXor1>(x));
    y = umax32(y, dppu<kDppXor1>(y));
    x = umax32(x, dppu<kDppXor2>(x));
    y = umax32(y, dppu<kDppXor2>(y));
    x = umax32(x, dppu<kDppHalfMirror>(x));
    y = umax32(y, dppu<kDppHalfMirror>(y));
    x = umax32(x, dppu<kDppMirror>(x));
    y = umax32(y, dppu<kDppMirror>(y));
    const uint32_t HA = rows_max(x), HB = rows_max(y);
    x = ah == HA ? (uint32_t)a : 0u;
    y = bh == HB ? (uint32_t)b : 0u;
    x = umax32(x, dppu<kDppXor1>(x));
    y = umax32(y, dppu<kDppXor1>(y));
    x = umax32(x, dppu<kDppXor2>(x));
    y = umax32(y, dppu<kDppXor2>(y));
    x = umax32(x, dppu<kDppHalfMirror>(x));
    y = umax32(y, dppu<kDppHalfMirror>(y));
    x = umax32(x, dppu<kDppMirror>(x));
    y = umax32(y, dppu<kDppMirror>(y));
    a = ((u64)HA << 32) | rows_max(x);
    b = ((u64)HB << 32) | rows_max(y);
}

// Top-2 over the wave; every lane holds a1 >= a2, keys unique apart from zeros.
__device__ __forceinline__ void wave_top2(u64 &a1, u64 &a2) {
    const u64 m1 = wave_max(a1);
    const u64 m2 = wave_max(a1 == m1 ? a2 : a1);
    a1 = m1;
    a2 = m2;
}

// Two independent top-2 reductions, interleaved.
__device__ __forceinline__ void wave_top2_pair(u64 &a1, u64 &a2, u64 &b1, u64 &b2) {
    u64 ma = a1, mb = b1;
    wave_max_pair(ma, mb);
    u64 sa = a1 == ma ? a2 : a1, sb = b1 == mb ? b2 : b1;
    wave_max_pair(sa, sb);
    a1 = ma;
    a2 = sa;
    b1 = mb;
    b2 = sb;
}

// ---- candidate lists (registers) --------------------------------------------------------

__device__ __forceinline__ u64 list_max(const u64 (&L)[kM]) {
    u64 m = L[0];
#pragma unroll
    for (int i = 1; i < kM; ++i) m = umax64(m, L[i]);
    return m;
}

// Insert exact candidate y; B (upper 48 bits only) bounds every candidate
// outside the list.  y's job is not in the list.  Without branches: y takes
// an empty slot, or evicts the smallest entry (which then joins the bound),
// or stays outside and becomes the bound.
__device__ __forceinline__ void list_insert(u64 (&L)[kM], u64 &B, u64 y) {
    const u64 yh = hi48(y);
    u64 mn = L[0];
    int mi = 0;
#pragma unroll
    for (int i = 1; i < kM; ++i) {
        const bool lt = L[i] < mn;
        mn = lt ? L[i] : mn;
        mi = lt ? i : mi;
    }
    const u64 mh = hi48(mn);
    const bool above = yh > B, full = mn != 0;
    const bool take = above && (!full || yh >= mh);
    B = (above && full) ? (yh < mh ? yh : umax64(B, mh)) : B;
#pragma unroll
    for (int i = 0; i < kM; ++i) L[i] = (take && mi == i) ? y : L[i];
}

__device__ __forceinline__ void list_drop_jobs(u64 (&L)[kM], int j1, int j2) {
#pragma unroll
    for (int i = 0; i < kM; ++i) {
        const int j = kidx(L[i]);
        if (L[i] != 0 && (j == j1 || j == j2)) L[i] = 0;
    }
}

// Number of lanes below this one whose bit is set in a wave ballot.
__device__ __forceinline__ int lanes_below(u64 bal, int lane) { return __popcll(bal & ((1ull << lane) - 1)); }

struct V3Params {
    const int32_t *A;      // nr x n (row stride n)
    const int32_t *AT;     // n x nr (row stride nr)
    int32_t *tau;          // in: start assignment; out: final assignment
    const int32_t *sigma;  // start inverse assignment
    const int32_t *d;      // start benefits d[c] = a[c][tau(c)]
    const u64 *lists;      // full-evaluation candidate lists [n][kScanListLen] (gain, job) keys
    const u64 *bb;         // full-evaluation bounds
    const int32_t *W;      // USEW: n x n, W[x][c] = a[x][tau0(c)] for the start assignment tau0
    u64 *words;            // 2 * G * kW exchange words
    int64_t *stats;        // [0] switches [1] gain sum [3] re-evaluations [4] stalled rounds
    const int32_t *flags;  // [0] != 0: range check failed, do nothing
    int32_t *err;          // set when a wait exceeds its spin limit (1) or a decision is invalid (2)
    int n;
    int nr;  // real agents; agents nr..n-1 are virtual (benefit 0 everywhere, no candidate list)
    int64_t max_switches;
};

__device__ __forceinline__ void put_word(u64 *p, u64 w) {
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// NPER: gathered words per thread (G * kW <= NPER * kT).  VIRT: the instance
// has virtual agents (nr < n; the square path compiles without their tests).
// USEW: square instances only; rows of A through the start assignment are read from W.
template <int NPER, bool VIRT, bool USEW>
__global__ __launch_bounds__(kT) void k_switch_v3(V3Params P) {
    static_assert(!(VIRT && USEW), "W is kept for square instances only");
    extern __shared__ __align__(16) u64 wl[];  // gathered words, G x (words of the round)
    // values reduced by this workgroup in a round: 0 best keys, 1 pending keys, 2 + j the
    // shares for the round's j-th target (written at the end of the previous round)
    __shared__ u64 vals[2 + kTargets][kT];
    __shared__ u64 pay[kT];    // job, partner and own job of each agent's best exchange
    __shared__ u64 pinfo[kT];  // benefit and job of each agent
    __shared__ u64 dec_key;    // largest decision key of the round; item number in the low byte
    __shared__ u64 dec_pay[1 + kTargets];  // per item: job << 48 | partner << 32 | own job << 16
    __shared__ int4 nx[kD];                // pending agents chosen this round: agent (-1: none), job, benefit
    __shared__ u64 nx_key0;                // key of the first chosen pending agent (0: none)
    __shared__ int2 tgc[2][kTargets];      // a round's targets (agent, job), by round parity
    __shared__ u64 pend[kD];               // wave 0: the pending keys when there are at most kD
    __shared__ int pend_at[kD];
    __shared__ u64 rcand[kT / 64][kMaxG];  // per wave: candidates of a list being rebuilt
    __shared__ u64 rsel[kT / 64][kM + 1];
    __shared__ u64 rlist[kTargets][kM + 1];  // rebuilt lists of the round's targets, then their bounds
    __shared__ int s_err;

    if (P.flags[0]) return;  // same decision in every workgroup
    const int G = gridDim.x, q = blockIdx.x, t = threadIdx.x, n = P.n, nr = VIRT ? P.nr : P.n;
    const int64_t nn = n, nt_ = VIRT ? (int64_t)nr : nn;  // row strides of A and of AT
    const int r = q * kT + t;
    const bool mine = r < n;
    const bool real = VIRT ? r < nr : mine;  // a virtual agent keeps no list: its exchanges are the real agents' moves
    auto is_real = [&](int x) { return !VIRT || x < nr; };
    const int lane = t & 63, wave = t >> 6;

    int tr = 0, dr = 0;
    bool moved = false;  // USEW: this agent has switched (its column of W is stale)
    u64 L[kM];
#pragma unroll
    for (int i = 0; i < kM; ++i) L[i] = 0;
    u64 B = 0;
    bool inflight = false;
    if (mine) {
        tr = P.tau[r];
        dr = P.d[r];
    }
    if (real) {
#pragma unroll
        for (int i = 0; i < kM && i < kScanListLen; ++i) {
            const u64 k = P.lists[(size_t)r * kScanListLen + i];
            if (k) {
                const int job = key_index(k);
                L[i] = le_key(key_gain(k), job, P.sigma[job]);
            }
        }
        const u64 b = P.bb[r];
        B = b ? hi48(le_key(key_gain(b), key_index(b), 0)) : 0;
    }
    if (t == 0) s_err = 0;
    int nt = 0;  // targets of the round (uniform)
    int S = 0, refreshes = 0, stalls = 0;
    int64_t gsum = 0;
    __syncthreads();

    for (uint32_t s = 0;; ++s) {
        const uint32_t tag = s & 0xFFu;
        const int kWa = kWShare + 2 * nt;  // words per workgroup this round
        u64 *buf = P.words + (size_t)(s & 1) * G * kW;
        const int2 *tg = tgc[s & 1];

        // ---- this workgroup's words ------------------------------------------------------
        {
            u64 lk = 0, pd = 0;
            if (mine) {
                const u64 b = list_max(L);
                if (b) {
                    lk = ak_key(kgain(b), r);
                } else if (!inflight && B != 0 && kgain(B) > 0) {
                    pd = ak_key(kgain(B), r);
                }
                pay[t] = ((u64)(uint32_t)kidx(b) << 48) | ((u64)(uint32_t)kpartner(b) << 32) |
                         ((u64)(uint32_t)tr << 16);
                pinfo[t] = ((u64)(uint32_t)dr << 32) | ((u64)(uint32_t)tr << 16);
            }
            vals[0][t] = lk;
            vals[1][t] = pd;
        }
        __syncthreads();
        // every thread has read the previous round's decision and pending choice
        if (t == 0) {
            dec_key = 0;
            nx_key0 = 0;
        }
        if (t < kD) nx[t] = make_int4(-1, 0, 0, 0);
        // wave w reduces value types w, w + 4 (together) and w + 8: 0 best, 1 pending (top-2),
        // 2 + j shares (top-2).  Word w of a workgroup always sits at the same place and is
        // always written by the same lane, every round (share words of inactive targets carry
        // only the tag), so no older word with a matching tag can be left anywhere in the buffer.
        {
            auto gather4 = [&](int ty, u64 &v1, u64 &v2) {
                v1 = vals[ty][lane];
                v2 = 0;
                top2_push(v1, v2, vals[ty][lane + 64]);
                top2_push(v1, v2, vals[ty][lane + 128]);
                top2_push(v1, v2, vals[ty][lane + 192]);
            };
            auto publish = [&](int ty, u64 v1, u64 v2) {
                if (ty >= 2 + nt) {
                    if (lane < 2) put_word(&buf[(size_t)q * kW + kWShare + 2 * (ty - 2) + lane], (u64)tag);
                } else if (ty == 0) {
                    if (lane == 0) {
                        const u64 w1 = v1 ? pay[kidx(v1) - q * kT] : 0;
                        put_word(&buf[(size_t)q * kW + kWBest], v1 | tag);
                        put_word(&buf[(size_t)q * kW + kWPay], (w1 & ~(u64)0xFF) | tag);
                    }
                } else if (lane < 2) {
                    const u64 v = lane == 0 ? v1 : v2;
                    if (ty == 1) {
                        const u64 info = v ? pinfo[kidx(v) - q * kT] : 0;
                        put_word(&buf[(size_t)q * kW + kWPend + lane], v | tag);
                        put_word(&buf[(size_t)q * kW + kWInfo + lane], (info & ~(u64)0xFF) | tag);
                    } else {
                        const u64 w = v ? (hi48(v) | ((v & 0xFF) << 8)) : 0;  // local partner in bits 15..8
                        put_word(&buf[(size_t)q * kW + kWShare + 2 * (ty - 2) + lane], w | tag);
                    }
                }
            };
            const int tA = wave, tB = wave + 4, tC = wave + 8;  // tA < 2 always holds for waves 0, 1
            u64 a1 = 0, a2 = 0, b1 = 0, b2 = 0;
            if (tA < 2 + nt) gather4(tA, a1, a2);
            if (tB < 2 + nt) gather4(tB, b1, b2);
            wave_top2_pair(a1, a2, b1, b2);
            publish(tA, a1, a2);
            publish(tB, b1, b2);
            u64 c1 = 0, c2 = 0;
            if (tC < 2 + nt) {
                gather4(tC, c1, c2);
                wave_top2(c1, c2);
            }
            publish(tC, c1, c2);
        }

        // ---- gather every workgroup's words ------------------------------------------------
        // the first kWa words of each workgroup, packed as wl[q * kWa + w]
        {
            const int NW = G * kWa;
            const uint32_t magic = (uint32_t)((0x100000000ull + (uint64_t)kWa - 1) / (uint64_t)kWa);
            u64 wv[NPER];
            int src[NPER];
#pragma unroll
            for (int i = 0; i < NPER; ++i) {
                const int x = t + i * kT;
                const int qq = (int)__umulhi((uint32_t)x, magic);  // x / kWa (exact for x < 2^16)
                src[i] = qq * kW + (x - qq * kWa);
                wv[i] = x < NW ? __hip_atomic_load(&buf[src[i]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : (u64)tag;
            }
            long long spins = 0;
            for (;;) {
                bool ready = true;
#pragma unroll
                for (int i = 0; i < NPER; ++i) ready &= (uint32_t)(wv[i] & 0xFFu) == tag;
                if (ready) break;
                if (++spins > kSpinLimit) {
                    s_err = 1;
                    atomicOr(P.err, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int i = 0; i < NPER; ++i) {
                    const int x = t + i * kT;
                    if (x < NW && (uint32_t)(wv[i] & 0xFFu) != tag)
                        wv[i] = __hip_atomic_load(&buf[src[i]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
#pragma unroll
            for (int i = 0; i < NPER; ++i) {
                const int x = t + i * kT;
                if (x < NW) wl[x] = wv[i];
            }
        }
        __syncthreads();
        if (s_err) break;

        // ---- maxima over workgroups (waves 1-3), pending agents to re-evaluate (wave 0) -----
        if (wave > 0) {
            // item 0: best exchange; item 1 + j: best share of target j.  Each wave turns its
            // items into decision candidates: a key (gain, agent) with the item number below
            // it, and the exchange's job, partner and own job.  Items go in pairs.
            auto item_max = [&](int it) {
                const int widx = it == 0 ? kWBest : kWShare + 2 * (it - 1);
                u64 m = 0;
                for (int qq = lane; qq < G; qq += 64) m = umax64(m, (wl[qq * kWa + widx] & ~(u64)0xFF) | (u64)qq);
                return m;
            };
            auto commit = [&](int it, u64 m) {
                if (hi48(m) == 0) return;
                u64 key, pw;
                if (it == 0) {
                    key = hi48(m);
                    pw = wl[(kidx(m) / kT) * kWa + kWPay] & ~(u64)0xFFFF;
                } else {
                    const int2 x = tg[it - 1];
                    key = ak_key(kgain(m), x.x);
                    const int partner = (int)(m & 0xFF) * kT + (int)((m >> 8) & 0xFF);
                    pw = ((u64)(uint32_t)kidx(m) << 48) | ((u64)(uint32_t)partner << 32) | ((u64)(uint32_t)x.y << 16);
                }
                dec_pay[it] = pw;
                atomicMax(&dec_key, key | (u64)(0xFF - it));  // equal keys: the lower item
            };
            for (int i0 = wave - 1; i0 <= nt; i0 += 6) {
                const int i1 = i0 + 3;
                u64 m0 = item_max(i0), m1 = i1 <= nt ? item_max(i1) : 0;
                wave_max_pair(m0, m1);
                if (lane == 0) {
                    commit(i0, m0);
                    if (i1 <= nt) commit(i1, m1);
                }
            }
        } else {
            // the kD largest of the 2G published pending keys (unique); the ranks nobody holds
            // keep the "none" written after the publication barrier
            constexpr int kPer = (2 * (NPER * kT / kW) + 63) / 64;  // keys per lane: G <= NPER * kT / kW
            u64 kk[kPer];
            int m = 0;
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int e = lane + 64 * i;
                kk[i] = e < 2 * G ? hi48(wl[(e >> 1) * kWa + kWPend + (e & 1)]) : 0;
                m += __popcll(__ballot(kk[i] != 0));
            }
            auto choose = [&](int rank, u64 key, int e) {
                const u64 info = wl[(e >> 1) * kWa + kWInfo + (e & 1)];
                nx[rank] = make_int4(kidx(key), (int)((info >> 16) & 0xFFFFu), (int)(uint32_t)(info >> 32), 0);
                if (rank == 0) nx_key0 = key;
            };
            if (m <= kD) {  // all of them: compact, then rank among themselves
                int c = 0;
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    const u64 bal = __ballot(kk[i] != 0);
                    if (kk[i]) {
                        const int at = c + lanes_below(bal, lane);
                        pend[at] = kk[i];
                        pend_at[at] = lane + 64 * i;
                    }
                    c += __popcll(bal);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                if (lane < m) {
                    const u64 me = pend[lane];
                    int rank = 0;
#pragma unroll
                    for (int i = 0; i < kD; ++i) rank += i < m && pend[i] > me;
                    choose(rank, me, pend_at[lane]);
                }
            } else {  // the kD largest by repeated maxima; the chosen agents' lookups after the loop
                      // (inside it, each was a dependent LDS round trip)
                int rk[kPer];
                u64 k0[kPer];
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    rk[i] = kD;
                    k0[i] = kk[i];
                }
                for (int rank = 0; rank < kD; ++rank) {
                    u64 mx = 0;
#pragma unroll
                    for (int i = 0; i < kPer; ++i) mx = umax64(mx, kk[i]);
                    const u64 top = wave_max(mx);
#pragma unroll
                    for (int i = 0; i < kPer; ++i) {
                        const bool hit = kk[i] == top;  // one lane, one slot: keys are unique
                        rk[i] = hit ? rank : rk[i];
                        kk[i] = hit ? 0 : kk[i];
                    }
                }
#pragma unroll
                for (int i = 0; i < kPer; ++i)
                    if (rk[i] < kD) choose(rk[i], k0[i], lane + 64 * i);
            }
        }
        __syncthreads();

        // ---- decide ---------------------------------------------------------------------------
        int nx_agent[kD], nx_tau[kD], nx_d[kD];
#pragma unroll
        for (int dd = 0; dd < kD; ++dd) {
            const int4 v = nx[dd];
            nx_agent[dd] = __builtin_amdgcn_readfirstlane(v.x);  // uniform
            nx_tau[dd] = __builtin_amdgcn_readfirstlane(v.y);
            nx_d[dd] = v.z;
        }
        int nref = 0;  // the chosen pending agents are a prefix
#pragma unroll
        for (int dd = 0; dd < kD; ++dd) nref += nx_agent[dd] >= 0;
        const u64 pkey0 = nx_key0;
        u64 best = 0;
        int bj = -1, bk = -1, bj0 = -1;  // job, partner and own job of the best exchange
        {
            const u64 win = dec_key;
            if (hi48(win)) {
                const u64 pw = dec_pay[0xFF - (int)(win & 0xFF)];
                best = hi48(win);
                bj = (int)((pw >> 48) & 0xFFFFu);
                bk = (int)((pw >> 32) & 0xFFFFu);
                bj0 = (int)((pw >> 16) & 0xFFFFu);
            }
        }
        if (P.max_switches >= 0 && S >= P.max_switches) break;
        const bool stall = nx_agent[0] >= 0 && pkey0 > best;  // pending bounds have gain > 0
        if (!stall && (best == 0 || kgain(best) <= 0)) break;

        int is = -1, js = -1, k = -1, j0 = -1, gw = 0;
        if (!stall) {
            is = kidx(best);
            js = bj;
            k = bk;
            j0 = bj0;
            gw = kgain(best);
            if (is < 0 || is >= n || js < 0 || js >= n || k < 0 || k >= n || j0 < 0 || j0 >= n || k == is) {
                if (t == 0) atomicOr(P.err, 2);  // cannot happen; never index with it
                break;
            }
        }

        // ---- loads of the round: the switch's changed candidates and the re-evaluations ---
        // Nothing loaded here is read before the owner rebuilds below, so every load of the
        // round is in flight at once (the two new benefits are issued last: no wait for
        // them may come before the other loads are issued).
        int tr2 = tr;  // job after this round's switch
        if (mine && !stall) tr2 = r == is ? js : (r == k ? j0 : tr);
        int a1 = 0, a2 = 0, w1 = 0, w2 = 0;
        const bool wcur = USEW && !moved;  // a[x][tau(r)] = W[x][r]
        // Every lane loads under uniform conditions only: a per-lane condition costs an exec-mask
        // branch around every load.  Lanes without an agent read column 0 and virtual agents column
        // 0 of AT (in bounds); values a lane does not need are never used, and a virtual agent's
        // own benefits (0) replace its AT values where they are used, after the loads' wait.
        const int rc = mine ? r : 0, rt = real ? r : 0;
        auto row_at_tau = [&](int x, int job) {  // a[x][job], job = tau(r) when W's column r is current
            if constexpr (USEW) return *(wcur ? P.W + (int64_t)x * nn + rc : P.A + (int64_t)x * nn + job);
            return P.A[(int64_t)x * nn + job];
        };
        if (!stall) {
            a1 = P.AT[(int64_t)js * nt_ + rt];  // a[r][j*]
            a2 = P.AT[(int64_t)j0 * nt_ + rt];  // a[r][j0]
            w1 = row_at_tau(is, tr);                 // a[i*][tau(r)]
            if (is_real(k)) w2 = row_at_tau(k, tr);  // a[k][tau(r)]
        }
        // (No branch may merge paths that hold loaded values in different registers: the
        // copy at the merge would wait for the loads.)
        int ra[kD], rb[kD];
#pragma unroll
        for (int dd = 0; dd < kD; ++dd) {
            const int x = nx_agent[dd];
            ra[dd] = rb[dd] = 0;
            if (dd < nref && x != is && x != k) {  // uniform
                ra[dd] = P.AT[(int64_t)nx_tau[dd] * nt_ + rt];  // a[r][tau(x)]
                // a[x][tau(r)] after the switch (W's column r is stale if r switches now)
                if constexpr (USEW)
                    rb[dd] = *(wcur && r != is && r != k ? P.W + (int64_t)x * nn + rc : P.A + (int64_t)x * nn + tr2);
                else
                    rb[dd] = P.A[(int64_t)x * nn + tr2];
            }
        }
        int dis = 0, dk = 0;
        if (!stall) {
            dis = P.A[(int64_t)is * nn + js];  // a[i*][j*]
            if (is_real(k)) dk = P.A[(int64_t)k * nn + j0];  // a[k][j0]
        }

        // ---- owners rebuild the lists of this round's targets (while the loads are in flight)
        // Done by the owner's wave alone: the bound is the largest workgroup second, the list
        // the workgroup bests above it (the kM largest when there are more).  The new list
        // goes through LDS to its owner.
        int myj = -1;  // this thread's rebuilt target, if any
        uint32_t own = 0;  // targets whose owner is in this wave (uniform)
#pragma unroll
        for (int j = 0; j < kTargets; ++j) {
            const int x = tg[j].x;
            if (j < nt && x / 64 == q * (kT / 64) + wave && x != is && x != k) own |= 1u << j;
        }
        own = __builtin_amdgcn_readfirstlane(own);
#pragma unroll 1
        for (int j = 0; j < nt; ++j) {
            if (!((own >> j) & 1u)) continue;
            const int x = tg[j].x;
            const int sw = kWShare + 2 * j;
            u64 sec = 0;
            for (int qq = lane; qq < G; qq += 64) sec = umax64(sec, hi48(wl[qq * kWa + sw + 1]));
            const u64 bnd = wave_max(sec);
            int cnt = 0;
            for (int base = 0; base < G; base += 64) {
                const int qq = base + lane;
                const u64 w = qq < G ? wl[qq * kWa + sw] : 0;
                const bool c = hi48(w) > bnd;
                const u64 bal = __ballot(c);
                if (c) rcand[wave][cnt + lanes_below(bal, lane)] = hi48(w) | (u64)(qq * kT + (int)((w >> 8) & 0xFF));
                cnt += __popcll(bal);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            if (cnt > kM) {  // keep the kM largest; the next one joins the bound
                for (int e = lane; e < cnt; e += 64) {
                    const u64 me = rcand[wave][e];
                    int rank = 0;
                    for (int i = 0; i < cnt; ++i) rank += rcand[wave][i] > me;
                    if (rank <= kM) rsel[wave][rank] = me;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            }
            if (lane <= kM) {
                u64 v;
                if (cnt > kM)
                    v = lane < kM ? rsel[wave][lane] : umax64(bnd, hi48(rsel[wave][kM]));
                else
                    v = lane < kM ? (lane < cnt ? rcand[wave][lane] : 0) : bnd;
                rlist[j][lane] = v;
            }
            if (r == x) myj = j;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // rlist is written; rcand is reused
        }
        if (myj >= 0) {
#pragma unroll
            for (int e = 0; e < kM; ++e) L[e] = rlist[myj][e];
            B = rlist[myj][kM];
            inflight = false;
        }

        // ---- apply the switch; shares for the next round's targets ---------------------------
        // Targets of the next round: i* (share g(r, i*)), k (g(r, k)), then the live pending
        // agents chosen in this round.  Shares go straight to vals.
        int2 *tgn = tgc[(s + 1) & 1];
        int jn = 0, nsw = 0;  // next round's targets; of them the switch's agents
        if (!stall) {
            ++S;
            gsum += gw;
            u64 s0 = 0, s1 = 0;
            if (mine) {
                const bool own_row = !VIRT || real;  // a virtual agent's benefits are 0
                const int g1 = ((own_row ? a1 : 0) + w1) - (dr + dis);  // g(r, i*)
                const int g2 = ((own_row ? a2 : 0) + w2) - (dr + dk);   // g(r, k)
                const bool switched = r == is || r == k;
                list_drop_jobs(L, js, j0);
                list_insert(L, B, le_key(g1, js, is));
                list_insert(L, B, le_key(g2, j0, k));
                const bool drop = switched || !real;  // (a virtual agent never keeps a list)
#pragma unroll
                for (int i = 0; i < kM; ++i) L[i] = drop ? 0 : L[i];
                B = drop ? 0 : B;
                inflight = switched ? false : inflight;
                s0 = r == is ? 0 : (r == k ? le_key(-gw, j0, t) : le_key(g1, tr, t));  // g(k, i*) after the switch
                s1 = r == k ? 0 : (r == is ? le_key(-gw, js, t) : le_key(g2, tr, t));  // g(i*, k) after the switch
                moved = moved || switched;
                tr = tr2;
                dr = r == is ? dis : (r == k ? dk : dr);
            }
            // a virtual partner keeps no list: only i* is then rebuilt
            nsw = is_real(k) ? 2 : 1;
            vals[2][t] = s0;
            if (nsw == 2) vals[3][t] = s1;
            if (t == 0) {
                tgn[0] = make_int2(is, js);
                if (nsw == 2) tgn[1] = make_int2(k, j0);
            }
            jn = nsw;
        } else {
            ++stalls;
        }
#pragma unroll
        for (int dd = 0; dd < kD; ++dd) {
            const int x = nx_agent[dd];
            if (dd < nref && x != is && x != k) {  // uniform
                u64 v = 0;
                if (mine && r != x)  // g(r, x) (a virtual agent's benefit a[r][tau(x)] is 0)
                    v = le_key((((!VIRT || real) ? ra[dd] : 0) + rb[dd]) - (dr + nx_d[dd]), tr, t);
                if (mine && r == x) inflight = true;
                vals[2 + jn][t] = v;
                if (t == 0) tgn[jn] = make_int2(x, nx_tau[dd]);
                ++jn;
            }
        }
        refreshes += jn - nsw;
        nt = jn;
    }

    if (mine) P.tau[r] = tr;
    if (t == 0 && q == 0) {
        P.stats[0] = S;
        P.stats[1] = gsum;
        P.stats[3] = refreshes;
        P.stats[4] = stalls;
    }
}

}  // namespace

int switch_v3_grid(int n) { return (n + kT - 1) / kT; }
size_t switch_v3_word_bytes(int n) { return 2 * (size_t)switch_v3_grid(n) * kW * sizeof(u64); }

hipError_t launch_switch_v3(const Instance &I, int64_t max_switches, void *words, int32_t *err, bool coop,
                            hipStream_t s) {
    V3Params P;
    P.A = I.A;
    P.AT = I.AT;
    P.tau = I.tau;
    P.sigma = I.sigma;
    P.d = I.d;
    P.lists = I.lists;
    P.bb = I.bb;
    P.W = I.W;
    P.words = (u64 *)words;
    P.stats = I.stats;
    P.flags = I.flags;
    P.err = err;
    P.n = I.n;
    P.nr = I.nr;
    P.max_switches = max_switches;
    const int grid = switch_v3_grid(I.n);
    if (grid < 1 || grid > kMaxG) return hipErrorInvalidValue;
    const size_t shm = (size_t)grid * kW * sizeof(u64);
    // the narrow gather when every workgroup's words fit 8 per thread
    const bool narrow = grid * kW <= 8 * kT, virt = I.nr < I.n, usew = I.W != nullptr && !virt;
    const void *kern = narrow ? (virt   ? (const void *)k_switch_v3<8, true, false>
                                 : usew ? (const void *)k_switch_v3<8, false, true>
                                        : (const void *)k_switch_v3<8, false, false>)
                              : (virt   ? (const void *)k_switch_v3<kGatherPer, true, false>
                                 : usew ? (const void *)k_switch_v3<kGatherPer, false, true>
                                        : (const void *)k_switch_v3<kGatherPer, false, false>);
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    void *args[] = {&P};
    if (!coop) return hipLaunchKernel(kern, dim3((unsigned)grid), dim3(kT), args, shm, s);
    return hipLaunchCooperativeKernel(kern, dim3((unsigned)grid), dim3(kT), args, (unsigned)shm, s);
}

}  // namespace dgs
