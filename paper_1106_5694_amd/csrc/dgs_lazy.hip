// Lazy DGS (Algorithm 1 with stale stored bests, Section 3.3) on gfx950: the
// switching phase of one pass as one cooperative launch over the whole grid.
//
// The pass starts from a full evaluation of every agent (ADE: best job,
// lowest job on ties) and every job (JDE: best agent to take it, its owner
// then taking that agent's job, lowest agent on ties), computed by the
// tile-pair evaluation.  Only positive improvements are stored.  Then, while
// a stored improvement is positive: the agent and the job with the largest
// stored values (lowest index on ties) are found; the agent's stored exchange
// is followed if its value is strictly larger than the job's, else the job's;
// the value followed is zeroed; the exchange is applied only if it raises f,
// and then the two agents and the two jobs it moves are evaluated afresh.
// Other stored values stay as they were (stale).
//
// Layout: G = ceil(n / 256) workgroups of 256 threads; thread t of workgroup
// q owns agent r = 256 q + t and job r.  It keeps in registers the agent's
// job and benefit, the job's owner and that owner's benefit, and the two
// stored entries:
//   agent r: value va (0: none), job ja, the current owner of ja and whether
//            the exchange (r takes ja, that owner takes tau(r)) raises f now;
//   job r:   value vj (0: none), agent ij, tau(ij) and whether the exchange
//            (ij takes r, the owner of r takes tau(ij)) raises f now.
// The stored values are stale by design; the "raises f now" flags are kept
// exact: an applied exchange changes them only for agent entries whose job
// changed owner and for job entries whose agent moved, and those threads
// recompute the flag from two entries of A.
//
// Rounds.  The workgroups meet once per round through tagged words (relaxed
// agent-scope atomics, double-buffered by round parity, every word rewritten
// every round, as in the switching loop).  A workgroup publishes its kM best
// agent entries and kM best job entries (key: value and index; payload: the
// flag and the exchange's agents and jobs), the key of its next entry on
// each side (a bound on everything it did not publish), and its shares of
// the four entities of the previous round's applied exchange: for agent i*
// the best gain g(i*, e) over its agents e keyed by job tau(e), for i*'s new
// job j* the same gains keyed by agent e (e takes j*, i* takes tau(e)), and
// likewise for the other agent and job.  Every workgroup then walks the same
// merged order: the best remaining entry of a side is known when it lies
// above every workgroup's bound of that side; the agent side is taken when
// its best is strictly larger than the job side's best (which can hold with
// one side unknown, against the bound), else the job side.  The entry taken
// is zeroed; the walk ends at the first taken entry whose exchange raises f
// (it is applied) or when the next choice is not known yet.  Entries taken
// before it failed the improvement guard.  The refreshed entities' new
// entries come from the shares.
#include "dgs_device.h"

namespace dgs {
namespace {

using namespace dev;

constexpr int kLT = 256;     // threads = agents = jobs per workgroup
constexpr int kM = 3;        // entries of each side published per workgroup and round
constexpr int kLMaxG = 102;  // G * kLW <= 8 * kLT (n <= 26112)
// words of a workgroup per round
constexpr int kWA = 0;            // agent entries: kM keys, then kM payloads
constexpr int kWJ = 2 * kM;       // job entries: kM keys, then kM payloads
constexpr int kWBnd = 4 * kM;     // bounds: agent side, job side
constexpr int kWSh = 4 * kM + 2;  // shares: i*, c* (keyed by job), j* key + info, t0* key + info
constexpr int kLW = kWSh + 6;     // 20
constexpr long long kLSpin = 1ll << 26;
// walk candidates per lane: kM per workgroup and side, plus two fresh entries
constexpr int kCand = (kLMaxG * kM + 2 + 63) / 64;

// Entry key: value (positive, 32 bits) | 0xFFFF - index (16) | 0 (8) | tag (8).
// Unsigned order of the upper 48 bits: value descending, index ascending.
__device__ __forceinline__ u64 ent_key(int v, int idx) {
    return ((u64)(uint32_t)v << 32) | ((u64)(0xFFFFu - (uint32_t)idx) << 16);
}
__device__ __forceinline__ int ent_val(u64 k) { return (int)(uint32_t)(k >> 32); }
__device__ __forceinline__ int ent_idx(u64 k) { return (int)(0xFFFFu - (uint32_t)((k >> 16) & 0xFFFFu)); }
__device__ __forceinline__ u64 untag(u64 k) { return k & ~(u64)0xFF; }
// Payload: raises-f flag (bit 56) | x (16) | owner (16) | other job (16) | tag.
// Agent entry of r: x = ja, owner = sigma(ja), other job = tau(r).
// Job entry of r:   x = ij, owner = sigma(r),  other job = tau(ij).
__device__ __forceinline__ u64 ent_pay(bool pass, int x, int owner, int t0) {
    return ((u64)pass << 56) | ((u64)(uint32_t)x << 40) | ((u64)(uint32_t)owner << 24) | ((u64)(uint32_t)t0 << 8);
}
__device__ __forceinline__ bool pay_pass(u64 p) { return (p >> 56) & 1; }
__device__ __forceinline__ int pay_x(u64 p) { return (int)((p >> 40) & 0xFFFFu); }
__device__ __forceinline__ int pay_owner(u64 p) { return (int)((p >> 24) & 0xFFFFu); }
__device__ __forceinline__ int pay_t0(u64 p) { return (int)((p >> 8) & 0xFFFFu); }
// Share key: gain biased (32) | 0xFFFF - index (16) | local partner (8) | tag (8);
// index = job tau(e) for an agent target, agent e for a job target.
__device__ __forceinline__ u64 sh_key(int g, int idx, int local) {
    return ((u64)((uint32_t)g ^ 0x80000000u) << 32) | ((u64)(0xFFFFu - (uint32_t)idx) << 16) |
           ((u64)(uint32_t)local << 8);
}
__device__ __forceinline__ int sh_gain(u64 k) { return (int)((uint32_t)(k >> 32) ^ 0x80000000u); }
__device__ __forceinline__ u64 hi48(u64 k) { return k & ~(u64)0xFFFF; }

struct LazyParams {
    const int32_t *A;
    const int32_t *AT;
    int32_t *tau;
    int32_t *sigma;
    int32_t *d;
    const u64 *ade;  // per agent: best key (gain, job) of the pass's evaluation
    const u64 *jde;  // per agent c: best key (gain, agent) over agents taking c's job
    u64 *words;      // 2 * G * kLW exchange words
    int64_t *stats;  // [0] switches, [1] gain sum, [5] switches of this pass, [7] attempts
    const int32_t *flags;
    int32_t *err;
    int n;
    int64_t max_switches;
};

__device__ __forceinline__ void put_word(u64 *p, u64 w) {
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The kM + 1 largest keys of the workgroup's 256 (unique apart from 0), by one
// wave: kM + 1 rounds of a wave maximum over four keys per lane.
__device__ __forceinline__ void top_keys(const u64 *vals, int lane, u64 (&out)[kM + 1]) {
    u64 k[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) k[u] = vals[lane + 64 * u];
#pragma unroll
    for (int m = 0; m <= kM; ++m) {
        const u64 mx = wave_max64(umax64(umax64(k[0], k[1]), umax64(k[2], k[3])));
        out[m] = mx;
#pragma unroll
        for (int u = 0; u < 4; ++u) k[u] = k[u] == mx ? 0 : k[u];
    }
}

// NPER: gathered words per thread (G * kLW <= NPER * kLT).
template <int NPER>
__global__ __launch_bounds__(kLT) void k_lazy_rounds(LazyParams P) {
    extern __shared__ __align__(16) u64 wl[];  // gathered words, G x kLW
    __shared__ u64 vals[6][kLT];               // 0 agent keys, 1 job keys, 2..5 shares (i*, c*, j*, t0*)
    __shared__ u64 pays[2][kLT];               // payloads of the entries (by local index)
    __shared__ int tauv[kLT];                  // tau of each agent (for the job shares' info)
    __shared__ u64 dec[16];                    // the walk's result (see below)
    __shared__ long long gpart[kLT / 64];
    __shared__ int s_err;

    if (P.flags[0]) return;  // same decision in every workgroup
    const int G = gridDim.x, q = blockIdx.x, t = threadIdx.x, n = P.n;
    const int64_t nn = n;
    const int r = q * kLT + t;
    const bool mine = r < n;
    const int lane = t & 63, wave = t >> 6;

    // ---- the pass's stored entries and state -------------------------------------------
    int tr = 0, dr = 0, so = 0, dso = 0;
    int va = 0, ja = 0, ca = 0;   // agent entry: value, job, owner of the job
    bool pa = false;              // agent entry raises f now
    int vj = 0, ij = 0, tij = 0;  // job entry: value, agent, tau(agent)
    bool pj = false;
    if (mine) {
        tr = P.tau[r];
        dr = P.d[r];
        so = P.sigma[r];
        dso = P.d[so];
        const u64 ka = P.ade[r];
        if (ka != 0 && key_gain(ka) > 0) {
            va = key_gain(ka);  // fresh: the stored value is the exchange's exact gain
            ja = key_index(ka);
            ca = P.sigma[ja];
            pa = true;
        }
        const u64 kj = P.jde[so];
        if (kj != 0 && key_gain(kj) > 0) {
            vj = key_gain(kj);
            ij = key_index(kj);
            tij = P.tau[ij];
            pj = true;
        }
    }
    if (t == 0) s_err = 0;
#pragma unroll
    for (int e = 2; e < 6; ++e) vals[e][t] = 0;
    // entities refreshed this round from the previous round's exchange: agents i*, c*, jobs
    // j*, t0* (-1: none)
    int ri = -1, rc = -1, rj = -1, rt = -1;
    int64_t S = P.stats[0];
    long long applied = 0, attempts = 0, gsum = 0;
    __syncthreads();

    for (uint32_t s = 0;; ++s) {
        // every round takes at least one stored value and an applied exchange sets at most
        // four: more rounds than this means a broken invariant (same in every workgroup)
        if ((long long)s > 2LL * n + 4 * applied + 16) {
            if (t == 0) atomicOr(P.err, 3);
            break;
        }
        const uint32_t tag = s & 0xFFu;
        u64 *buf = P.words + (size_t)(s & 1) * G * kLW;
        // ---- publication ------------------------------------------------------------------
        {
            const bool tgt_a = r == ri || r == rc, tgt_j = r == rj || r == rt;
            vals[0][t] = (mine && va > 0 && !tgt_a) ? ent_key(va, r) : 0;
            vals[1][t] = (mine && vj > 0 && !tgt_j) ? ent_key(vj, r) : 0;
            pays[0][t] = ent_pay(pa, ja, ca, tr);
            pays[1][t] = ent_pay(pj, ij, so, tij);
            tauv[t] = tr;
        }
        __syncthreads();
        if (wave < 2) {
            u64 top[kM + 1];
            top_keys(vals[wave], lane, top);
            const int base = wave == 0 ? kWA : kWJ;
            if (lane < kM) {
                const u64 k = top[lane];
                const u64 p = k ? pays[wave][ent_idx(k) - q * kLT] : 0;
                put_word(&buf[(size_t)q * kLW + base + lane], k | tag);
                put_word(&buf[(size_t)q * kLW + base + kM + lane], p | tag);
            } else if (lane == kM) {
                put_word(&buf[(size_t)q * kLW + kWBnd + wave], top[kM] | tag);
            }
        } else {
            // shares of the refreshed entities: wave 2 the agents (keyed by job), wave 3 the
            // jobs (keyed by agent, with the agent's job in an info word)
            const int ty0 = wave == 2 ? 2 : 4;
            u64 m0 = 0, m1 = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                m0 = umax64(m0, vals[ty0][lane + 64 * u]);
                m1 = umax64(m1, vals[ty0 + 1][lane + 64 * u]);
            }
            m0 = wave_max64(m0);
            m1 = wave_max64(m1);
            if (lane < 2) {
                const u64 m = lane == 0 ? m0 : m1;
                if (wave == 2) {
                    put_word(&buf[(size_t)q * kLW + kWSh + lane], m | tag);
                } else {
                    const int loc = (int)((m >> 8) & 0xFF);
                    put_word(&buf[(size_t)q * kLW + kWSh + 2 + 2 * lane], m | tag);
                    put_word(&buf[(size_t)q * kLW + kWSh + 3 + 2 * lane],
                             (m ? ((u64)(uint32_t)tauv[loc] << 8) : 0) | tag);
                }
            }
        }

        // ---- gather every workgroup's words ------------------------------------------------
        {
            const int NW = G * kLW;
            u64 wv[NPER];
#pragma unroll
            for (int i = 0; i < NPER; ++i) {
                const int x = t + i * kLT;
                wv[i] = x < NW ? __hip_atomic_load(&buf[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : (u64)tag;
            }
            long long spins = 0;
            for (;;) {
                bool ready = true;
#pragma unroll
                for (int i = 0; i < NPER; ++i) ready &= (uint32_t)(wv[i] & 0xFFu) == tag;
                if (ready) break;
                if (++spins > kLSpin) {
                    s_err = 1;
                    atomicOr(P.err, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int i = 0; i < NPER; ++i) {
                    const int x = t + i * kLT;
                    if (x < NW && (uint32_t)(wv[i] & 0xFFu) != tag)
                        wv[i] = __hip_atomic_load(&buf[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
#pragma unroll
            for (int i = 0; i < NPER; ++i) {
                const int x = t + i * kLT;
                if (x < NW) wl[x] = wv[i];
            }
        }
        __syncthreads();
        if (s_err) break;

        // ---- the walk (wave 0; identical in every workgroup) ----------------------------------
        // dec[0]: 1 applied, 2 stopped (the next choice is not known), 3 pass over, 4 switch
        //         budget reached
        // dec[1..4]: i, j, c, t0 of the applied exchange; dec[5]: entries taken in the round
        // dec[6], dec[7]: the smallest key taken on the agent / job side (0: none)
        // dec[8 + e], dec[12 + e]: key (0: none) and payload of refreshed entity e's new entry
        if (wave == 0) {
            u64 fk[4] = {0, 0, 0, 0}, fp[4] = {0, 0, 0, 0};
            if (ri >= 0) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int w = e < 2 ? kWSh + e : kWSh + 2 + 2 * (e - 2);
                    u64 m = 0;
                    for (int qq = lane; qq < G; qq += 64) m = umax64(m, hi48(wl[qq * kLW + w]) | (u64)qq);
                    m = wave_max64(m);
                    const int from = (int)(m & 0xFF);
                    const int g = sh_gain(m);
                    if (hi48(m) != 0 && g > 0) {
                        const u64 raw = wl[from * kLW + w];
                        const int idx = (int)(0xFFFFu - (uint32_t)((raw >> 16) & 0xFFFFu));
                        const int partner = from * kLT + (int)((raw >> 8) & 0xFF);
                        if (e < 2) {
                            // agent i* (c*) takes job idx from its owner `partner`, who takes
                            // i*'s new job j* (c*'s new job t0*)
                            fk[e] = ent_key(g, e == 0 ? ri : rc);
                            fp[e] = ent_pay(true, idx, partner, e == 0 ? rj : rt);
                        } else {
                            // agent idx takes job j* (t0*) from its owner i* (c*), who takes
                            // idx's job, sent in the info word
                            const int tidx = (int)((wl[from * kLW + w + 1] >> 8) & 0xFFFFu);
                            fk[e] = ent_key(g, e == 2 ? rj : rt);
                            fp[e] = ent_pay(true, idx, e == 2 ? ri : rc, tidx);
                        }
                    }
                }
            }
            u64 cA[kCand], cJ[kCand];
            const int NA = G * kM;
#pragma unroll
            for (int u = 0; u < kCand; ++u) {
                const int e = lane + 64 * u;
                u64 a = 0, b = 0;
                if (e < NA) {
                    a = untag(wl[(e / kM) * kLW + kWA + e % kM]);
                    b = untag(wl[(e / kM) * kLW + kWJ + e % kM]);
                } else if (e < NA + 2) {
                    a = fk[e - NA];
                    b = fk[2 + e - NA];
                }
                cA[u] = a;
                cJ[u] = b;
            }
            u64 bA = 0, bJ = 0;  // the largest key any workgroup did not publish (0: none)
            for (int qq = lane; qq < G; qq += 64) {
                bA = umax64(bA, untag(wl[qq * kLW + kWBnd]));
                bJ = umax64(bJ, untag(wl[qq * kLW + kWBnd + 1]));
            }
            bA = wave_max64(bA);
            bJ = wave_max64(bJ);
            int result = 2, ai = -1, aj = -1, ac = -1, at0 = -1, steps = 0;
            u64 lastA = 0, lastJ = 0;
            for (;;) {
                if (P.max_switches >= 0 && S >= P.max_switches) {
                    result = 4;
                    break;
                }
                u64 tA = 0, tJ = 0;
#pragma unroll
                for (int u = 0; u < kCand; ++u) {
                    tA = umax64(tA, cA[u]);
                    tJ = umax64(tJ, cJ[u]);
                }
                tA = wave_max64(tA);
                tJ = wave_max64(tJ);
                const bool knownA = bA == 0 || tA > bA, knownJ = bJ == 0 || tJ > bJ;
                const int vA = tA ? ent_val(tA) : 0, vJ = tJ ? ent_val(tJ) : 0;
                int side = -1;  // 0 agent, 1 job, -1 not known yet
                if (knownA && knownJ) {
                    if (!tA && !tJ) {
                        result = 3;  // no positive stored value left anywhere
                        break;
                    }
                    side = vA > vJ ? 0 : 1;
                } else if (knownJ) {
                    if (tJ && vJ >= ent_val(bA)) side = 1;
                } else if (knownA) {
                    if (tA && vA > ent_val(bJ)) side = 0;
                }
                if (side < 0) break;
                const u64 key = side == 0 ? tA : tJ;
                const int idx = ent_idx(key);
                u64 pay = 0;
                {
                    const int qq = idx / kLT, base = side == 0 ? kWA : kWJ;
                    bool found = false;
                    for (int m = 0; m < kM; ++m) {
                        if (untag(wl[qq * kLW + base + m]) == key) {
                            pay = wl[qq * kLW + base + kM + m];
                            found = true;
                        }
                    }
                    if (!found) {
                        const int e0 = side == 0 ? 0 : 2;
                        pay = fk[e0] == key ? fp[e0] : fp[e0 + 1];
                    }
                }
#pragma unroll
                for (int u = 0; u < kCand; ++u) {
                    if (side == 0 && cA[u] == key) cA[u] = 0;
                    if (side == 1 && cJ[u] == key) cJ[u] = 0;
                }
                if (side == 0)
                    lastA = key;
                else
                    lastJ = key;
                ++steps;
                if (pay_pass(pay)) {
                    result = 1;
                    ai = side == 0 ? idx : pay_x(pay);
                    aj = side == 0 ? pay_x(pay) : idx;
                    ac = pay_owner(pay);
                    at0 = pay_t0(pay);
                    break;
                }
            }
            if (lane == 0) {
                dec[0] = (u64)result;
                dec[1] = (u64)(int64_t)ai;
                dec[2] = (u64)(int64_t)aj;
                dec[3] = (u64)(int64_t)ac;
                dec[4] = (u64)(int64_t)at0;
                dec[5] = (u64)steps;
                dec[6] = lastA;
                dec[7] = lastJ;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    dec[8 + e] = fk[e];
                    dec[12 + e] = fp[e];
                }
            }
        }
        __syncthreads();

        // ---- everyone: the decision ---------------------------------------------------------
        const int result = (int)dec[0];
        const int is = (int)(int64_t)dec[1], js = (int)(int64_t)dec[2], k = (int)(int64_t)dec[3],
                  j0 = (int)(int64_t)dec[4];
        attempts += (long long)dec[5];
        const u64 lastA = dec[6], lastJ = dec[7];
        // entries taken in the walk are zeroed; refreshed entities take their new entries
        // (unless taken too).  A published entry was taken iff its key >= its side's last.
        if (mine) {
            if (r == ri || r == rc) {
                const int e = r == ri ? 0 : 1;
                const u64 fkey = dec[8 + e], fpay = dec[12 + e];
                const bool taken = fkey != 0 && lastA != 0 && fkey >= lastA;
                va = (fkey && !taken) ? ent_val(fkey) : 0;
                ja = pay_x(fpay);
                ca = pay_owner(fpay);
                pa = pay_pass(fpay);
            } else if (va > 0 && lastA != 0 && ent_key(va, r) >= lastA) {
                va = 0;
            }
            if (r == rj || r == rt) {
                const int e = r == rj ? 2 : 3;
                const u64 fkey = dec[8 + e], fpay = dec[12 + e];
                const bool taken = fkey != 0 && lastJ != 0 && fkey >= lastJ;
                vj = (fkey && !taken) ? ent_val(fkey) : 0;
                ij = pay_x(fpay);
                tij = pay_t0(fpay);
                pj = pay_pass(fpay);
            } else if (vj > 0 && lastJ != 0 && ent_key(vj, r) >= lastJ) {
                vj = 0;
            }
        }
        if (result == 3 || result == 4) break;
        if (result == 2) {  // nothing applied: no entity is refreshed next round
            ri = rc = rj = rt = -1;
#pragma unroll
            for (int e = 2; e < 6; ++e) vals[e][t] = 0;
            __syncthreads();  // dec is read by every thread before the next walk rewrites it
            continue;
        }
        if (is < 0 || is >= n || js < 0 || js >= n || k < 0 || k >= n || j0 < 0 || j0 >= n || k == is) {
            if (t == 0) atomicOr(P.err, 2);  // cannot happen; never index with it
            break;
        }
        ++S;
        ++applied;
        // loads: the two new benefits, each agent's two changed gains (four entries), and
        // for the threads whose raises-f flag changes, two entries each
        int tr2 = tr;
        if (mine) tr2 = r == is ? js : (r == k ? j0 : tr);
        int a1 = 0, a2 = 0, w1 = 0, w2 = 0;
        if (mine) {
            a1 = P.AT[(int64_t)js * nn + r];   // a[r][j*]
            a2 = P.AT[(int64_t)j0 * nn + r];   // a[r][j0]
            w1 = P.A[(int64_t)is * nn + tr2];  // a[i*][tau(r)] after the switch
            w2 = P.A[(int64_t)k * nn + tr2];   // a[k][tau(r)] after the switch
        }
        // agent entry whose job changed owner (ja in {j*, j0}), job entry whose agent moved
        // (ij in {i*, k}); the refreshed ones are replaced next round anyway
        const bool fixa = mine && va > 0 && r != is && r != k && (ja == js || ja == j0);
        const bool fixj = mine && vj > 0 && r != js && r != j0 && (ij == is || ij == k);
        const int na = ja == js ? is : k;    // new owner of ja
        const int tin = ij == is ? js : j0;  // new job of ij
        int xa1 = 0, xa2 = 0, xj1 = 0, xj2 = 0;
        if (fixa) {
            xa1 = P.AT[(int64_t)ja * nn + r];  // a[r][ja]
            xa2 = P.A[(int64_t)na * nn + tr];  // a[new owner][tau(r)]
        }
        if (fixj) {
            xj1 = P.AT[(int64_t)r * nn + ij];   // a[ij][r]
            xj2 = P.A[(int64_t)so * nn + tin];  // a[owner of r][new tau(ij)]
        }
        const int dis = P.A[(int64_t)is * nn + js];  // a[i*][j*]
        const int dk = P.A[(int64_t)k * nn + j0];    // a[k][j0]
        if (mine) {
            if (r == is) gsum += dis - dr;
            if (r == k) gsum += dk - dr;
            tr = tr2;
            dr = r == is ? dis : (r == k ? dk : dr);
            if (r == js) {
                so = is;
                dso = dis;
            } else if (r == j0) {
                so = k;
                dso = dk;
            }
            if (fixa) {
                ca = na;
                pa = (xa1 + xa2) - (dr + (na == is ? dis : dk)) > 0;
            }
            if (fixj) {
                tij = tin;
                pj = (xj1 + xj2) - ((ij == is ? dis : dk) + dso) > 0;
            }
        }
        // shares for the next round: g(r, i*) and g(r, k) after the switch
        {
            u64 s0 = 0, s1 = 0, s2 = 0, s3 = 0;
            if (mine) {
                const int g1 = (a1 + w1) - (dr + dis);  // g(r, i*)
                const int g2 = (a2 + w2) - (dr + dk);   // g(r, k)
                if (r != is) {
                    s0 = sh_key(g1, tr, t);  // agent i*, keyed by job tau(r)
                    s2 = sh_key(g1, r, t);   // job j* (owner i*), keyed by agent r
                }
                if (r != k) {
                    s1 = sh_key(g2, tr, t);
                    s3 = sh_key(g2, r, t);
                }
            }
            vals[2][t] = s0;
            vals[3][t] = s1;
            vals[4][t] = s2;
            vals[5][t] = s3;
        }
        ri = is;
        rc = k;
        rj = js;
        rt = j0;
        __syncthreads();  // dec is read by every thread before the next walk rewrites it
    }

    if (mine) {
        P.tau[r] = tr;
        P.sigma[r] = so;
        P.d[r] = dr;
    }
    // the gains of the applied exchanges (each counted by its two agents)
    long long v = gsum;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane == 0) gpart[wave] = v;
    __syncthreads();
    if (t == 0) {
        const long long g = gpart[0] + gpart[1] + gpart[2] + gpart[3];
        if (g) atomicAdd((unsigned long long *)&P.stats[1], (unsigned long long)g);
        if (q == 0) {
            P.stats[0] = S;
            P.stats[5] = applied;
            P.stats[7] += attempts;
        }
    }
}

}  // namespace

int lazy_grid(int n) { return (n + kLT - 1) / kLT; }
size_t lazy_word_bytes(int n) { return 2 * (size_t)lazy_grid(n) * kLW * sizeof(u64); }

hipError_t launch_lazy_pass(const Instance &I, const u64 *jde, void *words, int64_t max_switches, hipStream_t s) {
    LazyParams P{I.A, I.AT, I.tau, I.sigma, I.d, I.bk, jde, (u64 *)words, I.stats, I.flags, I.flags + 2, I.n,
                 max_switches};
    const int grid = lazy_grid(I.n);
    // every workgroup's words fit 8 gathered words per thread (n <= 26112)
    if (grid < 1 || grid * kLW > 8 * kLT) return hipErrorInvalidValue;
    const size_t shm = (size_t)grid * kLW * sizeof(u64);
    const void *kern = (const void *)k_lazy_rounds<8>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    void *args[] = {&P};
    return hipLaunchCooperativeKernel(kern, dim3((unsigned)grid), dim3(kLT), args, (unsigned)shm, s);
}

}  // namespace dgs
