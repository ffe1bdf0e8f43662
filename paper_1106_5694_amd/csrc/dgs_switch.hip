// Switching phase of DGS on gfx950 (Section 3.3, Algorithm 1 read as
// steepest ascent): repeatedly apply the best 2-exchange over all agents
// until none improves the objective.
//
// One cooperative grid of G workgroups; workgroup q owns the 256 agents
// [256 q, 256 q + 256), one per thread.  Each thread keeps its agent's
// candidate list in registers: up to kM exact candidates (packed keys
// (gain, job)) and a bound key that every candidate outside the list does
// not exceed, so the list maximum is the agent's exact best exchange.
//
// Per switch the workgroups meet once, through an all-to-all exchange of
// nine 64-bit words each.  Every word carries the round number in its low
// 16 bits and is written and read with relaxed agent-scope atomics, so a
// reader knows a word is current from the word alone: no cache flushes or
// fences are needed, and nothing else is shared between workgroups:
//   * each workgroup keeps a private replica of tau, sigma and d (current
//     benefit of every agent) and applies every switch to it;
//   * the cross terms of the exchange gain are read from the benefit matrix
//     and its transpose, which never change;
//   * W (W[r][c] = a[r][tau(c)]) is read and written only by the owner of row r.
//
// A switch (i*, j*) with partner k = sigma(j*) and j0 = tau(i*) changes, for
// every other agent r, only the candidates towards i* (job j*) and towards
// k (job j0).  Each thread applies those two to its list; by the symmetry
// g(r, c) = g(c, r) the same values are i*'s and k's candidates towards r,
// so every workgroup also publishes its top-3 for agents i* and k and the
// owners rebuild those two lists from all workgroups' shares.
//
// An agent whose list runs empty is re-evaluated in full by its workgroup
// after the workgroup has published its words, while it waits for the
// others; its bound is published as "pending".  If a pending bound could
// beat the best known exchange, the round applies no switch and is
// repeated with the re-evaluated lists (this is rare).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgs_device.h"
#include "dgs_internal.h"

namespace dgs {
namespace {

using namespace dev;

constexpr int kT = 256;      // threads per workgroup
// agents per workgroup: 128 while that keeps the grid within 256 workgroups, else 256
__host__ __device__ constexpr int rows_per_wg(int n) { return n <= 128 * 256 ? 128 : 256; }
constexpr int kM = 8;        // candidate list length
constexpr int kWords = 9;    // exchange words per workgroup per round
constexpr int kCand = 2 * kT;  // selection scratch (candidates above a bound)
constexpr long long kSpinLimit = 1ll << 27;
// Replicas of tau, sigma (16-bit) and d (32-bit) sit in LDS up to this size.
constexpr size_t kExLdsReplicaBytes = (size_t)8 * 16384 + 16;
constexpr int kMaxGrid = 256;                                  // n <= 65535
constexpr int kGatherPer = (kMaxGrid * kWords + kT - 1) / kT;  // words gathered per thread

// Short keys: (gain biased:32 | 0xFFFF - idx:16 | round tag:16).  Unsigned
// order of the upper 48 bits = (gain ascending, idx descending); 0 = none.
__device__ __forceinline__ u64 skey(int g, int idx) {
    return ((u64)((uint32_t)g ^ 0x80000000u) << 32) | ((u64)(0xFFFFu - (uint32_t)idx) << 16);
}
__device__ __forceinline__ int sgain(u64 k) { return (int)((uint32_t)(k >> 32) ^ 0x80000000u); }
__device__ __forceinline__ int sidx(u64 k) { return (int)(0xFFFFu - (uint32_t)((k >> 16) & 0xFFFFu)); }
__device__ __forceinline__ u64 kpart(u64 w) { return w & ~(u64)0xFFFF; }

// long key (gain, ~idx) of the full-scan kernel -> short key
__device__ __forceinline__ u64 from_long(u64 k) { return k ? skey(key_gain(k), key_index(k)) : 0; }

struct ExParams {
    const int32_t *A;
    const int32_t *AT;
    int32_t *W;
    int32_t *tau;          // in: start assignment; out: final assignment
    const int32_t *sigma;  // start inverse assignment
    const int32_t *d;      // start benefits d[c] = a[c][tau(c)]
    const u64 *lists;      // full-evaluation candidate lists [n][kScanListLen] (long form)
    const u64 *bb;         // full-evaluation bounds (long form)
    u64 *words;            // 2 * G * kWords exchange words
    unsigned char *rep;    // private replicas (global mode): G * n * 8 bytes
    int64_t *stats;        // [0] switches [1] gain sum [3] re-evaluations [4] stalled rounds
    const int32_t *flags;  // [0] != 0: range check failed, do nothing
    int32_t *err;          // set when a wait exceeds its spin limit
    int n;
    int rows;  // agents per workgroup
    int64_t max_switches;
};

// ---- small sorted-triple and list helpers --------------------------------------

__device__ __forceinline__ void top3_push(u64 &a1, u64 &a2, u64 &a3, u64 k) {
    if (k > a3) {  // rare after the first few: skip the insertion network
        const u64 lo1 = umin64(a1, k);
        a1 = umax64(a1, k);
        const u64 lo2 = umin64(a2, lo1);
        a2 = umax64(a2, lo1);
        a3 = umax64(a3, lo2);
    }
}

// merge sorted triples (keys unique, zeros sink)
__device__ __forceinline__ void top3_merge(u64 &a1, u64 &a2, u64 &a3, u64 b1, u64 b2, u64 b3) {
    const bool A = a1 >= b1;
    const u64 x1 = A ? a1 : b1;
    const u64 u1 = A ? a2 : b2, u2 = A ? a3 : b3;
    const u64 v1 = A ? b1 : a1, v2 = A ? b2 : a2;
    const u64 x2 = umax64(u1, v1);
    const u64 x3 = (u1 >= v1) ? umax64(u2, v1) : umax64(u1, v2);
    a1 = x1;
    a2 = x2;
    a3 = x3;
}

template <int N>
__device__ __forceinline__ void wave_max_n(u64 (&v)[N]) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = umax64(v[i], shfl_xor64(v[i], m));
    }
}

// Block-wide max of N values; every thread gets the results.
template <int N>
__device__ __forceinline__ void block_max_n(u64 (&v)[N], u64 *red) {
    wave_max_n<N>(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) red[w * N + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        u64 r = red[i];
#pragma unroll
        for (int x = 1; x < kT / 64; ++x) r = umax64(r, red[x * N + i]);
        v[i] = r;
    }
}

// Block-wide merge of sorted triples; every thread gets the result.
__device__ __forceinline__ void block_top3(u64 &a1, u64 &a2, u64 &a3, u64 *red) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        u64 b1 = shfl_xor64(a1, m), b2 = shfl_xor64(a2, m), b3 = shfl_xor64(a3, m);
        top3_merge(a1, a2, a3, b1, b2, b3);
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[3 * w] = a1;
        red[3 * w + 1] = a2;
        red[3 * w + 2] = a3;
    }
    __syncthreads();
    a1 = red[0];
    a2 = red[1];
    a3 = red[2];
#pragma unroll
    for (int x = 1; x < kT / 64; ++x) top3_merge(a1, a2, a3, red[3 * x], red[3 * x + 1], red[3 * x + 2]);
}

__device__ __forceinline__ u64 list_max(const u64 (&L)[kM]) {
    u64 m = L[0];
#pragma unroll
    for (int i = 1; i < kM; ++i) m = umax64(m, L[i]);
    return m;
}

__device__ __forceinline__ bool list_empty(const u64 (&L)[kM]) { return list_max(L) == 0; }

// Insert candidate y (exact value) into list L with bound B.
__device__ __forceinline__ void list_insert(u64 (&L)[kM], u64 &B, u64 y) {
    if (y <= B) return;  // outside the list, and y <= B already holds
    // slot with the smallest key (an empty slot has key 0)
    u64 mn = L[0];
    int mi = 0;
#pragma unroll
    for (int i = 1; i < kM; ++i) {
        if (L[i] < mn) {
            mn = L[i];
            mi = i;
        }
    }
    if (mn != 0) {
        if (y < mn) {  // full and y is below every entry: it stays outside
            B = y;
            return;
        }
        B = umax64(B, mn);  // evict the smallest entry
    }
#pragma unroll
    for (int i = 0; i < kM; ++i)
        if (i == mi) L[i] = y;
}

// Remove entries whose job is j1 or j2.
__device__ __forceinline__ void list_drop_jobs(u64 (&L)[kM], int j1, int j2) {
#pragma unroll
    for (int i = 0; i < kM; ++i) {
        const int j = sidx(L[i]);
        if (L[i] != 0 && (j == j1 || j == j2)) L[i] = 0;
    }
}

// Wave 0 selects the kM largest of cand[0..cnt) into out[0..kM) and the
// (kM+1)-th into out[kM] (0 if none).  Destroys cand.  Keys are unique.
__device__ __forceinline__ void wave_select(u64 *cand, int cnt, u64 *out) {
    const int lane = threadIdx.x & 63;
    for (int round = 0; round <= kM; ++round) {
        u64 m = 0;
        int mi = -1;
        for (int i = lane; i < cnt; i += 64) {
            if (cand[i] > m) {
                m = cand[i];
                mi = i;
            }
        }
        u64 v = m;
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) v = umax64(v, shfl_xor64(v, s));
        if (v != 0 && m == v) cand[mi] = 0;
        if (lane == 0) out[round] = v;
    }
}

__device__ __forceinline__ bool spin_load(u64 *p, uint32_t tag, u64 &out) {
    long long spins = 0;
    for (;;) {
        u64 v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v & 0xFFFFu) == tag) {
            out = v;
            return true;
        }
        if (++spins > kSpinLimit) return false;
        __builtin_amdgcn_s_sleep(1);
    }
}

template <bool kLdsReplica>
__global__ __launch_bounds__(kT) void k_switch_ex(ExParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ u64 red[4 * 8];
    __shared__ u64 cand[kCand];
    __shared__ u64 sel[kM + 1];
    __shared__ int cand_n;
    __shared__ int dirty_list[kT];
    __shared__ int dirty_n;
    __shared__ int win_pay[2];
    __shared__ int s_err;

    if (P.flags[0]) return;  // same decision in every workgroup
    const int G = gridDim.x, q = blockIdx.x, t = threadIdx.x, n = P.n;
    const int64_t nn = n;

    uint16_t *rt;
    uint16_t *rs;
    int32_t *rd;
    u64 *wl = (u64 *)smem;  // gathered exchange words, G * kWords
    const size_t wl_bytes = ((size_t)G * kWords * sizeof(u64) + 15) & ~(size_t)15;
    if (kLdsReplica) {
        unsigned char *rb = smem + wl_bytes;
        rt = (uint16_t *)rb;
        rs = rt + n;
        rd = (int32_t *)(rb + (((size_t)4 * n + 15) & ~(size_t)15));
    } else {
        unsigned char *base = P.rep + (size_t)q * (size_t)n * 8;
        rt = (uint16_t *)base;
        rs = rt + n;
        rd = (int32_t *)(base + (size_t)4 * n);
    }
    for (int c = t; c < n; c += kT) {
        rt[c] = (uint16_t)P.tau[c];
        rs[c] = (uint16_t)P.sigma[c];
        rd[c] = P.d[c];
    }
    if (t == 0) s_err = 0;

    const int R = P.rows;
    const int r = q * R + t;  // this thread's agent (threads t < R own one each)
    const bool mine = t < R && r < n;
    u64 L[kM];
#pragma unroll
    for (int i = 0; i < kM; ++i) L[i] = 0;
    u64 B = 0;
    if (mine) {
#pragma unroll
        for (int i = 0; i < kM && i < kScanListLen; ++i) L[i] = from_long(P.lists[(size_t)r * kScanListLen + i]);
        B = from_long(P.bb[r]);
    }
    bool dirty = false;
    __syncthreads();

    int pis = -1, pk = -1;          // agents switched last: lists come from the shares
    u64 ppi1 = 0, ppi2 = 0, ppi3 = 0;  // this workgroup's top-3 share for pis
    u64 ppk1 = 0, ppk2 = 0, ppk3 = 0;  // ... and for pk
    int64_t S = 0, gsum = 0, rescans = 0, stalls = 0;

    for (uint32_t s = 0;; ++s) {
        const uint32_t tag = s & 0xFFFFu;
        u64 *buf = P.words + (size_t)(s & 1) * G * kWords;

        // -- best owned agent, and the bound of the pending ones -------------------
        u64 lk = 0, pend = 0;
        if (mine && r != pis && r != pk) {
            if (!dirty) {
                const u64 b = list_max(L);
                if (b) lk = skey(sgain(b), r);
            } else {
                pend = skey(sgain(B), r);
            }
        }
        {
            u64 v[2] = {lk, pend};
            block_max_n<2>(v, red);
            if (t == 0) {
                // job of the best owned agent (its owner thread posts it below)
                win_pay[0] = 0xFFFF;
            }
            __syncthreads();
            if (v[0] != 0 && lk == v[0]) win_pay[0] = sidx(list_max(L));
            if (t == 0) dirty_n = 0;
            __syncthreads();
            if (t < kWords) {
                u64 w;
                switch (t) {
                    case 0: w = v[0]; break;
                    case 1: w = (u64)(uint32_t)win_pay[0] << 16; break;
                    case 2: w = v[1]; break;
                    case 3: w = ppi1; break;
                    case 4: w = ppi2; break;
                    case 5: w = ppi3; break;
                    case 6: w = ppk1; break;
                    case 7: w = ppk2; break;
                    default: w = ppk3; break;
                }
                __hip_atomic_store(&buf[(size_t)q * kWords + t], kpart(w) | tag, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }

        // -- full re-evaluation of owned agents whose list ran empty ---------------
        // (overlaps the wait for the other workgroups' words)
        if (dirty) dirty_list[atomicAdd(&dirty_n, 1)] = r;
        __syncthreads();
        const int nd = dirty_n;
        for (int e = 0; e < nd; ++e) {
            const int rr = dirty_list[e];
            const int32_t *Wr = P.W + (int64_t)rr * nn;
            const int32_t *Tr = P.AT + (int64_t)rt[rr] * nn;
            const int dr = rd[rr];
            u64 t1 = 0, t2 = 0, t3 = 0;
            int g3 = INT32_MIN;  // gain of t3: most candidates fail this int32 test
            auto consider = [&](int c, int g) {
                if (g >= g3 && c != rr) {
                    top3_push(t1, t2, t3, skey(g, rt[c]));
                    g3 = t3 ? sgain(t3) : INT32_MIN;
                }
            };
            if ((n & 3) == 0) {
                // 8 int4 loads of each row in flight per thread
                constexpr int U = 8;
                for (int base = 4 * t; base < n; base += 4 * kT * U) {
                    int4 wv[U], tv[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int c4 = base + u * 4 * kT;
                        if (c4 < n) {
                            wv[u] = *(const int4 *)(Wr + c4);
                            tv[u] = *(const int4 *)(Tr + c4);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int c4 = base + u * 4 * kT;
                        if (c4 < n) {
                            const int4 dv = *(const int4 *)(rd + c4);
                            consider(c4, (wv[u].x + tv[u].x) - (dr + dv.x));
                            consider(c4 + 1, (wv[u].y + tv[u].y) - (dr + dv.y));
                            consider(c4 + 2, (wv[u].z + tv[u].z) - (dr + dv.z));
                            consider(c4 + 3, (wv[u].w + tv[u].w) - (dr + dv.w));
                        }
                    }
                }
            } else {
                constexpr int U = 8;
                for (int base = t; base < n; base += kT * U) {
                    int wv[U], tv[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int c = base + u * kT;
                        if (c < n) {
                            wv[u] = Wr[c];
                            tv[u] = Tr[c];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int c = base + u * kT;
                        if (c < n) consider(c, (wv[u] + tv[u]) - (dr + rd[c]));
                    }
                }
            }
            u64 b3[1] = {t3};
            block_max_n<1>(b3, red);
            if (t == 0) cand_n = 0;
            __syncthreads();
            if (t1 > b3[0]) cand[atomicAdd(&cand_n, 1)] = t1;
            if (t2 > b3[0]) cand[atomicAdd(&cand_n, 1)] = t2;
            __syncthreads();
            if (t < 64) wave_select(cand, cand_n, sel);
            __syncthreads();
            if (mine && r == rr) {
#pragma unroll
                for (int i = 0; i < kM; ++i) L[i] = sel[i];
                B = umax64(b3[0], sel[kM]);
                dirty = false;
            }
            __syncthreads();
        }
        rescans += nd;

        // -- gather every workgroup's words -----------------------------------------
        // All loads are issued at once; a word is current when its tag matches.
        {
            const int NW = G * kWords;
            u64 wv[kGatherPer];
#pragma unroll
            for (int i = 0; i < kGatherPer; ++i) {
                const int x = t + i * kT;
                wv[i] = x < NW ? __hip_atomic_load(&buf[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : (u64)tag;
            }
            long long spins = 0;
            for (;;) {
                bool ready = true;
#pragma unroll
                for (int i = 0; i < kGatherPer; ++i) ready &= (uint32_t)(wv[i] & 0xFFFFu) == tag;
                if (ready) break;
                if (++spins > kSpinLimit) {
                    s_err = 1;
                    atomicOr(P.err, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int i = 0; i < kGatherPer; ++i) {
                    const int x = t + i * kT;
                    if ((uint32_t)(wv[i] & 0xFFFFu) != tag)
                        wv[i] = __hip_atomic_load(&buf[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
#pragma unroll
            for (int i = 0; i < kGatherPer; ++i) {
                const int x = t + i * kT;
                if (x < NW) wl[x] = kpart(wv[i]) | (wv[i] & 0xFFFFu);
            }
        }
        __syncthreads();
        u64 x0 = 0, x1 = 0, x2 = 0, xi1 = 0, xi2 = 0, xi3 = 0, xk1 = 0, xk2 = 0, xk3 = 0;
        if (t < G) {
            const u64 *w = wl + (size_t)t * kWords;
            x0 = kpart(w[0]);
            x1 = w[1];
            x2 = kpart(w[2]);
            xi1 = kpart(w[3]);
            xi2 = kpart(w[4]);
            xi3 = kpart(w[5]);
            xk1 = kpart(w[6]);
            xk2 = kpart(w[7]);
            xk3 = kpart(w[8]);
        }
        u64 v[6] = {x0, x2, xi1, xk1, xi3, xk3};
        block_max_n<6>(v, red);
        if (s_err) break;
        // v: [0] best owned (all) [1] pending max [2] best share of pis [3] of pk
        //    [4] bound of pis's shares [5] of pk's shares
        if (v[0] != 0 && x0 == v[0]) win_pay[0] = (int)((x1 >> 16) & 0xFFFFu);
        __syncthreads();
        u64 best = v[0];
        int bj = (v[0] != 0) ? win_pay[0] : -1;
        if (pis >= 0 && v[2] != 0) {
            const u64 c2 = skey(sgain(v[2]), pis);
            if (c2 > best) {
                best = c2;
                bj = sidx(v[2]);
            }
        }
        if (pk >= 0 && v[3] != 0) {
            const u64 c2 = skey(sgain(v[3]), pk);
            if (c2 > best) {
                best = c2;
                bj = sidx(v[3]);
            }
        }

        // owners rebuild the lists of the two agents switched last
        for (int which = 0; which < 2; ++which) {
            const int row = which == 0 ? pis : pk;
            if (row < 0 || row / R != q) continue;  // uniform across the workgroup
            const u64 bnd = which == 0 ? v[4] : v[5];
            if (t == 0) cand_n = 0;
            __syncthreads();
            if (t < G) {
                const u64 c1 = which == 0 ? xi1 : xk1;
                const u64 c2 = which == 0 ? xi2 : xk2;
                if (c1 > bnd) cand[atomicAdd(&cand_n, 1)] = c1;
                if (c2 > bnd) cand[atomicAdd(&cand_n, 1)] = c2;
            }
            __syncthreads();
            if (t < 64) wave_select(cand, cand_n, sel);
            __syncthreads();
            if (mine && r == row) {
#pragma unroll
                for (int i = 0; i < kM; ++i) L[i] = sel[i];
                B = umax64(bnd, sel[kM]);
                dirty = false;
            }
            __syncthreads();
        }

        const bool stall = v[1] != 0 && v[1] > best && sgain(v[1]) > 0;
        if (stall) {
            // a pending agent might hold the best exchange: no switch this round;
            // its list is exact by now and is published next round.
            ++stalls;
            pis = pk = -1;
            ppi1 = ppi2 = ppi3 = ppk1 = ppk2 = ppk3 = 0;
            continue;
        }
        const int gw = best ? sgain(best) : 0;
        if (best == 0 || gw <= 0 || (P.max_switches >= 0 && S >= P.max_switches)) break;

        // -- apply the switch ------------------------------------------------------------
        const int is = sidx(best);
        const int js = bj;
        if (is < 0 || is >= n || js < 0 || js >= n) {  // cannot happen; never index with it
            if (t == 0) atomicOr(P.err, 2);
            break;
        }
        const int k = rs[js];
        const int j0 = rt[is];
        // every load of this switch is issued before the replicas change
        const int dis = P.A[(int64_t)is * nn + js];  // a[i*][j*]
        const int dk = P.A[(int64_t)k * nn + j0];    // a[k][j0]
        int a1 = 0, a2 = 0, w1 = 0, w2 = 0, tr = 0, dr = 0;
        if (mine) {
            if (r == is) {
                a2 = P.AT[(int64_t)j0 * nn + is];  // a[i*][j0]: new W[i*][k]
            } else if (r == k) {
                a1 = P.AT[(int64_t)js * nn + k];  // a[k][j*]: new W[k][i*]
            } else {
                tr = rt[r];
                dr = rd[r];
                a1 = P.AT[(int64_t)js * nn + r];  // a[r][j*]: new W[r][i*]
                a2 = P.AT[(int64_t)j0 * nn + r];  // a[r][j0]: new W[r][k]
                w1 = P.A[(int64_t)is * nn + tr];  // a[i*][tau(r)]
                w2 = P.A[(int64_t)k * nn + tr];   // a[k][tau(r)]
            }
        }
        ++S;
        gsum += gw;
        __syncthreads();  // everyone has read rt/rs/rd for this switch
        if (t == 0) {
            rt[is] = (uint16_t)js;
            rt[k] = (uint16_t)j0;
            rs[js] = (uint16_t)is;
            rs[j0] = (uint16_t)k;
            rd[is] = dis;
            rd[k] = dk;
        }
        // (the next reads of the replicas come after further barriers)

        // -- the two changed candidates of every owned agent ---------------------------
        u64 si1 = 0, si2 = 0, si3 = 0, sk1 = 0, sk2 = 0, sk3 = 0;
        if (mine) {
            int32_t *Wr = P.W + (int64_t)r * nn;
            if (r == is) {
                sk1 = skey(-gw, js);  // g(k, i*) = -gain, job of i* is j*
#pragma unroll
                for (int i = 0; i < kM; ++i) L[i] = 0;
                B = 0;
                Wr[is] = dis;
                Wr[k] = a2;
            } else if (r == k) {
                si1 = skey(-gw, j0);  // g(i*, k) = -gain, job of k is j0
#pragma unroll
                for (int i = 0; i < kM; ++i) L[i] = 0;
                B = 0;
                Wr[is] = a1;
                Wr[k] = dk;
            } else {
                const int g1 = (a1 + w1) - (dr + dis);  // g(r, i*)
                const int g2 = (a2 + w2) - (dr + dk);   // g(r, k)
                Wr[is] = a1;
                Wr[k] = a2;
                list_drop_jobs(L, js, j0);
                list_insert(L, B, skey(g1, js));
                list_insert(L, B, skey(g2, j0));
                dirty = list_empty(L);
                si1 = skey(g1, tr);
                sk1 = skey(g2, tr);
            }
        }
        block_top3(si1, si2, si3, red);
        block_top3(sk1, sk2, sk3, red);
        ppi1 = si1;
        ppi2 = si2;
        ppi3 = si3;
        ppk1 = sk1;
        ppk2 = sk2;
        ppk3 = sk3;
        pis = is;
        pk = k;
    }

    if (mine) P.tau[r] = rt[r];
    if (t == 0) {
        if (rescans) atomicAdd((unsigned long long *)&P.stats[3], (unsigned long long)rescans);
        if (stalls) atomicAdd((unsigned long long *)&P.stats[4], (unsigned long long)stalls);
        if (q == 0) {
            P.stats[0] = S;
            P.stats[1] = gsum;
        }
    }
}

}  // namespace

// ---- host side ---------------------------------------------------------------------------

int switch_ex_grid(int n) { return (n + rows_per_wg(n) - 1) / rows_per_wg(n); }
size_t switch_ex_word_bytes(int n) { return 2 * (size_t)switch_ex_grid(n) * kWords * sizeof(u64); }
bool switch_ex_lds_replica(int n) { return (size_t)8 * n + 16 <= kExLdsReplicaBytes; }
size_t switch_ex_replica_bytes(int n) {
    return switch_ex_lds_replica(n) ? 0 : (size_t)switch_ex_grid(n) * (size_t)n * 8;
}

hipError_t launch_switch_ex(const Instance &I, int64_t max_switches, void *words, void *replica,
                            int32_t *err, bool coop, hipStream_t s) {
    ExParams P;
    P.A = I.A;
    P.AT = I.AT;
    P.W = I.W;
    P.tau = I.tau;
    P.sigma = I.sigma;
    P.d = I.d;
    P.lists = I.lists;
    P.bb = I.bb;
    P.words = (u64 *)words;
    P.rep = (unsigned char *)replica;
    P.stats = I.stats;
    P.flags = I.flags;
    P.err = err;
    P.n = I.n;
    P.rows = rows_per_wg(I.n);
    P.max_switches = max_switches;
    const int grid = switch_ex_grid(I.n);
    void *args[] = {&P};
    const size_t wl_bytes = ((size_t)grid * kWords * sizeof(u64) + 15) & ~(size_t)15;
    if (switch_ex_lds_replica(I.n)) {
        const size_t shm = wl_bytes + (((size_t)4 * I.n + 15) & ~(size_t)15) + (size_t)4 * I.n;
        hipError_t e = hipFuncSetAttribute((const void *)k_switch_ex<true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        if (!coop) {
            hipLaunchKernelGGL(k_switch_ex<true>, dim3((unsigned)grid), dim3(kT), shm, s, P);
            return hipGetLastError();
        }
        return hipLaunchCooperativeKernel((const void *)k_switch_ex<true>, dim3((unsigned)grid), dim3(kT), args,
                                          (unsigned)shm, s);
    }
    hipError_t e = hipFuncSetAttribute((const void *)k_switch_ex<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)wl_bytes);
    if (e != hipSuccess) return e;
    if (!coop) {
        hipLaunchKernelGGL(k_switch_ex<false>, dim3((unsigned)grid), dim3(kT), wl_bytes, s, P);
        return hipGetLastError();
    }
    return hipLaunchCooperativeKernel((const void *)k_switch_ex<false>, dim3((unsigned)grid), dim3(kT), args,
                                      (unsigned)wl_bytes, s);
}

}  // namespace dgs
