// Batched DGS on gfx950: many independent instances (n <= kBatchMaxN).  The
// greedy starts and the switching run in persistent launches whose workgroups
// take instances from a device-side queue (largest first) and work on each one
// alone; the transposes and the difference evaluations of all instances are
// spread over the whole device between them:
//   1. greedy start (Section 3.1) with the value-range check fused in: agents
//      in order; thread t owns columns t, t + BLOCK, ...; one block max per
//      agent over the free columns (each thread tracks its own columns'
//      taken flags in registers);
//   2. AT = A^T of every instance, tile by tile, by the workgroups of the greedy
//      launch once no instance is left for them (hidden under the largest
//      instances' greedy starts, which would otherwise also transpose alone);
//   3. difference evaluation of every agent (Algorithm 2), for every instance
//      at once: k_batch_pairs scores the tile pairs of all instances (each
//      entry read once); the switching launch starts each agent from the top-2
//      of its partials (best exchange, bound);
//   4. switching (Algorithm 1 as steepest ascent): block max over the
//      agents' list maxima, apply, update every agent's two changed
//      candidates, rebuild the two switched agents' lists from the same
//      values (g(r, c) = g(c, r)), re-evaluate agents whose list ran empty.
// Results are identical to the single-instance path.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgs_device.h"
#include "dgs_internal.h"

namespace dgs {
namespace {

using namespace dev;

constexpr int kBM = 4;  // candidate list length per agent
constexpr int kMaxAbsB = 536870911;

// (gain:32 | 0xFFFF - row:16 | job:16): unsigned order = (gain asc, row desc);
// the job rides along (rows are unique).
__device__ __forceinline__ u64 wkey(int g, int row, int job) {
    return ((u64)((uint32_t)g ^ 0x80000000u) << 32) | ((u64)(0xFFFFu - (uint32_t)row) << 16) | (uint32_t)job;
}
__device__ __forceinline__ int wrow(u64 k) { return (int)(0xFFFFu - (uint32_t)((k >> 16) & 0xFFFFu)); }
__device__ __forceinline__ int wjob(u64 k) { return (int)(uint32_t)(k & 0xFFFFu); }

template <int BLOCK>
struct Red {
    static constexpr int W = BLOCK / 64;
};

// Block max of one u64; `slot` alternates between two LDS rows so that one
// barrier per call suffices.
template <int BLOCK>
__device__ __forceinline__ u64 bmax1(u64 v, u64 *red, int &slot) {
    v = wave_max64(v);
    u64 *row = red + slot * Red<BLOCK>::W;
    slot ^= 1;
    if ((threadIdx.x & 63) == 0) row[threadIdx.x >> 6] = v;
    __syncthreads();
    u64 r = row[0];
#pragma unroll
    for (int i = 1; i < Red<BLOCK>::W; ++i) r = umax64(r, row[i]);
    return r;
}

template <int BLOCK>
__device__ __forceinline__ void btop2(u64 &a1, u64 &a2, u64 *red, int &slot) {
    wave_top2(a1, a2);
    u64 *row = red + slot * 2 * Red<BLOCK>::W;
    slot ^= 1;
    if ((threadIdx.x & 63) == 0) {
        row[2 * (threadIdx.x >> 6)] = a1;
        row[2 * (threadIdx.x >> 6) + 1] = a2;
    }
    __syncthreads();
    a1 = row[0];
    a2 = row[1];
#pragma unroll
    for (int i = 1; i < Red<BLOCK>::W; ++i) top2_merge(a1, a2, row[2 * i], row[2 * i + 1]);
}

// Unsorted list of kBM exact candidates (0 = empty) plus bound.
__device__ __forceinline__ u64 lmax(const u64 *L) {
    u64 m = L[0];
#pragma unroll
    for (int i = 1; i < kBM; ++i) m = umax64(m, L[i]);
    return m;
}
__device__ __forceinline__ void ldrop(u64 *L, int j1, int j2) {
#pragma unroll
    for (int i = 0; i < kBM; ++i) {
        const int j = key_index(L[i]);
        if (L[i] != 0 && (j == j1 || j == j2)) L[i] = 0;
    }
}
__device__ __forceinline__ void linsert(u64 *L, u64 &B, u64 y) {
    if (y <= B) return;
    u64 mn = L[0];
    int mi = 0;
#pragma unroll
    for (int i = 1; i < kBM; ++i)
        if (L[i] < mn) {
            mn = L[i];
            mi = i;
        }
    if (mn != 0) {
        if (y < mn) {
            B = y;
            return;
        }
        B = umax64(B, mn);
    }
#pragma unroll
    for (int i = 0; i < kBM; ++i)
        if (i == mi) L[i] = y;
}

// Full evaluation of agent r by one wave (row of A staged in `arow`).
// Returns top-2 keys (gain, job) over partners c != r in lane 0..63 (all lanes).
// Both rows are loaded with every load in flight at once (one memory round
// trip per agent).
__device__ __forceinline__ void wave_eval_row(const int32_t *A, const int32_t *AT, int n, int r,
                                              const uint16_t *rt, const int32_t *rd, int32_t *arow, u64 &b1,
                                              u64 &b2) {
    constexpr int kPer = kBatchMaxN / 64;
    const int lane = threadIdx.x & 63;
    const int32_t *Ar = A + (int64_t)r * n;
    const int32_t *Tr = AT + (int64_t)rt[r] * n;
    int av[kPer], tv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int c = lane + 64 * u;
        av[u] = c < n ? Ar[c] : 0;
        tv[u] = c < n ? Tr[c] : 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // earlier reads of arow are done
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int c = lane + 64 * u;
        if (c < n) arow[c] = av[u];
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // the row is in LDS for every lane
    const int dr = rd[r];
    b1 = 0;
    b2 = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int c = lane + 64 * u;
        if (c < n && c != r) top2_push(b1, b2, mk_key((arow[rt[c]] + tv[u]) - (dr + rd[c]), rt[c]));
    }
    wave_top2(b1, b2);
}

// PHASE 0: the greedy start with the range check (tau and res[0], res[4] out); then,
// once no instance is left, the transposes AT = A^T of all instances, tiles taken from
// queue word 2 (they hide under the largest instances' greedy starts).  PHASE 1: the
// switching, each agent starting from the top-2 of its partials from k_batch_pairs
// (which runs between the two launches).  Each phase takes the instances from its own
// queue word, largest first.
template <int BLOCK, int PHASE>
__global__ __launch_bounds__(BLOCK) void k_batch_solve(const BatchItem *items, const int32_t *order, int count,
                                                        int32_t *queue, int64_t max_switches, int64_t tiles) {
    constexpr int RPT = kBatchMaxN / BLOCK;  // agents (and columns) per thread
    constexpr int NW = BLOCK / 64;
    __shared__ uint16_t rt[kBatchMaxN];
    __shared__ uint16_t rs[kBatchMaxN];
    __shared__ int32_t rd[kBatchMaxN];
    __shared__ int32_t rowbuf[NW][kBatchMaxN + 64];  // per-wave staged rows
    __shared__ u64 red[4 * NW];
    __shared__ int s_item;
    __shared__ int dirty_list[kBatchMaxN];
    __shared__ int dirty_n;

    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    int slot = 0;

    for (;;) {
        if (t == 0) s_item = atomicAdd(&queue[PHASE], 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= count) break;
        const BatchItem I = items[order[it]];
        const int n = I.n;
        const int32_t *A = I.A;
        if constexpr (PHASE == 0) {
        // ---- 1. greedy start + range check -----------------------------------------------
        bool taken[RPT];
#pragma unroll
        for (int u = 0; u < RPT; ++u) taken[u] = false;
        int bad = 0;
        int64_t f0 = 0;
        // rows are loaded kAhead agents ahead, every load unconditional (clamped addresses,
        // values outside the instance unused) so that each wait covers exactly one row
        constexpr int kAhead = 4;
        int nv[kAhead][RPT];
#pragma unroll
        for (int d = 0; d < kAhead; ++d) {
            const int32_t *Ar = A + (int64_t)min(d, n - 1) * n;
#pragma unroll
            for (int u = 0; u < RPT; ++u) nv[d][u] = Ar[min(t + u * BLOCK, n - 1)];
        }
        for (int i0 = 0; i0 < n; i0 += kAhead) {
#pragma unroll
            for (int d = 0; d < kAhead; ++d) {
                const int i = i0 + d;
                if (i >= n) break;
                int v[RPT];
#pragma unroll
                for (int u = 0; u < RPT; ++u) v[u] = nv[d][u];
                {
                    const int32_t *Ar = A + (int64_t)min(i + kAhead, n - 1) * n;
#pragma unroll
                    for (int u = 0; u < RPT; ++u) nv[d][u] = Ar[min(t + u * BLOCK, n - 1)];
                }
                u64 best = 0;
#pragma unroll
                for (int u = 0; u < RPT; ++u) {
                    const int c = t + u * BLOCK;
                    if (c < n) {
                        bad |= (v[u] > kMaxAbsB) | (v[u] < -kMaxAbsB);
                        if (!taken[u]) best = umax64(best, mk_key(v[u], c));
                    }
                }
                best = bmax1<BLOCK>(best, red, slot);
                const int c = best ? key_index(best) : 0;  // a free column always exists
                if (c % BLOCK == t) {
#pragma unroll
                    for (int u = 0; u < RPT; ++u)
                        if (u == c / BLOCK) taken[u] = true;
                }
                if (t == 0) {
                    rt[i] = (uint16_t)c;
                    rs[c] = (uint16_t)i;
                    rd[i] = key_gain(best);
                }
                f0 += key_gain(best);
            }
        }
        {
            u64 b = bad ? 1 : 0;
            b = bmax1<BLOCK>(b, red, slot);
            bad = (int)b;
        }
        if (bad) {
            if (t == 0) {
                I.res[4] = DGS_E_RANGE;
                I.res[0] = I.res[1] = I.res[2] = I.res[3] = 0;
            }
            __syncthreads();
            continue;
        }

        for (int r = t; r < n; r += BLOCK) I.tau[r] = rt[r];
        if (t == 0) {
            I.res[0] = f0;
            I.res[4] = DGS_OK;
        }
        __syncthreads();
        continue;
        } else {
        // (AT = A^T was written by the greedy launch, the evaluation's partials by
        // k_batch_pairs)
        if (I.res[4] != DGS_OK) {  // the range check failed (same in every thread)
            __syncthreads();
            continue;
        }
        // the greedy start: tau, sigma and the benefits d
        for (int r = t; r < n; r += BLOCK) {
            const int j = I.tau[r];
            rt[r] = (uint16_t)j;
            rs[j] = (uint16_t)r;
            rd[r] = A[(int64_t)r * n + j];
        }
        const int64_t f0 = I.res[0];
        __syncthreads();
        // ---- 3 (end). each agent's best exchange and bound: the top-2 of its partials --------
        u64 L[RPT][kBM];
        u64 B[RPT];
        const int nb = (n + 63) >> 6;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int r = t + u * BLOCK;
#pragma unroll
            for (int i = 0; i < kBM; ++i) L[u][i] = 0;
            u64 b1 = 0, b2 = 0;
            if (r < n) {
                const u64 *pp = I.part + (size_t)r * nb * 2;
                for (int x = 0; x < nb; ++x) top2_merge(b1, b2, pp[2 * x], pp[2 * x + 1]);
            }
            L[u][0] = b1;
            B[u] = b2;
        }

        // ---- 4. switching ---------------------------------------------------------------------
        int64_t S = 0, gsum = 0, rescans = 0;
        for (;;) {
            u64 mine = 0;
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int r = t + u * BLOCK;
                if (r < n) {
                    const u64 b = lmax(L[u]);
                    if (b) mine = umax64(mine, wkey(key_gain(b), r, key_index(b)));
                }
            }
            const u64 best = bmax1<BLOCK>(mine, red, slot);
            const int gw = best ? (int)((uint32_t)(best >> 32) ^ 0x80000000u) : 0;
            if (best == 0 || gw <= 0 || (max_switches >= 0 && S >= max_switches)) break;
            const int is = wrow(best), js = wjob(best);
            const int k = rs[js], j0 = rt[is];
            const int dis = A[(int64_t)is * n + js];
            const int dk = A[(int64_t)k * n + j0];
            // loads of the two changed candidates of every owned agent
            int a1[RPT], a2[RPT], w1[RPT], w2[RPT], dr[RPT], tr[RPT];
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int r = t + u * BLOCK;
                a1[u] = a2[u] = w1[u] = w2[u] = dr[u] = tr[u] = 0;
                if (r < n && r != is && r != k) {
                    tr[u] = rt[r];
                    dr[u] = rd[r];
                    a1[u] = I.AT[(int64_t)js * n + r];
                    a2[u] = I.AT[(int64_t)j0 * n + r];
                    w1[u] = A[(int64_t)is * n + tr[u]];
                    w2[u] = A[(int64_t)k * n + tr[u]];
                }
            }
            ++S;
            gsum += gw;
            __syncthreads();  // every thread has read rt / rs / rd
            if (t == 0) {
                rt[is] = (uint16_t)js;
                rt[k] = (uint16_t)j0;
                rs[js] = (uint16_t)is;
                rs[j0] = (uint16_t)k;
                rd[is] = dis;
                rd[k] = dk;
                dirty_n = 0;
            }
            u64 pi1 = 0, pi2 = 0, pk1 = 0, pk2 = 0;  // candidates of agents i* and k
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int r = t + u * BLOCK;
                if (r >= n) continue;
                if (r == is) {
                    top2_push(pk1, pk2, mk_key(-gw, js));
                    continue;
                }
                if (r == k) {
                    top2_push(pi1, pi2, mk_key(-gw, j0));
                    continue;
                }
                const int g1 = (a1[u] + w1[u]) - (dr[u] + dis);
                const int g2 = (a2[u] + w2[u]) - (dr[u] + dk);
                ldrop(L[u], js, j0);
                linsert(L[u], B[u], mk_key(g1, js));
                linsert(L[u], B[u], mk_key(g2, j0));
                top2_push(pi1, pi2, mk_key(g1, tr[u]));
                top2_push(pk1, pk2, mk_key(g2, tr[u]));
            }
            __syncthreads();  // dirty_n reset and replicas visible
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int r = t + u * BLOCK;
                if (r < n && r != is && r != k && lmax(L[u]) == 0) dirty_list[atomicAdd(&dirty_n, 1)] = r;
            }
            btop2<BLOCK>(pi1, pi2, red, slot);
            btop2<BLOCK>(pk1, pk2, red, slot);
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int r = t + u * BLOCK;
                if (r == is || r == k) {
#pragma unroll
                    for (int i = 0; i < kBM; ++i) L[u][i] = 0;
                    L[u][0] = r == is ? pi1 : pk1;
                    B[u] = r == is ? pi2 : pk2;
                }
            }
            __syncthreads();
            const int nd = dirty_n;
            // full re-evaluation of agents whose list ran empty, one per wave
            for (int e = w; e < nd; e += NW) {
                const int r = dirty_list[e];
                u64 b1, b2;
                wave_eval_row(A, I.AT, n, r, rt, rd, rowbuf[w], b1, b2);
                if (lane == 0) {
                    I.lists[2 * r] = b1;
                    I.lists[2 * r + 1] = b2;
                }
            }
            rescans += nd;
            __syncthreads();
            if (nd) {
#pragma unroll
                for (int u = 0; u < RPT; ++u) {
                    const int r = t + u * BLOCK;
                    if (r < n && r != is && r != k && lmax(L[u]) == 0) {
                        L[u][0] = I.lists[2 * r];
                        B[u] = I.lists[2 * r + 1];
                    }
                }
            }
        }

        // ---- 5. output ---------------------------------------------------------------------------
        for (int r = t; r < n; r += BLOCK) I.tau[r] = rt[r];
        if (t == 0) {
            I.res[0] = f0;
            I.res[1] = f0 + gsum;
            I.res[2] = S;
            I.res[3] = rescans;
            I.res[4] = DGS_OK;
        }
        __syncthreads();
        }
    }
    if constexpr (PHASE == 0) {
        // ---- 2. transposes of all instances: chunks of tiles from queue word 2 --------------
        // Tile g belongs to the last item x (table order) with items[x].tile0 <= g; a chunk
        // searches once and then walks forward.
        constexpr int kChunk = 8;
        int32_t(*tile)[65] = reinterpret_cast<int32_t(*)[65]>(&rowbuf[0][0]);  // 64 x 65 of the row buffers
        static_assert(NW * (kBatchMaxN + 64) >= 64 * 65, "tile fits the row buffers");
        for (;;) {
            if (t == 0) s_item = atomicAdd(&queue[2], kChunk);
            __syncthreads();
            const int64_t g0 = s_item;
            __syncthreads();
            if (g0 >= tiles) break;
            int x = 0, hi = count - 1;
            while (x < hi) {
                const int mid = (x + hi + 1) >> 1;
                if (items[mid].tile0 <= g0)
                    x = mid;
                else
                    hi = mid - 1;
            }
            for (int64_t g = g0; g < g0 + kChunk && g < tiles; ++g) {
                while (x + 1 < count && items[x + 1].tile0 <= g) ++x;
                const int32_t *A = items[x].A;
                int32_t *AT = items[x].AT;
                const int n = items[x].n, nt = (n + 63) >> 6;
                const int local = (int)(g - items[x].tile0), bi = local / nt, bj = local % nt;
                constexpr int RW = 64 / NW;  // rows per wave
                int v[RW];
#pragma unroll
                for (int k = 0; k < RW; ++k) {
                    const int row = bi * 64 + w + NW * k, col = bj * 64 + lane;
                    v[k] = (row < n && col < n) ? A[(int64_t)row * n + col] : 0;
                }
#pragma unroll
                for (int k = 0; k < RW; ++k) tile[w + NW * k][lane] = v[k];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < RW; ++k) {
                    const int col = bj * 64 + w + NW * k, row = bi * 64 + lane;
                    if (col < n && row < n) AT[(int64_t)col * n + row] = tile[lane][w + NW * k];
                }
                __syncthreads();  // the tile is rewritten next
            }
        }
    }
}

// The difference evaluation of every instance over the whole device: workgroup g scores
// tile pair g of the batch (the last item x, in table order, with items[x].pair0 <= g;
// an item whose range check failed is skipped).  Tile pair (I, K), I <= K, of an
// instance: g(i, k) = a[i][tau(k)] + a[k][tau(i)] - d(i) - d(k) for i in block I, k in
// block K, both tiles read from A^T through tau (row tau(x) of A^T holds a[.][tau(x)]);
// per (agent, partner block) the top-2 keys (gain, job) into the instance's partials.
__global__ __launch_bounds__(512) void k_batch_pairs(const BatchItem *items, int count) {
    constexpr int BLOCK = 512, Q = BLOCK / 64, E = 64 / Q, LD = (64 * 64 / 4) / BLOCK;
    __shared__ int32_t tA[64][65];
    __shared__ int32_t tB[64][65];
    __shared__ int32_t dI[64], dK[64], jI[64], jK[64];
    const int64_t g = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].pair0 <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    if (items[lo].res[4] != DGS_OK) return;
    const int32_t *A = items[lo].A, *AT = items[lo].AT, *tau = items[lo].tau;
    u64 *part = items[lo].part;
    const int n = items[lo].n, nb = (n + 63) >> 6;
    int bI, bK;
    pair_of(g - items[lo].pair0, nb, bI, bK);
    const int i0 = bI * 64, k0 = bK * 64, t = threadIdx.x;
    auto row = [&](int x) { return AT + (int64_t)tau[x] * n; };
    if ((n % 4 == 0) && i0 + 64 <= n && k0 + 64 <= n) {
        int4 va[LD], vb[LD];
#pragma unroll
        for (int u = 0; u < LD; ++u) {
            const int e = t + u * BLOCK;
            const int r = e >> 4, c4 = (e & 15) * 4;
            va[u] = *(const int4 *)(row(i0 + r) + k0 + c4);
            vb[u] = *(const int4 *)(row(k0 + r) + i0 + c4);
        }
#pragma unroll
        for (int u = 0; u < LD; ++u) {
            const int e = t + u * BLOCK;
            const int r = e >> 4, c4 = (e & 15) * 4;
            tA[r][c4] = va[u].x;
            tA[r][c4 + 1] = va[u].y;
            tA[r][c4 + 2] = va[u].z;
            tA[r][c4 + 3] = va[u].w;
            tB[r][c4] = vb[u].x;
            tB[r][c4 + 1] = vb[u].y;
            tB[r][c4 + 2] = vb[u].z;
            tB[r][c4 + 3] = vb[u].w;
        }
    } else {
        for (int e = t; e < 64 * 64; e += BLOCK) {
            const int r = e >> 6, c = e & 63;
            tA[r][c] = (i0 + r < n && k0 + c < n) ? row(i0 + r)[k0 + c] : 0;
            tB[r][c] = (k0 + r < n && i0 + c < n) ? row(k0 + r)[i0 + c] : 0;
        }
    }
    if (t < 64) {
        const int x = i0 + t;
        jI[t] = x < n ? tau[x] : 0;
        dI[t] = x < n ? A[(int64_t)x * n + tau[x]] : 0;
    } else if (t < 128) {
        const int x = k0 + t - 64;
        jK[t - 64] = x < n ? tau[x] : 0;
        dK[t - 64] = x < n ? A[(int64_t)x * n + tau[x]] : 0;
    }
    __syncthreads();
    const int rt = t / Q, q = t % Q;
    u64 a1 = 0, a2 = 0, c1 = 0, c2 = 0;  // row rt of I against K; row rt of K against I
    if (bI != bK && i0 + 64 <= n && k0 + 64 <= n) {
        const int di = dI[rt], dk = dK[rt];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int c = q * E + e;
            top2_push(a1, a2, mk_key((tA[rt][c] + tB[c][rt]) - (di + dK[c]), jK[c]));
            top2_push(c1, c2, mk_key((tA[c][rt] + tB[rt][c]) - (dI[c] + dk), jI[c]));
        }
    } else {
        if (i0 + rt < n) {
            const int di = dI[rt];
            for (int e = 0; e < E; ++e) {
                const int k = q * E + e;
                if (k0 + k >= n || (bI == bK && k == rt)) continue;
                top2_push(a1, a2, mk_key((tA[rt][k] + tB[k][rt]) - (di + dK[k]), jK[k]));
            }
        }
        if (bI != bK && k0 + rt < n) {
            const int dk = dK[rt];
            for (int e = 0; e < E; ++e) {
                const int i = q * E + e;
                if (i0 + i >= n) continue;
                top2_push(c1, c2, mk_key((tA[i][rt] + tB[rt][i]) - (dI[i] + dk), jI[i]));
            }
        }
    }
    // merge the Q threads of each row (adjacent lanes; lane distances as template arguments)
    static_assert(Q == 8, "three merge steps");
    top2_merge(a1, a2, xor_lanes64<1>(a1), xor_lanes64<1>(a2));
    top2_merge(c1, c2, xor_lanes64<1>(c1), xor_lanes64<1>(c2));
    top2_merge(a1, a2, xor_lanes64<2>(a1), xor_lanes64<2>(a2));
    top2_merge(c1, c2, xor_lanes64<2>(c1), xor_lanes64<2>(c2));
    top2_merge(a1, a2, xor_lanes64<4>(a1), xor_lanes64<4>(a2));
    top2_merge(c1, c2, xor_lanes64<4>(c1), xor_lanes64<4>(c2));
    if (q == 0 && i0 + rt < n) {
        u64 *o = part + ((size_t)(i0 + rt) * nb + bK) * 2;
        o[0] = a1;
        o[1] = a2;
    }
    if (q == 0 && bI != bK && k0 + rt < n) {
        u64 *o = part + ((size_t)(k0 + rt) * nb + bI) * 2;
        o[0] = c1;
        o[1] = c2;
    }
}

}  // namespace

int batch_grid_limit(int block) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = block == 512
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_solve<512, 1>, 512, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_solve<256, 1>, 256, 0);
    if (e != hipSuccess || per < 1) return 0;
    return cus * per;
}

hipError_t launch_batch(const BatchItem *items, const int32_t *order, int count, int32_t *queue,
                        int64_t max_switches, const BatchTotals &tot, int block, int grid, hipStream_t s) {
    if (count < 1) return hipSuccess;
    // the greedy launch fills the device: workgroups without an instance transpose at once
    static int full[2] = {-1, -1};
    int &f = full[block == 512];
    if (f < 0) f = batch_grid_limit(block);
    const int grid0 = f > grid ? f : grid;
    if (block == 512)
        hipLaunchKernelGGL((k_batch_solve<512, 0>), dim3((unsigned)grid0), dim3(512), 0, s, items, order, count,
                           queue, max_switches, tot.tiles);
    else
        hipLaunchKernelGGL((k_batch_solve<256, 0>), dim3((unsigned)grid0), dim3(256), 0, s, items, order, count,
                           queue, max_switches, tot.tiles);
    hipLaunchKernelGGL(k_batch_pairs, dim3((unsigned)tot.pairs), dim3(512), 0, s, items, count);
    if (block == 512)
        hipLaunchKernelGGL((k_batch_solve<512, 1>), dim3((unsigned)grid), dim3(512), 0, s, items, order, count, queue,
                           max_switches, tot.tiles);
    else
        hipLaunchKernelGGL((k_batch_solve<256, 1>), dim3((unsigned)grid), dim3(256), 0, s, items, order, count, queue,
                           max_switches, tot.tiles);
    return hipGetLastError();
}

}  // namespace dgs
