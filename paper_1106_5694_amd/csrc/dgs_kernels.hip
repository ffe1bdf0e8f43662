// Deep Greedy Switching on gfx950: device kernels.
//
// Notation follows the paper (Roverso et al., arXiv:1106.5694, Section 3):
// a_ij benefit of agent i for job j; tau(i) job of agent i; sigma(j) agent of
// job j; switch(i, j, sigma) gives job j to agent i and i's old job to
// sigma(j).  Gains are exact int32 (|a| <= 2^29 - 1 is checked first).
//
// Working layout (built once per solve):
//   AT[j][i] = a_ij                      (transpose of the input)
//   W[r][c]  = a[r][tau(c)]              (benefit of agent r for agent c's job)
//   d[c]     = W[c][c]                   (current benefit of agent c)
// With it the gain of the 2-exchange between agents r and c is
//   g(r, c) = W[r][c] + W[c][r] - d[r] - d[c] = W[r][c] + AT[tau(r)][c] - d[r] - d[c]
// (the second form reads row r of W and row tau(r) of AT, both contiguous),
// and g(r, c) = g(c, r).  Agent r's candidate towards agent c is ranked by
// the packed key (gain, job tau(c)): larger gain first, lower job on ties
// (ADE, Algorithm 2, takes the first strictly better job in index order).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgs_device.h"
#include "dgs_internal.h"

namespace dgs {

namespace {

using namespace dev;

constexpr int kMaxAbs = 536870911;  // 2^29 - 1
constexpr int kLoopBlock = 256;

// ---- ingest ------------------------------------------------------------------

__global__ void k_range_check(const int32_t *__restrict__ A, int64_t count, int32_t *flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (; i < count; i += stride) {
        int v = A[i];
        bad |= (v > kMaxAbs) | (v < -kMaxAbs);
    }
    if (bad) atomicOr(flag, 1);
}

// ---- greedy start (Section 3.1) ----------------------------------------------
// Agents in index order; each takes the free job of largest benefit, lowest
// job on ties.  One workgroup; the taken-job bitmap lives in LDS.
constexpr int kGreedyBlock = 1024;

__global__ __launch_bounds__(kGreedyBlock) void k_greedy_wg(const int32_t *__restrict__ A, int n,
                                                              int32_t *tau, int32_t *sigma) {
    extern __shared__ uint32_t taken[];
    __shared__ u64 red[3 * kGreedyBlock / 64];
    const int words = (n + 31) >> 5;
    for (int w = threadIdx.x; w < words; w += blockDim.x) taken[w] = 0u;
    __syncthreads();
    for (int i = 0; i < n; ++i) {
        const int32_t *Ai = A + (int64_t)i * n;
        u64 best = 0;
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            if (!((taken[j >> 5] >> (j & 31)) & 1u)) best = umax64(best, mk_key(Ai[j], j));
        }
        best = block_max<kGreedyBlock>(best, red);
        if (threadIdx.x == 0) {
            int j = key_index(best);
            tau[i] = j;
            sigma[j] = i;
            taken[j >> 5] |= 1u << (j & 31);
        }
        __syncthreads();
    }
}

__global__ void k_fill(int32_t *p, int n, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// sigma = tau^-1, flagging a tau that is not a permutation.
__global__ void k_invert_checked(const int32_t *__restrict__ tau, int n, int32_t *sigma, int32_t *flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int j = tau[i];
    if (j < 0 || j >= n) {
        atomicOr(flag, 1);
        return;
    }
    int old = atomicExch(&sigma[j], i);
    if (old != -1) atomicOr(flag, 1);
}

// ---- layout build ---------------------------------------------------------------

__global__ __launch_bounds__(256) void k_transpose(const int32_t *__restrict__ A, int32_t *__restrict__ AT,
                                                     int n) {
    __shared__ int32_t tile[64][65];
    const int bx = blockIdx.x * 64, by = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        int row = by + r, col = bx + tx;
        if (row < n && col < n) tile[r][tx] = A[(int64_t)row * n + col];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        int row = bx + r, col = by + tx;
        if (row < n && col < n) AT[(int64_t)row * n + col] = tile[tx][r];
    }
}

// W[r][c] = a[r][tau(c)] = AT[tau(c)][r]: a transpose whose source rows are
// picked through tau.  Each 64 x 64 tile reads 64 row segments of AT and
// writes 64 row segments of W, both coalesced, through an LDS tile.
__global__ __launch_bounds__(256) void k_build_w(const int32_t *__restrict__ AT, const int32_t *__restrict__ tau,
                                                   int n, int32_t *__restrict__ W) {
    __shared__ int32_t tile[64][65];
    const int bx = blockIdx.x * 64, by = blockIdx.y * 64;  // bx: agents r, by: agents c
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int c = ty; c < 64; c += 4) {
        const int cc = by + c, rr = bx + tx;
        if (cc < n && rr < n) tile[c][tx] = AT[(int64_t)tau[cc] * n + rr];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int rr = bx + r, cc = by + tx;
        if (rr < n && cc < n) W[(int64_t)rr * n + cc] = tile[tx][r];
    }
}

// d[r] = a[r][tau(r)] and f0 = sum of d.
__global__ __launch_bounds__(256) void k_benefits(const int32_t *__restrict__ A, const int32_t *__restrict__ tau,
                                                    int n, int32_t *d, unsigned long long *f0) {
    __shared__ long long part[4];
    const int r = blockIdx.x * 256 + threadIdx.x;
    long long v = 0;
    if (r < n) {
        const int x = A[(int64_t)r * n + tau[r]];
        d[r] = x;
        v = x;
    }
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(f0, (unsigned long long)(part[0] + part[1] + part[2] + part[3]));
}

// ---- difference evaluation of every agent (Algorithm 2) ---------------------------
// One workgroup per agent r: top-2 keys over partners c != r.  The best is
// the agent's exchange (gain, job); the second is the bound kept with it.
__global__ __launch_bounds__(256) void k_scan_rows(const int32_t *__restrict__ W, const int32_t *__restrict__ AT,
                                                     const int32_t *__restrict__ tau,
                                                     const int32_t *__restrict__ sigma,
                                                     const int32_t *__restrict__ d, int n, u64 *bk, u64 *bb,
                                                     int32_t *bc) {
    __shared__ u64 red[3 * 256 / 64];
    const int r = blockIdx.x;
    const int32_t *Wr = W + (int64_t)r * n;
    const int32_t *Tr = AT + (int64_t)tau[r] * n;
    const int dr = d[r];
    u64 b1 = 0, b2 = 0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        if (c == r) continue;
        int g = (Wr[c] + Tr[c]) - (dr + d[c]);
        top2_push(b1, b2, mk_key(g, tau[c]));
    }
    block_top2<256>(b1, b2, red);
    if (threadIdx.x == 0) {
        bk[r] = b1;
        bb[r] = b2;
        bc[r] = b1 ? sigma[key_index(b1)] : -1;
    }
}

__global__ void k_export_best(const u64 *__restrict__ bk, int n, int64_t *gain, int32_t *job) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    u64 k = bk[r];
    gain[r] = k ? (int64_t)key_gain(k) : INT64_MIN;
    job[r] = k ? key_index(k) : -1;
}

// ---- switching phase: device-resident loop -----------------------------------------
//
// One cooperative grid; workgroup q owns agents [q*R, (q+1)*R).  Each
// iteration applies one switch (steepest ascent: the best exchange over
// all agents, Section 3.3 / Algorithm 1):
//   1. every workgroup publishes its best owned agent (key (gain, agent))
//      and its share of the two agents switched last (below); one grid
//      barrier; every workgroup reduces all records to the same winner;
//   2. the winner (i*, j*, partner k, j0 = old job of i*) is applied: the
//      owners update tau, sigma, d and W's columns i*, k;
//   3. every owned agent r gets its two changed candidates g(r, i*) (job j*)
//      and g(r, k) (job j0); by symmetry the same values are agent i*'s and
//      agent k's candidates towards r, so the full re-evaluation of i* and
//      k (Algorithm 1 re-evaluates the agents of the switch) is spread over
//      all workgroups as partial top-2 records merged after the barrier;
//   4. an agent whose best pointed at job j0 or j* and that no new candidate
//      beats above its bound is re-evaluated in full by its owner.
// Every gain of agent r other than the two candidates is unchanged by the
// switch, so the kept (best, bound) pair stays exact.
struct LoopRec {
    u64 lkey;          // key(gain, agent) of the workgroup's best agent
    u64 pi1, pi2;      // partial top-2 of agent i* (keys (gain, job))
    u64 pk1, pk2;      // partial top-2 of agent k
    int32_t lj, lc, lj0;  // best agent's job, partner, current job
    int32_t pic, pkc;     // partners of pi1, pk1
    int32_t pad[3];
};

struct LoopParams {
    const int32_t *AT;
    int32_t *W;
    int32_t *tau;
    int32_t *sigma;
    int32_t *d;
    u64 *bk;
    u64 *bb;
    int32_t *bc;
    LoopRec *recs;
    uint32_t *bar;
    int64_t *stats;
    const int32_t *flags;  // [0] != 0: the benefit range check failed; do nothing
    int n;
    int rows_per_wg;
    int64_t max_switches;
};

__device__ __forceinline__ void grid_barrier(uint32_t *bar, uint32_t target) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(bar, 1u);
        // wrap-safe: the counter only grows, by one per workgroup per barrier
        while ((int32_t)(__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0)
            __builtin_amdgcn_s_sleep(1);
        __threadfence();
    }
    __syncthreads();
    __threadfence();
}

// Best owned agent (excluding ex1, ex2) -> (key(gain, agent), job, partner, tau).
struct LocalBest {
    u64 key;
    int j, c, j0;
};

__device__ LocalBest local_best(const LoopParams &P, int r0, int r1, int ex1, int ex2, u64 *red,
                                int *pay) {
    u64 best = 0;
    for (int r = r0 + (int)threadIdx.x; r < r1; r += kLoopBlock) {
        if (r == ex1 || r == ex2) continue;
        u64 b = P.bk[r];
        if (b) best = umax64(best, mk_key(key_gain(b), r));
    }
    u64 m = block_max<kLoopBlock>(best, red);
    LocalBest L{m, -1, -1, -1};
    if (m) {
        int row = key_index(m);
        if (row >= r0 + (int)threadIdx.x && ((row - r0) % kLoopBlock) == (int)threadIdx.x && row < r1) {
            pay[0] = key_index(P.bk[row]);
            pay[1] = P.bc[row];
            pay[2] = P.tau[row];
        }
        __syncthreads();
        L.j = pay[0];
        L.c = pay[1];
        L.j0 = pay[2];
    }
    return L;
}

__global__ __launch_bounds__(kLoopBlock) void k_switch_loop(LoopParams P) {
    extern __shared__ int exh[];  // rows needing a full re-evaluation (<= rows_per_wg)
    __shared__ u64 red[3 * kLoopBlock / 64];
    __shared__ int pay[4];
    __shared__ u64 win_key;
    __shared__ int win_pay[3];
    __shared__ int n_exh;

    const int G = gridDim.x, q = blockIdx.x, t = threadIdx.x;
    if (P.flags[0]) return;  // same decision in every workgroup
    const int n = P.n;
    const int64_t nn = n;
    const int r0 = min(n, q * P.rows_per_wg), r1 = min(n, r0 + P.rows_per_wg);

    int prev_is = -1, prev_k = -1, prev_js = -1, prev_j0 = -1;
    int64_t S = 0, gsum = 0, rescans = 0;

    {
        LocalBest L = local_best(P, r0, r1, -1, -1, red, pay);
        if (t == 0) {
            LoopRec rec{};
            rec.lkey = L.key;
            rec.lj = L.j;
            rec.lc = L.c;
            rec.lj0 = L.j0;
            rec.pic = rec.pkc = -1;
            P.recs[q] = rec;
        }
    }

    for (uint32_t s = 0;; ++s) {
        grid_barrier(P.bar, (s + 1) * (uint32_t)G);

        // -- 1. winner ---------------------------------------------------------
        const LoopRec *R = P.recs + (size_t)(s & 1) * G;
        u64 wk = 0;
        int wslot = -1;
        Best2 mi{0, 0, -1}, mk{0, 0, -1};
        for (int x = t; x < G; x += kLoopBlock) {
            const LoopRec &rec = R[x];
            if (rec.lkey > wk) {
                wk = rec.lkey;
                wslot = x;
            }
            best2_merge(mi, rec.pi1, rec.pi2, rec.pic);
            best2_merge(mk, rec.pk1, rec.pk2, rec.pkc);
        }
        u64 wmax = block_max<kLoopBlock>(wk, red);
        if (wmax && wk == wmax) {
            win_pay[0] = R[wslot].lj;
            win_pay[1] = R[wslot].lc;
            win_pay[2] = R[wslot].lj0;
        }
        block_best2<kLoopBlock>(mi, red);
        block_best2<kLoopBlock>(mk, red);
        // block_best2 ends with a barrier after the LDS writes, so win_pay is visible.
        int wj = win_pay[0], wc = win_pay[1], wj0 = win_pay[2];
        if (wmax == 0) wj = wc = wj0 = -1;
        if (prev_is >= 0 && mi.k1) {
            u64 k2 = mk_key(key_gain(mi.k1), prev_is);
            if (k2 > wmax) {
                wmax = k2;
                wj = key_index(mi.k1);
                wc = mi.c1;
                wj0 = prev_js;
            }
        }
        if (prev_k >= 0 && mk.k1) {
            u64 k2 = mk_key(key_gain(mk.k1), prev_k);
            if (k2 > wmax) {
                wmax = k2;
                wj = key_index(mk.k1);
                wc = mk.c1;
                wj0 = prev_j0;
            }
        }
        if (t == 0) {
            if (prev_is >= r0 && prev_is < r1) {
                P.bk[prev_is] = mi.k1;
                P.bb[prev_is] = mi.k2;
                P.bc[prev_is] = mi.c1;
            }
            if (prev_k >= r0 && prev_k < r1) {
                P.bk[prev_k] = mk.k1;
                P.bb[prev_k] = mk.k2;
                P.bc[prev_k] = mk.c1;
            }
            n_exh = 0;
        }
        const int wg = wmax ? key_gain(wmax) : 0;
        if (wmax == 0 || wg <= 0 || (P.max_switches >= 0 && S >= P.max_switches)) break;
        const int is = key_index(wmax), js = wj, k = wc, j0 = wj0;
        ++S;
        gsum += wg;
        __syncthreads();

        // -- 2./3. apply and update owned agents ---------------------------------
        const int dis = P.AT[(int64_t)js * nn + is];  // a[i*][j*]
        const int dk = P.AT[(int64_t)j0 * nn + k];    // a[k][j0]
        Best2 pi{0, 0, -1}, pk{0, 0, -1};
        for (int r = r0 + t; r < r1; r += kLoopBlock) {
            int32_t *Wr = P.W + (int64_t)r * nn;
            if (r == is) {
                Wr[is] = dis;
                Wr[k] = P.AT[(int64_t)j0 * nn + is];
                P.tau[is] = js;
                P.d[is] = dis;
                P.sigma[js] = is;
                best2_push(pk, mk_key(-wg, js), is);  // g(k, i*) = -gain, job of i* = j*
            } else if (r == k) {
                Wr[is] = P.AT[(int64_t)js * nn + k];
                Wr[k] = dk;
                P.tau[k] = j0;
                P.d[k] = dk;
                P.sigma[j0] = k;
                best2_push(pi, mk_key(-wg, j0), k);  // g(i*, k) = -gain, job of k = j0
            } else {
                const int a1 = P.AT[(int64_t)js * nn + r];  // new W[r][i*] = a[r][j*]
                const int a2 = P.AT[(int64_t)j0 * nn + r];  // new W[r][k]  = a[r][j0]
                const int w1 = P.W[(int64_t)is * nn + r];   // W[i*][r] = a[i*][tau(r)]
                const int w2 = P.W[(int64_t)k * nn + r];    // W[k][r]  = a[k][tau(r)]
                const int dr = P.d[r], tr = P.tau[r];
                const int x1 = (a1 + w1) - (dr + dis);      // g(r, i*)
                const int x2 = (a2 + w2) - (dr + dk);       // g(r, k)
                Wr[is] = a1;
                Wr[k] = a2;
                u64 b = P.bk[r], bnd = P.bb[r];
                int c = P.bc[r];
                const int bj = key_index(b);
                if (b && (bj == js || bj == j0)) b = 0;
                const u64 y1 = mk_key(x1, js);
                if (y1 > bnd) {
                    if (y1 > b) {
                        if (b) bnd = b;
                        b = y1;
                        c = is;
                    } else {
                        bnd = y1;
                    }
                }
                const u64 y2 = mk_key(x2, j0);
                if (y2 > bnd) {
                    if (y2 > b) {
                        if (b) bnd = b;
                        b = y2;
                        c = k;
                    } else {
                        bnd = y2;
                    }
                }
                P.bk[r] = b;
                P.bb[r] = bnd;
                P.bc[r] = c;
                if (!b) exh[atomicAdd(&n_exh, 1)] = r;
                best2_push(pi, mk_key(x1, tr), r);
                best2_push(pk, mk_key(x2, tr), r);
            }
        }
        block_best2<kLoopBlock>(pi, red);
        block_best2<kLoopBlock>(pk, red);

        // -- 4. full re-evaluation of exhausted agents ----------------------------
        const int ne = n_exh;
        for (int e = 0; e < ne; ++e) {
            const int r = exh[e];
            const int32_t *Wr = P.W + (int64_t)r * nn;
            const int32_t *Tr = P.AT + (int64_t)P.tau[r] * nn;
            const int dr = P.d[r];
            u64 b1 = 0, b2 = 0;
            for (int c = t; c < n; c += kLoopBlock) {
                if (c == r) continue;
                int tc, dc;
                if (c == is) {
                    tc = js;
                    dc = dis;
                } else if (c == k) {
                    tc = j0;
                    dc = dk;
                } else {
                    tc = P.tau[c];
                    dc = P.d[c];
                }
                const int gg = (Wr[c] + Tr[c]) - (dr + dc);
                top2_push(b1, b2, mk_key(gg, tc));
            }
            block_top2<kLoopBlock>(b1, b2, red);
            if (t == 0) {
                P.bk[r] = b1;
                P.bb[r] = b2;
                const int jb = key_index(b1);
                P.bc[r] = (jb == js) ? is : (jb == j0) ? k : P.sigma[jb];
            }
            __syncthreads();
        }
        rescans += ne;

        // -- publish ----------------------------------------------------------------
        LocalBest L = local_best(P, r0, r1, is, k, red, pay);
        if (t == 0) {
            LoopRec rec;
            rec.lkey = L.key;
            rec.lj = L.j;
            rec.lc = L.c;
            rec.lj0 = L.j0;
            rec.pi1 = pi.k1;
            rec.pi2 = pi.k2;
            rec.pic = pi.c1;
            rec.pk1 = pk.k1;
            rec.pk2 = pk.k2;
            rec.pkc = pk.c1;
            rec.pad[0] = rec.pad[1] = rec.pad[2] = 0;
            P.recs[(size_t)((s + 1) & 1) * G + q] = rec;
        }
        prev_is = is;
        prev_k = k;
        prev_js = js;
        prev_j0 = j0;
    }
    if (t == 0) {
        if (rescans) atomicAdd((unsigned long long *)&P.stats[3], (unsigned long long)rescans);
        if (q == 0) {
            P.stats[0] = S;
            P.stats[1] = gsum;
        }
    }
}

}  // namespace

// ---- host launchers ----------------------------------------------------------------------

size_t loop_record_bytes() { return sizeof(LoopRec); }

int loop_grid_size(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_switch_loop, kLoopBlock, 0) != hipSuccess)
        return 0;
    if (per_cu < 1) return 0;
    return cus;
}

hipError_t launch_range_check(const int32_t *A, int64_t count, int32_t *flag, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_range_check, dim3((unsigned)blocks), dim3(256), 0, s, A, count, flag);
    return hipGetLastError();
}

hipError_t launch_greedy(const int32_t *A, int32_t n, int32_t *tau, int32_t *sigma, hipStream_t s) {
    size_t shm = sizeof(uint32_t) * (size_t)((n + 31) / 32);
    hipLaunchKernelGGL(k_greedy_wg, dim3(1), dim3(kGreedyBlock), shm, s, A, n, tau, sigma);
    return hipGetLastError();
}

hipError_t launch_fill(int32_t *p, int32_t n, int32_t v, hipStream_t s) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_invert_checked(const int32_t *tau, int32_t n, int32_t *sigma, int32_t *flag,
                                 hipStream_t s) {
    unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, sigma, n, -1);
    hipLaunchKernelGGL(k_invert_checked, dim3(blocks), dim3(256), 0, s, tau, n, sigma, flag);
    return hipGetLastError();
}

hipError_t launch_transpose(const int32_t *A, int32_t *AT, int32_t n, hipStream_t s) {
    unsigned t = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(k_transpose, dim3(t, t), dim3(256), 0, s, A, AT, n);
    return hipGetLastError();
}

hipError_t launch_build_w(const int32_t *A, const int32_t *AT, const int32_t *tau, int32_t n, int32_t *W,
                          int32_t *d, int64_t *f0, hipStream_t s) {
    const unsigned t = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(k_build_w, dim3(t, t), dim3(256), 0, s, AT, tau, n, W);
    hipLaunchKernelGGL(k_benefits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, tau, n, d,
                       (unsigned long long *)f0);
    return hipGetLastError();
}

hipError_t launch_benefits(const int32_t *A, const int32_t *tau, int32_t n, int32_t *d, int64_t *f, hipStream_t s) {
    hipLaunchKernelGGL(k_benefits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, tau, n, d,
                       (unsigned long long *)f);
    return hipGetLastError();
}

hipError_t launch_scan_rows(const Instance &I, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_rows, dim3((unsigned)I.n), dim3(256), 0, s, I.W, I.AT, I.tau, I.sigma, I.d,
                       I.n, I.bk, I.bb, I.bc);
    return hipGetLastError();
}

hipError_t launch_switch_loop(const Instance &I, int64_t max_switches, int grid, hipStream_t s) {
    LoopParams P;
    P.AT = I.AT;
    P.W = I.W;
    P.tau = I.tau;
    P.sigma = I.sigma;
    P.d = I.d;
    P.bk = I.bk;
    P.bb = I.bb;
    P.bc = I.bc;
    P.recs = (LoopRec *)I.recs;
    P.bar = I.barrier;
    P.stats = I.stats;
    P.flags = I.flags;
    P.n = I.n;
    if (grid > I.n) grid = I.n;
    if (grid < 1) grid = 1;
    P.rows_per_wg = (I.n + grid - 1) / grid;
    P.max_switches = max_switches;
    void *args[] = {&P};
    size_t shm = sizeof(int) * (size_t)P.rows_per_wg;
    return hipLaunchCooperativeKernel((const void *)k_switch_loop, dim3((unsigned)grid), dim3(kLoopBlock), args,
                                      (unsigned)shm, s);
}

hipError_t launch_export_best(const Instance &I, int64_t *gain_out, int32_t *job_out, hipStream_t s) {
    hipLaunchKernelGGL(k_export_best, dim3((unsigned)((I.n + 255) / 256)), dim3(256), 0, s, I.bk, I.n,
                       gain_out, job_out);
    return hipGetLastError();
}

}  // namespace dgs
