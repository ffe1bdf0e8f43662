// Difference evaluation of every agent (Section 3.2, Algorithm 2) on gfx950,
// reading every entry of the benefit matrix once.
//
// With W[r][c] = a[r][tau(c)] and d[c] = W[c][c], the 2-exchange of agents
// i and k gains g(i, k) = W[i][k] + W[k][i] - d[i] - d[k] = g(k, i).  The
// agents are cut into blocks of kTile; the workgroup of block pair (I, K),
// I <= K, loads the two tiles of the pair once and scores every pair
// (i in I, k in K) for both agents: for agent i the candidate is
// (g, job tau(k)), for agent k it is (g, job tau(i)).  Ties: larger gain,
// then lower job.
//
// g is symmetric in the two tiles, so it can be read from V = W^T, and row x
// of V is row tau(x) of A^T (V[x][y] = a[y][tau(x)] = W[y][x]): the kernel
// reads the transpose through tau, and no assignment-ordered matrix is ever
// built (a switch changes tau, not the matrix).
//
// Two reductions of the scores:
//   * lists (the steepest-ascent solve): a top-2 per agent and partner
//     block; k_scan_reduce merges an agent's blocks into its best exchange,
//     a candidate list and a bound for everything outside the list;
//   * both sides (Parallel DGS and lazy DGS): per agent and partner block
//     the best candidate keyed by job (the agent side, ADE) and the best
//     keyed by partner agent (for agent c: the best agent to take c's job,
//     the job side, JDE, lowest agent on ties); k_scan_best keeps the best
//     of each.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgs_device.h"
#include "dgs_internal.h"

namespace dgs {
namespace {

using namespace dev;

constexpr int kTile = 64;
constexpr int kScanBlock = 512;  // 8 threads per tile row
constexpr int kPad = kTile + 1;
constexpr int kListLen = kScanListLen;

struct ScanParams {
    const int32_t *AT;    // A^T (n x nr); tile row x is row tau[x] of it
    const int32_t *tau;
    const int32_t *d;
    u64 *part;  // [nr][nb][2]
    int n;      // agents (with the virtual ones of a rectangular instance)
    int nr;     // real agents: entries of virtual agents y >= nr are 0, and only real agents get results
    int nb;
};

// One workgroup of BLOCK threads per tile pair: BLOCK / 64 threads per tile
// row, each scoring 64 / (BLOCK / 64) partners on each side; interior pairs
// (no bounds, no diagonal) take an unrolled path.
// kBoth: slot 0 of a partial is the best candidate keyed by the partner's
// job tau(k), slot 1 the best keyed by the partner agent k itself.
// Otherwise the two slots are the top-2 by job.
template <int BLOCK, bool kBoth>
__global__ __launch_bounds__(BLOCK) void k_scan_pairs_b(ScanParams P) {
    constexpr int Q = BLOCK / 64;  // threads per tile row
    constexpr int E = kTile / Q;   // partners per thread
    constexpr int LD = (kTile * kTile / 4) / BLOCK;  // int4 loads per thread per tile
    __shared__ int32_t tA[kTile][kPad];  // tA[i][k] = W[I*T + i][K*T + k]
    __shared__ int32_t tB[kTile][kPad];  // tB[k][i] = W[K*T + k][I*T + i]
    __shared__ int32_t dI[kTile], dK[kTile], jI[kTile], jK[kTile];
    int I, K;
    pair_of((long long)blockIdx.x, P.nb, I, K);
    const int n = P.n, nr = P.nr;
    const int i0 = I * kTile, k0 = K * kTile;
    const int t = threadIdx.x;
    const bool full = (nr % 4 == 0) && i0 + kTile <= nr && k0 + kTile <= nr;
    auto row = [&](int x) { return P.AT + (int64_t)P.tau[x] * nr; };
    if (full) {
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
        for (int e = t; e < kTile * kTile; e += BLOCK) {
            const int r = e >> 6, c = e & 63;
            tA[r][c] = (i0 + r < n && k0 + c < nr) ? row(i0 + r)[k0 + c] : 0;
            tB[r][c] = (k0 + r < n && i0 + c < nr) ? row(k0 + r)[i0 + c] : 0;
        }
    }
    if (t < kTile) {
        dI[t] = i0 + t < n ? P.d[i0 + t] : 0;
        jI[t] = i0 + t < n ? P.tau[i0 + t] : 0;
    } else if (t < 2 * kTile) {
        const int x = t - kTile;
        dK[x] = k0 + x < n ? P.d[k0 + x] : 0;
        jK[x] = k0 + x < n ? P.tau[k0 + x] : 0;
    }
    __syncthreads();

    // the both-sides reduction reads only bests: a top-1 per key kind
    // (partner job x, partner agent y) suffices
    auto push = [](u64 &b1, u64 &b2, int g, int x, int y) {
        if constexpr (kBoth) {
            b1 = umax64(b1, mk_key(g, x));
            b2 = umax64(b2, mk_key(g, y));
        } else {
            top2_push(b1, b2, mk_key(g, x));
        }
    };
    const int rt = t / Q, q = t % Q;
    u64 a1 = 0, a2 = 0, c1 = 0, c2 = 0;  // row rt of I against K; row rt of K against I
    if (I != K && i0 + kTile <= n && k0 + kTile <= n) {
        const int di = dI[rt], dk = dK[rt];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int c = q * E + e;
            push(a1, a2, (tA[rt][c] + tB[c][rt]) - (di + dK[c]), jK[c], k0 + c);
            push(c1, c2, (tA[c][rt] + tB[rt][c]) - (dI[c] + dk), jI[c], i0 + c);
        }
    } else {
        if (i0 + rt < n) {
            const int di = dI[rt];
            for (int e = 0; e < E; ++e) {
                const int k = q * E + e;
                if (k0 + k >= n || (I == K && k == rt)) continue;
                push(a1, a2, (tA[rt][k] + tB[k][rt]) - (di + dK[k]), jK[k], k0 + k);
            }
        }
        if (I != K && k0 + rt < n) {
            const int dk = dK[rt];
            for (int e = 0; e < E; ++e) {
                const int i = q * E + e;
                if (i0 + i >= n) continue;
                push(c1, c2, (tA[i][rt] + tB[rt][i]) - (dI[i] + dk), jI[i], i0 + i);
            }
        }
    }
    // merge the Q threads of each row (adjacent lanes)
#pragma unroll
    for (int m = 1; m < Q; m <<= 1) {
        if constexpr (kBoth) {
            a1 = umax64(a1, shfl_xor64(a1, m));
            a2 = umax64(a2, shfl_xor64(a2, m));
            c1 = umax64(c1, shfl_xor64(c1, m));
            c2 = umax64(c2, shfl_xor64(c2, m));
        } else {
            top2_merge(a1, a2, shfl_xor64(a1, m), shfl_xor64(a2, m));
            top2_merge(c1, c2, shfl_xor64(c1, m), shfl_xor64(c2, m));
        }
    }
    if (q == 0 && i0 + rt < nr) {
        u64 *o = P.part + ((size_t)(i0 + rt) * P.nb + K) * 2;
        o[0] = a1;
        o[1] = a2;
    }
    if (q == 0 && I != K && k0 + rt < nr) {
        u64 *o = P.part + ((size_t)(k0 + rt) * P.nb + I) * 2;
        o[0] = c1;
        o[1] = c2;
    }
}

// One wave per agent: the best of its nb block bests of each key kind (no
// list, no bound): by job into bk (with the partner sigma(job) into bc, if
// given), by partner agent into ba.
__global__ __launch_bounds__(256) void k_scan_best(const u64 *__restrict__ part, int n, int nb,
                                                    const int32_t *__restrict__ sigma, u64 *bk, int32_t *bc,
                                                    u64 *ba) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    const u64 *p = part + (size_t)r * nb * 2;
    u64 m = 0, y = 0;
    for (int x = lane; x < nb; x += 64) {
        m = umax64(m, p[2 * x]);
        y = umax64(y, p[2 * x + 1]);
    }
    m = wave_max64(m);
    y = wave_max64(y);
    if (lane == 0) {
        bk[r] = m;
        ba[r] = y;
        if (bc) bc[r] = m ? sigma[key_index(m)] : -1;
    }
}

// One wave per agent: merge its nb block top-2s into the agent's candidate
// list.  Every candidate that is not a block's best is <= its block's
// second, so B = max over blocks of the second is a bound for everything
// outside the block bests; the list is the kListLen best block bests above
// B, and the bound is B or the next block best above it.
__global__ __launch_bounds__(256) void k_scan_reduce(const u64 *__restrict__ part, int n, int nb,
                                                      const int32_t *__restrict__ sigma, u64 *bk, u64 *bb,
                                                      int32_t *bc, u64 *lists) {
    constexpr int kPer = 8;  // block bests held per lane: nb <= 512 (n <= 32768) stays in registers
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    const u64 *p = part + (size_t)r * nb * 2;
    u64 bnd = 0;
    u64 best[kPer];
#pragma unroll
    for (int m = 0; m < kPer; ++m) best[m] = 0;
    const bool regs = nb <= 64 * kPer;
    if (regs) {
#pragma unroll
        for (int m = 0; m < kPer; ++m) {
            const int x = lane + 64 * m;
            if (x < nb) {
                best[m] = p[2 * x];
                bnd = umax64(bnd, p[2 * x + 1]);
            }
        }
    } else {
        for (int x = lane; x < nb; x += 64) bnd = umax64(bnd, p[2 * x + 1]);
    }
    bnd = wave_max64(bnd);
    // up to kListLen + 1 rounds of "largest block best above the bound"
    u64 taken_max = ~(u64)0;  // keys already emitted are >= this
    u64 out = 0;              // lane i < kListLen keeps entry i
    u64 first = 0;
    for (int round = 0; round <= kListLen; ++round) {
        u64 m1 = 0;
        if (regs) {
#pragma unroll
            for (int m = 0; m < kPer; ++m)
                if (best[m] > bnd && best[m] < taken_max) m1 = umax64(m1, best[m]);
        } else {
            for (int x = lane; x < nb; x += 64) {
                const u64 k = p[2 * x];
                if (k > bnd && k < taken_max) m1 = umax64(m1, k);
            }
        }
        m1 = wave_max64(m1);
        if (m1 == 0) break;
        if (round == kListLen) {
            bnd = m1;  // the next block best above B becomes the bound
            break;
        }
        if (round == 0) first = m1;
        if (lane == round) out = m1;
        taken_max = m1;
    }
    if (lane < kListLen) lists[(size_t)r * kListLen + lane] = out;
    if (lane == 0) {
        bk[r] = first;
        bb[r] = bnd;
        bc[r] = first ? sigma[key_index(first)] : -1;
    }
}

}  // namespace

size_t scan_pairs_scratch_bytes(int n) {
    const size_t nb = ((size_t)n + kTile - 1) / kTile;
    return (size_t)n * nb * 2 * sizeof(u64);
}

// Tile pairs (I, K), I <= K, with a real agent in block I: the first ones of
// the row-major triangular order (pairs of two virtual blocks score nothing
// a real agent needs).
static long long scan_pairs_count(int nb, int nbr) {
    return (long long)nbr * nb - (long long)nbr * (nbr - 1) / 2;
}

hipError_t launch_scan_best_transposed(const Instance &I, void *scratch, hipStream_t s, u64 *by_job,
                                       int32_t *partner, u64 *by_agent) {
    const int nb = (I.n + kTile - 1) / kTile, nbr = (I.nr + kTile - 1) / kTile;
    ScanParams P{I.AT, I.tau, I.d, (u64 *)scratch, I.n, I.nr, nb};
    hipLaunchKernelGGL((k_scan_pairs_b<kScanBlock, true>), dim3((unsigned)scan_pairs_count(nb, nbr)),
                       dim3(kScanBlock), 0, s, P);
    hipLaunchKernelGGL(k_scan_best, dim3((unsigned)((I.nr + 3) / 4)), dim3(256), 0, s, (const u64 *)scratch, I.nr,
                       nb, I.sigma, by_job, partner, by_agent);
    return hipGetLastError();
}

hipError_t launch_scan_pairs(const Instance &I, void *scratch, hipStream_t s) {
    const int nb = (I.n + kTile - 1) / kTile, nbr = (I.nr + kTile - 1) / kTile;
    ScanParams P{I.AT, I.tau, I.d, (u64 *)scratch, I.n, I.nr, nb};
    hipLaunchKernelGGL((k_scan_pairs_b<kScanBlock, false>), dim3((unsigned)scan_pairs_count(nb, nbr)),
                       dim3(kScanBlock), 0, s, P);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)((I.nr + 3) / 4)), dim3(256), 0, s, (const u64 *)scratch, I.nr,
                       nb, I.sigma, I.bk, I.bb, I.bc, I.lists);
    return hipGetLastError();
}

}  // namespace dgs
