// Deep Greedy Switching on gfx950: device kernels.
//
// Notation follows the paper (Roverso et al., arXiv:1106.5694, Section 3):
// a_ij benefit of agent i for job j; tau(i) job of agent i; sigma(j) agent of
// job j; switch(i, j, sigma) gives job j to agent i and i's old job to
// sigma(j).  Gains are exact int32 (|a| <= 2^29 - 1 is checked first).
//
// Working layout (built once per solve):
//   AT[j][i] = a_ij                      (transpose of the input)
//   d[c]     = a[c][tau(c)]              (current benefit of agent c)
// With W[r][c] = a[r][tau(c)] (benefit of agent r for agent c's job) the
// gain of the 2-exchange between agents r and c is
//   g(r, c) = W[r][c] + W[c][r] - d[r] - d[c],  g(r, c) = g(c, r),
// and column c of W is row tau(c) of AT, so the evaluation reads AT through
// tau.  The steepest-ascent switching loop reads rows of W, so W is built for
// it once from the start assignment (k_permuted); the loop reads W's column c
// only while agent c still holds its start job.  Agent r's candidate towards agent c is ranked
// by the packed key (gain, job tau(c)): larger gain first, lower job on ties
// (ADE, Algorithm 2, takes the first strictly better job in index order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "dgs_device.h"
#include "dgs_internal.h"

namespace dgs {

namespace {

using namespace dev;

constexpr int kMaxAbs = 536870911;  // 2^29 - 1

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

// AT (cols x rows) = A^T for A (rows x cols): 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void k_transpose(const int32_t *__restrict__ A, int32_t *__restrict__ AT,
                                                     int rows, int cols) {
    __shared__ int32_t tile[64][65];
    const int bx = blockIdx.x * 64, by = blockIdx.y * 64;  // column and row offsets in A
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        int row = by + r, col = bx + tx;
        if (row < rows && col < cols) tile[r][tx] = A[(int64_t)row * cols + col];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        int row = bx + r, col = by + tx;
        if (row < cols && col < rows) AT[(int64_t)row * rows + col] = tile[tx][r];
    }
}

// W[r][c] = a[r][tau(c)] for the rows r of A (n columns): one workgroup per row r, the
// row staged through LDS in chunks of kPermChunk columns (one chunk for
// n <= kPermChunk), then every column c takes its entry tau(c) from LDS.  With
// VEC4 (n a multiple of 4) rows, tau and W move 16 bytes per thread and access.
constexpr int kPermChunk = 16384;
constexpr int kPermThreads = 512;
template <bool VEC4>
__global__ __launch_bounds__(kPermThreads) void k_permuted(const int32_t *__restrict__ A,
                                                             const int32_t *__restrict__ tau, int n,
                                                             int32_t *__restrict__ W) {
    extern __shared__ int4 prow4[];  // min(n, kPermChunk) entries
    int32_t *prow = reinterpret_cast<int32_t *>(prow4);
    const int t = threadIdx.x;
    const int32_t *Ar = A + (int64_t)blockIdx.x * n;
    int32_t *Wr = W + (int64_t)blockIdx.x * n;
    for (int h0 = 0; h0 < n; h0 += kPermChunk) {
        const int len = min(kPermChunk, n - h0);
        if (VEC4) {
            const int4 *src = reinterpret_cast<const int4 *>(Ar + h0);
            for (int i = t; i < len / 4; i += kPermThreads) prow4[i] = src[i];
        } else {
            for (int i = t; i < len; i += kPermThreads) prow[i] = Ar[h0 + i];
        }
        __syncthreads();
        if (VEC4) {
            const int4 *tv = reinterpret_cast<const int4 *>(tau);
            int4 *dst = reinterpret_cast<int4 *>(Wr);
            for (int c = t; c < n / 4; c += kPermThreads) {
                const int4 j = tv[c];
                const int j0 = j.x - h0, j1 = j.y - h0, j2 = j.z - h0, j3 = j.w - h0;
                if (len == n) {  // one chunk: every entry of a permutation is in LDS
                    auto at = [&](int j) { return (unsigned)j < (unsigned)len ? prow[j] : 0; };
                    dst[c] = make_int4(at(j0), at(j1), at(j2), at(j3));
                } else {
                    if ((unsigned)j0 < (unsigned)len) Wr[4 * c] = prow[j0];
                    if ((unsigned)j1 < (unsigned)len) Wr[4 * c + 1] = prow[j1];
                    if ((unsigned)j2 < (unsigned)len) Wr[4 * c + 2] = prow[j2];
                    if ((unsigned)j3 < (unsigned)len) Wr[4 * c + 3] = prow[j3];
                }
            }
        } else {
            for (int c = t; c < n; c += kPermThreads) {
                const int j = tau[c] - h0;
                if ((unsigned)j < (unsigned)len) Wr[c] = prow[j];
            }
        }
        __syncthreads();  // the next chunk overwrites the row buffer
    }
}

// d[r] = a[r][tau(r)] (0 for the virtual agents r >= nr) and f0 = sum of d.
__global__ __launch_bounds__(256) void k_benefits(const int32_t *__restrict__ A, const int32_t *__restrict__ tau,
                                                    int n, int nr, int32_t *d, unsigned long long *f0) {
    __shared__ long long part[4];
    const int r = blockIdx.x * 256 + threadIdx.x;
    long long v = 0;
    if (r < n) {
        const int x = r < nr ? A[(int64_t)r * n + tau[r]] : 0;
        d[r] = x;
        v = x;
    }
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(f0, (unsigned long long)(part[0] + part[1] + part[2] + part[3]));
}

__global__ void k_export_best(const u64 *__restrict__ bk, int n, int64_t *gain, int32_t *job) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    u64 k = bk[r];
    gain[r] = k ? (int64_t)key_gain(k) : INT64_MIN;
    job[r] = k ? key_index(k) : -1;
}

}  // namespace

// ---- host launchers ----------------------------------------------------------------------

hipError_t launch_range_check(const int32_t *A, int64_t count, int32_t *flag, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_range_check, dim3((unsigned)blocks), dim3(256), 0, s, A, count, flag);
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

hipError_t launch_transpose(const int32_t *A, int32_t *AT, int32_t rows, int32_t cols, hipStream_t s) {
    const unsigned tc = (unsigned)((cols + 63) / 64), tr = (unsigned)((rows + 63) / 64);
    hipLaunchKernelGGL(k_transpose, dim3(tc, tr), dim3(256), 0, s, A, AT, rows, cols);
    return hipGetLastError();
}

hipError_t launch_permuted(const int32_t *A, const int32_t *tau, int32_t rows, int32_t n, int32_t *W,
                           hipStream_t s) {
    if (rows < 1 || n < 1) return hipSuccess;
    const int shm = (int)(std::min(n, kPermChunk) * sizeof(int32_t));
    auto al16 = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
    const bool vec4 = n % 4 == 0 && al16(A) && al16(tau) && al16(W);  // every row then starts 16-byte aligned
    const void *kern = vec4 ? (const void *)k_permuted<true> : (const void *)k_permuted<false>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, shm);
    if (e != hipSuccess) return e;
    if (vec4)
        hipLaunchKernelGGL(k_permuted<true>, dim3((unsigned)rows), dim3(kPermThreads), (unsigned)shm, s, A, tau, n, W);
    else
        hipLaunchKernelGGL(k_permuted<false>, dim3((unsigned)rows), dim3(kPermThreads), (unsigned)shm, s, A, tau, n, W);
    return hipGetLastError();
}

hipError_t launch_benefits(const int32_t *A, const int32_t *tau, int32_t n, int32_t nr, int32_t *d, int64_t *f,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_benefits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, tau, n, nr, d,
                       (unsigned long long *)f);
    return hipGetLastError();
}

hipError_t launch_export_best(const Instance &I, int64_t *gain_out, int32_t *job_out, hipStream_t s) {
    hipLaunchKernelGGL(k_export_best, dim3((unsigned)((I.n + 255) / 256)), dim3(256), 0, s, I.bk, I.n,
                       gain_out, job_out);
    return hipGetLastError();
}

}  // namespace dgs
