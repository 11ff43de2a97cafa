// Least squares on top of TSQR (Sec. 1, the remark on solving least squares
// problems with a QR factorisation): with A = QR and C = Q^T B (full m x m Q,
// applied through the tree of Q factors), X solves R X = C(0:n, :) and, Q
// preserving norms, the residual norm of column j is ||C(n:m, j)||_2.
// The factorisation and Q^T B are the TSQR kernels; this file holds the two
// steps after them.
#include "tsqr_common.hpp"

namespace tsqr {

// Back substitution R X = C for the k columns of C, the first n rows of B,
// which X overwrites.  One thread per column; R (upper n x n, padded to NC
// with zeros) is staged in LDS and read at one address per step by every lane.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_trsm_upper(int n, const T* __restrict__ R, int64_t ldr,
                                                    T* __restrict__ B, int64_t ldb, int64_t k) {
    __shared__ T sR[NC * NC];
    for (int e = threadIdx.x; e < NC * NC; e += blockDim.x) {
        const int i = e / NC, j = e - i * NC;
        sR[e] = (i < n && j < n && j >= i) ? R[(int64_t)i * ldr + j] : T(0);
    }
    __syncthreads();
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= k) return;
    T x[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) x[i] = (i < n) ? B[(int64_t)i * ldb + col] : T(0);
    // x_i = (c_i - sum_{j > i} R_ij x_j) / R_ii, last row first; the padded
    // entries are zero in both R and x, so they add nothing
#pragma unroll
    for (int i = NC - 1; i >= 0; --i) {
        if (i < n) {
            T s = x[i];
#pragma unroll
            for (int j = i + 1; j < NC; ++j) s -= sR[i * NC + j] * x[j];
            x[i] = s / sR[i * NC + i];
        }
    }
#pragma unroll
    for (int i = 0; i < NC; ++i)
        if (i < n) B[(int64_t)i * ldb + col] = x[i];
}

// Sums of squares of rows [r0, m) of the k columns of B, one partial sum per
// chunk of `rows` rows: part[chunk * k + col], accumulated in FP64.
// Workgroup (group of 64 columns, chunk); wave w takes rows w, w + 4, ... of
// the chunk, and the four waves' sums are added in a fixed order, so the
// result does not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(256) void k_colsq_part(int64_t r0, int64_t m, int64_t rows, const T* __restrict__ B,
                                                    int64_t ldb, int64_t k, double* __restrict__ part) {
    __shared__ double s[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.x * 64 + lane;
    const int64_t a = r0 + (int64_t)blockIdx.y * rows;
    const int64_t e = (a + rows < m) ? a + rows : m;
    double acc = 0.0;
    if (col < k) {
        for (int64_t i = a + w; i < e; i += 4) {
            const double v = (double)B[i * ldb + col];
            acc += v * v;
        }
    }
    s[w][lane] = acc;
    __syncthreads();
    if (w == 0 && col < k) part[(int64_t)blockIdx.y * k + col] = (s[0][lane] + s[1][lane]) + (s[2][lane] + s[3][lane]);
}

// rnorm[col] = sqrt(sum over chunks, in chunk order, of the partial sums).
template <typename T>
__global__ __launch_bounds__(256) void k_colsq_final(int64_t nchunks, const double* __restrict__ part, int64_t k,
                                                     T* __restrict__ rnorm) {
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= k) return;
    double acc = 0.0;
    for (int64_t c = 0; c < nchunks; ++c) acc += part[c * k + col];
    rnorm[col] = (T)sqrt(acc);
}

template <typename T>
static hipError_t trsm_t(int64_t n, const T* R, int64_t ldr, T* B, int64_t ldb, int64_t k, hipStream_t st) {
    const unsigned grid = (unsigned)((k + 255) / 256);
    const int NC = n <= 8 ? 8 : n <= 16 ? 16 : n <= 32 ? 32 : 64;
    if (NC == 8)
        k_trsm_upper<T, 8><<<grid, 256, 0, st>>>((int)n, R, ldr, B, ldb, k);
    else if (NC == 16)
        k_trsm_upper<T, 16><<<grid, 256, 0, st>>>((int)n, R, ldr, B, ldb, k);
    else if (NC == 32)
        k_trsm_upper<T, 32><<<grid, 256, 0, st>>>((int)n, R, ldr, B, ldb, k);
    else
        k_trsm_upper<T, 64><<<grid, 256, 0, st>>>((int)n, R, ldr, B, ldb, k);
    return hipGetLastError();
}

hipError_t launch_trsm_upper(bool f64, int64_t n, const void* R, int64_t ldr, void* B, int64_t ldb, int64_t k,
                             hipStream_t st) {
    if (k <= 0) return hipSuccess;
    if (n < 1 || n > 64 || (k + 255) / 256 > 0x7fffffff) return hipErrorInvalidValue;
    return f64 ? trsm_t<double>(n, (const double*)R, ldr, (double*)B, ldb, k, st)
               : trsm_t<float>(n, (const float*)R, ldr, (float*)B, ldb, k, st);
}

hipError_t launch_colnorm(bool f64, int64_t r0, int64_t m, const void* B, int64_t ldb, int64_t k, void* rnorm,
                          hipStream_t st) {
    if (k <= 0) return hipSuccess;
    if ((k + 63) / 64 > 0x7fffffff) return hipErrorInvalidValue;
    const int64_t len = m > r0 ? m - r0 : 0;
    // chunks of at least 512 rows, at most 1024 chunks, at most 2^23 partial sums
    int64_t nchunks = (len + 511) / 512;
    if (nchunks > 1024) nchunks = 1024;
    const int64_t cap = ((int64_t)1 << 23) / k;
    if (nchunks > cap) nchunks = cap;
    if (nchunks < 1) nchunks = 1;
    const int64_t rows = (len + nchunks - 1) / nchunks;
    double* part = nullptr;
    hipError_t e = hipMallocAsync((void**)&part, (size_t)(nchunks * k) * sizeof(double), st);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)((k + 63) / 64), (unsigned)nchunks);
    const unsigned gridf = (unsigned)((k + 255) / 256);
    if (f64) {
        k_colsq_part<double><<<grid, 256, 0, st>>>(r0, m, rows, (const double*)B, ldb, k, part);
        k_colsq_final<double><<<gridf, 256, 0, st>>>(nchunks, part, k, (double*)rnorm);
    } else {
        k_colsq_part<float><<<grid, 256, 0, st>>>(r0, m, rows, (const float*)B, ldb, k, part);
        k_colsq_final<float><<<gridf, 256, 0, st>>>(nchunks, part, k, (float*)rnorm);
    }
    e = hipGetLastError();
    const hipError_t ef = hipFreeAsync(part, st);
    return e != hipSuccess ? e : ef;
}

}  // namespace tsqr
