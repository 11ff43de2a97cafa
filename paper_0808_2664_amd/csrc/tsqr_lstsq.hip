// Least squares on top of TSQR (Sec. 1, the remark on solving least squares
// problems with a QR factorisation): with A = QR and C = Q^T B (full m x m Q,
// applied through the tree of Q factors), X solves R X = C(0:n, :) and, Q
// preserving norms, the residual norm of column j is ||C(n:m, j)||_2.
// The factorisation and Q^T B are the TSQR kernels; this file holds the two
// steps after them.
#include "tsqr_common.hpp"

namespace tsqr {

// Back substitution R X = C for the k columns of C, the first n rows of B,
// which X overwrites.  One wave per column: lane i holds row i of R (zeros
// left of the diagonal, so the update below leaves rows under step j alone)
// and c_i.  Step j, last row first: lane j forms x_j = c_j / R_jj, every lane
// takes x_j from lane j and subtracts R_ij x_j.  The waves of a workgroup
// take consecutive columns.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_trsm_upper(int n, const T* __restrict__ R, int64_t ldr,
                                                    T* __restrict__ B, int64_t ldb, int64_t k) {
    const int lane = threadIdx.x & 63;
    const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= k) return;  // uniform over the wave
    T r[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) r[j] = (lane < n && j < n && j >= lane) ? R[(int64_t)lane * ldr + j] : T(0);
    T c = (lane < n) ? B[(int64_t)lane * ldb + col] : T(0);
    T x = T(0);
#pragma unroll
    for (int j = NC - 1; j >= 0; --j) {
        if (j < n) {
            const T q = c / ((lane == j) ? r[j] : T(1));
            const T xj = dev::shfl(q, j);
            if (lane == j) x = q;
            c -= r[j] * xj;
        }
    }
    if (lane < n) B[(int64_t)lane * ldb + col] = x;
}

// Sums of squares of rows [r0, m) of the k columns of B, one partial sum per
// chunk of `rows` rows: part[chunk * k + col], accumulated in FP64.
// Workgroup (group of CW columns, chunk), CW = 32 for k <= 32 (a wave then
// reads two rows per load), else 64.  Slot (wave w, row-in-wave h) takes rows
// s, s + 4 (64 / CW), ... of the chunk with four independent sums; the sums
// and slots are added in a fixed order, so the result does not depend on
// scheduling.
template <typename T>
__global__ __launch_bounds__(256) void k_colsq_part(int64_t r0, int64_t m, int64_t rows, const T* __restrict__ B,
                                                    int64_t ldb, int64_t k, double* __restrict__ part) {
    __shared__ double s[4][64];
    const int cw = (k <= 32) ? 32 : 64, rpw = 64 / cw;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int h = lane / cw, c = lane - h * cw;
    const int64_t col = (int64_t)blockIdx.x * cw + c;
    const int64_t a = r0 + (int64_t)blockIdx.y * rows;
    const int64_t e = (a + rows < m) ? a + rows : m;
    const int64_t step = 4 * rpw;  // rows between one slot's consecutive rows
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (col < k) {
        int64_t i = a + w * rpw + h;
        for (; i + 3 * step < e; i += 4 * step) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = (double)B[(i + u * step) * ldb + col];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] += v[u] * v[u];
        }
        for (int u = 0; i < e; i += step, ++u) {
            const double v = (double)B[i * ldb + col];
            acc[u & 3] += v * v;
        }
    }
    s[w][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (w == 0 && h == 0 && col < k) {
        double t = 0.0;
        for (int ww = 0; ww < 4; ++ww)
            for (int hh = 0; hh < rpw; ++hh) t += s[ww][hh * cw + c];
        part[(int64_t)blockIdx.y * k + col] = t;
    }
}

// rnorm[col] = sqrt of the sum of the column's partial sums: one workgroup
// per column, thread t adding partials t, t + 256, ..., then a fixed-order
// tree over the 256 threads.
template <typename T>
__global__ __launch_bounds__(256) void k_colsq_final(int64_t nchunks, const double* __restrict__ part, int64_t k,
                                                     T* __restrict__ rnorm) {
    __shared__ double s[256];
    const int64_t col = blockIdx.x;
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int64_t c = t; c < nchunks; c += 256) acc += part[c * k + col];
    s[t] = acc;
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
        if (t < half) s[t] += s[t + half];
        __syncthreads();
    }
    if (t == 0) rnorm[col] = (T)sqrt(s[0]);
}

template <typename T>
static hipError_t trsm_t(int64_t n, const T* R, int64_t ldr, T* B, int64_t ldb, int64_t k, hipStream_t st) {
    const unsigned grid = (unsigned)((k + 3) / 4);
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
    if (n < 1 || n > 64 || (k + 3) / 4 > 0x7fffffff) return hipErrorInvalidValue;
    return f64 ? trsm_t<double>(n, (const double*)R, ldr, (double*)B, ldb, k, st)
               : trsm_t<float>(n, (const float*)R, ldr, (float*)B, ldb, k, st);
}

hipError_t launch_colnorm(bool f64, int64_t r0, int64_t m, const void* B, int64_t ldb, int64_t k, void* rnorm,
                          hipStream_t st) {
    if (k <= 0) return hipSuccess;
    if (k > 0x7fffffff) return hipErrorInvalidValue;
    const int64_t len = m > r0 ? m - r0 : 0;
    // chunks of at least 256 rows, at most 4096 chunks, at most 2^23 partial sums
    int64_t nchunks = (len + 255) / 256;
    if (nchunks > 4096) nchunks = 4096;
    const int64_t cap = ((int64_t)1 << 23) / k;
    if (nchunks > cap) nchunks = cap;
    if (nchunks < 1) nchunks = 1;
    const int64_t rows = (len + nchunks - 1) / nchunks;
    double* part = nullptr;
    hipError_t e = ws_malloc((void**)&part, (size_t)(nchunks * k) * sizeof(double), st);
    if (e != hipSuccess) return e;
    const int cw = (k <= 32) ? 32 : 64;
    const dim3 grid((unsigned)((k + cw - 1) / cw), (unsigned)nchunks);
    const unsigned gridf = (unsigned)k;
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
