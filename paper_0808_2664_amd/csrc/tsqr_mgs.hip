// Modified Gram-Schmidt, the other comparison algorithm of Sec. 2.3 (beside
// CholeskyQR): fast but unstable, its loss of orthogonality grows with the
// condition number of A.  Provided so that TSQR can be compared with it on
// the same device.
//
// Right-looking MGS: step j takes r_jj = ||a_j||, q_j = a_j / r_jj and, for
// every later column, r_jc = q_j^T a_c and a_c -= r_jc q_j.  Each step needs
// inner products over all m rows, a reduction across the whole matrix, so
// the path is n + 1 streaming passes over the rows, each fused with the
// previous step's update:
//   pass j: apply step j-1 (a_c -= (r_{j-1,c} / r_{j-1,j-1}) a_{j-1} for
//           c >= j, and q_{j-1} = a_{j-1} / r_{j-1,j-1}), then the partial
//           sums s_jc = a_j^T a_c over the workgroup's rows (c >= j);
//   reduce j: the partial sums added in a fixed order; r_jj = sqrt(s_jj),
//           r_jc = s_jc / r_jj (= q_j^T a_c) and the next pass's
//           coefficients s_jc / s_jj and 1 / r_jj.
// Q (row-major) is written by pass 0 from A and updated in place after that.
// A row of n <= 64 columns is one wave-wide load: lane c holds column c, and
// a_j's entry is taken from lane j (v_readlane).  Rank deficiency (s_jj = 0)
// is not detected: Inf/NaN propagate.
#include "tsqr_common.hpp"

namespace tsqr {

namespace {

constexpr int kMgsRows = 1024;  // rows per workgroup (chunk) of a pass

template <typename T>
__device__ __forceinline__ T rdlane_u(T x, int j);
template <>
__device__ __forceinline__ double rdlane_u(double x, int j) {
    struct P { int lo, hi; };
    P p = __builtin_bit_cast(P, x);
    p.lo = __builtin_amdgcn_readlane(p.lo, j);
    p.hi = __builtin_amdgcn_readlane(p.hi, j);
    return __builtin_bit_cast(double, p);
}
template <>
__device__ __forceinline__ float rdlane_u(float x, int j) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), j));
}

// One pass (see above).  coef[c] = r_{j-1,c} / r_{j-1,j-1} for c >= j and
// coef[64] = 1 / r_{j-1,j-1}, written by the previous reduce; part[chunk][c]
// receives the chunk's partial sums for c >= j (zero elsewhere).
template <typename T>
__global__ __launch_bounds__(256) void k_mgs_pass(int64_t m, int n, int j, const T* __restrict__ src, int64_t lds,
                                                  T* __restrict__ Q, int64_t ldq, const T* __restrict__ coef,
                                                  T* __restrict__ part) {
    __shared__ T red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kMgsRows;
    const int64_t r1 = (r0 + kMgsRows < m) ? r0 + kMgsRows : m;
    const bool upd = j > 0;
    const T cf = (upd && lane >= j && lane < n) ? coef[lane] : T(0);
    const T inv = upd ? coef[64] : T(1);
    // lanes that read and write: the columns from j - 1 on
    const bool live = lane < n && lane >= (upd ? j - 1 : 0);
    T acc[4] = {T(0), T(0), T(0), T(0)};
    // wave w takes rows r0 + w, r0 + w + 4, ...; four rows per iteration
    int64_t i = r0 + w;
    for (; i + 12 < r1; i += 16) {
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = live ? src[(i + 4 * u) * lds + lane] : T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (upd) {
                const T v = rdlane_u(x[u], j - 1);
                x[u] = (lane == j - 1) ? v * inv : fma(-cf, v, x[u]);
            }
            if (live) Q[(i + 4 * u) * ldq + lane] = x[u];
            if (j < n) {
                const T xj = rdlane_u(x[u], j);
                acc[u] = fma(xj, (lane >= j) ? x[u] : T(0), acc[u]);
            }
        }
    }
    for (; i < r1; i += 4) {
        T x = live ? src[i * lds + lane] : T(0);
        if (upd) {
            const T v = rdlane_u(x, j - 1);
            x = (lane == j - 1) ? v * inv : fma(-cf, v, x);
        }
        if (live) Q[i * ldq + lane] = x;
        if (j < n) {
            const T xj = rdlane_u(x, j);
            acc[0] = fma(xj, (lane >= j) ? x : T(0), acc[0]);
        }
    }
    if (j >= n) return;
    red[w][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (w == 0) part[(int64_t)blockIdx.x * 64 + lane] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Reduce of step j: one wave, lane c sums part[*][c] over the chunks (four
// strided running sums, then their sum: a fixed order).
template <typename T>
__global__ __launch_bounds__(64) void k_mgs_reduce(int n, int j, int64_t nchunks, const T* __restrict__ part,
                                                   T* __restrict__ R, int64_t ldr, T* __restrict__ coef) {
    const int lane = threadIdx.x;
    T s[4] = {T(0), T(0), T(0), T(0)};
    int64_t c = 0;
    for (; c + 3 < nchunks; c += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] += part[(c + u) * 64 + lane];
    }
    for (; c < nchunks; ++c) s[0] += part[c * 64 + lane];
    const T sc = (s[0] + s[1]) + (s[2] + s[3]);
    const T sjj = rdlane_u(sc, j);
    const T rjj = sqrt(sjj);
    if (lane < n) R[(int64_t)j * ldr + lane] = (lane > j) ? sc / rjj : ((lane == j) ? rjj : T(0));
    if (lane < n) coef[lane] = (lane > j) ? sc / sjj : T(0);
    if (lane == 0) coef[64] = T(1) / rjj;
}

template <typename T>
hipError_t mgs_t(int64_t m, int n, const T* A, int64_t lda, T* Q, int64_t ldq, T* R, int64_t ldr, hipStream_t st) {
    const int64_t nchunks = (m + kMgsRows - 1) / kMgsRows;
    if (nchunks > 0x7fffffff) return hipErrorInvalidValue;
    void* ws = nullptr;
    hipError_t e = ws_malloc(&ws, (size_t)(nchunks * 64 + 128) * sizeof(T), st);
    if (e != hipSuccess) return e;
    T* part = (T*)ws;
    T* coef = part + nchunks * 64;
    for (int j = 0; j <= n && e == hipSuccess; ++j) {
        const T* src = (j == 0) ? A : Q;
        const int64_t ls = (j == 0) ? lda : ldq;
        k_mgs_pass<T><<<(unsigned)nchunks, 256, 0, st>>>(m, n, j, src, ls, Q, ldq, coef, part);
        if (j < n) k_mgs_reduce<T><<<1, 64, 0, st>>>(n, j, nchunks, part, R, ldr, coef);
        e = hipGetLastError();
    }
    hipError_t e2 = hipFreeAsync(ws, st);
    return e != hipSuccess ? e : e2;
}

}  // namespace

hipError_t launch_mgs(bool f64, int64_t m, int64_t n, const void* A, int64_t lda, void* Q, int64_t ldq, void* R,
                      int64_t ldr, hipStream_t st) {
    if (f64) return mgs_t<double>(m, (int)n, (const double*)A, lda, (double*)Q, ldq, (double*)R, ldr, st);
    return mgs_t<float>(m, (int)n, (const float*)A, lda, (float*)Q, ldq, (float*)R, ldr, st);
}

}  // namespace tsqr
