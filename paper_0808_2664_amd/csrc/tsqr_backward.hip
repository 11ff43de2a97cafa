// Reverse-mode derivative (adjoint) of the thin QR map A -> (Q, R) with
// diag(R) > 0, for the differentiable TSQR.  Not in the paper: the published
// QR adjoint (Walter & Lehmann; Liao, Liu, Wang & Xiang, "copyltu" form):
//     M  = R triu(dR)^T - dQ^T Q,   C = tril(M) + tril(M, -1)^T,
//     dA = (dQ + Q C) R^{-T} = dQ Y + Q X,   Y = R^{-T},  X = C R^{-T}.
// The m-long contraction dQ^T Q is reduced like the TSQR tree: row chunks,
// each a sum of MFMA products, then the chunk partials in a fixed order.
// The n x n work (M, C, R^{-1}) runs in one workgroup per matrix; R^{-1} uses
// the same block recurrence as the T factors (inverse of an upper triangle:
// T12 = -T11 U12 T22).  dA is one streaming pass over dQ and Q on MFMA.
// CholeskyQR, the comparison algorithm of Sec. 2.3, reuses the Gram kernels.
#include "tsqr_common.hpp"

namespace tsqr {
using namespace dev;

// Partial Gram dQ^T Q over rows [ch*CR, (ch+1)*CR) of matrix b.  SYM: dQ and
// Q are the same matrix; only the tiles on and above the diagonal are formed
// (the others are written as zeros) and the matrix is read once.
template <typename T, int NC, bool SYM = false>
__global__ __launch_bounds__(256) void k_gram(int64_t m, int n, const T* __restrict__ dQ, int64_t lddq, int64_t sdq,
                                              const T* __restrict__ Q, int64_t ldq, int64_t sq, int64_t CR,
                                              T* __restrict__ part) {
    typedef Mfma<T> M;
    typedef typename M::acc acc_t;
    constexpr int NCP = NC < 16 ? 16 : NC;
    constexpr int NP = NCP / 16;
    __shared__ T red[4][16][17];
    const int b = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const T* dq = dQ + (int64_t)b * sdq;
    const T* q = Q + (int64_t)b * sq;
    const int64_t lo = (int64_t)ch * CR, hi = (lo + CR < m) ? lo + CR : m;
    acc_t acc[NP][NP];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int c = 0; c < NP; ++c) acc[p][c] = acc_t{0, 0, 0, 0};
    // a 64-row step's rows (4 per lane and column tile), loaded one step
    // ahead of the products that use them; the products and their order are
    // those of a plain loop over the steps
    auto load_step = [&](int64_t r0, T (&a)[4][NP], T (&bq)[4][NP]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = r0 + M::orow(l4, i);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int cc = 16 * p + l16;
                const bool ok = (r < hi) && (cc < n);
                a[i][p] = ok ? dq[r * lddq + cc] : T(0);
                bq[i][p] = SYM ? a[i][p] : (ok ? q[r * ldq + cc] : T(0));
            }
        }
    };
    T a[4][NP], bq[4][NP];
    int64_t r0 = lo + 16 * wv;
    if (r0 < hi) load_step(r0, a, bq);
    for (; r0 < hi; r0 += 64) {
        T na[4][NP], nb[4][NP];
        if (r0 + 64 < hi) load_step(r0 + 64, na, nb);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int c = 0; c < NP; ++c)
                    if (!SYM || c >= p) acc[p][c] = M::mma(a[i][p], bq[i][c], acc[p][c]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                a[i][p] = na[i][p];
                bq[i][p] = nb[i][p];
            }
    }
    T* out = part + ((int64_t)b * nch + ch) * NCP * NCP;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int c = 0; c < NP; ++c) {
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wv][M::orow(l4, r)][l16] = acc[p][c][r];
            __syncthreads();
            {
                const int i = tid >> 4, j = tid & 15;
                T s = red[0][i][j] + red[1][i][j];
                s += red[2][i][j];
                s += red[3][i][j];
                out[(16 * p + i) * NCP + 16 * c + j] = s;
            }
            __syncthreads();
        }
}

// G[b] = sum over chunks of the partials, in a fixed order: wave w of a
// workgroup adds chunks w, w + 4, w + 8, ... for 64 consecutive entries (one
// per lane, so the loads are coalesced) into four running sums (chunks
// w + 16 t + 4 u go to sum u), then the sums and the four waves' results are
// added in order.  Sixteen independent streams per entry keep the loads in
// flight.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_gram_reduce(int nch, const T* __restrict__ part, T* __restrict__ G) {
    constexpr int NCP = NC < 16 ? 16 : NC;
    __shared__ T red[4][64];
    const int b = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    const bool ok = e < NCP * NCP;
    const T* p = part + (int64_t)b * nch * NCP * NCP + (ok ? e : 0);
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    int c = wv;
    for (; c + 12 < nch; c += 16) {
        s0 += p[(int64_t)c * NCP * NCP];
        s1 += p[(int64_t)(c + 4) * NCP * NCP];
        s2 += p[(int64_t)(c + 8) * NCP * NCP];
        s3 += p[(int64_t)(c + 12) * NCP * NCP];
    }
    for (; c < nch; c += 4) s0 += p[(int64_t)c * NCP * NCP];
    red[wv][lane] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (wv == 0 && ok) G[(int64_t)b * NCP * NCP + e] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Per matrix: X = copyltu(R triu(dR)^T - G) R^{-T} and Y = R^{-T}.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_adjoint_small(int n, const T* __restrict__ R, int64_t ldr, int64_t sr,
                                                       const T* __restrict__ dR, int64_t lddr, int64_t sdr,
                                                       const T* __restrict__ G, int has_dq, T* __restrict__ XY) {
    constexpr int NCP = NC < 16 ? 16 : NC;
    __shared__ T Rs[NCP][NCP + 1];
    __shared__ T Ui[NCP][NCP + 1];  // R^{-1}, built in place
    __shared__ T Cm[NCP][NCP + 1];
    __shared__ T tmp[(NCP / 2) * (NCP / 2)];
    const int b = blockIdx.x, tid = threadIdx.x;
    const T* r = R + (int64_t)b * sr;
    const T* dr = dR ? dR + (int64_t)b * sdr : nullptr;
    const T* g = G + (int64_t)b * NCP * NCP;
    for (int e = tid; e < NCP * NCP; e += 256) {
        const int i = e / NCP, j = e - i * NCP;
        const T v = (i < n && j < n && j >= i) ? r[i * ldr + j] : T(0);
        Rs[i][j] = v;
        Ui[i][j] = (i == j) ? ((i < n) ? T(1) / v : T(0)) : v;
    }
    __syncthreads();
    // M = R triu(dR)^T - G  (Cm holds M)
    for (int e = tid; e < NCP * NCP; e += 256) {
        const int i = e / NCP, j = e - i * NCP;
        T a = T(0);
        if (i < n && j < n) {
            if (dr) {
                const int k0 = i > j ? i : j;
                for (int k = k0; k < n; ++k) a = fma(Rs[i][k], dr[j * lddr + k], a);
            }
            if (has_dq) a -= g[i * NCP + j];
        }
        Cm[i][j] = a;
    }
    // R^{-1} by the block recurrence on diagonal blocks of size 1, 2, 4, ...
    for (int s = 1; s < NCP; s *= 2) {
        const int npairs = NCP / (2 * s), ss = s * s;
        __syncthreads();
        for (int e = tid; e < npairs * ss; e += 256) {
            const int pr = e / ss, rem = e - pr * ss, i = rem / s, jj = rem - i * s;
            const int o = 2 * s * pr;
            T a = T(0);
            for (int l = 0; l <= jj; ++l) a = fma(Ui[o + i][o + s + l], Ui[o + s + l][o + s + jj], a);
            tmp[e] = a;
        }
        __syncthreads();
        for (int e = tid; e < npairs * ss; e += 256) {
            const int pr = e / ss, rem = e - pr * ss, i = rem / s, jj = rem - i * s;
            const int o = 2 * s * pr;
            T a = T(0);
            for (int l = i; l < s; ++l) a = fma(Ui[o + i][o + l], tmp[pr * ss + l * s + jj], a);
            Ui[o + i][o + s + jj] = -a;
        }
    }
    __syncthreads();
    // X = C R^{-T}, C = copyltu(M);  Y = R^{-T}
    T* X = XY + (int64_t)b * 2 * NCP * NCP;
    T* Y = X + NCP * NCP;
    for (int e = tid; e < NCP * NCP; e += 256) {
        const int i = e / NCP, j = e - i * NCP;
        T a = T(0);
        if (i < n && j < n) {
            for (int k = j; k < n; ++k) {
                const T c = (i >= k) ? Cm[i][k] : Cm[k][i];
                a = fma(c, Ui[j][k], a);
            }
        }
        X[i * NCP + j] = a;
        Y[i * NCP + j] = (i < n && j < n && i >= j) ? Ui[j][i] : T(0);
    }
}

// dA = dQ Y + Q X over 256-row blocks (4 waves x 64 rows).
// VEC (n a multiple of 16 and rows of dQ and Q aligned to 16 bytes): each
// lane reads four consecutive entries of its row per load group (columns
// 16h + 4 l4 .. +3), so a wave's load covers 16 rows in runs of 64 (FP32) or
// 128 (FP64) bytes instead of 16 or 32; the K order of the products follows
// (step 4h + j takes column 16h + 4 l4 + j), a permutation of the same sum.
template <typename T, int NC, bool VEC>
__global__ __launch_bounds__(256) void k_adjoint_stream(int64_t m, int n, const T* __restrict__ dQ, int64_t lddq,
                                                        int64_t sdq, const T* __restrict__ Q, int64_t ldq,
                                                        int64_t sq, const T* __restrict__ XY, T* __restrict__ dA,
                                                        int64_t ldda, int64_t sda) {
    typedef Mfma<T> M;
    typedef typename M::acc acc_t;
    constexpr int NCP = NC < 16 ? 16 : NC;
    constexpr int NP = NCP / 16;
    constexpr int NK = NCP / 4;
    __shared__ T Xs[NCP][NCP + 1];
    __shared__ T Ys[NCP][NCP + 1];
    const int b = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const T* xy = XY + (int64_t)b * 2 * NCP * NCP;
    for (int e = tid; e < NCP * NCP; e += 256) {
        const int i = e / NCP, j = e - i * NCP;
        Xs[i][j] = xy[e];
        Ys[i][j] = xy[NCP * NCP + e];
    }
    __syncthreads();
    const T* dq = dQ ? dQ + (int64_t)b * sdq : nullptr;
    const T* q = Q + (int64_t)b * sq;
    T* da = dA + (int64_t)b * sda;
    const int64_t base = (int64_t)blockIdx.x * 256 + 64 * wv;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int64_t rr = base + 16 * s + l16;  // A-operand row of this lane
        T adq[NK], aq[NK];
        if constexpr (VEC) {
            typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type V;
            constexpr int PER = 16 / (int)sizeof(T);  // entries of one 16-byte load
            const bool ok = rr < m;
#pragma unroll
            for (int h = 0; h < NP; ++h)
#pragma unroll
                for (int v = 0; v < 4 / PER; ++v) {
                    const int cc = 16 * h + 4 * l4 + PER * v;
                    const V z = V{};
                    const V a = (ok && dq) ? *(const V*)(dq + rr * lddq + cc) : z;
                    const V b = ok ? *(const V*)(q + rr * ldq + cc) : z;
                    const T* pa = (const T*)&a;
                    const T* pb = (const T*)&b;
#pragma unroll
                    for (int j = 0; j < PER; ++j) {
                        adq[4 * h + PER * v + j] = pa[j];
                        aq[4 * h + PER * v + j] = pb[j];
                    }
                }
        } else {
#pragma unroll
            for (int k4 = 0; k4 < NK; ++k4) {
                const int cc = 4 * k4 + l4;
                const bool ok = (rr < m) && (cc < n);
                adq[k4] = (ok && dq) ? dq[rr * lddq + cc] : T(0);
                aq[k4] = ok ? q[rr * ldq + cc] : T(0);
            }
        }
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            acc_t u = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int k4 = 0; k4 < NK; ++k4) {
                const int kr = VEC ? 16 * (k4 >> 2) + 4 * l4 + (k4 & 3) : 4 * k4 + l4;
                u = M::mma(adq[k4], Ys[kr][16 * c + l16], u);
                u = M::mma(aq[k4], Xs[kr][16 * c + l16], u);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = base + 16 * s + M::orow(l4, r);
                const int col = 16 * c + l16;
                if (row < m && col < n) da[row * ldda + col] = u[r];
            }
        }
    }
}

// CholeskyQR (Sec. 2.3: the fast, conditionally stable alternative to TSQR):
// R = upper Cholesky factor of G = A^T A, Q = A R^{-1}.  The Gram matrix
// reuses k_gram (symmetric form) and k_gram_reduce, the product A R^{-1} is
// k_rmul_stream with R^{-1} taken from Y of XY; this kernel does the n x n
// part in one workgroup:
// Cholesky of G in LDS, R^{-1} column by column, and R written out, or
// R Rprev when Rprev is given (the second pass of CholeskyQR2: R = R2 R1).
// A pivot that is not positive gives NaN (sqrt of a negative), which
// propagates to Q and R.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_chol_small(int n, const T* __restrict__ G, T* R, int64_t ldr, const T* Rprev,
                                                    int64_t ldp, T* __restrict__ XY) {
    constexpr int NCP = NC < 16 ? 16 : NC;
    __shared__ T Gs[NCP][NCP + 1];
    __shared__ T Ui[NCP][NCP + 1];
    __shared__ T Pv[NCP][NCP + 1];
    const int tid = threadIdx.x;
    for (int e = tid; e < NCP * NCP; e += 256) {
        const int i = e / NCP, j = e - i * NCP;
        Gs[i][j] = (i < n && j < n) ? G[i * NCP + j] : T(0);
        Pv[i][j] = (Rprev && i < n && j < n && j >= i) ? Rprev[(int64_t)i * ldp + j] : T(0);
    }
    __syncthreads();
    // right-looking Cholesky: row j of the upper triangle becomes row j of R
    for (int j = 0; j < n; ++j) {
        if (tid == 0) Gs[j][j] = sqrt(Gs[j][j]);
        __syncthreads();
        for (int c = j + 1 + tid; c < n; c += 256) Gs[j][c] /= Gs[j][j];
        __syncthreads();
        // thread (column tid % 64, row phase tid / 64) updates rows i > j
        {
            const int c = tid & 63;
            if (c > j && c < n) {
                const T rjc = Gs[j][c];
                for (int i = j + 1 + (tid >> 6); i <= c; i += 4) Gs[i][c] -= Gs[j][i] * rjc;
            }
        }
        __syncthreads();
    }
    // column c of R^{-1}: back substitution R x = e_c
    if (tid < NCP) {
        const int c = tid;
        for (int i = NCP - 1; i >= 0; --i) {
            T v = T(0);
            if (c < n && i <= c) {
                v = (i == c) ? T(1) : T(0);
                for (int l = i + 1; l <= c; ++l) v -= Gs[i][l] * Ui[l][c];
                v /= Gs[i][i];
            }
            Ui[i][c] = v;
        }
    }
    __syncthreads();
    T* X = XY;
    T* Y = XY + NCP * NCP;
    for (int e = tid; e < NCP * NCP; e += 256) {
        const int i = e / NCP, j = e - i * NCP;
        X[e] = T(0);
        Y[e] = Ui[i][j];
        if (i < n && j < n) {
            T v = T(0);
            if (j >= i) {
                if (Rprev) {
                    for (int l = i; l <= j; ++l) v += Gs[i][l] * Pv[l][j];
                } else {
                    v = Gs[i][j];
                }
            }
            R[(int64_t)i * ldr + j] = v;
        }
    }
}

// Q = A M for the n x n upper triangle M = R^{-1} (CholeskyQR's second
// step), over 512-row blocks (4 waves x 8 groups of 16 rows).  The K index of
// MFMA step k4 in lane group l4 is NK l4 + k4, so a lane reads NK consecutive
// entries of its row; the next group's rows are loaded while the current one
// is multiplied.  A wave loads a group's rows whole before writing them, so Q
// may be A itself.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_rmul_stream(int64_t m, int n, const T* A, int64_t lda,
                                                     const T* __restrict__ Mg, T* Q, int64_t ldq) {
    typedef Mfma<T> M;
    typedef typename M::acc acc_t;
    constexpr int NCP = NC < 16 ? 16 : NC;
    constexpr int NP = NCP / 16;
    constexpr int NK = NCP / 4;
    constexpr int GR = 8;  // groups of 16 rows per wave
    __shared__ T Ms[NCP][NCP + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    for (int e = tid; e < NCP * NCP; e += 256) {
        const int i = e / NCP, j = e - i * NCP;
        Ms[i][j] = Mg[e];
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (64 * GR) + (16 * GR) * wv;
    T a[NK], an[NK];
    auto load = [&](int g, T* dst) {
        const int64_t rr = base + 16 * g + l16;
#pragma unroll
        for (int k4 = 0; k4 < NK; ++k4) {
            const int cc = NK * l4 + k4;
            dst[k4] = (rr < m && cc < n) ? A[rr * lda + cc] : T(0);
        }
    };
    load(0, a);
    for (int g = 0; g < GR; ++g) {
        if (base + 16 * g >= m) break;
        if (g + 1 < GR) load(g + 1, an);
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            acc_t u = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int k4 = 0; k4 < NK; ++k4) u = M::mma(a[k4], Ms[NK * l4 + k4][16 * c + l16], u);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = base + 16 * g + M::orow(l4, r);
                const int col = 16 * c + l16;
                if (row < m && col < n) Q[row * ldq + col] = u[r];
            }
        }
#pragma unroll
        for (int k4 = 0; k4 < NK; ++k4) a[k4] = an[k4];
    }
}

template <typename T, int NC>
static hipError_t cholqr_nc(int64_t m, int n, const T* A, int64_t lda, T* Q, int64_t ldq, T* R, int64_t ldr,
                            int passes, hipStream_t st) {
    constexpr int NCP = NC < 16 ? 16 : NC;
    // about 512 chunks: two workgroups per CU for the Gram, and a partial-sum
    // buffer small enough (16 MB at n = 64) to be cheap to allocate per call
    int64_t CR = (m + 511) / 512;
    CR = ((CR + 255) / 256) * 256;
    if (CR < 256) CR = 256;
    const int64_t nch = (m + CR - 1) / CR;
    const size_t bytes = (size_t)(nch + 1 + 2) * NCP * NCP * sizeof(T);
    void* ws = nullptr;
    hipError_t e = ws_malloc(&ws, bytes, st);
    if (e != hipSuccess) return e;
    T* part = (T*)ws;
    T* G = part + (size_t)nch * NCP * NCP;
    T* XY = G + (size_t)NCP * NCP;
    const T* src = A;
    int64_t lds = lda;
    for (int p = 0; p < passes; ++p) {
        k_gram<T, NC, true><<<dim3((unsigned)nch, 1), 256, 0, st>>>(m, n, src, lds, 0, src, lds, 0, CR, part);
        k_gram_reduce<T, NC><<<dim3((NCP * NCP + 63) / 64, 1), 256, 0, st>>>((int)nch, part, G);
        k_chol_small<T, NC><<<1, 256, 0, st>>>(n, G, R, ldr, p > 0 ? R : nullptr, ldr, XY);
        // Q = src R^{-1} (Y of XY); each wave reads its rows whole before
        // writing them, so the second pass may run in place on Q
        k_rmul_stream<T, NC><<<(unsigned)((m + 511) / 512), 256, 0, st>>>(m, n, src, lds, XY + NCP * NCP, Q, ldq);
        src = Q;
        lds = ldq;
    }
    e = hipGetLastError();
    hipError_t e2 = hipFreeAsync(ws, st);
    return e != hipSuccess ? e : e2;
}

template <typename T>
static hipError_t cholqr_t(int64_t m, int n, const T* A, int64_t lda, T* Q, int64_t ldq, T* R, int64_t ldr, int passes,
                           hipStream_t st) {
    if (n <= 16) return cholqr_nc<T, 16>(m, n, A, lda, Q, ldq, R, ldr, passes, st);
    if (n <= 32) return cholqr_nc<T, 32>(m, n, A, lda, Q, ldq, R, ldr, passes, st);
    return cholqr_nc<T, 64>(m, n, A, lda, Q, ldq, R, ldr, passes, st);
}

hipError_t launch_cholqr(bool f64, int64_t m, int64_t n, const void* A, int64_t lda, void* Q, int64_t ldq, void* R,
                         int64_t ldr, int passes, hipStream_t st) {
    if (f64)
        return cholqr_t<double>(m, (int)n, (const double*)A, lda, (double*)Q, ldq, (double*)R, ldr, passes, st);
    return cholqr_t<float>(m, (int)n, (const float*)A, lda, (float*)Q, ldq, (float*)R, ldr, passes, st);
}

template <typename T, int NC>
static hipError_t backward_nc(int64_t batch, int64_t m, int n, const T* Q, int64_t ldq, int64_t sq, const T* R,
                              int64_t ldr, int64_t sr, const T* dQ, int64_t lddq, int64_t sdq, const T* dR,
                              int64_t lddr, int64_t sdr, T* dA, int64_t ldda, int64_t sda, hipStream_t st) {
    constexpr int NCP = NC < 16 ? 16 : NC;
    // chunks of whole 64-row steps, ~2048 workgroups in total
    int64_t CR = (m * batch + 2047) / 2048;
    CR = ((CR + 255) / 256) * 256;
    if (CR < 256) CR = 256;
    const int64_t nch = (m + CR - 1) / CR;
    const size_t es = sizeof(T);
    const size_t bytes = (size_t)batch * (nch + 1 + 2) * NCP * NCP * es;
    void* ws = nullptr;
    hipError_t e = ws_malloc(&ws, bytes, st);
    if (e != hipSuccess) return e;
    T* part = (T*)ws;
    T* G = part + (size_t)batch * nch * NCP * NCP;
    T* XY = G + (size_t)batch * NCP * NCP;
    if (dQ) {
        k_gram<T, NC><<<dim3((unsigned)nch, (unsigned)batch), 256, 0, st>>>(m, n, dQ, lddq, sdq, Q, ldq, sq, CR, part);
        k_gram_reduce<T, NC><<<dim3((NCP * NCP + 63) / 64, (unsigned)batch), 256, 0, st>>>((int)nch, part, G);
    }
    k_adjoint_small<T, NC><<<(unsigned)batch, 256, 0, st>>>(n, R, ldr, sr, dR, lddr, sdr, G, dQ ? 1 : 0, XY);
    // 16-byte loads: n fills the padded width, and every row start of dQ and
    // Q (base, leading dimension, member stride) is 16-byte aligned
    const int64_t al = 16 / (int64_t)es;
    auto aligned = [&](const T* p, int64_t ld, int64_t s) {
        return p == nullptr || (((uintptr_t)p % 16) == 0 && ld % al == 0 && (batch == 1 || s % al == 0));
    };
    const dim3 grid((unsigned)((m + 255) / 256), (unsigned)batch);
    if (n == NCP && aligned(dQ, lddq, sdq) && aligned(Q, ldq, sq))
        k_adjoint_stream<T, NC, true><<<grid, 256, 0, st>>>(m, n, dQ, lddq, sdq, Q, ldq, sq, XY, dA, ldda, sda);
    else
        k_adjoint_stream<T, NC, false><<<grid, 256, 0, st>>>(m, n, dQ, lddq, sdq, Q, ldq, sq, XY, dA, ldda, sda);
    e = hipGetLastError();
    hipError_t e2 = hipFreeAsync(ws, st);
    return e != hipSuccess ? e : e2;
}

template <typename T>
static hipError_t backward_t(int64_t batch, int64_t m, int n, const T* Q, int64_t ldq, int64_t sq, const T* R,
                             int64_t ldr, int64_t sr, const T* dQ, int64_t lddq, int64_t sdq, const T* dR, int64_t lddr,
                             int64_t sdr, T* dA, int64_t ldda, int64_t sda, hipStream_t st) {
    if (n <= 16)
        return backward_nc<T, 16>(batch, m, n, Q, ldq, sq, R, ldr, sr, dQ, lddq, sdq, dR, lddr, sdr, dA, ldda, sda, st);
    if (n <= 32)
        return backward_nc<T, 32>(batch, m, n, Q, ldq, sq, R, ldr, sr, dQ, lddq, sdq, dR, lddr, sdr, dA, ldda, sda, st);
    return backward_nc<T, 64>(batch, m, n, Q, ldq, sq, R, ldr, sr, dQ, lddq, sdq, dR, lddr, sdr, dA, ldda, sda, st);
}

hipError_t launch_backward(bool f64, int64_t batch, int64_t m, int64_t n, const void* Q, int64_t ldq, int64_t sq,
                           const void* R, int64_t ldr, int64_t sr, const void* dQ, int64_t lddq, int64_t sdq,
                           const void* dR, int64_t lddr, int64_t sdr, void* dA, int64_t ldda, int64_t sda,
                           hipStream_t st) {
    if (f64)
        return backward_t<double>(batch, m, (int)n, (const double*)Q, ldq, sq, (const double*)R, ldr, sr,
                                  (const double*)dQ, lddq, sdq, (const double*)dR, lddr, sdr, (double*)dA, ldda, sda,
                                  st);
    return backward_t<float>(batch, m, (int)n, (const float*)Q, ldq, sq, (const float*)R, ldr, sr, (const float*)dQ,
                             lddq, sdq, (const float*)dR, lddr, sdr, (float*)dA, ldda, sda, st);
}

}  // namespace tsqr
