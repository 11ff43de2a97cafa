// TSQR factorisation kernels for gfx950 (paper Sec. 2.1).
//
//  * k_chain_factor: one workgroup per chain (a contiguous range of rows).
//    It runs sequential TSQR on a flat tree (Sec. 2.1): the first block is a
//    plain Householder QR; every later block is factored stacked under the
//    R factor kept in LDS, so A is read once and the reflectors written once
//    (Table 4, Eq. TSQR_seq_runtime: 2mn words).
//  * k_tree_combine: one workgroup per tree node; folds the R factors of the
//    node's children into the first child's R, one stacked-triangle QR per
//    child (Sec. 2.1, Eqs. TSQR_binarytree_2/3).  Reflector j of such a step
//    touches the head row j and only the rows of the lower triangle that are
//    nonzero, so the stored bottom reflectors stay upper triangular (the
//    zeros of the triangles stay exact zeros).
//
// Local QR (the engine hh_factor): Householder reflectors with unit topmost
// entry (Sec. 5.2 normalisation), beta = -sign(alpha)||x||, sign(0) = +1,
// tau = 0 for a zero tail.  The per-block compact-WY factor T of the block
// Householder form I - Y T Y^T (Schreiber-Van Loan, cited in Sec. 2.1 and
// used for the trailing update in Sec. 3.1) is built at the end of every
// block from the Gram entries y_i^T v_j gathered during the factorisation.
//
// Register tile: the block's rows x NC columns are spread over 8*NW row-lanes
// and 8 column-lanes (lane = row-lane + 8 * column-lane inside a wave), each
// thread holding RPT rows x NC/8 columns.  Column reductions are 8-lane DPP
// sums inside a wave plus one LDS exchange across waves.
#include "tsqr_common.hpp"

namespace tsqr {
using namespace dev;

template <typename T, int NC, int NW>
struct FactorSmem {
    T R[NC][NC];                       // head rows (R factor kept on chip)
    T PT[NC][NC + 1];                  // Gram entries P (strict upper), then T
    T tmp[(NC / 2) * (NC / 2) + 1];    // T-build scratch
    T tau[NC];
    T redn[2][NW];
    T alpha[2];
    T redw[2][NW][NC];
};

// Factor the register tile.  tile_mode: the head of reflector j is tile row j
// (first block of a chain: plain Householder QR).  Otherwise the head is row j
// of the on-chip R (sm.R), and all tile rows belong to the reflector's tail.
template <typename T, int NC, int RPT, int NW>
__device__ __forceinline__ void hh_factor(T (&x)[RPT][NC / 8], FactorSmem<T, NC, NW>& sm, int n, bool tile_mode) {
    constexpr int CPT = NC / 8;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int rl = lane & 7, cl = lane >> 3;
    const int rbase = rl + 8 * wv;
#pragma unroll
    for (int jt = 0; jt < CPT; ++jt) {
        for (int jc = 0; jc < 8; ++jc) {
            const int j = 8 * jt + jc;
            if (j >= n) break;
            const int buf = j & 1;
            // ---- phase 1: alpha and sigma^2 = ||tail of column j||^2
            T s = T(0);
            if (cl == jc) {
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const int r = rbase + 8 * NW * q;
                    const T xv = x[q][jt];
                    if (!tile_mode || r > j) s = fma(xv, xv, s);
                    if (tile_mode && r == j) sm.alpha[buf] = xv;
                }
            }
            s = sum8(s);
            if (rl == 0 && cl == jc) sm.redn[buf][wv] = s;
            T Rrow[CPT];
            T alpha_r = T(0);
            if (!tile_mode) {
                alpha_r = sm.R[j][j];
#pragma unroll
                for (int t = 0; t < CPT; ++t) {
                    const int c = cl + 8 * t;
                    Rrow[t] = (c > j) ? sm.R[j][c] : T(0);
                }
            }
            __syncthreads();
            T sigma2 = sum8((rl < NW) ? sm.redn[buf][rl < NW ? rl : 0] : T(0));
            const T alpha = tile_mode ? sm.alpha[buf] : alpha_r;
            T beta, tau, scale;
            if (sigma2 == T(0)) {
                tau = T(0);
                beta = alpha;
                scale = T(0);
            } else {
                const T nrm = sqrt(fma(alpha, alpha, sigma2));
                beta = (alpha >= T(0)) ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scale = T(1) / (alpha - beta);
            }
            // ---- phase 2: reflector entries for this thread's rows
            T v[RPT];
            const int src = rl + 8 * jc;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int r = rbase + 8 * NW * q;
                const T xj = shfl(x[q][jt], src);
                T vv = xj * scale;
                if (tile_mode) vv = (r < j) ? T(0) : ((r == j) ? T(1) : vv);
                v[q] = vv;
                if (cl == jc) {
                    if (!tile_mode || r > j) x[q][jt] = vv;
                    else if (r == j) x[q][jt] = beta;
                }
            }
            // ---- phase 3: v^T x for every column this thread holds
            //      (columns < j: Gram entries for T; columns > j: w for the update)
            T acc[CPT];
#pragma unroll
            for (int t = 0; t < CPT; ++t) {
                T a = T(0);
#pragma unroll
                for (int q = 0; q < RPT; ++q) a = fma(v[q], x[q][t], a);
                acc[t] = sum8(a);
            }
            if (rl == 0) {
#pragma unroll
                for (int t = 0; t < CPT; ++t) sm.redw[buf][wv][cl + 8 * t] = acc[t];
            }
            __syncthreads();
            T w[CPT];
#pragma unroll
            for (int t = 0; t < CPT; ++t) {
                T p = (rl < NW) ? sm.redw[buf][rl < NW ? rl : 0][cl + 8 * t] : T(0);
                w[t] = sum8(p);
                if (!tile_mode) w[t] += Rrow[t];
            }
            // ---- phase 4: record Gram entries, tau and the new head row
            if (wv == 0 && rl == 0) {
#pragma unroll
                for (int t = 0; t < CPT; ++t) {
                    const int c = cl + 8 * t;
                    if (c < j) sm.PT[c][j] = w[t];
                    if (!tile_mode) {
                        if (c > j) sm.R[j][c] = fma(-tau, w[t], Rrow[t]);
                        else if (c == j) sm.R[j][j] = beta;
                    }
                }
                if (cl == 0) sm.tau[j] = tau;
            }
            // ---- phase 5: rank-1 update of the trailing columns
#pragma unroll
            for (int t = 0; t < CPT; ++t) {
                if (t < jt) continue;
                const int c = cl + 8 * t;
                if (c > j) {
                    const T tw = tau * w[t];
#pragma unroll
                    for (int q = 0; q < RPT; ++q) x[q][t] = fma(-v[q], tw, x[q][t]);
                }
            }
        }
    }
}

// T of the block reflector I - V T V^T from P = strict upper part of V^T V and
// tau, by the block recurrence T12 = -T11 P12 T22 on diagonal blocks of size
// 1, 2, 4, ...  (in place in sm.PT; columns >= n stay zero).
template <typename T, int NC, int NW>
__device__ __forceinline__ void build_T(FactorSmem<T, NC, NW>& sm, int n) {
    constexpr int NT = 64 * NW;
    const int tid = threadIdx.x;
    for (int i = tid; i < NC; i += NT) sm.PT[i][i] = (i < n) ? sm.tau[i] : T(0);
    __syncthreads();
    for (int s = 1; s < NC; s *= 2) {
        const int npairs = NC / (2 * s);
        const int ss = s * s;
        for (int e = tid; e < npairs * ss; e += NT) {
            const int pr = e / ss, rem = e - pr * ss, i = rem / s, jj = rem - i * s;
            const int o = 2 * s * pr;
            T a = T(0);
            for (int l = 0; l <= jj; ++l) a = fma(sm.PT[o + i][o + s + l], sm.PT[o + s + l][o + s + jj], a);
            sm.tmp[e] = a;
        }
        __syncthreads();
        for (int e = tid; e < npairs * ss; e += NT) {
            const int pr = e / ss, rem = e - pr * ss, i = rem / s, jj = rem - i * s;
            const int o = 2 * s * pr;
            T a = T(0);
            for (int l = i; l < s; ++l) a = fma(sm.PT[o + i][o + l], sm.tmp[pr * ss + l * s + jj], a);
            sm.PT[o + i][o + s + jj] = -a;
        }
        __syncthreads();
    }
}

template <typename T, int NC, int NW>
__device__ __forceinline__ void smem_init(FactorSmem<T, NC, NW>& sm) {
    T* p = &sm.PT[0][0];
    for (int e = threadIdx.x; e < NC * (NC + 1); e += 64 * NW) p[e] = T(0);
    T* r = &sm.R[0][0];
    for (int e = threadIdx.x; e < NC * NC; e += 64 * NW) r[e] = T(0);
    __syncthreads();
}

template <typename T, int NC, int NW>
__device__ __forceinline__ void store_T_tau(FactorSmem<T, NC, NW>& sm, int n, T* __restrict__ Tout,
                                            T* __restrict__ tauout) {
    for (int e = threadIdx.x; e < n * n; e += 64 * NW) {
        const int i = e / n, j = e - i * n;
        if (i <= j) Tout[j * (j + 1) / 2 + i] = sm.PT[i][j];
    }
    for (int i = threadIdx.x; i < n; i += 64 * NW) tauout[i] = sm.tau[i];
}

template <typename T, int NC, int RPT, int NW>
__global__ __launch_bounds__(64 * NW) void k_chain_factor(Geom g, T* __restrict__ A, int64_t lda,
                                                          T* __restrict__ tau_blk, T* __restrict__ T_blk,
                                                          T* __restrict__ Rbuf) {
    __shared__ FactorSmem<T, NC, NW> sm;
    constexpr int CPT = NC / 8, ROWS = 8 * NW * RPT;
    const int c = blockIdx.x;
    const int n = (int)g.n;
    const int tri = n * (n + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, rl = lane & 7, cl = lane >> 3;
    const int rbase = rl + 8 * wv;
    smem_init(sm);
    const int64_t start = chain_start(g, c), end = chain_end(g, c);
    const int nb = chain_nblocks(g, c);
    const int64_t blk0 = chain_blk0(g, c);
    for (int b = 0; b < nb; ++b) {
        const int64_t r0 = start + (int64_t)b * ROWS;
        const int rows = (int)((end - r0) < ROWS ? (end - r0) : ROWS);
        T x[RPT][CPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = rbase + 8 * NW * q;
#pragma unroll
            for (int t = 0; t < CPT; ++t) {
                const int cc = cl + 8 * t;
                x[q][t] = (r < rows && cc < n) ? A[(r0 + r) * lda + cc] : T(0);
            }
        }
        hh_factor<T, NC, RPT, NW>(x, sm, n, b == 0);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = rbase + 8 * NW * q;
#pragma unroll
            for (int t = 0; t < CPT; ++t) {
                const int cc = cl + 8 * t;
                if (r < rows && cc < n) A[(r0 + r) * lda + cc] = x[q][t];
                if (b == 0 && r < n && cc >= r && cc < n) sm.R[r][cc] = x[q][t];
            }
        }
        __syncthreads();
        build_T(sm, n);
        store_T_tau(sm, n, T_blk + (blk0 + b) * tri, tau_blk + (blk0 + b) * n);
        __syncthreads();
    }
    T* Rc = Rbuf + (int64_t)c * n * n;
    for (int e = tid; e < n * n; e += 64 * NW) {
        const int i = e / n, j = e - i * n;
        Rc[e] = (j >= i) ? sm.R[i][j] : T(0);
    }
}

// One node of the reduction tree at level `lev`: fold children
// i + t*stride (t = 1..arity-1) into the R of child i.
template <typename T, int NC, int NW>
__global__ __launch_bounds__(64 * NW) void k_tree_combine(Geom g, int lev, T* __restrict__ Rbuf,
                                                          T* __restrict__ Ynode, T* __restrict__ Tnode,
                                                          T* __restrict__ tau_node) {
    __shared__ FactorSmem<T, NC, NW> sm;
    constexpr int CPT = NC / 8;
    constexpr int RPT = (NC / (8 * NW)) > 0 ? NC / (8 * NW) : 1;
    const int n = (int)g.n;
    const int tri = n * (n + 1) / 2;
    const int64_t stride = ipow(g.arity, lev - 1);
    const int64_t i0 = (int64_t)blockIdx.x * g.arity * stride;
    if (i0 + stride >= g.W) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, rl = lane & 7, cl = lane >> 3;
    const int rbase = rl + 8 * wv;
    smem_init(sm);
    const T* Ra = Rbuf + i0 * n * n;
    for (int e = tid; e < n * n; e += 64 * NW) {
        const int i = e / n, j = e - i * n;
        sm.R[i][j] = Ra[e];
    }
    __syncthreads();
    for (int t1 = 1; t1 < g.arity; ++t1) {
        const int64_t c = i0 + t1 * stride;
        if (c >= g.W) break;
        const T* Rc = Rbuf + c * n * n;
        T x[RPT][CPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = rbase + 8 * NW * q;
#pragma unroll
            for (int t = 0; t < CPT; ++t) {
                const int cc = cl + 8 * t;
                x[q][t] = (r < n && cc < n) ? Rc[r * n + cc] : T(0);
            }
        }
        hh_factor<T, NC, RPT, NW>(x, sm, n, false);
        T* Yc = Ynode + c * n * n;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = rbase + 8 * NW * q;
#pragma unroll
            for (int t = 0; t < CPT; ++t) {
                const int cc = cl + 8 * t;
                if (r < n && cc < n) Yc[r * n + cc] = x[q][t];
            }
        }
        __syncthreads();
        build_T(sm, n);
        store_T_tau(sm, n, Tnode + c * tri, tau_node + c * n);
        __syncthreads();
    }
    T* Rw = Rbuf + i0 * n * n;
    for (int e = tid; e < n * n; e += 64 * NW) {
        const int i = e / n, j = e - i * n;
        Rw[e] = (j >= i) ? sm.R[i][j] : T(0);
    }
}

template <typename T>
__global__ void k_copy_r(int64_t n, const T* __restrict__ Rsrc, T* __restrict__ R, int64_t ldr, int zero_lower) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int64_t i = e / n, j = e - i * n;
    if (j >= i) R[i * ldr + j] = Rsrc[e];
    else if (zero_lower) R[i * ldr + j] = T(0);
}

template <typename T, int NC>
static hipError_t factor_nc(const Geom& g, T* A, int64_t lda, const Work& wk, hipStream_t st) {
    T* tau_blk = (T*)wk.tau_blk;
    T* T_blk = (T*)wk.T_blk;
    T* Rbuf = (T*)wk.Rbuf;
    phase_begin(0, st);
    switch (g.h) {
        case 64: k_chain_factor<T, NC, 2, 4><<<g.W, 256, 0, st>>>(g, A, lda, tau_blk, T_blk, Rbuf); break;
        case 128: k_chain_factor<T, NC, 4, 4><<<g.W, 256, 0, st>>>(g, A, lda, tau_blk, T_blk, Rbuf); break;
        case 256: k_chain_factor<T, NC, 8, 4><<<g.W, 256, 0, st>>>(g, A, lda, tau_blk, T_blk, Rbuf); break;
        default: return hipErrorInvalidValue;
    }
    phase_end(0, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int lev = 1; lev <= g.levels; ++lev) {
        const int64_t stride = ipow(g.arity, lev - 1);
        const int64_t span = stride * g.arity;
        const int nodes = (int)((g.W + span - 1) / span);
        k_tree_combine<T, NC, 1><<<nodes, 64, 0, st>>>(g, lev, Rbuf, (T*)wk.Ynode, (T*)wk.Tnode, (T*)wk.tau_node);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
static hipError_t factor_t(const Geom& g, T* A, int64_t lda, const Work& wk, hipStream_t st) {
    switch (g.NC) {
        case 8: return factor_nc<T, 8>(g, A, lda, wk, st);
        case 16: return factor_nc<T, 16>(g, A, lda, wk, st);
        case 32: return factor_nc<T, 32>(g, A, lda, wk, st);
        case 64: return factor_nc<T, 64>(g, A, lda, wk, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_factor(bool f64, const Geom& g, void* A, int64_t lda, const Work& wk, hipStream_t st) {
    return f64 ? factor_t<double>(g, (double*)A, lda, wk, st) : factor_t<float>(g, (float*)A, lda, wk, st);
}

hipError_t launch_copy_r(bool f64, int64_t n, const void* Rsrc, void* R, int64_t ldr, bool zero_lower,
                         hipStream_t st) {
    const int64_t tot = n * n;
    const int nb = (int)((tot + 255) / 256);
    if (f64)
        k_copy_r<double><<<nb, 256, 0, st>>>(n, (const double*)Rsrc, (double*)R, ldr, zero_lower ? 1 : 0);
    else
        k_copy_r<float><<<nb, 256, 0, st>>>(n, (const float*)Rsrc, (float*)R, ldr, zero_lower ? 1 : 0);
    return hipGetLastError();
}

}  // namespace tsqr
