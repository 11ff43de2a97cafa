// Householder engine shared by the TSQR kernels (plain and batched).
// See tsqr_factor.hip for the description of the method and the layout.
#pragma once
#include "tsqr_common.hpp"

namespace tsqr {
using namespace dev;

template <typename T, int NC, int NW>
struct FSmem {
    static constexpr int NCP = NC < 16 ? 16 : NC;
    // RG[i][j], i <= j: Gram entries v_i^T v_j, turned in place into T.
    // RG[j+1][i], i <= j: R[i][j] (the on-chip R, shifted below the diagonal).
    T RG[NCP + 1][NCP + 1];
    union U {
        T Wpart[NW][16][NCP];  // per-wave partial V_p^T X
        T trans[NW][16][17];   // per-wave 16x16 transpose
        T tmp[(NCP / 2) * (NCP / 2)];
    } u;
    T Wp[16][NCP + 1];
    T tau[NCP];
    T redw[2][NW][16];
    T hrow[2][16];
};

// ---- lane helpers ----------------------------------------------------------
__device__ __forceinline__ double swapsum(double x, bool sixteen) {
    struct P { int lo, hi; };
    P p = __builtin_bit_cast(P, x);
    if (sixteen) {
        auto a = __builtin_amdgcn_permlane16_swap(p.lo, p.lo, false, false);
        auto b = __builtin_amdgcn_permlane16_swap(p.hi, p.hi, false, false);
        P d0 = {(int)a[0], (int)b[0]}, d1 = {(int)a[1], (int)b[1]};
        return __builtin_bit_cast(double, d0) + __builtin_bit_cast(double, d1);
    } else {
        auto a = __builtin_amdgcn_permlane32_swap(p.lo, p.lo, false, false);
        auto b = __builtin_amdgcn_permlane32_swap(p.hi, p.hi, false, false);
        P d0 = {(int)a[0], (int)b[0]}, d1 = {(int)a[1], (int)b[1]};
        return __builtin_bit_cast(double, d0) + __builtin_bit_cast(double, d1);
    }
}
__device__ __forceinline__ float swapsum(float x, bool sixteen) {
    int v = __builtin_bit_cast(int, x);
    auto a = sixteen ? __builtin_amdgcn_permlane16_swap(v, v, false, false)
                     : __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return __builtin_bit_cast(float, (int)a[0]) + __builtin_bit_cast(float, (int)a[1]);
}
// Sum over the 4 lanes {l%16 + 16k}; all four get the same bits.
template <typename T>
__device__ __forceinline__ T sum4(T x) {
    return swapsum(swapsum(x, true), false);
}
// Value of lane J of this lane's 16-lane row.
template <int J>
__device__ __forceinline__ double bcast16(double x) {
    long long v = __builtin_bit_cast(long long, x);
    v = __builtin_amdgcn_update_dpp(0ll, v, 0x150 + J, 0xF, 0xF, false);
    return __builtin_bit_cast(double, v);
}
template <int J>
__device__ __forceinline__ float bcast16(float x) {
    int v = __builtin_bit_cast(int, x);
    v = __builtin_amdgcn_update_dpp(0, v, 0x150 + J, 0xF, 0xF, false);
    return __builtin_bit_cast(float, v);
}

// Runtime-index form; folds to one DPP instruction once the column loop is unrolled.
template <typename T>
__device__ __forceinline__ T bcast16r(T x, int j) {
    switch (j) {
        case 0: return bcast16<0>(x);
        case 1: return bcast16<1>(x);
        case 2: return bcast16<2>(x);
        case 3: return bcast16<3>(x);
        case 4: return bcast16<4>(x);
        case 5: return bcast16<5>(x);
        case 6: return bcast16<6>(x);
        case 7: return bcast16<7>(x);
        case 8: return bcast16<8>(x);
        case 9: return bcast16<9>(x);
        case 10: return bcast16<10>(x);
        case 11: return bcast16<11>(x);
        case 12: return bcast16<12>(x);
        case 13: return bcast16<13>(x);
        case 14: return bcast16<14>(x);
        default: return bcast16<15>(x);
    }
}

template <typename T, int NC, int NW>
__device__ __forceinline__ T& TM(FSmem<T, NC, NW>& sm, int i, int j) { return sm.RG[i][j]; }
template <typename T, int NC, int NW>
__device__ __forceinline__ T& RM(FSmem<T, NC, NW>& sm, int i, int j) { return sm.RG[j + 1][i]; }

// T12 = -T11 P12 T22 for diagonal blocks of size s in [slo, shi), over the
// columns [base, base + span) of RG (upper triangle: Gram entries -> T).
template <typename T, int NC, int NW>
__device__ __forceinline__ void t_levels(FSmem<T, NC, NW>& sm, int slo, int shi, int base, int span) {
    constexpr int NT = 64 * NW;
    const int tid = threadIdx.x;
    for (int s = slo; s < shi && s < span; s *= 2) {
        const int npairs = span / (2 * s);
        const int ss = s * s;
        for (int e = tid; e < npairs * ss; e += NT) {
            const int pr = e / ss, rem = e - pr * ss, i = rem / s, jj = rem - i * s;
            const int o = base + 2 * s * pr;
            T a = T(0);
            for (int l = 0; l <= jj; ++l) a = fma(sm.RG[o + i][o + s + l], sm.RG[o + s + l][o + s + jj], a);
            sm.u.tmp[e] = a;
        }
        __syncthreads();
        for (int e = tid; e < npairs * ss; e += NT) {
            const int pr = e / ss, rem = e - pr * ss, i = rem / s, jj = rem - i * s;
            const int o = base + 2 * s * pr;
            T a = T(0);
            for (int l = i; l < s; ++l) a = fma(sm.RG[o + i][o + l], sm.u.tmp[pr * ss + l * s + jj], a);
            sm.RG[o + i][o + s + jj] = -a;
        }
        __syncthreads();
    }
}

// Householder reflector entry masks for the first block of a chain: in rows
// r < n of that block the reflector of column c is 0 above row c and 1 on it.
template <typename T>
__device__ __forceinline__ T vmask(T x, int r, int c) {
    return (r > c) ? x : ((r == c) ? T(1) : T(0));
}

// Householder scalars from alpha and sigma^2 = ||tail||^2 (sigma^2 > 0):
// nrm = sqrt(alpha^2 + sigma^2), beta = -sign(alpha) nrm (sign(0) = +1),
// tau = (beta - alpha)/beta = 1 + |alpha|/nrm, scale = 1/(alpha - beta).
// Hardware reciprocal / reciprocal square root refined by Newton steps.
__device__ __forceinline__ void hh_scalars(double alpha, double sigma2, double& beta, double& tau, double& scale) {
    const double s = fma(alpha, alpha, sigma2);
    double y = __builtin_amdgcn_rsq(s);
    double e = fma(-s * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-s * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    double nrm = s * y;
    nrm = fma(fma(-nrm, nrm, s), 0.5 * y, nrm);
    const double aa = fabs(alpha);
    beta = (alpha >= 0.0) ? -nrm : nrm;
    tau = fma(aa, y, 1.0);
    const double d = aa + nrm;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    scale = (alpha >= 0.0) ? r : -r;
}
__device__ __forceinline__ void hh_scalars(float alpha, float sigma2, float& beta, float& tau, float& scale) {
    const float s = fmaf(alpha, alpha, sigma2);
    float y = __builtin_amdgcn_rsqf(s);
    y = fmaf(0.5f * y, fmaf(-s * y, y, 1.0f), y);
    float nrm = s * y;
    nrm = fmaf(fmaf(-nrm, nrm, s), 0.5f * y, nrm);
    const float aa = fabsf(alpha);
    beta = (alpha >= 0.0f) ? -nrm : nrm;
    tau = fmaf(aa, y, 1.0f);
    const float d = aa + nrm;
    float r = __builtin_amdgcn_rcpf(d);
    r = fmaf(r, fmaf(-d, r, 1.0f), r);
    scale = (alpha >= 0.0f) ? r : -r;
}

// Factor one block held in registers (see the file comment).  TILE: first
// block of a chain (heads inside the tile); otherwise heads are the on-chip R.
template <typename T, int NC, int NW, int SG, bool TILE>
__device__ __forceinline__ void factor_block(T (&x)[SG][4][(NC < 16 ? 16 : NC) / 16], FSmem<T, NC, NW>& sm,
                                             int n) {
    typedef Mfma<T> M;
    typedef typename M::acc acc_t;
    constexpr int NCP = NC < 16 ? 16 : NC;
    constexpr int NP = NCP / 16;
    constexpr int NT = 64 * NW;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int rbase = wv * 16 * SG;

    for (int p = 0; p < NP; ++p) {
        const int c0 = 16 * p;
        if (c0 >= n) break;
        const int c = c0 + l16;
        T xp[SG][4];
#pragma unroll
        for (int q = 0; q < NP; ++q)
            if (q == p) {
#pragma unroll
                for (int s = 0; s < SG; ++s)
#pragma unroll
                    for (int i = 0; i < 4; ++i) xp[s][i] = x[s][i][q];
            }
        // ------------------------------------------------ panel: column by column
        // One reduction per column: g_c = sum over the tail rows of x_j * x_c
        // for every panel column c (g_j = sigma^2).  With v = head + scale*x_j
        // (tail), v^T x_c = head_c + scale * g_c, so the Householder scalars
        // and the update coefficients follow from the same sums.
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int j = c0 + jj;
            if (j >= n) break;
            __builtin_amdgcn_sched_barrier(0);
            const int buf = jj & 1;
            T a = T(0);
#pragma unroll
            for (int s = 0; s < SG; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = rbase + 16 * s + M::orow(l4, i);
                    const T xv = xp[s][i];
                    const T xj = bcast16r(xv, jj);
                    a = fma((!TILE || r > j) ? xj : T(0), xv, a);
                    if (TILE && r == j) sm.hrow[buf][l16] = xv;
                }
            a = sum4(a);
            if (l4 == 0) sm.redw[buf][wv][l16] = a;
            T rhead = T(0), alpha_r = T(0);
            if (!TILE) {
                alpha_r = RM(sm, j, j);
                if (c > j && c < n) rhead = RM(sm, j, c);
            }
            __syncthreads();
            T g = T(0), sigma2 = T(0);
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                g += sm.redw[buf][ww][l16];
                sigma2 += sm.redw[buf][ww][jj];
            }
            const T alpha = TILE ? sm.hrow[buf][jj] : alpha_r;
            const T headc = TILE ? sm.hrow[buf][l16] : rhead;
            T beta, tau, scale;
            if (sigma2 == T(0)) {
                tau = T(0);
                beta = alpha;
                scale = T(0);
            } else {
                hh_scalars(alpha, sigma2, beta, tau, scale);
            }
            const T w = fma(scale, g, headc);
            const T tw = (c > j && c < n) ? tau * w : T(0);
#pragma unroll
            for (int s = 0; s < SG; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = rbase + 16 * s + M::orow(l4, i);
                    const T xv = xp[s][i];
                    T vb = bcast16r(xv, jj) * scale;
                    if (TILE) vb = (r < j) ? T(0) : ((r == j) ? T(1) : vb);
                    T nx = fma(-vb, tw, xv);
                    if (l16 == jj) {
                        if (!TILE || r > j) nx = vb;
                        else if (r == j) nx = beta;
                    }
                    xp[s][i] = nx;
                }
            if (wv == 0 && l4 == 0) {
                if (c < j) TM(sm, c, j) = w;
                if (!TILE) {
                    if (c > j && c < n) RM(sm, j, c) = fma(-tau, w, rhead);
                    else if (c == j) RM(sm, j, j) = beta;
                }
                if (l16 == 0) sm.tau[j] = tau;
            }
        }
#pragma unroll
        for (int q = 0; q < NP; ++q)
            if (q == p) {
#pragma unroll
                for (int s = 0; s < SG; ++s)
#pragma unroll
                    for (int i = 0; i < 4; ++i) x[s][i][q] = xp[s][i];
            }
        // V_p as an MFMA operand (unit heads / zeros above in the first block)
#pragma unroll
        for (int s = 0; s < SG; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = rbase + 16 * s + M::orow(l4, i);
                xp[s][i] = (c < n) ? (TILE ? vmask(xp[s][i], r, c) : xp[s][i]) : T(0);
            }
        __syncthreads();
        // T of the panel: diagonal 16 x 16 block of the block's T
        for (int i = tid; i < 16; i += NT) TM(sm, c0 + i, c0 + i) = (c0 + i < n) ? sm.tau[c0 + i] : T(0);
        __syncthreads();
        t_levels(sm, 1, 16, c0, 16);

        // ------------------------------------------------ V_p^T X over all other column tiles
        acc_t acc[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) acc[q] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            if (q == p || 16 * q >= n) continue;
#pragma unroll
            for (int s = 0; s < SG; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = rbase + 16 * s + M::orow(l4, i);
                    T b = x[s][i][q];
                    if (TILE && q < p) b = vmask(b, r, 16 * q + l16);
                    acc[q] = M::mma(xp[s][i], b, acc[q]);
                }
        }
#pragma unroll
        for (int q = 0; q < NP; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.u.Wpart[wv][M::orow(l4, r)][16 * q + l16] = acc[q][r];
        __syncthreads();
        for (int e = tid; e < 16 * NCP; e += NT) {
            const int r = e / NCP, cc = e - r * NCP;
            T sum = T(0);
#pragma unroll
            for (int w = 0; w < NW; ++w) sum += sm.u.Wpart[w][r][cc];
            const bool valid = (c0 + r < n) && (cc < n);
            if (cc < c0) {
                if (valid) TM(sm, cc, c0 + r) = sum;  // Gram block V_q^T V_p
                sm.u.Wpart[0][r][cc] = T(0);
            } else if (cc < c0 + 16 || !valid) {
                sm.u.Wpart[0][r][cc] = T(0);
            } else {
                if (!TILE) sum += RM(sm, c0 + r, cc);
                sm.u.Wpart[0][r][cc] = sum;
            }
        }
        __syncthreads();
        // W' = T_pp^T W (16 x trailing columns)
        for (int e = tid; e < 16 * NCP; e += NT) {
            const int r = e / NCP, cc = e - r * NCP;
            T a = T(0);
            if (cc >= c0 + 16) {
                for (int l = 0; l <= r; ++l) a = fma(sm.RG[c0 + l][c0 + r], sm.u.Wpart[0][l][cc], a);
            }
            sm.Wp[r][cc] = a;
        }
        __syncthreads();
        if (!TILE) {
            for (int e = tid; e < 16 * NCP; e += NT) {
                const int r = e / NCP, cc = e - r * NCP;
                if (cc >= c0 + 16 && cc < n && c0 + r < n) RM(sm, c0 + r, cc) -= sm.Wp[r][cc];
            }
        }
        // X -= V_p W' on the trailing column tiles
        if (p + 1 < NP && c0 + 16 < n) {
#pragma unroll
            for (int s = 0; s < SG; ++s) {
#pragma unroll
                for (int i = 0; i < 4; ++i) sm.u.trans[wv][M::orow(l4, i)][l16] = xp[s][i];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                T a4[4];
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) a4[q4] = sm.u.trans[wv][l16][4 * q4 + l4];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    if (q <= p) continue;
                    acc_t u = acc_t{0, 0, 0, 0};
#pragma unroll
                    for (int q4 = 0; q4 < 4; ++q4) u = M::mma(a4[q4], sm.Wp[4 * q4 + l4][16 * q + l16], u);
#pragma unroll
                    for (int i = 0; i < 4; ++i) x[s][i][q] -= u[i];
                }
            }
        }
        __syncthreads();
    }
}

template <typename T, int NC, int NW>
__device__ __forceinline__ void smem_init(FSmem<T, NC, NW>& sm) {
    constexpr int NCP = NC < 16 ? 16 : NC;
    T* p = &sm.RG[0][0];
    for (int e = threadIdx.x; e < (NCP + 1) * (NCP + 1); e += 64 * NW) p[e] = T(0);
    __syncthreads();
}

// Full block T (levels of size >= 16) and the stores of T (packed) and tau.
template <typename T, int NC, int NW>
__device__ __forceinline__ void finish_T(FSmem<T, NC, NW>& sm, int n, T* __restrict__ Tout, T* __restrict__ tauout) {
    constexpr int NCP = NC < 16 ? 16 : NC;
    __syncthreads();
    t_levels(sm, 16, NCP, 0, NCP);
    for (int e = threadIdx.x; e < n * n; e += 64 * NW) {
        const int i = e / n, j = e - i * n;
        if (i <= j) Tout[j * (j + 1) / 2 + i] = sm.RG[i][j];
    }
    for (int i = threadIdx.x; i < n; i += 64 * NW) tauout[i] = sm.tau[i];
    __syncthreads();
}

template <typename T, int NC, int NW, int SG>
__device__ __forceinline__ void load_tile(T (&x)[SG][4][(NC < 16 ? 16 : NC) / 16], const T* __restrict__ A,
                                          int64_t lda, int64_t r0, int rows, int n) {
    typedef Mfma<T> M;
    constexpr int NP = (NC < 16 ? 16 : NC) / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, l16 = lane & 15, l4 = lane >> 4;
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = wv * 16 * SG + 16 * s + M::orow(l4, i);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int cc = 16 * p + l16;
                x[s][i][p] = (r < rows && cc < n) ? A[(r0 + r) * lda + cc] : T(0);
            }
        }
}

template <typename T, int NC, int NW, int SG>
__device__ __forceinline__ void store_tile(const T (&x)[SG][4][(NC < 16 ? 16 : NC) / 16], T* __restrict__ A,
                                           int64_t lda, int64_t r0, int rows, int n) {
    typedef Mfma<T> M;
    constexpr int NP = (NC < 16 ? 16 : NC) / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, l16 = lane & 15, l4 = lane >> 4;
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = wv * 16 * SG + 16 * s + M::orow(l4, i);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int cc = 16 * p + l16;
                if (r < rows && cc < n) A[(r0 + r) * lda + cc] = x[s][i][p];
            }
        }
}


template <int NC>
struct CombineShape {
    static constexpr int NCP = NC < 16 ? 16 : NC;
    static constexpr int NW = NCP / 16;  // one 16-row group per wave
    static constexpr int SG = 1;
};

// Flat tree of one chain (sequential TSQR, Sec. 2.1): block 0 plain, every
// later block stacked under the on-chip R.  Writes reflectors over A, the
// per-block T and tau, and the chain's R into Rbuf[c].
template <typename T, int NC, int NW, int SG>
__device__ __forceinline__ void chain_body(FSmem<T, NC, NW>& sm, const Geom& g, T* __restrict__ A, int64_t lda,
                                           T* __restrict__ tau_blk, T* __restrict__ T_blk, T* __restrict__ Rbuf,
                                           int c) {
    typedef Mfma<T> M;
    constexpr int NP = (NC < 16 ? 16 : NC) / 16;
    constexpr int ROWS = NW * 16 * SG;
    const int n = (int)g.n;
    const int tri = n * (n + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    smem_init(sm);
    const int64_t start = chain_start(g, c), end = chain_end(g, c);
    const int nb = chain_nblocks(g, c);
    const int64_t blk0 = chain_blk0(g, c);
    for (int b = 0; b < nb; ++b) {
        const int64_t r0 = start + (int64_t)b * ROWS;
        const int rows = (int)((end - r0) < ROWS ? (end - r0) : ROWS);
        T x[SG][4][NP];
        load_tile<T, NC, NW, SG>(x, A, lda, r0, rows, n);
        if (b == 0) {
            factor_block<T, NC, NW, SG, true>(x, sm, n);
#pragma unroll
            for (int s = 0; s < SG; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = wv * 16 * SG + 16 * s + M::orow(l4, i);
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        const int cc = 16 * p + l16;
                        if (r < n && cc >= r && cc < n) RM(sm, r, cc) = x[s][i][p];
                    }
                }
        } else {
            factor_block<T, NC, NW, SG, false>(x, sm, n);
        }
        store_tile<T, NC, NW, SG>(x, A, lda, r0, rows, n);
        finish_T(sm, n, T_blk + (blk0 + b) * tri, tau_blk + (blk0 + b) * n);
    }
    T* Rc = Rbuf + (int64_t)c * n * n;
    for (int e = tid; e < n * n; e += 64 * NW) {
        const int i = e / n, j = e - i * n;
        Rc[e] = (j >= i) ? RM(sm, i, j) : T(0);
    }
}

// One tree node (Sec. 2.1): fold the R factors of children
// i0 + t*stride (t = 1..arity-1, those below W) into Rbuf[i0], one
// stacked-triangle QR per child; the child's reflectors, T and tau go to
// its node slot.
template <typename T, int NC, int NW, int SG>
__device__ __forceinline__ void combine_body(FSmem<T, NC, NW>& sm, const Geom& g, T* __restrict__ Rbuf, int64_t i0,
                                             int64_t stride, int arity, T* __restrict__ Ynode,
                                             T* __restrict__ Tnode, T* __restrict__ tau_node) {
    constexpr int NP = (NC < 16 ? 16 : NC) / 16;
    const int n = (int)g.n;
    const int tri = n * (n + 1) / 2;
    const int tid = threadIdx.x;
    smem_init(sm);
    const T* Ra = Rbuf + i0 * n * n;
    for (int e = tid; e < n * n; e += 64 * NW) {
        const int i = e / n, j = e - i * n;
        if (j >= i) RM(sm, i, j) = Ra[e];
    }
    __syncthreads();
    for (int t1 = 1; t1 < arity; ++t1) {
        const int64_t c = i0 + t1 * stride;
        if (c >= g.W) break;
        T x[SG][4][NP];
        load_tile<T, NC, NW, SG>(x, Rbuf + c * n * n, n, 0, n, n);
        factor_block<T, NC, NW, SG, false>(x, sm, n);
        store_tile<T, NC, NW, SG>(x, Ynode + c * n * n, n, 0, n, n);
        finish_T(sm, n, Tnode + c * tri, tau_node + c * n);
    }
    T* Rw = Rbuf + i0 * n * n;
    for (int e = tid; e < n * n; e += 64 * NW) {
        const int i = e / n, j = e - i * n;
        Rw[e] = (j >= i) ? RM(sm, i, j) : T(0);
    }
}

}  // namespace tsqr
