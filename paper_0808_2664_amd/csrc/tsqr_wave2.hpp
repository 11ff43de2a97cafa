// Two-wave chain engine of the factor kernel (gfx950, wave64), for n > 32.
//
// The chain (the flat tree of sequential TSQR, Sec. 2.1) is reduced by one
// workgroup of two waves that split the columns: wave A owns column tiles 0
// and 1 (columns 0..31), wave B tiles 2 and 3 (columns 32..63).  In a block
// stacked under the chain's R, the reflector of column j acts on R's row j
// and on the block's rows only, so the entries of R in a column are touched
// only by the reflectors of that column's panel and of earlier panels
// applied to that column: each wave owns R's entries in its own columns,
// and the only data that passes between the waves is wave A's reflectors
// of panels 0 and 1 (their tails, stored to HBM as the factor's output
// anyway) and the two diagonal blocks of T.  So wave A runs ahead: per block
// it factors panels 0 and 1 and publishes them, then goes on to the next
// block; wave B applies panels 0 and 1 of that block to its columns, then
// factors panels 2 and 3.  Two independent instruction streams share each
// SIMD (two waves per SIMD), where the one-wave engine (tsqr_wave.hpp) runs
// one latency-bound column sweep at a time.
//
// Wave B carries five of the six block-reflector updates of a block, wave A
// one, so with the implicit Q kept the off-diagonal blocks of T (Gram blocks
// V_a^T V_c and the T recurrence) go to wave A: once wave B has published a
// block (its reflectors in HBM, its diagonal T blocks in LDS), wave A forms
// that block's off-diagonal T blocks between two blocks of its own.
//
// Every step is the arithmetic of the one-wave engine on a column subset:
// the same reflectors (Sec. 5.2 convention), the same compact form
// I - V T V^T per block (T upper triangular, forward product), the same
// panel-of-16 sweep with one lane reduction per column.  The R of the chain
// is published at the end for the tree, which runs in a second launch.
#pragma once
#include "tsqr_wave.hpp"

namespace tsqr {

constexpr int kW2Ring = 2;  // blocks wave A may run ahead of wave B

template <typename T>
struct W2Smem {
    static constexpr int NCP = 64;
    static constexpr int RP = 64 * 65 / 2;
    T R[RP];                     // the chain's R (packed by rows); columns 0..31 wave A's, 32..63 wave B's
    T scr[2][16][17];            // per-wave transposes and the sweep's staging target
    T tdA[kW2Ring][2][16][17];   // wave A's diagonal T blocks (panels 0, 1), one slot per block in flight
    T tdB[kW2Ring][2][16][17];   // wave B's diagonal T blocks (panels 2, 3), one slot per block in flight
                                 // (entries below the diagonals stay zero)
    T scl[2][16];                // per-wave scales of the current panel's columns
    T zero;                      // holds 0
    int ready;                   // blocks whose panels 0 and 1 wave A has published
    int used;                    // blocks whose slot wave B has released (R only)
    int swept;                   // blocks wave B has published (implicit Q kept)
};

// LDS flag helpers (workgroup scope).
__device__ __forceinline__ int lds_load_acq(const int* p) {
    const int v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return v;
}
__device__ __forceinline__ void lds_store_rel(int* p, int v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Wait until *p >= v (the other wave of this workgroup is resident and
// never waits on this one for the value it is to write).
__device__ __forceinline__ void lds_wait_ge(const int* p, int v) {
    while (__builtin_amdgcn_readfirstlane(lds_load_acq(p)) < v) __builtin_amdgcn_s_sleep(1);
}

// ---- tile I/O: column tile p (columns 16p..16p+15) of a block of `rows`
// rows at row r0, in the tile layout (lane: column 16p + l16, rows
// 16s + orow(l4, i)); entries past the block's rows or past column n are
// zero on load and not written on store.
template <typename T, int SG, int p>
__device__ __forceinline__ void v_load_tile(T (&v)[SG][4], const T* __restrict__ A, int64_t lda, int64_t r0, int rows,
                                            int n) {
    typedef Mfma<T> M;
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    const int cc = 16 * p + l16;
    if (rows == 16 * SG && cc < n) {
        const T* __restrict__ pb = A + (r0 + M::orow(l4, 0)) * lda + cc;
#pragma unroll
        for (int s = 0; s < SG; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) v[s][i] = pb[(int64_t)(16 * s + M::orow(0, i) - M::orow(0, 0)) * lda];
        return;
    }
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * s + M::orow(l4, i);
            v[s][i] = (r < rows && cc < n) ? A[(r0 + r) * lda + cc] : T(0);
        }
}
// This wave's two tiles P0 and P0 + 1.
template <typename T, int SG, int P0>
__device__ __forceinline__ void x_load_tiles(T (&x)[SG][4][2], const T* __restrict__ A, int64_t lda, int64_t r0,
                                             int rows, int n) {
    T v0[SG][4], v1[SG][4];
    v_load_tile<T, SG, P0>(v0, A, lda, r0, rows, n);
    v_load_tile<T, SG, P0 + 1>(v1, A, lda, r0, rows, n);
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            x[s][i][0] = v0[s][i];
            x[s][i][1] = v1[s][i];
        }
}
template <typename T, int SG, int P0, int t>
__device__ __forceinline__ void x_store_tile(const T (&x)[SG][4][2], T* __restrict__ A, int64_t lda, int64_t r0,
                                             int rows, int n) {
    typedef Mfma<T> M;
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    const int cc = 16 * (P0 + t) + l16;
    if (cc >= n) return;
    if (rows == 16 * SG) {
        T* __restrict__ pb = A + (r0 + M::orow(l4, 0)) * lda + cc;
#pragma unroll
        for (int s = 0; s < SG; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) pb[(int64_t)(16 * s + M::orow(0, i) - M::orow(0, 0)) * lda] = x[s][i][t];
        return;
    }
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * s + M::orow(l4, i);
            if (r < rows) A[(r0 + r) * lda + cc] = x[s][i][t];
        }
}

// Panel p (global index; tile p - P0 of this wave's two tiles x[.][.][0..1])
// of one block: the column sweep, the delayed scaling of the reflector tails,
// tau, and the panel's diagonal T block (into td and, with WQ, into Tout).
// MODE 0: the chain's first block (heads inside the tile); MODE 1: a block
// stacked under the on-chip R.
template <typename T, int SG, int MODE, bool WQ, int P0, int p>
__device__ __forceinline__ void w2_sweep(T (&x)[SG][4][2], W2Smem<T>& sm, T (&scr)[16][17], T (&td)[16][17],
                                         T (&scl)[16], const int n_, T* __restrict__ Tout, T* __restrict__ tauout) {
    typedef Mfma<T> M;
    constexpr int c0 = 16 * p;
    sweep_panel<T, W2Smem<T>::NCP, MODE, SG, 2, p - P0, p, SG>(x, sm.R, td, &scr[0][0], scl, &sm.zero, n_);
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    const int c = c0 + l16;
    const int n = opaque_s(n_);
    wave_sync();
    if (WQ && l4 == 0 && c < n) tauout[c] = td[l16][l16];
    if constexpr (WQ) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = c0 + M::orow(l4, r);
            if (i <= c && c < n) Tout[tpi(i, c)] = td[M::orow(l4, r)][l16];
        }
    }
}

// Apply panel p's block reflector (tails v in the tile layout, the panel's
// diagonal T block td) to this wave's tiles q in [Q0, P0 + 2):
// W = V^T X (+ R's rows of panel p in MODE 1), W' = T^T W, R rows -= W',
// X -= V W'.  In MODE 0 the heads lie inside v (masked here to the unit
// lower trapezoid) and R's rows are rows of the tile.
template <typename T, int SG, int MODE, int P0, int p, int Q0>
__device__ __forceinline__ void w2_apply(T (&x)[SG][4][2], const T (&v)[SG][4], W2Smem<T>& sm, T (&scr)[16][17],
                                         const T (&td)[16][17], const int n_) {
    typedef Mfma<T> M;
    typedef typename M::acc acc_t;
    constexpr int NCP = 64;
    constexpr int c0 = 16 * p;
    constexpr int S0 = (MODE == 0) ? p : 0;
    constexpr int Q1 = P0 + 2;
    const int n = opaque_s(n_);
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    acc_t w0[2];
    sfor<Q0, Q1>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        w0[q - P0] = acc_t{0, 0, 0, 0};
        if constexpr (MODE != 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = c0 + M::orow(l4, r), cc = 16 * q + l16;
                const T rv = sm.R[rpi<NCP>(i, cc)];
                w0[q - P0][r] = (i < n && cc < n) ? rv : T(0);
            }
        }
    });
    sfor<S0, SG>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            T a = v[s][i];
            if constexpr (MODE == 0 && s == p) a = vmask(a, M::orow(l4, i), l16);
            sfor<Q0, Q1>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                w0[q - P0] = M::mma(a, x[s][i][q - P0], w0[q - P0]);
            });
        }
    });
    // -W' = -T^T W
    T ntpp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) ntpp[r] = -td[M::orow(l4, r)][l16];
    acc_t nw[2];
    sfor<Q0, Q1>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        nw[q - P0] = acc_t{0, 0, 0, 0};
    });
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
        sfor<Q0, Q1>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            nw[q - P0] = M::mma(ntpp[kc], w0[q - P0][kc], nw[q - P0]);
        });
    }
    if constexpr (MODE != 0) {
        sfor<Q0, Q1>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = c0 + M::orow(l4, r), cc = 16 * q + l16;
                if (i < n && cc < n) sm.R[rpi<NCP>(i, cc)] += nw[q - P0][r];
            }
        });
    }
    // X -= V W'
    sfor<S0, SG>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            T a = v[s][i];
            if constexpr (MODE == 0 && s == p) a = vmask(a, M::orow(l4, i), l16);
            scr[M::orow(l4, i)][l16] = a;
        }
        wave_sync();
        T vt[4];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) vt[kc] = scr[l16][M::orow(l4, kc)];
        wave_sync();
        acc_t u[2];
        sfor<Q0, Q1>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            u[q - P0] = acc_t{x[s][0][q - P0], x[s][1][q - P0], x[s][2][q - P0], x[s][3][q - P0]};
        });
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            sfor<Q0, Q1>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                u[q - P0] = M::mma(vt[kc], nw[q - P0][kc], u[q - P0]);
            });
        }
        sfor<Q0, Q1>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
#pragma unroll
            for (int r = 0; r < 4; ++r) x[s][r][q - P0] = u[q - P0][r];
        });
    });
}

// MODE 0: rows of row group g of the block are rows of R; once final, this
// wave's entries of them (its columns >= the row) go to the on-chip R.
template <typename T, int SG, int P0, int g>
__device__ __forceinline__ void w2_rows_to_r(const T (&x)[SG][4][2], W2Smem<T>& sm, const int n_) {
    typedef Mfma<T> M;
    constexpr int NCP = 64;
    const int n = opaque_s(n_);
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 16 * g + M::orow(l4, i);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int cc = 16 * (P0 + t) + l16;
            if (r < n && cc >= r && cc < n) sm.R[rpi<NCP>(r, cc)] = x[g][i][t];
        }
    }
}

// Gram block P = V_a^T V_c of two reflector tiles (a < c, both in the tile
// layout) in the A-operand layout; rows where V_c vanishes (above panel c's
// heads in the first block) are skipped and V_c's heads masked.
template <typename T, int SG, int MODE, int c>
__device__ __forceinline__ typename Mfma<T>::acc w2_gram(const T (&va)[SG][4], const T (&vc)[SG][4]) {
    typedef Mfma<T> M;
    typedef typename M::acc acc_t;
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    acc_t P = acc_t{0, 0, 0, 0};
    sfor<(MODE == 0 ? c : 0), SG>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            T b = vc[s][i];
            if constexpr (MODE == 0 && s == c) b = vmask(b, M::orow(l4, i), l16);
            P = M::mma(b, va[s][i], P);
        }
    });
    return P;
}

// The two diagonal T blocks a (D and A operand layouts) of a 16 x 17 LDS block.
template <typename T>
__device__ __forceinline__ void w2_tblock(const T (&td)[16][17], T (&tD)[4], T (&tA)[4]) {
    typedef Mfma<T> M;
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        tD[r] = td[M::orow(l4, r)][l16];
        tA[r] = td[l16][M::orow(l4, r)];
    }
}

// T_ab = -T_aa * Y, Y = sum_c P_ac T_cb (all 16 x 16, P in A layout, the
// T_cb in D layout); returns T_ab in D layout.
template <typename T>
__device__ __forceinline__ typename Mfma<T>::acc w2_tnext(const T (&tAaa)[4], typename Mfma<T>::acc y) {
    typedef Mfma<T> M;
    typedef typename M::acc acc_t;
    acc_t t = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) t = M::mma(tAaa[kc], y[kc], t);
    return -t;
}

template <typename T>
__device__ __forceinline__ void w2_tstore(T* __restrict__ Tout, int a, int b, const typename Mfma<T>::acc& t, int n) {
    typedef Mfma<T> M;
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    const int jx = 16 * b + l16;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (jx < n) Tout[tpi(16 * a + M::orow(l4, r), jx)] = t[r];
}

// Off-diagonal blocks of one block's T (wave A, after wave B published the
// block): T_ab = -T_aa sum_{c=a+1..b} P_ac T_cb for b = 1..3, a = b-1..0,
// with the Gram blocks P_ac = V_a^T V_c of the four reflector tiles read back
// from HBM and the diagonal blocks from the block's LDS slot.
template <typename T, int SG, int MODE>
__device__ __forceinline__ void w2_tblocks(W2Smem<T>& sm, const T* __restrict__ A, int64_t lda, int64_t r0, int rows,
                                           int n, int slot, T* __restrict__ Tout) {
    typedef Mfma<T> M;
    typedef typename M::acc acc_t;
    acc_t P01, P02, P03, P12, P13, P23;
    {
        T v2[SG][4], v3[SG][4];
        v_load_tile<T, SG, 2>(v2, A, lda, r0, rows, n);
        v_load_tile<T, SG, 3>(v3, A, lda, r0, rows, n);
        P23 = w2_gram<T, SG, MODE, 3>(v2, v3);
        T v0[SG][4];
        v_load_tile<T, SG, 0>(v0, A, lda, r0, rows, n);
        P02 = w2_gram<T, SG, MODE, 2>(v0, v2);
        P03 = w2_gram<T, SG, MODE, 3>(v0, v3);
        T v1[SG][4];
        v_load_tile<T, SG, 1>(v1, A, lda, r0, rows, n);
        P01 = w2_gram<T, SG, MODE, 1>(v0, v1);
        P12 = w2_gram<T, SG, MODE, 2>(v1, v2);
        P13 = w2_gram<T, SG, MODE, 3>(v1, v3);
    }
    T tD0[4], tA0[4], tD1[4], tA1[4], tD2[4], tA2[4], tD3[4], tA3[4];
    w2_tblock<T>(sm.tdA[slot][0], tD0, tA0);
    w2_tblock<T>(sm.tdA[slot][1], tD1, tA1);
    w2_tblock<T>(sm.tdB[slot][0], tD2, tA2);
    w2_tblock<T>(sm.tdB[slot][1], tD3, tA3);
    (void)tD0;
    (void)tA3;
    // column block 1
    acc_t y = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) y = M::mma(P01[kc], tD1[kc], y);
    const acc_t t01 = w2_tnext<T>(tA0, y);
    w2_tstore<T>(Tout, 0, 1, t01, n);
    // column block 2
    y = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) y = M::mma(P12[kc], tD2[kc], y);
    const acc_t t12 = w2_tnext<T>(tA1, y);
    y = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) y = M::mma(P01[kc], t12[kc], y);
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) y = M::mma(P02[kc], tD2[kc], y);
    const acc_t t02 = w2_tnext<T>(tA0, y);
    w2_tstore<T>(Tout, 1, 2, t12, n);
    w2_tstore<T>(Tout, 0, 2, t02, n);
    // column block 3
    y = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) y = M::mma(P23[kc], tD3[kc], y);
    const acc_t t23 = w2_tnext<T>(tA2, y);
    w2_tstore<T>(Tout, 2, 3, t23, n);
    y = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) y = M::mma(P12[kc], t23[kc], y);
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) y = M::mma(P13[kc], tD3[kc], y);
    const acc_t t13 = w2_tnext<T>(tA1, y);
    w2_tstore<T>(Tout, 1, 3, t13, n);
    y = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) y = M::mma(P01[kc], t13[kc], y);
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) y = M::mma(P02[kc], t23[kc], y);
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) y = M::mma(P03[kc], tD3[kc], y);
    const acc_t t03 = w2_tnext<T>(tA0, y);
    w2_tstore<T>(Tout, 0, 3, t03, n);
}

// One chain of the two-wave engine; the chain's R is left in sm.R (both
// waves' columns complete when this returns, after a workgroup barrier).
template <typename T, bool WQ>
__device__ __forceinline__ void w2_chain(W2Smem<T>& sm, const Geom& g, int ch, T* __restrict__ A, int64_t lda,
                                         T* __restrict__ tau_blk, T* __restrict__ T_blk) {
    typedef Mfma<T> M;
    typedef typename M::acc acc_t;
    constexpr int SG = 4, H = 64;
    const int n = (int)g.n;
    const int64_t tri = (int64_t)n * (n + 1) / 2;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = lane_id();
    for (int e = threadIdx.x; e < W2Smem<T>::RP; e += 128) sm.R[e] = T(0);
    for (int e = threadIdx.x; e < kW2Ring * 2 * 16 * 17; e += 128) {
        (&sm.tdA[0][0][0][0])[e] = T(0);
        (&sm.tdB[0][0][0][0])[e] = T(0);
    }
    if (threadIdx.x == 0) {
        sm.zero = T(0);
        sm.ready = 0;
        sm.used = 0;
        sm.swept = 0;
    }
    __syncthreads();
    const int64_t start = chain_start(g, ch), end = chain_end(g, ch);
    const int nb = chain_nblocks(g, ch);
    const int64_t blk0 = chain_blk0(g, ch);
    T x[SG][4][2];
    auto rows_of = [&](int b) {
        const int64_t r0 = start + (int64_t)b * H;
        return (int)((end - r0) < H ? (end - r0) : H);
    };
    if (wv == 0) {
        // ---------------------------------------------------------------- wave A
        x_load_tiles<T, SG, 0>(x, A, lda, start, rows_of(0), n);
        for (int b = 0; b < nb; ++b) {
            const int64_t r0 = start + (int64_t)b * H;
            const int rows = rows_of(b);
            const int slot = b % kW2Ring;
            T* Tout = T_blk + (blk0 + b) * tri;
            T* tauout = tau_blk + (blk0 + b) * n;
            // the slot's previous block must have been released by wave B (with
            // the implicit Q kept, wave A's wait for block b - 1 below implies it)
            if (!WQ && b >= kW2Ring) lds_wait_ge(&sm.used, b - kW2Ring + 1);
            auto blockA = [&](auto mc) {
                constexpr int MODE = decltype(mc)::value;
                w2_sweep<T, SG, MODE, WQ, 0, 0>(x, sm, sm.scr[0], sm.tdA[slot][0], sm.scl[0], n, Tout, tauout);
                x_store_tile<T, SG, 0, 0>(x, A, lda, r0, rows, n);
                {
                    T v0[SG][4];
#pragma unroll
                    for (int s = 0; s < SG; ++s)
#pragma unroll
                        for (int i = 0; i < 4; ++i) v0[s][i] = x[s][i][0];
                    w2_apply<T, SG, MODE, 0, 0, 1>(x, v0, sm, sm.scr[0], sm.tdA[slot][0], n);
                }
                if constexpr (MODE == 0) w2_rows_to_r<T, SG, 0, 0>(x, sm, n);
                if (16 < n) {
                    w2_sweep<T, SG, MODE, WQ, 0, 1>(x, sm, sm.scr[0], sm.tdA[slot][1], sm.scl[0], n, Tout, tauout);
                    if constexpr (MODE == 0) w2_rows_to_r<T, SG, 0, 1>(x, sm, n);
                } else {
                    // panel 1 lies beyond n: its diagonal T block is zero
                    for (int e = lane; e < 16 * 17; e += 64) (&sm.tdA[slot][1][0][0])[e] = T(0);
                    wave_sync();
                }
                x_store_tile<T, SG, 0, 1>(x, A, lda, r0, rows, n);
                // the tails are in HBM (L2) before wave B is told
                pub_wait();
                lds_store_rel(&sm.ready, b + 1);
            };
            if (b == 0) blockA(ic_t<0>{});
            else blockA(ic_t<1>{});
            if constexpr (WQ) {
                // the previous block's off-diagonal T blocks, once wave B has published it
                if (b >= 1) {
                    lds_wait_ge(&sm.swept, b);
                    const int pb = b - 1;
                    T* Tprev = T_blk + (blk0 + pb) * tri;
                    if (pb == 0) w2_tblocks<T, SG, 0>(sm, A, lda, r0 - H, rows_of(pb), n, pb % kW2Ring, Tprev);
                    else w2_tblocks<T, SG, 1>(sm, A, lda, r0 - H, rows_of(pb), n, pb % kW2Ring, Tprev);
                }
            }
            if (b + 1 < nb) x_load_tiles<T, SG, 0>(x, A, lda, r0 + H, rows_of(b + 1), n);
        }
        if (WQ && nb > 0) {
            lds_wait_ge(&sm.swept, nb);
            const int pb = nb - 1;
            T* Tprev = T_blk + (blk0 + pb) * tri;
            const int64_t rp = start + (int64_t)pb * H;
            if (pb == 0) w2_tblocks<T, SG, 0>(sm, A, lda, rp, rows_of(pb), n, pb % kW2Ring, Tprev);
            else w2_tblocks<T, SG, 1>(sm, A, lda, rp, rows_of(pb), n, pb % kW2Ring, Tprev);
        }
    } else {
        // ---------------------------------------------------------------- wave B
        x_load_tiles<T, SG, 2>(x, A, lda, start, rows_of(0), n);
        for (int b = 0; b < nb; ++b) {
            const int64_t r0 = start + (int64_t)b * H;
            const int rows = rows_of(b);
            const int slot = b % kW2Ring;
            T* Tout = T_blk + (blk0 + b) * tri;
            T* tauout = tau_blk + (blk0 + b) * n;
            lds_wait_ge(&sm.ready, b + 1);
            auto blockB = [&](auto mc) {
                constexpr int MODE = decltype(mc)::value;
                // panels 0 and 1 of this block (wave A's reflectors) on tiles 2, 3
                {
                    T v[SG][4];
                    v_load_tile<T, SG, 0>(v, A, lda, r0, rows, n);
                    w2_apply<T, SG, MODE, 2, 0, 2>(x, v, sm, sm.scr[1], sm.tdA[slot][0], n);
                    if constexpr (MODE == 0) w2_rows_to_r<T, SG, 2, 0>(x, sm, n);
                }
                if (16 < n) {
                    T v[SG][4];
                    v_load_tile<T, SG, 1>(v, A, lda, r0, rows, n);
                    w2_apply<T, SG, MODE, 2, 1, 2>(x, v, sm, sm.scr[1], sm.tdA[slot][1], n);
                    if constexpr (MODE == 0) w2_rows_to_r<T, SG, 2, 1>(x, sm, n);
                }
                wave_sync();
                // without an implicit Q the slot's T blocks are no longer read
                if constexpr (!WQ) lds_store_rel(&sm.used, b + 1);
                // panels 2 and 3 (columns beyond n are zero: no skip needed
                // past panel 2, which n > 32 reaches)
                w2_sweep<T, SG, MODE, WQ, 2, 2>(x, sm, sm.scr[1], sm.tdB[slot][0], sm.scl[1], n, Tout, tauout);
                x_store_tile<T, SG, 2, 0>(x, A, lda, r0, rows, n);
                {
                    T v2[SG][4];
#pragma unroll
                    for (int s = 0; s < SG; ++s)
#pragma unroll
                        for (int i = 0; i < 4; ++i) v2[s][i] = x[s][i][0];
                    w2_apply<T, SG, MODE, 2, 2, 3>(x, v2, sm, sm.scr[1], sm.tdB[slot][0], n);
                }
                if constexpr (MODE == 0) w2_rows_to_r<T, SG, 2, 2>(x, sm, n);
                if (48 < n) {
                    w2_sweep<T, SG, MODE, WQ, 2, 3>(x, sm, sm.scr[1], sm.tdB[slot][1], sm.scl[1], n, Tout, tauout);
                    if constexpr (MODE == 0) w2_rows_to_r<T, SG, 2, 3>(x, sm, n);
                } else {
                    for (int e = lane; e < 16 * 17; e += 64) (&sm.tdB[slot][1][0][0])[e] = T(0);
                    wave_sync();
                }
                x_store_tile<T, SG, 2, 1>(x, A, lda, r0, rows, n);
                if constexpr (WQ) {
                    // tails in HBM (L2), diagonal T blocks in LDS: wave A may form
                    // this block's off-diagonal T blocks
                    pub_wait();
                    lds_store_rel(&sm.swept, b + 1);
                }
            };
            if (b == 0) blockB(ic_t<0>{});
            else blockB(ic_t<1>{});
            if (b + 1 < nb) x_load_tiles<T, SG, 2>(x, A, lda, r0 + H, rows_of(b + 1), n);
        }
    }
    __syncthreads();
}

// The chain kernel of the two-wave engine: chain blockIdx.x, its reflectors
// (and tau, T with WQ) written, its packed R published to its slot of Rbuf
// (the layout the tree launch reads).
template <typename T, bool WQ>
__global__ __launch_bounds__(128, 2) void k_chain2(Geom g, T* __restrict__ A, int64_t lda, T* __restrict__ tau_blk,
                                                   T* __restrict__ T_blk, T* __restrict__ Rbuf) {
    __shared__ W2Smem<T> sm;
    const int ch = (int)blockIdx.x;
    w2_chain<T, WQ>(sm, g, ch, A, lda, tau_blk, T_blk);
    T* dst = Rbuf + (int64_t)ch * rslot<4>(g.n);
    for (int e = threadIdx.x; e < W2Smem<T>::RP; e += 128) dst[e] = sm.R[e];
}

}  // namespace tsqr
