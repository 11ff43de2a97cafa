// Application of the implicit "tree of Q factors" (paper Sec. 1 and 2.1):
// B <- Q^T B, B <- Q B and the explicit thin Q = Q [I_n; 0].
//
// Q = diag(Q_chain) * (tree steps), never multiplied out (Sec. 2.1, remark
// after Eq. TSQR_binarytree_4).  Every factor is a block reflector
// I - V T V^T (compact WY, Schreiber-Van Loan, Sec. 2.1 / Sec. 3.1):
//   * chain block 0: V = unit lower trapezoidal reflectors of the block;
//   * chain block b >= 1 and every tree step: V = [I_n ; Y] acting on the
//     carried n-row slab (the R rows) stacked over the block's rows.
// For a block with slab S and rows X (Q^T direction):
//     W = T^T (S + Y^T X),   S -= W,   X -= Y W.
// This is the per-row-block trailing update of CAQR (Sec. 3.1, "applied to
// their submatrices in an embarrassingly parallel fashion", then the tree
// pairs exchanging only b rows).  The two products are dense contractions
// and run on the MFMA units (v_mfma_f64_16x16x4 / v_mfma_f32_16x16x4);
// FP32 compute with FP64 storage is the mixed-precision CAQR update.
//
// Workgroup = 4 waves, each owning H/4 rows of the block; 16 columns of B per
// workgroup.  Workgroups are numbered so that all column tiles of one chain
// land on the same XCD (dispatch is round robin over the 8 XCDs), so the
// block's reflectors are fetched from HBM once and re-read from that XCD's L2.
#include "tsqr_common.hpp"

namespace tsqr {
using namespace dev;

template <typename S, typename C, int NC>
struct ApplySmem {
    static constexpr int NCP = NC < 16 ? 16 : NC;
    union U {
        C Wpart[4][NCP][16];
        C trans[4][16][17];
    } u;
    C Wp[NCP][17];
    S slab[NCP][16];
    C Tl[NCP * (NCP + 1) / 2 + 16];
};

// One block reflector applied to a (rows x 16) column tile.
//   Yg/ldy/yrow0: reflector rows of the block; Bg/ldb/brow0: the tile rows;
//   top: chain block 0 (unit lower trapezoid, no separate slab);
//   MODE_QT uses T^T, MODE_Q / MODE_FORMQ use T.  MODE_FORMQ treats the
//   input rows as zero (explicit Q of [I; 0]).
template <typename S, typename C, int NC, int H, int MODE>
__device__ __forceinline__ void apply_block(ApplySmem<S, C, NC>& sm, int n, const S* __restrict__ Yg, int64_t ldy,
                                            int64_t yrow0, S* __restrict__ Bg, int64_t ldb, int64_t brow0, int rows,
                                            int64_t col0, int64_t k, bool top, const S* __restrict__ Tpk) {
    typedef Mfma<C> M;
    typedef typename M::acc acc_t;
    constexpr int NCP = ApplySmem<S, C, NC>::NCP;
    constexpr int NP = NCP / 16;
    constexpr int RW = H / 4;
    constexpr int SG = RW / 16;
    static_assert(SG >= 1, "block height too small");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int l16 = lane & 15, l4 = lane >> 4;
    const int tri = n * (n + 1) / 2;

    for (int e = tid; e < tri; e += 256) sm.Tl[e] = (C)Tpk[e];

    C ynat[SG][4][NP];
    S bt[SG][4];
#pragma unroll
    for (int s = 0; s < SG; ++s) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = wv * RW + 16 * s + M::orow(l4, i);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int cc = 16 * p + l16;
                C yv = C(0);
                if (r < rows && cc < n) yv = (C)Yg[(yrow0 + r) * ldy + cc];
                if (top && r < n) yv = (cc < r) ? yv : (cc == r ? C(1) : C(0));
                ynat[s][i][p] = yv;
            }
            const int64_t col = col0 + l16;
            S b = S(0);
            if (MODE != MODE_QT && top && r < n) b = sm.slab[r][l16];
            else if (MODE != MODE_FORMQ && r < rows && col < k) b = Bg[(brow0 + r) * ldb + col];
            bt[s][i] = b;
        }
    }

    // W partial = Y^T X over this wave's rows
    acc_t acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = acc_t{0, 0, 0, 0};
    if (!(MODE == MODE_FORMQ && !top)) {
#pragma unroll
        for (int s = 0; s < SG; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const C bv = (C)bt[s][i];
#pragma unroll
                for (int p = 0; p < NP; ++p) acc[p] = M::mma(ynat[s][i][p], bv, acc[p]);
            }
    }
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) sm.u.Wpart[wv][16 * p + M::orow(l4, r)][l16] = acc[p][r];
    __syncthreads();
    for (int e = tid; e < NCP * 16; e += 256) {
        const int j = e >> 4, cc = e & 15;
        C sum = sm.u.Wpart[0][j][cc] + sm.u.Wpart[1][j][cc];
        sum += sm.u.Wpart[2][j][cc];
        sum += sm.u.Wpart[3][j][cc];
        if (!top && j < n) sum += (C)sm.slab[j][cc];
        sm.u.Wpart[0][j][cc] = sum;
    }
    __syncthreads();
    // W' = T^T W (Q^T) or T W (Q); T upper triangular, packed by columns
    if (wv < NP) {
        acc_t a2 = acc_t{0, 0, 0, 0};
        const int m = 16 * wv + l16;
        const int qlo = (MODE == MODE_QT) ? 0 : 4 * wv;
        const int qhi = (MODE == MODE_QT) ? 4 * wv + 4 : NCP / 4;
        for (int q = qlo; q < qhi; ++q) {
            const int kk = 4 * q + l4;
            const int ti = (MODE == MODE_QT) ? kk : m;
            const int tj = (MODE == MODE_QT) ? m : kk;
            const C a = (ti <= tj && tj < n) ? sm.Tl[tj * (tj + 1) / 2 + ti] : C(0);
            a2 = M::mma(a, sm.u.Wpart[0][kk][l16], a2);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) sm.Wp[16 * wv + M::orow(l4, r)][l16] = a2[r];
    }
    __syncthreads();
    if (!top) {
        for (int e = tid; e < n * 16; e += 256) {
            const int j = e >> 4, cc = e & 15;
            sm.slab[j][cc] -= (S)sm.Wp[j][cc];
        }
    }
    // X -= Y W'
#pragma unroll
    for (int s = 0; s < SG; ++s) {
        acc_t u = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int i = 0; i < 4; ++i) sm.u.trans[wv][M::orow(l4, i)][l16] = ynat[s][i][p];
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const C a = sm.u.trans[wv][l16][4 * q + l4];
                const C bb = sm.Wp[16 * p + 4 * q + l4][l16];
                u = M::mma(a, bb, u);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) bt[s][i] -= (S)u[i];
    }
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = wv * RW + 16 * s + M::orow(l4, i);
            const int64_t col = col0 + l16;
            if (r < rows && col < k) Bg[(brow0 + r) * ldb + col] = bt[s][i];
            if (MODE == MODE_QT && top && r < n) sm.slab[r][l16] = bt[s][i];
        }
    __syncthreads();
}

// Reflector entry as an operand when the heads lie in the block: zero above
// the head row, one on it.
template <typename C>
__device__ __forceinline__ C vunit(C x, int r, int c) {
    return (r > c) ? x : ((r == c) ? C(1) : C(0));
}

// ---------------------------------------------------------------- 64-row blocks
// The chain kernel for 64-row blocks: four waves, wave w owning rows
// 16w..16w+15 of each block and (for w < n/16) the slab tile w.  The next
// block's reflectors, rows of B and T fragments are loaded into registers
// while the current block is processed.  Per block:
//   1. partial W_w = Y_w^T X_w on each wave (16 rows), to LDS;
//   2. wave p sums the partials of tile p (+ its slab tile) -> W_p, to LDS;
//   3. wave p: W'_p from T's blocks (loaded straight into the A-operand
//      layout) and the W tiles; slab tile p -= W'_p; W'_p to LDS;
//   4. every wave: X_w -= Y_w W' (Y_w transposed through its LDS tile).
template <typename S, typename C, int NP>
struct Apply64Smem {
    C part[4][NP][4][64];  // per-wave partials; part[0] holds the sums
    C wp[NP][4][64];       // W' tiles (MFMA D layout, lane-major)
    C trans[4][16][17];    // per-wave transposes
};

template <typename S, typename C, int NP, int MODE>
struct Apply64Regs {
    C y[4][NP];  // Y rows 16w + orow(l4, i), columns 16p + l16
    C x[4];      // B rows 16w + orow(l4, i), column col
    C t[NP][4];  // T fragments of this wave's W' tile (A-operand layout)
};

template <typename S, typename C, int NP, int MODE>
__device__ __forceinline__ void apply64_load(Apply64Regs<S, C, NP, MODE>& R, int wv, int l16, int l4, int n,
                                             const S* __restrict__ Y, int64_t ldy, const S* __restrict__ Tb,
                                             const S* __restrict__ B, int64_t ldb, int64_t r0, int rows, bool top,
                                             int64_t col, bool colok) {
    typedef Mfma<C> M;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 16 * wv + M::orow(l4, i);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int cc = 16 * p + l16;
            C v = (r < rows && cc < n) ? (C)Y[(r0 + r) * ldy + cc] : C(0);
            if (top) v = (cc < n) ? vunit(v, r, cc) : C(0);
            R.y[i][p] = v;
        }
        R.x[i] = (MODE != MODE_FORMQ && r < rows && colok) ? (C)B[(r0 + r) * ldb + col] : C(0);
    }
    // T fragments for output tile p = wv: QT uses (T_qp)^T (q <= p), Q uses T_pq (q >= p)
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            int ti, tj;
            if (MODE == MODE_QT) {
                ti = 16 * q + M::orow(l4, kc);
                tj = 16 * wv + l16;
            } else {
                ti = 16 * wv + l16;
                tj = 16 * q + M::orow(l4, kc);
            }
            const bool ok = wv < NP && ti <= tj && tj < n;
            R.t[q][kc] = ok ? (C)Tb[(int64_t)tj * (tj + 1) / 2 + ti] : C(0);
        }
}

template <typename S, typename C, int NP, int MODE>
__device__ __forceinline__ void apply64_block(Apply64Smem<S, C, NP>& sm, Apply64Regs<S, C, NP, MODE>& R,
                                              C (&sl)[4], int wv, int l16, int l4, int n, S* __restrict__ B,
                                              int64_t ldb, int64_t r0, int rows, bool top, int64_t col, bool colok) {
    typedef Mfma<C> M;
    typedef typename M::acc acc_t;
    const int lane = threadIdx.x & 63;
    // first block in the Q direction: its first n rows are the slab
    if (MODE != MODE_QT && top && wv < NP) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * wv + M::orow(l4, i);
            if (r < n) R.x[i] = sl[i];
        }
    }
    // Explicit Q, blocks past the first: the block's rows of B are zero, so
    // W is the slab itself and steps 1-2 reduce to publishing the slab tiles.
    if (MODE == MODE_FORMQ && !top) {
        if (wv < NP) {
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.part[0][wv][r][lane] = sl[r];
        }
        __syncthreads();
    } else {
    // 1. partial W over this wave's rows
    {
        acc_t acc[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[p] = acc_t{0, 0, 0, 0};
        if (!(MODE == MODE_FORMQ && !top)) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int p = 0; p < NP; ++p) acc[p] = M::mma(R.y[i][p], R.x[i], acc[p]);
        }
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.part[wv][p][r][lane] = acc[p][r];
    }
    __syncthreads();
    // 2. wave p: W_p = sum of partials (+ slab tile p)
    if (wv < NP) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            C v = sm.part[0][wv][r][lane] + sm.part[1][wv][r][lane];
            v += sm.part[2][wv][r][lane];
            v += sm.part[3][wv][r][lane];
            if (!top) v += sl[r];
            sm.part[0][wv][r][lane] = v;
        }
    }
    __syncthreads();
    }
    // 3. wave p: -W'_p, slab tile p
    if (wv < NP) {
        acc_t nw = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                if (MODE == MODE_QT ? (q > wv) : (q < wv)) continue;
                nw = M::mma(-R.t[q][kc], sm.part[0][q][kc][lane], nw);
            }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            sm.wp[wv][r][lane] = nw[r];
            if (!top) sl[r] += nw[r];
        }
    }
    __syncthreads();
    // 4. X -= Y W'
    {
        acc_t u = acc_t{R.x[0], R.x[1], R.x[2], R.x[3]};
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int i = 0; i < 4; ++i) sm.trans[wv][M::orow(l4, i)][l16] = R.y[i][p];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            C yt[4];
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) yt[kc] = sm.trans[wv][l16][M::orow(l4, kc)];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) u = M::mma(yt[kc], sm.wp[p][kc][lane], u);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * wv + M::orow(l4, i);
            if (MODE == MODE_QT && top && wv < NP && r < n) sl[i] = u[i];
            if (r < rows && colok) B[(r0 + r) * ldb + col] = (S)u[i];
        }
    }
}

template <typename S, typename C, int NP, int MODE>
__global__ __launch_bounds__(256, 2) void k_chain_apply64(Geom g, const S* __restrict__ Y, int64_t ldy,
                                                          const S* __restrict__ T_blk, S* __restrict__ B,
                                                          int64_t ldb, int64_t k, int ntiles) {
    typedef Mfma<C> M;
    __shared__ Apply64Smem<S, C, NP> sm;
    const int gid = blockIdx.x;
    const int x8 = gid & 7, yq = gid >> 3;
    const int chain = (yq / ntiles) * 8 + x8;
    const int tile = yq - (yq / ntiles) * ntiles;
    if (chain >= g.W) return;
    const int n = (int)g.n;
    const int64_t tri = (int64_t)n * (n + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const int64_t col = (int64_t)tile * 16 + l16;
    const bool colok = col < k;
    const int64_t start = chain_start(g, chain), end = chain_end(g, chain);
    const int nb = chain_nblocks(g, chain);
    const int64_t blk0 = chain_blk0(g, chain);
    // slab tile wv (D layout = the natural rows 16wv + orow(l4, i) of the chain's first rows)
    C sl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = 16 * wv + M::orow(l4, i);
        sl[i] = (MODE != MODE_QT && wv < NP && j < n && colok) ? (C)B[(start + j) * ldb + col] : C(0);
    }
    Apply64Regs<S, C, NP, MODE> cur, nxt;
    auto blk = [&](int bi) { return (MODE == MODE_QT) ? bi : nb - 1 - bi; };
    auto load = [&](Apply64Regs<S, C, NP, MODE>& R, int bi) {
        const int b = blk(bi);
        const int64_t r0 = start + (int64_t)b * 64;
        const int rows = (int)((end - r0) < 64 ? (end - r0) : 64);
        apply64_load<S, C, NP, MODE>(R, wv, l16, l4, n, Y, ldy, T_blk + (blk0 + b) * tri, B, ldb, r0, rows, b == 0,
                                     col, colok);
    };
    auto run = [&](Apply64Regs<S, C, NP, MODE>& R, int bi) {
        const int b = blk(bi);
        const int64_t r0 = start + (int64_t)b * 64;
        const int rows = (int)((end - r0) < 64 ? (end - r0) : 64);
        apply64_block<S, C, NP, MODE>(sm, R, sl, wv, l16, l4, n, B, ldb, r0, rows, b == 0, col, colok);
    };
    load(cur, 0);
    for (int bi = 0; bi < nb; bi += 2) {
        if (bi + 1 < nb) load(nxt, bi + 1);
        run(cur, bi);
        if (bi + 1 >= nb) break;
        if (bi + 2 < nb) load(cur, bi + 2);
        run(nxt, bi + 1);
    }
    if (MODE == MODE_QT && wv < NP) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = 16 * wv + M::orow(l4, i);
            if (j < n && colok) B[(start + j) * ldb + col] = (S)sl[i];
        }
    }
}

template <typename S, typename C, int NC, int H, int MODE>
__global__ __launch_bounds__(256) void k_chain_apply(Geom g, const S* __restrict__ Y, int64_t ldy,
                                                     const S* __restrict__ T_blk, S* __restrict__ B, int64_t ldb,
                                                     int64_t k, int ntiles) {
    __shared__ ApplySmem<S, C, NC> sm;
    const int gid = blockIdx.x;
    const int x8 = gid & 7, y = gid >> 3;
    const int chain = (y / ntiles) * 8 + x8;
    const int tile = y - (y / ntiles) * ntiles;
    if (chain >= g.W) return;
    const int n = (int)g.n;
    const int tri = n * (n + 1) / 2;
    const int64_t col0 = (int64_t)tile * 16;
    const int64_t start = chain_start(g, chain), end = chain_end(g, chain);
    const int nb = chain_nblocks(g, chain);
    const int64_t blk0 = chain_blk0(g, chain);
    const int tid = threadIdx.x;
    if (MODE != MODE_QT) {
        for (int e = tid; e < n * 16; e += 256) {
            const int j = e >> 4, cc = e & 15;
            const int64_t col = col0 + cc;
            sm.slab[j][cc] = (col < k) ? B[(start + j) * ldb + col] : S(0);
        }
        __syncthreads();
    }
    for (int bi = 0; bi < nb; ++bi) {
        const int b = (MODE == MODE_QT) ? bi : nb - 1 - bi;
        const int64_t r0 = start + (int64_t)b * H;
        const int rows = (int)((end - r0) < H ? (end - r0) : H);
        apply_block<S, C, NC, H, MODE>(sm, n, Y, ldy, r0, B, ldb, r0, rows, col0, k, b == 0,
                                       T_blk + (blk0 + b) * tri);
    }
    if (MODE == MODE_QT) {
        for (int e = tid; e < n * 16; e += 256) {
            const int j = e >> 4, cc = e & 15;
            const int64_t col = col0 + cc;
            if (col < k) B[(start + j) * ldb + col] = sm.slab[j][cc];
        }
    }
}

template <typename S, typename C, int NC, int MODE>
__global__ __launch_bounds__(256) void k_node_apply(Geom g, int lev, const S* __restrict__ Ynode,
                                                    const S* __restrict__ Tnode, S* __restrict__ B, int64_t ldb,
                                                    int64_t k, int ntiles) {
    __shared__ ApplySmem<S, C, NC> sm;
    const int node = blockIdx.x / ntiles;
    const int tile = blockIdx.x - node * ntiles;
    const int64_t stride = ipow(g.arity, lev - 1);
    const int64_t i0 = (int64_t)node * g.arity * stride;
    if (i0 + stride >= g.W) return;
    const int n = (int)g.n;
    const int tri = n * (n + 1) / 2;
    const int64_t col0 = (int64_t)tile * 16;
    const int tid = threadIdx.x;
    const int64_t sa = chain_start(g, (int)i0);
    for (int e = tid; e < n * 16; e += 256) {
        const int j = e >> 4, cc = e & 15;
        const int64_t col = col0 + cc;
        sm.slab[j][cc] = (col < k) ? B[(sa + j) * ldb + col] : S(0);
    }
    __syncthreads();
    int nch = 0;
    for (int t1 = 1; t1 < g.arity && i0 + (int64_t)t1 * stride < g.W; ++t1) nch = t1;
    for (int ti = 0; ti < nch; ++ti) {
        const int t1 = (MODE == MODE_QT) ? ti + 1 : nch - ti;
        const int64_t c = i0 + (int64_t)t1 * stride;
        const int64_t sc = chain_start(g, (int)c);
        apply_block<S, C, NC, 64, MODE>(sm, n, Ynode + c * n * n, n, 0, B, ldb, sc, n, col0, k, false,
                                        Tnode + c * tri);
    }
    for (int e = tid; e < n * 16; e += 256) {
        const int j = e >> 4, cc = e & 15;
        const int64_t col = col0 + cc;
        if (col < k) B[(sa + j) * ldb + col] = sm.slab[j][cc];
    }
}

template <typename T>
__global__ void k_init_formq(int64_t n, T* __restrict__ Q, int64_t ldq) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int64_t i = e / n, j = e - i * n;
    Q[i * ldq + j] = (i == j) ? T(1) : T(0);
}

template <typename S, typename C, int NC, int H, int MODE>
static hipError_t chain_apply_launch(const Geom& g, const S* Y, int64_t ldy, const Work& wk, S* B, int64_t ldb,
                                     int64_t k, hipStream_t st) {
    const int ntiles = (int)((k + 15) / 16);
    const int groups = (g.W + 7) / 8;
    const int64_t grid = (int64_t)groups * 8 * ntiles;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    constexpr int NP = NC <= 16 ? 1 : NC / 16;
    phase_begin(1 + MODE, st);
    if constexpr (H == 64)
        k_chain_apply64<S, C, NP, MODE><<<(int)grid, 256, 0, st>>>(g, Y, ldy, (const S*)wk.T_blk, B, ldb, k, ntiles);
    else
        k_chain_apply<S, C, NC, H, MODE><<<(int)grid, 256, 0, st>>>(g, Y, ldy, (const S*)wk.T_blk, B, ldb, k, ntiles);
    phase_end(1 + MODE, st);
    return hipGetLastError();
}

template <typename S, typename C, int NC, int MODE>
static hipError_t node_apply_launch(const Geom& g, int lev, const Work& wk, S* B, int64_t ldb, int64_t k,
                                    hipStream_t st) {
    const int ntiles = (int)((k + 15) / 16);
    const int64_t stride = ipow(g.arity, lev - 1);
    const int64_t span = stride * g.arity;
    const int64_t nodes = (g.W + span - 1) / span;
    const int64_t grid = nodes * ntiles;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    k_node_apply<S, C, NC, MODE><<<(int)grid, 256, 0, st>>>(g, lev, (const S*)wk.Ynode, (const S*)wk.Tnode, B, ldb,
                                                            k, ntiles);
    return hipGetLastError();
}

template <typename S, typename C, int NC, int MODE>
static hipError_t chain_apply_h(const Geom& g, const S* Y, int64_t ldy, const Work& wk, S* B, int64_t ldb, int64_t k,
                                hipStream_t st) {
    if (g.h != 64) return hipErrorInvalidValue;
    return chain_apply_launch<S, C, NC, 64, MODE>(g, Y, ldy, wk, B, ldb, k, st);
}

template <typename S, typename C, int NC, int MODE>
static hipError_t apply_mode(const Geom& g, const S* Y, int64_t ldy, const Work& wk, S* B, int64_t ldb, int64_t k,
                             hipStream_t st) {
    hipError_t e = hipSuccess;
    if (MODE == MODE_QT) {
        e = chain_apply_h<S, C, NC, MODE>(g, Y, ldy, wk, B, ldb, k, st);
        for (int lev = 1; lev <= g.levels && e == hipSuccess; ++lev)
            e = node_apply_launch<S, C, NC, MODE>(g, lev, wk, B, ldb, k, st);
    } else {
        for (int lev = g.levels; lev >= 1 && e == hipSuccess; --lev)
            e = node_apply_launch<S, C, NC, MODE>(g, lev, wk, B, ldb, k, st);
        if (e == hipSuccess) e = chain_apply_h<S, C, NC, MODE>(g, Y, ldy, wk, B, ldb, k, st);
    }
    return e;
}

template <typename S, typename C, int NC>
static hipError_t apply_nc(const Geom& g, const S* Y, int64_t ldy, const Work& wk, S* B, int64_t ldb, int64_t k,
                           int mode, hipStream_t st) {
    switch (mode) {
        case MODE_QT: return apply_mode<S, C, NC, MODE_QT>(g, Y, ldy, wk, B, ldb, k, st);
        case MODE_Q: return apply_mode<S, C, NC, MODE_Q>(g, Y, ldy, wk, B, ldb, k, st);
        case MODE_FORMQ: return apply_mode<S, C, NC, MODE_FORMQ>(g, Y, ldy, wk, B, ldb, k, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename S, typename C>
static hipError_t apply_sc(const Geom& g, const S* Y, int64_t ldy, const Work& wk, S* B, int64_t ldb, int64_t k,
                           int mode, hipStream_t st) {
    switch (g.NC) {
        case 8: return apply_nc<S, C, 8>(g, Y, ldy, wk, B, ldb, k, mode, st);
        case 16: return apply_nc<S, C, 16>(g, Y, ldy, wk, B, ldb, k, mode, st);
        case 32: return apply_nc<S, C, 32>(g, Y, ldy, wk, B, ldb, k, mode, st);
        case 64: return apply_nc<S, C, 64>(g, Y, ldy, wk, B, ldb, k, mode, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_apply(bool store_f64, bool compute_f64, const Geom& g, const void* Y, int64_t ldy, const Work& wk,
                        void* B, int64_t ldb, int64_t k, int mode, hipStream_t st) {
    if (store_f64 && compute_f64)
        return apply_sc<double, double>(g, (const double*)Y, ldy, wk, (double*)B, ldb, k, mode, st);
    if (store_f64 && !compute_f64)
        return apply_sc<double, float>(g, (const double*)Y, ldy, wk, (double*)B, ldb, k, mode, st);
    if (!store_f64 && !compute_f64)
        return apply_sc<float, float>(g, (const float*)Y, ldy, wk, (float*)B, ldb, k, mode, st);
    return hipErrorInvalidValue;
}

template <typename T>
__global__ void k_fill_identity(int64_t m, int64_t n, T* __restrict__ Q, int64_t ldq) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * n) return;
    const int64_t i = e / n, j = e - i * n;
    Q[i * ldq + j] = (i == j) ? T(1) : T(0);
}

hipError_t launch_fill_identity(bool f64, int64_t m, int64_t n, void* Q, int64_t ldq, hipStream_t st) {
    const int64_t nb = (m * n + 255) / 256;
    if (f64) k_fill_identity<double><<<(unsigned)nb, 256, 0, st>>>(m, n, (double*)Q, ldq);
    else k_fill_identity<float><<<(unsigned)nb, 256, 0, st>>>(m, n, (float*)Q, ldq);
    return hipGetLastError();
}

hipError_t launch_init_formq(bool f64, int64_t n, void* Q, int64_t ldq, hipStream_t st) {
    const int nb = (int)((n * n + 255) / 256);
    if (f64) k_init_formq<double><<<nb, 256, 0, st>>>(n, (double*)Q, ldq);
    else k_init_formq<float><<<nb, 256, 0, st>>>(n, (float*)Q, ldq);
    return hipGetLastError();
}

}  // namespace tsqr
