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
// FP32 compute with FP64 storage is the mixed-precision CAQR update: the
// products take FP32 operands (the FP64 values rounded) and accumulate in
// FP32 from zero, and each product is then added to the FP64 values of the
// slab and of B, which stay FP64 throughout (only Q^T is offered in this
// form; it is the trailing update).
//
// Workgroup = 4 waves, each owning 16 rows of a 64-row block; 16 columns of B
// per workgroup.  Workgroups are numbered so that all column tiles of one
// chain land on the same XCD (dispatch is round robin over the 8 XCDs), so the
// block's reflectors are fetched from HBM once and re-read from that XCD's L2.
// Q^T runs the chains in one launch and every tree level in a second one;
// Q and the explicit Q run the tree levels top-down, one launch per level,
// then the chains.
#include <type_traits>

#include "tsqr_common.hpp"

namespace tsqr {
using namespace dev;

template <typename C>
__device__ __forceinline__ C vunit(C x, int r, int c) {
    return (r > c) ? x : ((r == c) ? C(1) : C(0));
}

// FP32 products on FP64 storage (S != C): products start from zero and are
// added to the storage-type values afterwards; with S == C the product
// accumulates onto the values directly (one rounding fewer, same as before).
template <typename S, typename C>
constexpr bool kMixed = !std::is_same<S, C>::value;
// accumulator-shaped storage of the slab in the storage type
template <typename S, typename C>
using SAcc = typename Mfma<typename std::conditional<std::is_same<S, C>::value, C, S>::type>::acc;
template <typename To, typename From>
__device__ __forceinline__ To vcvt(From v) {
    return __builtin_convertvector(v, To);
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

// Held in the storage type: a prefetched value is converted to the compute
// type only where it is used, so the load's latency stays hidden.
template <typename S, typename C, int NP, int MODE>
struct Apply64Regs {
    S y[4][NP];  // Y rows 16w + orow(l4, i), columns 16p + l16
    S x[4];      // B rows 16w + orow(l4, i), column col
    S t[NP][4];  // T fragments of this wave's W' tile (A-operand layout)
};

// PUB: the rows of B were published by another workgroup of this launch.
template <typename S, typename C, int NP, int MODE, bool PUB = false>
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
            S v = (r < rows && cc < n) ? Y[(r0 + r) * ldy + cc] : S(0);
            if (top) v = (cc < n) ? vunit(v, r, cc) : S(0);
            R.y[i][p] = v;
        }
        const S* bp = B + (r0 + r) * ldb + col;
        R.x[i] = (MODE != MODE_FORMQ && r < rows && colok) ? (PUB ? pub_load(bp) : *bp) : S(0);
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
            R.t[q][kc] = ok ? Tb[(int64_t)tj * (tj + 1) / 2 + ti] : S(0);
        }
}

template <typename S, typename C, int NP, int MODE>
__device__ __forceinline__ void apply64_block(Apply64Smem<S, C, NP>& sm, Apply64Regs<S, C, NP, MODE>& R,
                                              S (&sl)[4], int wv, int l16, int l4, int n, S* __restrict__ B,
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
            for (int r = 0; r < 4; ++r) sm.part[0][wv][r][lane] = (C)sl[r];
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
                for (int p = 0; p < NP; ++p) acc[p] = M::mma((C)R.y[i][p], (C)R.x[i], acc[p]);
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
            if (!top) v += (C)sl[r];
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
                nw = M::mma(-(C)R.t[q][kc], sm.part[0][q][kc][lane], nw);
            }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            sm.wp[wv][r][lane] = nw[r];
            if (!top) sl[r] += (S)nw[r];
        }
    }
    __syncthreads();
    // 4. X -= Y W'
    {
        acc_t u = kMixed<S, C> ? acc_t{0, 0, 0, 0} : acc_t{(C)R.x[0], (C)R.x[1], (C)R.x[2], (C)R.x[3]};
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int i = 0; i < 4; ++i) sm.trans[wv][M::orow(l4, i)][l16] = (C)R.y[i][p];
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
            const S o = kMixed<S, C> ? R.x[i] + (S)u[i] : (S)u[i];
            if (MODE == MODE_QT && top && wv < NP && r < n) sl[i] = o;
            if (r < rows && colok) B[(r0 + r) * ldb + col] = o;
        }
    }
}

// Tree levels of Q^T in one launch (Sec. 2.1: the nodes of the tree of Q
// factors are applied bottom-up).  Workgroup (node, tile) applies level-1
// node `node` to one 16-column tile of B: child 0's slab (its chain's top n
// rows of B) and each further child's slab are combined with that child's
// node reflectors.  Then, level by level, the last of a node's children to
// arrive (an arrival count per node and tile, zero at launch) applies the
// node; the others leave.  Slabs pass between workgroups with
// device-coherent stores and loads.
template <typename S, typename C, int NP>
__global__ __launch_bounds__(256, 2) void k_qt_tree64(Geom g, int ntiles, S* __restrict__ B, int64_t ldb, int64_t k,
                                                      const S* __restrict__ Ynode, const S* __restrict__ Tnode,
                                                      int* __restrict__ cnt) {
    typedef Mfma<C> M;
    __shared__ Apply64Smem<S, C, NP> sm;
    __shared__ int s_old;
    const int node = blockIdx.x / ntiles;
    const int tile = blockIdx.x - node * ntiles;
    const int n = (int)g.n;
    const int64_t tri = (int64_t)n * (n + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const int64_t col = (int64_t)tile * 16 + l16;
    const bool colok = col < k;
    int cur = node * g.arity;
    if (cur >= g.W) return;
    for (int lev = 1; lev <= g.levels; ++lev) {
        const int64_t stride = ipow(g.arity, lev - 1);
        const int64_t span = stride * g.arity;
        const int i0 = (int)((cur / span) * span);
        int nch = (int)((g.W - i0 + stride - 1) / stride);
        if (nch > g.arity) nch = g.arity;
        if (nch <= 1) continue;  // unpaired: carried up unchanged
        if (lev > 1) {
            pub_wait();  // this workgroup's slab stores have landed
            __syncthreads();
            if (tid == 0) s_old = atomicAdd(cnt + (((int64_t)(lev - 2) * g.W + i0) * ntiles + tile), 1);
            __syncthreads();
            if (s_old != nch - 1) return;
        }
        const int64_t sa = chain_start(g, i0);
        S sl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = 16 * wv + M::orow(l4, i);
            sl[i] = (wv < NP && j < n && colok) ? pub_load(B + (sa + j) * ldb + col) : S(0);
        }
        for (int t = 1; t < nch; ++t) {
            const int64_t ch = i0 + t * stride;
            S* Bc = B + chain_start(g, (int)ch) * ldb;
            Apply64Regs<S, C, NP, MODE_QT> R;
            apply64_load<S, C, NP, MODE_QT, true>(R, wv, l16, l4, n, Ynode + ch * n * n, n, Tnode + ch * tri, Bc,
                                                  ldb, 0, n, false, col, colok);
            apply64_block<S, C, NP, MODE_QT>(sm, R, sl, wv, l16, l4, n, Bc, ldb, 0, n, false, col, colok);
        }
        if (wv < NP) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = 16 * wv + M::orow(l4, i);
                if (j < n && colok) pub_store(B + (sa + j) * ldb + col, sl[i]);
            }
        }
        cur = i0;
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
    S sl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = 16 * wv + M::orow(l4, i);
        sl[i] = (MODE != MODE_QT && wv < NP && j < n && colok) ? B[(start + j) * ldb + col] : S(0);
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
            if (j < n && colok) B[(start + j) * ldb + col] = sl[i];
        }
    }
}

// ---- wide chain kernel: n = 64, 64 columns of B per workgroup ---------------
//
// Each of the four waves owns one 16-column tile of B over all 64 rows of a
// block, so W = V^T [S; X], W' = T^T W (Q^T) or T W (Q), S -= W' and
// X -= Y W' need no reduction across waves.  The block's rows of X are held
// in the MFMA accumulator layout (x[4r + i] = row 16r + orow(l4, i)); the
// V^T X product sums over the rows in that same order, so x is also its B
// operand, and W and W' are used as B operands exactly as the products leave
// them: no transposes.  The block's Y (64 x 64, row pitch 66) and -T (a
// full 64 x 64 matrix, zero below the diagonal) are staged once per
// workgroup in LDS (in the compute type) and read as A operands.
// Four waves: two workgroups per CU (two waves per SIMD, 256 registers), the
// next block's rows of B loaded after the block's stores and its Y and T
// after the block's barrier, while the other workgroup computes.  Two waves
// (32 columns): one wave per SIMD, the next block's Y, T and rows of B
// loaded into registers (in the storage type) during X -= Y W'.
constexpr int WY_PITCH = 66;
constexpr int W_TRI = 64 * 65 / 2;

template <typename C>
struct WideSmem {
    C Y[64][WY_PITCH];
    C T[W_TRI];
};

// Global access at a wave-uniform base plus a 32-bit per-lane byte offset:
// the form the scalar-base vector memory instructions take, so no per-lane
// 64-bit address arithmetic is spent on it.
// (The offset passes through an empty asm so the optimiser does not fold it
// into a 64-bit per-lane address computed once outside the block loop.)
template <typename T>
__device__ __forceinline__ T ld_off(const T* base, uint32_t off) {
    asm volatile("" : "+v"(off));
    return *(const T*)((const char*)base + off);
}
template <typename T>
__device__ __forceinline__ void st_off(T* base, uint32_t off, T v) {
    asm volatile("" : "+v"(off));
    *(T*)((char*)base + off) = v;
}

template <typename T>
__device__ __forceinline__ T pub_load_off(const T* base, uint32_t off) {
    asm volatile("" : "+v"(off));
    return pub_load((const T*)((const char*)base + off));
}
template <typename T>
__device__ __forceinline__ void pub_store_off(T* base, uint32_t off, T v) {
    asm volatile("" : "+v"(off));
    pub_store((T*)((char*)base + off), v);
}

// Row pitch of the full -T staged in LDS (WideSmemF below).
constexpr int WT_PITCH = 65;
// Index in WideSmemF::Tn of entry e of a T packed column by column.
__device__ __forceinline__ int wide_tdst(int e) {
    int j = (int)((__builtin_sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    j -= (j * (j + 1) / 2 > e) ? 1 : 0;
    j += ((j + 1) * (j + 2) / 2 <= e) ? 1 : 0;
    return (e - j * (j + 1) / 2) * WT_PITCH + j;
}

// Entry (i, j), i <= j, of a block's T staged as is (packed column by column).
template <typename C>
__device__ __forceinline__ C wide_t(const WideSmem<C>& sm, int i, int j) {
    return sm.T[j * (j + 1) / 2 + i];
}

// The chain kernel's LDS: the block's Y, and -T as a full 64 x 64 matrix
// (zero below the diagonal), so an A operand of W' = T^T W or T W is one
// read at a lane offset fixed for the kernel, with no triangle test.
template <typename C>
struct WideSmemF {
    C Y[64][WY_PITCH];
    C Tn[64][WT_PITCH];
};

// TW waves per workgroup (2 or 4), so 16 TW columns of B per workgroup;
// with four waves two workgroups share a CU (two waves per SIMD).
template <typename S, typename C, int MODE, int TW>
__global__ __launch_bounds__(64 * TW, TW == 4 ? 2 : 1) void k_chain_apply_w(
    Geom g, const S* __restrict__ Y, int64_t ldy, const S* __restrict__ T_blk, S* __restrict__ B, int64_t ldb, int64_t k,
    int ngroups) {
    constexpr int NT = 64 * TW, YS = 64 / TW, TSN = (W_TRI + NT - 1) / NT;
    typedef Mfma<C> M;
    typedef typename M::acc acc_t;
    __shared__ WideSmemF<C> sm;
    const int gid = blockIdx.x;
    const int x8 = gid & 7, yq = gid >> 3;
    const int chain = (yq / ngroups) * 8 + x8;
    const int grp = yq - (yq / ngroups) * ngroups;
    if (chain >= g.W) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const int64_t col = (int64_t)grp * (16 * TW) + 16 * wv + l16;
    const bool colok = col < k;
    const int64_t start = chain_start(g, chain), end = chain_end(g, chain);
    const int nb = chain_nblocks(g, chain);
    const int64_t blk0 = chain_blk0(g, chain);
    auto blk = [&](int bi) { return (MODE == MODE_QT) ? bi : nb - 1 - bi; };
    // Full blocks of a workgroup whose columns are all inside B take the fast
    // accesses: a uniform row base and a 32-bit lane offset (rows
    // 16r + orow(l4, i) of a block: base row 16r, offset boff[i]).
    const bool colall = (int64_t)grp * (16 * TW) + 16 * TW <= k &&
                        (int64_t)(16 * ldb + k) * (int64_t)sizeof(S) < ((int64_t)1 << 31) &&
                        (int64_t)(64 * ldy) * (int64_t)sizeof(S) < ((int64_t)1 << 31);
    const int wvu = __builtin_amdgcn_readfirstlane(wv);
    uint32_t boff[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) boff[i] = (uint32_t)(((int64_t)M::orow(l4, i) * ldb + col) * (int64_t)sizeof(S));
    const uint32_t loff = (uint32_t)(lane * (int)sizeof(S)), toff0 = (uint32_t)(tid * (int)sizeof(S));
    // row of register kk = 4r + i of the accumulator layout
    auto xrow = [&](int kk) { return 16 * (kk >> 2) + M::orow(l4, kk & 3); };
    // staging of one block's Y (rows TW t + wv, column lane) and packed T
    S ys[YS], ts[TSN];
    auto stage_load = [&](int bi) {
        const int b = blk(bi);
        const int64_t r0 = start + (int64_t)b * 64;
        const int rows = (int)((end - r0) < 64 ? (end - r0) : 64);
        if (rows == 64 && colall) {
#pragma unroll
            for (int t = 0; t < YS; ++t) ys[t] = ld_off(Y + (r0 + TW * t + wvu) * ldy, loff);
        } else {
#pragma unroll
            for (int t = 0; t < YS; ++t) {
                const int r = TW * t + wv;
                ys[t] = (r < rows) ? Y[(r0 + r) * ldy + lane] : S(0);
            }
        }
        const S* Tb = T_blk + (blk0 + b) * W_TRI;
#pragma unroll
        for (int t = 0; t < TSN; ++t) {
            if ((t + 1) * NT <= W_TRI) {
                ts[t] = ld_off(Tb + NT * t, toff0);
            } else {
                const int e = tid + NT * t;
                ts[t] = (e < W_TRI) ? Tb[e] : S(0);
            }
        }
    };
    // where packed entry e = tid + NT t of T goes in Tn: kept in registers
    // with two waves (one per SIMD), recomputed with four (256 registers)
    int tdp[TW == 4 ? 1 : TSN];
    if constexpr (TW != 4) {
#pragma unroll
        for (int t = 0; t < TSN; ++t) tdp[t] = wide_tdst(tid + NT * t);
    }
    auto tdst = [&](int t) {
        if constexpr (TW == 4) return wide_tdst(tid + NT * t);
        else return tdp[t];
    };
    auto stage_store = [&](int bi) {
        const bool top = blk(bi) == 0;
#pragma unroll
        for (int t = 0; t < YS; ++t) {
            const int r = TW * t + wv;
            sm.Y[r][lane] = (C)(top ? vunit(ys[t], r, lane) : ys[t]);
        }
#pragma unroll
        for (int t = 0; t < TSN; ++t) {
            const int e = tid + NT * t;
            if (e < W_TRI) (&sm.Tn[0][0])[tdst(t)] = -(C)ts[t];
        }
    };
    S xn[16];
    auto x_load = [&](int bi) {
        const int b = blk(bi);
        const int64_t r0 = start + (int64_t)b * 64;
        const int rows = (int)((end - r0) < 64 ? (end - r0) : 64);
        const bool zero = (MODE == MODE_FORMQ) || (MODE != MODE_QT && b == 0);  // zero rows / the slab
        if (!zero && rows == 64 && colall) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int i = 0; i < 4; ++i) xn[4 * r + i] = ld_off(B + (r0 + 16 * r) * ldb, boff[i]);
            return;
        }
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int r = xrow(kk);
            xn[kk] = (!zero && r < rows && colok) ? B[(r0 + r) * ldb + col] : S(0);
        }
    };
    // slab S (the chain's first 64 rows), accumulator layout
    SAcc<S, C> sl[4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * p + M::orow(l4, i);
            if (MODE == MODE_QT) sl[p][i] = S(0);
            else if (colall) sl[p][i] = ld_off(B + (start + 16 * p) * ldb, boff[i]);
            else sl[p][i] = colok ? B[(start + r) * ldb + col] : S(0);
        }
    // Tn below the diagonal is zero for every block (staging writes the rest)
    for (int e = tid; e < 64 * WT_PITCH; e += NT) {
        const int i = e / WT_PITCH, j = e - i * WT_PITCH;
        if (i > j) (&sm.Tn[0][0])[e] = C(0);
    }
    S x[16];
    stage_load(0);
    x_load(0);
    stage_store(0);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) x[kk] = xn[kk];
    for (int bi = 0; bi < nb; ++bi) {
        const int b = blk(bi);
        const bool top = b == 0;
        const bool more = bi + 1 < nb;
        // the first block in the Q direction holds the slab in its rows
        if (MODE != MODE_QT && top) {
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int i = 0; i < 4; ++i) x[4 * p + i] = sl[p][i];
        }
        // W = V^T [S; X]
        acc_t w[4];
        const bool xzero = (MODE == MODE_FORMQ) && !top;
        C xc[16];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) xc[kk] = (C)x[kk];
        // (scheduling fences between the products' groups keep the operand
        // reads from LDS from all being hoisted ahead: two waves share a SIMD)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            w[p] = top ? acc_t{0, 0, 0, 0} : vcvt<acc_t>(sl[p]);
            if (!xzero) {
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) w[p] = M::mma(sm.Y[xrow(kk)][16 * p + l16], xc[kk], w[p]);
            }
            if constexpr (TW == 4) __builtin_amdgcn_sched_barrier(0);
        }
        // W' = T^T W (Q^T) or T W (Q); kept negated
        acc_t nw[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            nw[p] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (MODE == MODE_QT ? (q > p) : (q < p)) continue;
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) {
                    const C a = (MODE == MODE_QT) ? sm.Tn[16 * q + M::orow(l4, kc)][16 * p + l16]
                                                  : sm.Tn[16 * p + l16][16 * q + M::orow(l4, kc)];
                    nw[p] = M::mma(a, w[q][kc], nw[p]);
                }
            }
            if constexpr (TW == 4) __builtin_amdgcn_sched_barrier(0);
        }
        // S -= W'
        if (!top) {
#pragma unroll
            for (int p = 0; p < 4; ++p) sl[p] += vcvt<SAcc<S, C>>(nw[p]);
        }
        // two waves (one per SIMD): the next block's loads fly during X -= Y W'
        if (TW != 4 && more) {
            stage_load(bi + 1);
            x_load(bi + 1);
        }
        // X -= Y W'
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            acc_t u = kMixed<S, C> ? acc_t{0, 0, 0, 0} : acc_t{xc[4 * r], xc[4 * r + 1], xc[4 * r + 2], xc[4 * r + 3]};
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) u = M::mma(sm.Y[16 * r + l16][16 * p + M::orow(l4, kc)], nw[p][kc], u);
#pragma unroll
            for (int i = 0; i < 4; ++i) x[4 * r + i] = kMixed<S, C> ? x[4 * r + i] + (S)u[i] : (S)u[i];
            if constexpr (TW == 4) __builtin_amdgcn_sched_barrier(0);
        }
        if (MODE == MODE_QT && top) {
            // the chain's first block becomes the slab
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int i = 0; i < 4; ++i) sl[p][i] = x[4 * p + i];
        } else {
            const int64_t r0 = start + (int64_t)b * 64;
            const int rows = (int)((end - r0) < 64 ? (end - r0) : 64);
            if (rows == 64 && colall) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int i = 0; i < 4; ++i) st_off(B + (r0 + 16 * r) * ldb, boff[i], x[4 * r + i]);
            } else {
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) {
                    const int r = xrow(kk);
                    if (r < rows && colok) B[(r0 + r) * ldb + col] = x[kk];
                }
            }
        }
        // four waves (two per SIMD): the next block's rows are loaded after
        // this block's stores, whose registers they reuse, and its Y and T
        // after the barrier (no registers to hold them through the block);
        // the other workgroup on the CU computes meanwhile
        if (TW == 4 && more) x_load(bi + 1);
        if (more) {
            __syncthreads();  // every wave is done with this block's Y and T
            if constexpr (TW == 4) stage_load(bi + 1);
            stage_store(bi + 1);
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) x[kk] = xn[kk];
        }
    }
    if (MODE == MODE_QT && colall) {
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int i = 0; i < 4; ++i) st_off(B + (start + 16 * p) * ldb, boff[i], sl[p][i]);
    } else if (MODE == MODE_QT && colok) {
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int i = 0; i < 4; ++i) B[(start + 16 * p + M::orow(l4, i)) * ldb + col] = sl[p][i];
    }
}

// Tree levels of Q^T for n = 64, two waves (32 columns) per workgroup: the
// form of k_qt_tree_w below with T packed in LDS and one workgroup's steps
// in registers (one wave per SIMD), as
// k_qt_tree64 (level-1 node per workgroup, then the last arrival performs a
// node), each wave owning a 16-column tile over all 64 slab rows as in
// k_chain_apply_w; a step's Y_node and T_node are staged in LDS.
// A node's reflector tails sit in the positions of a child's upper triangle
// (Sec. 2.1: the stacked-triangle QR), so the 16 x 16 tiles of Y_node below
// the block diagonal are exact zeros and their products are skipped (here
// and in k_node_apply_w); the results are the same bits.
template <typename S, typename C, int TW>
__global__ __launch_bounds__(64 * TW, 1) void k_qt_tree_w2(Geom g, int ngroups, S* __restrict__ B, int64_t ldb,
                                                          int64_t k, const S* __restrict__ Ynode,
                                                          const S* __restrict__ Tnode, int* __restrict__ cnt) {
    constexpr int NT = 64 * TW, YS = 64 / TW, TSN = (W_TRI + NT - 1) / NT;
    typedef Mfma<C> M;
    typedef typename M::acc acc_t;
    __shared__ WideSmem<C> sm;
    __shared__ int s_old;
    const int node = blockIdx.x / ngroups;
    const int grp = blockIdx.x - node * ngroups;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const int64_t col = (int64_t)grp * (16 * TW) + 16 * wv + l16;
    const bool colok = col < k;
    auto xrow = [&](int kk) { return 16 * (kk >> 2) + M::orow(l4, kk & 3); };
    int cur = node * g.arity;
    if (cur >= g.W) return;
    bool staged = false;  // LDS holds a previous step's operands
    for (int lev = 1; lev <= g.levels; ++lev) {
        const int64_t stride = ipow(g.arity, lev - 1);
        const int64_t span = stride * g.arity;
        const int i0 = (int)((cur / span) * span);
        int nch = (int)((g.W - i0 + stride - 1) / stride);
        if (nch > g.arity) nch = g.arity;
        if (nch <= 1) continue;  // unpaired: carried up unchanged
        if (lev > 1) {
            pub_wait();  // this workgroup's slab stores have landed
            __syncthreads();
            if (tid == 0) s_old = atomicAdd(cnt + (((int64_t)(lev - 2) * g.W + i0) * ngroups + grp), 1);
            __syncthreads();
            if (s_old != nch - 1) return;
        }
        const int64_t sa = chain_start(g, i0);
        SAcc<S, C> sl[4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                sl[p][i] = colok ? pub_load(B + (sa + 16 * p + M::orow(l4, i)) * ldb + col) : S(0);
        for (int t = 1; t < nch; ++t) {
            const int64_t ch = i0 + t * stride;
            S* Bc = B + chain_start(g, (int)ch) * ldb;
            // stage Y_node (64 x 64, row-major) and T_node
            S ys[YS], ts[TSN];
            const S* Yc = Ynode + ch * 4096;
            const S* Tc = Tnode + ch * W_TRI;
#pragma unroll
            for (int u = 0; u < YS; ++u) ys[u] = Yc[(TW * u + wv) * 64 + lane];
#pragma unroll
            for (int u = 0; u < TSN; ++u) {
                const int e = tid + NT * u;
                ts[u] = (e < W_TRI) ? Tc[e] : S(0);
            }
            S x[16];
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) x[kk] = colok ? pub_load(Bc + xrow(kk) * ldb + col) : S(0);
            if (staged) __syncthreads();  // every wave is done with the previous step's operands
#pragma unroll
            for (int u = 0; u < YS; ++u) sm.Y[TW * u + wv][lane] = (C)ys[u];
#pragma unroll
            for (int u = 0; u < TSN; ++u) {
                const int e = tid + NT * u;
                if (e < W_TRI) sm.T[e] = (C)ts[u];
            }
            __syncthreads();
            staged = true;
            // W = S + Y^T X;  W' = T^T W (negated);  S -= W';  X -= Y W'
            acc_t w[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                w[p] = vcvt<acc_t>(sl[p]);
#pragma unroll
                for (int kk = 0; kk < 16; ++kk)
                    if ((kk >> 2) <= p) w[p] = M::mma(sm.Y[xrow(kk)][16 * p + l16], (C)x[kk], w[p]);
            }
            acc_t nw[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                nw[p] = acc_t{0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q <= p; ++q)
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc) {
                        const int ti = 16 * q + M::orow(l4, kc);
                        const int tj = 16 * p + l16;
                        const C a = (ti <= tj) ? wide_t(sm, ti, tj) : C(0);
                        nw[p] = M::mma(-a, w[q][kc], nw[p]);
                    }
            }
#pragma unroll
            for (int p = 0; p < 4; ++p) sl[p] += vcvt<SAcc<S, C>>(nw[p]);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                acc_t u = kMixed<S, C> ? acc_t{0, 0, 0, 0}
                                       : acc_t{(C)x[4 * r], (C)x[4 * r + 1], (C)x[4 * r + 2], (C)x[4 * r + 3]};
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc)
                        if (p >= r) u = M::mma(sm.Y[16 * r + l16][16 * p + M::orow(l4, kc)], nw[p][kc], u);
#pragma unroll
                for (int i = 0; i < 4; ++i) x[4 * r + i] = kMixed<S, C> ? x[4 * r + i] + (S)u[i] : (S)u[i];
            }
            if (colok) {
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) Bc[xrow(kk) * ldb + col] = x[kk];
            }
        }
        if (colok) {
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int i = 0; i < 4; ++i) pub_store(B + (sa + 16 * p + M::orow(l4, i)) * ldb + col, (S)sl[p][i]);
        }
        cur = i0;
    }
}

// Tree levels of Q^T for n = 64 with 64 columns per workgroup, as
// k_qt_tree64 (level-1 node per workgroup, then the last arrival performs a
// node), each wave owning a 16-column tile over all 64 slab rows as in
// k_chain_apply_w; a step's Y_node and T_node are staged in LDS.
// A node's reflector tails sit in the positions of a child's upper triangle
// (Sec. 2.1: the stacked-triangle QR), so the 16 x 16 tiles of Y_node below
// the block diagonal are exact zeros and their products are skipped (here
// and in k_node_apply_w); the results are the same bits.
template <typename S, typename C, int TW>
__global__ __launch_bounds__(64 * TW, TW == 4 ? 2 : 1) void k_qt_tree_w(Geom g, int ngroups, S* __restrict__ B, int64_t ldb,
                                                          int64_t k, const S* __restrict__ Ynode,
                                                          const S* __restrict__ Tnode, int* __restrict__ cnt) {
    constexpr int NT = 64 * TW, YS = 64 / TW;
    typedef Mfma<C> M;
    typedef typename M::acc acc_t;
    __shared__ WideSmemF<C> sm;
    __shared__ int s_old;
    const int node = blockIdx.x / ngroups;
    const int grp = blockIdx.x - node * ngroups;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const int64_t col = (int64_t)grp * (16 * TW) + 16 * wv + l16;
    const bool colok = col < k;
    auto xrow = [&](int kk) { return 16 * (kk >> 2) + M::orow(l4, kk & 3); };
    int cur = node * g.arity;
    if (cur >= g.W) return;
    // as in k_chain_apply_w: uniform row bases and 32-bit lane offsets when
    // every column of the workgroup lies inside B
    const bool colall = (int64_t)grp * (16 * TW) + 16 * TW <= k &&
                        (int64_t)(16 * ldb + k) * (int64_t)sizeof(S) < ((int64_t)1 << 31);
    uint32_t boff[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) boff[i] = (uint32_t)(((int64_t)M::orow(l4, i) * ldb + col) * (int64_t)sizeof(S));
    // -T is staged over the whole 64 x 64 square (entry i, j of thread
    // tid + NT u, i = e / 64, j = e % 64), zeros below the diagonal included:
    // a workgroup applies few steps, so no separate clearing pass
    constexpr int TSF = 4096 / NT;
    bool staged = false;  // LDS holds a previous step's operands
    for (int lev = 1; lev <= g.levels; ++lev) {
        const int64_t stride = ipow(g.arity, lev - 1);
        const int64_t span = stride * g.arity;
        const int i0 = (int)((cur / span) * span);
        int nch = (int)((g.W - i0 + stride - 1) / stride);
        if (nch > g.arity) nch = g.arity;
        if (nch <= 1) continue;  // unpaired: carried up unchanged
        if (lev > 1) {
            pub_wait();  // this workgroup's slab stores have landed
            __syncthreads();
            if (tid == 0) s_old = atomicAdd(cnt + (((int64_t)(lev - 2) * g.W + i0) * ngroups + grp), 1);
            __syncthreads();
            if (s_old != nch - 1) return;
        }
        const int64_t sa = chain_start(g, i0);
        SAcc<S, C> sl[4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (colall) sl[p][i] = pub_load_off(B + (sa + 16 * p) * ldb, boff[i]);
                else sl[p][i] = colok ? pub_load(B + (sa + 16 * p + M::orow(l4, i)) * ldb + col) : S(0);
            }
        for (int t = 1; t < nch; ++t) {
            const int64_t ch = i0 + t * stride;
            S* Bc = B + chain_start(g, (int)ch) * ldb;
            // stage Y_node (64 x 64, row-major) and T_node
            S ys[YS], ts[TSF];
            const S* Yc = Ynode + ch * 4096;
            const S* Tc = Tnode + ch * W_TRI;
#pragma unroll
            for (int u = 0; u < YS; ++u) ys[u] = Yc[(TW * u + wv) * 64 + lane];
#pragma unroll
            for (int u = 0; u < TSF; ++u) {
                const int e = tid + NT * u, i = e >> 6, j = e & 63;
                ts[u] = (i <= j) ? Tc[j * (j + 1) / 2 + i] : S(0);
            }
            S x[16];
            if (colall) {
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) x[kk] = pub_load_off(Bc + 16 * (kk >> 2) * ldb, boff[kk & 3]);
            } else {
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) x[kk] = colok ? pub_load(Bc + xrow(kk) * ldb + col) : S(0);
            }
            if (staged) __syncthreads();  // every wave is done with the previous step's operands
#pragma unroll
            for (int u = 0; u < YS; ++u) sm.Y[TW * u + wv][lane] = (C)ys[u];
#pragma unroll
            for (int u = 0; u < TSF; ++u) {
                const int e = tid + NT * u;
                sm.Tn[e >> 6][e & 63] = -(C)ts[u];
            }
            __syncthreads();
            staged = true;
            // W = S + Y^T X;  W' = T^T W (negated);  S -= W';  X -= Y W'
            acc_t w[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                w[p] = vcvt<acc_t>(sl[p]);
#pragma unroll
                for (int kk = 0; kk < 16; ++kk)
                    if ((kk >> 2) <= p) w[p] = M::mma(sm.Y[xrow(kk)][16 * p + l16], (C)x[kk], w[p]);
                if constexpr (TW == 4) __builtin_amdgcn_sched_barrier(0);
            }
            acc_t nw[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                nw[p] = acc_t{0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q <= p; ++q)
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc)
                        nw[p] = M::mma(sm.Tn[16 * q + M::orow(l4, kc)][16 * p + l16], w[q][kc], nw[p]);
                if constexpr (TW == 4) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int p = 0; p < 4; ++p) sl[p] += vcvt<SAcc<S, C>>(nw[p]);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                acc_t u = kMixed<S, C> ? acc_t{0, 0, 0, 0}
                                       : acc_t{(C)x[4 * r], (C)x[4 * r + 1], (C)x[4 * r + 2], (C)x[4 * r + 3]};
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc)
                        if (p >= r) u = M::mma(sm.Y[16 * r + l16][16 * p + M::orow(l4, kc)], nw[p][kc], u);
#pragma unroll
                for (int i = 0; i < 4; ++i) x[4 * r + i] = kMixed<S, C> ? x[4 * r + i] + (S)u[i] : (S)u[i];
                if constexpr (TW == 4) __builtin_amdgcn_sched_barrier(0);
            }
            if (colall) {
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) st_off(Bc + 16 * (kk >> 2) * ldb, boff[kk & 3], x[kk]);
            } else if (colok) {
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) Bc[xrow(kk) * ldb + col] = x[kk];
            }
        }
        if (colall) {
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int i = 0; i < 4; ++i) pub_store_off(B + (sa + 16 * p) * ldb, boff[i], (S)sl[p][i]);
        } else if (colok) {
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int i = 0; i < 4; ++i) pub_store(B + (sa + 16 * p + M::orow(l4, i)) * ldb + col, (S)sl[p][i]);
        }
        cur = i0;
    }
}

// One tree level of Q or the explicit Q for n = 64 with 16 TW columns per
// workgroup, as k_node_apply64 (the node's steps, last child first), each
// wave owning a 16-column tile over all 64 slab rows.
template <typename S, typename C, int MODE, int TW>
__global__ __launch_bounds__(64 * TW, 1) void k_node_apply_w(Geom g, int lev, int ngroups, S* __restrict__ B,
                                                             int64_t ldb, int64_t k, const S* __restrict__ Ynode,
                                                             const S* __restrict__ Tnode) {
    constexpr int NT = 64 * TW, YS = 64 / TW, TSN = (W_TRI + NT - 1) / NT;
    typedef Mfma<C> M;
    typedef typename M::acc acc_t;
    __shared__ WideSmem<C> sm;
    const int node = blockIdx.x / ngroups;
    const int grp = blockIdx.x - node * ngroups;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const int64_t col = (int64_t)grp * (16 * TW) + 16 * wv + l16;
    const bool colok = col < k;
    auto xrow = [&](int kk) { return 16 * (kk >> 2) + M::orow(l4, kk & 3); };
    const int64_t stride = ipow(g.arity, lev - 1);
    const int64_t i0 = (int64_t)node * g.arity * stride;
    int nch = (int)((g.W - i0 + stride - 1) / stride);
    if (nch > g.arity) nch = g.arity;
    if (nch <= 1) return;
    const int64_t sa = chain_start(g, (int)i0);
    SAcc<S, C> sl[4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int i = 0; i < 4; ++i) sl[p][i] = colok ? B[(sa + 16 * p + M::orow(l4, i)) * ldb + col] : S(0);
    bool staged = false;
    for (int t = nch - 1; t >= 1; --t) {
        const int64_t ch = i0 + t * stride;
        S* Bc = B + chain_start(g, (int)ch) * ldb;
        S ys[YS], ts[TSN];
        const S* Yc = Ynode + ch * 4096;
        const S* Tc = Tnode + ch * W_TRI;
#pragma unroll
        for (int u = 0; u < YS; ++u) ys[u] = Yc[(TW * u + wv) * 64 + lane];
#pragma unroll
        for (int u = 0; u < TSN; ++u) {
            const int e = tid + NT * u;
            ts[u] = (e < W_TRI) ? Tc[e] : S(0);
        }
        S x[16];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) x[kk] = (MODE != MODE_FORMQ && colok) ? Bc[xrow(kk) * ldb + col] : S(0);
        if (staged) __syncthreads();  // every wave is done with the previous step's operands
#pragma unroll
        for (int u = 0; u < YS; ++u) sm.Y[TW * u + wv][lane] = (C)ys[u];
#pragma unroll
        for (int u = 0; u < TSN; ++u) {
            const int e = tid + NT * u;
            if (e < W_TRI) sm.T[e] = (C)ts[u];
        }
        __syncthreads();
        staged = true;
        // W = S + Y^T X (X = 0 for the explicit Q);  W' = T W (negated);  S -= W';  X -= Y W'
        acc_t w[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            w[p] = vcvt<acc_t>(sl[p]);
            if (MODE != MODE_FORMQ) {
#pragma unroll
                for (int kk = 0; kk < 16; ++kk)
                    if ((kk >> 2) <= p) w[p] = M::mma(sm.Y[xrow(kk)][16 * p + l16], (C)x[kk], w[p]);
            }
        }
        acc_t nw[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            nw[p] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int q = p; q < 4; ++q)
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) {
                    const int ti = 16 * q + M::orow(l4, kc);
                    const int tj = 16 * p + l16;
                    const C a = (tj <= ti) ? wide_t(sm, tj, ti) : C(0);
                    nw[p] = M::mma(-a, w[q][kc], nw[p]);
                }
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) sl[p] += vcvt<SAcc<S, C>>(nw[p]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            acc_t u = kMixed<S, C> ? acc_t{0, 0, 0, 0}
                                       : acc_t{(C)x[4 * r], (C)x[4 * r + 1], (C)x[4 * r + 2], (C)x[4 * r + 3]};
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int kc = 0; kc < 4; ++kc)
                    if (p >= r) u = M::mma(sm.Y[16 * r + l16][16 * p + M::orow(l4, kc)], nw[p][kc], u);
#pragma unroll
            for (int i = 0; i < 4; ++i) x[4 * r + i] = kMixed<S, C> ? x[4 * r + i] + (S)u[i] : (S)u[i];
        }
        if (colok) {
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) Bc[xrow(kk) * ldb + col] = x[kk];
        }
    }
    if (colok) {
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int i = 0; i < 4; ++i) B[(sa + 16 * p + M::orow(l4, i)) * ldb + col] = (S)sl[p][i];
    }
}

// The explicit Q's tree levels (binary tree, n = 64) in one launch.  Top
// down, a node's step maps its slab S to its children's slabs: with the
// children's rows zero (the explicit Q starts from [I_n; 0]), child 0 gets
// S - W' and child 1 gets -Y W', W' = T S.  So the slab arriving at a level-1
// node depends only on the steps along the path from the member's root, and
// each workgroup (level-1 node, 16 TW columns) recomputes its own path from
// S = I: every step along a path is the same arithmetic as in
// k_node_apply_w, so the slabs are the same bits, and the ten levels cost
// ten steps of one workgroup instead of ten dependent launches.  Only the
// level-1 slabs are written (the two chains' top rows), so no workgroup
// reads what another writes.
template <typename S, typename C, int TW>
__global__ __launch_bounds__(64 * TW, 2) void k_formq_paths_w(Geom g, int ngroups, S* __restrict__ B, int64_t ldb,
                                                              int64_t k, const S* __restrict__ Ynode,
                                                              const S* __restrict__ Tnode, const S* __restrict__ sgnR,
                                                              int64_t sgn_ldr, int64_t sgn_sr) {
    constexpr int NT = 64 * TW, YS = 64 / TW, TSN = (W_TRI + NT - 1) / NT;
    typedef Mfma<C> M;
    typedef typename M::acc acc_t;
    __shared__ WideSmem<C> sm;
    const int node1 = blockIdx.x / ngroups;
    const int grp = blockIdx.x - node1 * ngroups;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const int64_t col = (int64_t)grp * (16 * TW) + 16 * wv + l16;
    const bool colok = col < k;
    auto xrow = [&](int kk) { return 16 * (kk >> 2) + M::orow(l4, kk & 3); };
    const int c1 = 2 * node1;
    if (c1 >= g.W) return;
    // the member's root slab: I_n, or D = diag(sign R_jj) (sign(0) = +1);
    // D's entries are +-1, so every later step gives the bits of I_n's
    // result with column j negated where d_j = -1
    S dcol = S(1);
    if (sgnR && colok && sgnR[(int64_t)(c1 / g.cpm) * sgn_sr + col * sgn_ldr + col] < S(0)) dcol = S(-1);
    SAcc<S, C> sl[4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int i = 0; i < 4; ++i) sl[p][i] = (16 * p + M::orow(l4, i) == col) ? dcol : S(0);
    bool staged = false;
    for (int lev = g.levels; lev >= 1; --lev) {
        const int64_t stride = ipow(2, lev - 1), span = 2 * stride;
        const int64_t i0 = (c1 / span) * span;
        const int nch = (g.W - i0 > stride) ? 2 : 1;
        const int t = (int)((c1 - i0) / stride);  // the child on this path (0 at level 1)
        if (nch == 1) {
            if (lev == 1 && colok) {
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        B[(chain_start(g, c1) + 16 * p + M::orow(l4, i)) * ldb + col] = (S)sl[p][i];
            }
            continue;  // unpaired: carried down unchanged
        }
        const int64_t ch = i0 + stride;
        S ys[YS], ts[TSN];
        const S* Yc = Ynode + ch * 4096;
        const S* Tc = Tnode + ch * W_TRI;
#pragma unroll
        for (int u = 0; u < YS; ++u) ys[u] = Yc[(TW * u + wv) * 64 + lane];
#pragma unroll
        for (int u = 0; u < TSN; ++u) {
            const int e = tid + NT * u;
            ts[u] = (e < W_TRI) ? Tc[e] : S(0);
        }
        if (staged) __syncthreads();  // every wave is done with the previous step's operands
#pragma unroll
        for (int u = 0; u < YS; ++u) sm.Y[TW * u + wv][lane] = (C)ys[u];
#pragma unroll
        for (int u = 0; u < TSN; ++u) {
            const int e = tid + NT * u;
            if (e < W_TRI) sm.T[e] = (C)ts[u];
        }
        __syncthreads();
        staged = true;
        // W = S;  W' = T W (negated)
        acc_t w[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) w[p] = vcvt<acc_t>(sl[p]);
        acc_t nw[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            nw[p] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int q = p; q < 4; ++q)
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) {
                    const int ti = 16 * q + M::orow(l4, kc);
                    const int tj = 16 * p + l16;
                    const C a = (tj <= ti) ? wide_t(sm, tj, ti) : C(0);
                    nw[p] = M::mma(-a, w[q][kc], nw[p]);
                }
        }
        // child 1: X = -Y W' (the product of k_node_apply_w with X = 0)
        S x[16];
        const bool want1 = (lev == 1) || (t == 1);
        if (want1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                acc_t u = acc_t{0, 0, 0, 0};
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc)
                        if (p >= r) u = M::mma(sm.Y[16 * r + l16][16 * p + M::orow(l4, kc)], nw[p][kc], u);
#pragma unroll
                for (int i = 0; i < 4; ++i) x[4 * r + i] = kMixed<S, C> ? S(0) + (S)u[i] : (S)u[i];
            }
        }
        // child 0: S - W'
#pragma unroll
        for (int p = 0; p < 4; ++p) sl[p] += vcvt<SAcc<S, C>>(nw[p]);
        if (lev == 1) {
            if (colok) {
                S* B0 = B + chain_start(g, c1) * ldb;
                S* B1 = B + chain_start(g, c1 + 1) * ldb;
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int i = 0; i < 4; ++i) B0[(16 * p + M::orow(l4, i)) * ldb + col] = (S)sl[p][i];
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) B1[xrow(kk) * ldb + col] = x[kk];
            }
        } else if (t == 1) {
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int i = 0; i < 4; ++i) sl[p][i] = x[4 * p + i];
        }
    }
}

__global__ void k_apply_zero(int* __restrict__ p, int64_t count) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = 0;
}

template <typename T>
__global__ void k_init_formq(int64_t n, int64_t mb, T* __restrict__ Q, int64_t ldq, const T* __restrict__ sgnR,
                             int64_t sgn_ldr, int64_t sgn_sr) {
    // member blockIdx.y's root slab: I_n, or D = diag(sign R_jj) (sign(0) = +1)
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int64_t i = e / n, j = e - i * n;
    T d = T(1);
    if (i == j && sgnR && sgnR[(int64_t)blockIdx.y * sgn_sr + j * sgn_ldr + j] < T(0)) d = T(-1);
    Q[((int64_t)blockIdx.y * mb + i) * ldq + j] = (i == j) ? d : T(0);
}

// Layout of an apply with n = 64: the wide kernels (a 16-column tile over all
// 64 rows per wave) hold one workgroup per CU; when that gives fewer
// workgroups than CUs (few chains and few columns, e.g. the update of the
// next panel's 64 columns in CAQR), the narrow kernels' four times as many
// workgroups finish sooner.  One decision per apply (chains, tree levels).
static bool use_wide(const Geom& g, int64_t k) {
    if (g.n != 64 || k <= 16) return false;
    const int64_t tw = k <= 32 ? 2 : 4;
    return (int64_t)g.W * ((k + 16 * tw - 1) / (16 * tw)) >= 256;
}

bool apply_wide(const Geom& g, int64_t k) { return use_wide(g, k); }

template <typename S, typename C, int NC, int H, int MODE>
static hipError_t chain_apply_launch(const Geom& g, const S* Y, int64_t ldy, const Work& wk, S* B, int64_t ldb,
                                     int64_t k, hipStream_t st) {
    const int ntiles = (int)((k + 15) / 16);
    const int groups = (g.W + 7) / 8;
    const int64_t grid = (int64_t)groups * 8 * ntiles;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    constexpr int NP = NC <= 16 ? 1 : NC / 16;
    phase_begin(1 + MODE, st);
    static_assert(H == 64, "the chain kernel takes 64-row blocks");
    if constexpr (NP == 4) {
        if (use_wide(g, k)) {
            // 16 TW columns per workgroup, TW = 2 or 4 waves
            const int tw = k <= 32 ? 2 : 4;
            const int ngroups = (int)((k + 16 * tw - 1) / (16 * tw));
            const int64_t gw = (int64_t)groups * 8 * ngroups;
            const S* Tb = (const S*)wk.T_blk;
            if (tw == 4)
                k_chain_apply_w<S, C, MODE, 4><<<(int)gw, 256, 0, st>>>(g, Y, ldy, Tb, B, ldb, k, ngroups);
            else
                k_chain_apply_w<S, C, MODE, 2><<<(int)gw, 128, 0, st>>>(g, Y, ldy, Tb, B, ldb, k, ngroups);
            phase_end(1 + MODE, st);
            return hipGetLastError();
        }
    }
    k_chain_apply64<S, C, NP, MODE><<<(int)grid, 256, 0, st>>>(g, Y, ldy, (const S*)wk.T_blk, B, ldb, k, ntiles);
    phase_end(1 + MODE, st);
    return hipGetLastError();
}

// All tree levels of Q^T in one launch; arrival counts (levels above the
// first) live in a stream-ordered allocation cleared by a fill kernel.
template <typename S, typename C, int NC>
static hipError_t qt_tree_launch(const Geom& g, const Work& wk, S* B, int64_t ldb, int64_t k, hipStream_t st) {
    if (g.levels == 0) return hipSuccess;
    constexpr int NP = NC <= 16 ? 1 : NC / 16;
    const bool wide = NP == 4 && use_wide(g, k);
    const int tw = k <= 32 ? 2 : 4;  // waves (16-column tiles) per workgroup of the wide kernel
    const int ntiles = wide ? (int)((k + 16 * tw - 1) / (16 * tw)) : (int)((k + 15) / 16);  // column groups
    const int64_t nodes = (g.W + g.arity - 1) / g.arity;
    int* cnt = nullptr;
    const int64_t ncnt = (int64_t)g.W * (g.levels > 1 ? g.levels - 1 : 1) * ntiles;
    hipError_t e = ws_malloc((void**)&cnt, (size_t)ncnt * sizeof(int), st);
    if (e != hipSuccess) return e;
    k_apply_zero<<<(unsigned)((ncnt + 255) / 256), 256, 0, st>>>(cnt, ncnt);
    const S *Yn = (const S*)wk.Ynode, *Tn = (const S*)wk.Tnode;
    const unsigned gridt = (unsigned)(nodes * ntiles);
    if (wide && tw == 4)
        k_qt_tree_w<S, C, 4><<<gridt, 256, 0, st>>>(g, ntiles, B, ldb, k, Yn, Tn, cnt);
    else if (wide)
        k_qt_tree_w2<S, C, 2><<<gridt, 128, 0, st>>>(g, ntiles, B, ldb, k, Yn, Tn, cnt);
    else
        k_qt_tree64<S, C, NP><<<(unsigned)(nodes * ntiles), 256, 0, st>>>(g, ntiles, B, ldb, k, (const S*)wk.Ynode,
                                                                           (const S*)wk.Tnode, cnt);
    e = hipGetLastError();
    hipError_t e2 = hipFreeAsync(cnt, st);
    return e != hipSuccess ? e : e2;
}

// One tree level of Q (explicit Q or Q*B; Sec. 2.1, the tree of Q factors
// applied top-down): workgroup (node, tile) applies the node's steps, last
// child first, to [slab of child 0; slab of child t] for one 16-column tile.
// For the explicit Q the slabs of children t >= 1 are still zero here.
template <typename S, typename C, int NP, int MODE>
__global__ __launch_bounds__(256, 2) void k_node_apply64(Geom g, int lev, int ntiles, S* __restrict__ B,
                                                         int64_t ldb, int64_t k, const S* __restrict__ Ynode,
                                                         const S* __restrict__ Tnode) {
    typedef Mfma<C> M;
    __shared__ Apply64Smem<S, C, NP> sm;
    const int node = blockIdx.x / ntiles;
    const int tile = blockIdx.x - node * ntiles;
    const int n = (int)g.n;
    const int64_t tri = (int64_t)n * (n + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
    const int64_t col = (int64_t)tile * 16 + l16;
    const bool colok = col < k;
    const int64_t stride = ipow(g.arity, lev - 1);
    const int64_t i0 = (int64_t)node * g.arity * stride;
    int nch = (int)((g.W - i0 + stride - 1) / stride);
    if (nch > g.arity) nch = g.arity;
    if (nch <= 1) return;
    const int64_t sa = chain_start(g, (int)i0);
    S sl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = 16 * wv + M::orow(l4, i);
        sl[i] = (wv < NP && j < n && colok) ? B[(sa + j) * ldb + col] : S(0);
    }
    for (int t = nch - 1; t >= 1; --t) {
        const int64_t ch = i0 + t * stride;
        S* Bc = B + chain_start(g, (int)ch) * ldb;
        Apply64Regs<S, C, NP, MODE> R;
        apply64_load<S, C, NP, MODE>(R, wv, l16, l4, n, Ynode + ch * n * n, n, Tnode + ch * tri, Bc, ldb, 0, n, false,
                                     col, colok);
        apply64_block<S, C, NP, MODE>(sm, R, sl, wv, l16, l4, n, Bc, ldb, 0, n, false, col, colok);
    }
    if (wv < NP) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = 16 * wv + M::orow(l4, i);
            if (j < n && colok) B[(sa + j) * ldb + col] = sl[i];
        }
    }
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
    constexpr int NP = NC <= 16 ? 1 : NC / 16;
    if constexpr (NP == 4) {
        if (use_wide(g, k)) {
            const int tw = k <= 32 ? 2 : 4;
            const int ngroups = (int)((k + 16 * tw - 1) / (16 * tw));
            const unsigned gw = (unsigned)(nodes * ngroups);
            const S *Yn = (const S*)wk.Ynode, *Tn = (const S*)wk.Tnode;
            if (tw == 4)
                k_node_apply_w<S, C, MODE, 4><<<gw, 256, 0, st>>>(g, lev, ngroups, B, ldb, k, Yn, Tn);
            else
                k_node_apply_w<S, C, MODE, 2><<<gw, 128, 0, st>>>(g, lev, ngroups, B, ldb, k, Yn, Tn);
            return hipGetLastError();
        }
    }
    k_node_apply64<S, C, NP, MODE><<<(int)grid, 256, 0, st>>>(g, lev, ntiles, B, ldb, k, (const S*)wk.Ynode,
                                                              (const S*)wk.Tnode);
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
        if (e == hipSuccess) e = qt_tree_launch<S, C, NC>(g, wk, B, ldb, k, st);
    } else {
        bool done = false;
        if constexpr (MODE == MODE_FORMQ && NC == 64 && !kMixed<S, C>) {
            // the explicit Q's binary tree: every level in one launch (paths)
            if (g.levels >= 1 && g.arity == 2 && use_wide(g, k) && k > 32) {
                const int ngroups = (int)((k + 63) / 64);
                const int64_t gw = (int64_t)((g.W + 1) / 2) * ngroups;
                if (gw > 0x7fffffff) return hipErrorInvalidValue;
                k_formq_paths_w<S, C, 4><<<(unsigned)gw, 256, 0, st>>>(g, ngroups, B, ldb, k, (const S*)wk.Ynode,
                                                                       (const S*)wk.Tnode, (const S*)wk.sgnR,
                                                                       wk.sgn_ldr, wk.sgn_sr);
                e = hipGetLastError();
                done = true;
            }
        }
        for (int lev = g.levels; !done && lev >= 1 && e == hipSuccess; --lev)
            e = node_apply_launch<S, C, NC, MODE>(g, lev, wk, B, ldb, k, st);
        if (e == hipSuccess) e = chain_apply_h<S, C, NC, MODE>(g, Y, ldy, wk, B, ldb, k, st);
    }
    return e;
}

template <typename S, typename C, int NC>
static hipError_t apply_nc(const Geom& g, const S* Y, int64_t ldy, const Work& wk, S* B, int64_t ldb, int64_t k,
                           int mode, hipStream_t st) {
    if constexpr (kMixed<S, C>) {
        // FP32 products on FP64 storage: the trailing update (Q^T) only
        if (mode != MODE_QT) return hipErrorInvalidValue;
        return apply_mode<S, C, NC, MODE_QT>(g, Y, ldy, wk, B, ldb, k, st);
    } else {
        switch (mode) {
            case MODE_QT: return apply_mode<S, C, NC, MODE_QT>(g, Y, ldy, wk, B, ldb, k, st);
            case MODE_Q: return apply_mode<S, C, NC, MODE_Q>(g, Y, ldy, wk, B, ldb, k, st);
            case MODE_FORMQ: return apply_mode<S, C, NC, MODE_FORMQ>(g, Y, ldy, wk, B, ldb, k, st);
            default: return hipErrorInvalidValue;
        }
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

hipError_t launch_init_formq(bool f64, int64_t members, int64_t mb, int64_t n, void* Q, int64_t ldq, const void* sgnR,
                             int64_t sgn_ldr, int64_t sgn_sr, hipStream_t st) {
    if (members < 1 || members > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n * n + 255) / 256), (unsigned)members);
    if (f64)
        k_init_formq<double><<<grid, 256, 0, st>>>(n, mb, (double*)Q, ldq, (const double*)sgnR, sgn_ldr, sgn_sr);
    else
        k_init_formq<float><<<grid, 256, 0, st>>>(n, mb, (float*)Q, ldq, (const float*)sgnR, sgn_ldr, sgn_sr);
    return hipGetLastError();
}

}  // namespace tsqr
