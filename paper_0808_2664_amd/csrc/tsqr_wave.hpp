// One-wave Householder engine of the TSQR kernels (gfx950, wave64).
//
// A single wave owns one chain of row blocks (the flat tree of sequential
// TSQR, Sec. 2.1) and, on the reduction tree, the nodes it reaches last.  No
// workgroup barrier is ever taken: every reduction is a lane exchange inside
// the wave, so the 8 XCDs x 32 CUs run up to 8 independent chains per CU and
// the latency of one chain's column steps is hidden by the others.
//
// Register tile (the MFMA operand layout).  A block of 16*SG rows (SG = 4:
// 64-row blocks, so a lane holds at most 64 entries of an n <= 64 tile) and
// NCP = 16*NP columns sits in x[s][i][q]: lane l holds column 16q + l%16 of row
// 16s + orow(l/16, i).  Column c therefore lives in the 4 lanes l%16 == c%16 of
// one register group, and its reductions are one DPP broadcast per register
// plus two lane swaps (v_permlane16/32_swap).
//
// Local QR of one block (wave_block): blocked Householder QR in panels of 16
// columns.  Reflectors follow Sec. 5.2 (unit topmost entry): for column j,
// beta = -sign(alpha)||x||, sign(0) = +1, tau = (beta - alpha)/beta, and
// tau = 0 when the tail below the head is zero.  A panel is reduced column by
// column with one lane reduction per column: g_c = sum over the tail rows of
// x_j x_c for every column c at once gives sigma^2 = g_j and
// v_j^T x_c = head_c + scale_j g_c.  The panel then updates the trailing
// columns as the block reflector I - V T V^T (the compact form cited in
// Sec. 2.1 and used by the trailing update of Sec. 3.1): W = V^T X,
// W' = T^T W and X -= V W' are three MFMA products.  T is the forward
// block-reflector factor, upper triangular, grown panel by panel
// (T12 = -T11 (V1^T V2) T22): the panel's diagonal block is built during the
// column sweep from the in-panel Gram entries, the off-diagonal blocks by MFMA
// from the Gram blocks V_q^T V_p that the W product yields.
//
// Three block kinds (MODE):
//   0  first block of a chain: the heads lie inside the tile (rows < n);
//   1  a block stacked under the on-chip R of its chain (heads = R rows);
//   2  a tree node: the tile is a child's upper triangular R, stacked under
//      the node's R (Sec. 2.1, Eqs. TSQR_binarytree_2/3).  Row group s of the
//      tile is zero in panels p < s, so panel p works on groups 0..p only and
//      the zeros of the triangle stay exact.
// The on-chip R (packed upper triangle) and a 16 x 17 staging tile are the
// wave's only LDS.
#pragma once
#include <type_traits>

#include "tsqr_common.hpp"

namespace tsqr {
using namespace dev;

template <int I>
using ic_t = std::integral_constant<int, I>;

// Compile-time loop: f(ic_t<B>), ..., f(ic_t<E-1>).
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
    if constexpr (B < E) {
        f(ic_t<B>{});
        sfor<B + 1, E>(static_cast<F&&>(f));
    }
}

// ---- lane helpers -----------------------------------------------------------
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
// Sum over the 4 lanes {l%16 + 16k}; the four lanes get the same bits (each
// stage adds the same two operands in the same order).
template <typename T>
__device__ __forceinline__ T sum4(T x) {
    return swapsum(swapsum(x, true), false);
}
// Value of lane J of this lane's 16-lane row (DPP row_newbcast).
// Every lane is written, so no old value is needed.
template <int J>
__device__ __forceinline__ double bcast16(double x) {
    long long v = __builtin_bit_cast(long long, x);
    v = __builtin_amdgcn_mov_dpp(v, 0x150 + J, 0xF, 0xF, true);
    return __builtin_bit_cast(double, v);
}
template <int J>
__device__ __forceinline__ float bcast16(float x) {
    int v = __builtin_bit_cast(int, x);
    v = __builtin_amdgcn_mov_dpp(v, 0x150 + J, 0xF, 0xF, true);
    return __builtin_bit_cast(float, v);
}
// Value of lane L (wave-uniform).
template <int L>
__device__ __forceinline__ double rdlane(double x) {
    struct P { int lo, hi; };
    P p = __builtin_bit_cast(P, x);
    p.lo = __builtin_amdgcn_readlane(p.lo, L);
    p.hi = __builtin_amdgcn_readlane(p.hi, L);
    return __builtin_bit_cast(double, p);
}
template <int L>
__device__ __forceinline__ float rdlane(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), L));
}

// The lane id and n, made opaque to the optimiser.  The sweep is fully
// unrolled; without this the compiler hoists every column's lane masks and
// bounds out of the sweep and runs out of scalar registers holding them.
__device__ __forceinline__ int lane_id() {
    int l = threadIdx.x & 63;
    asm volatile("" : "+v"(l));
    return l;
}
__device__ __forceinline__ int opaque_s(int v) {
    asm volatile("" : "+s"(v));
    return v;
}

// ---- FMA with a broadcast operand -----------------------------------------------
// The column sweep multiplies every value of a lane by the value of column jj
// in the same row (DPP row_newbcast).  The compiler emits the broadcast as a
// separate move for 64-bit operands; v_fmac with a DPP source does both in
// one instruction.  These are written out here for the unmasked row groups
// [0, NS) of one panel tile x[.][.][L]:
//   dot_bc:  a[i] += bcast(x[s][i]) * x[s][i]   (s ascending; the sums of the
//            plain code, bit for bit)
//   upd_bc:  x[s][i] += bcast(x[s][i]) * coef   (in place: lane J of each row
//            has coef = 0, so the value it broadcasts is the same before and
//            after the write)
// Hazards the compiler does not see through inline asm are covered by the
// leading s_nop: a DPP read needs 2 wait states after a VALU write of any of
// its VGPRs and 5 after an EXEC write; the first column of a sweep (GUARD)
// follows the block-reflector products, whose MFMA results need 18 before a
// VALU reads them.  Inside one statement an accumulator is rewritten every
// fourth instruction (>= 2 wait states).  Every value written here is
// rewritten by compiler-visible VALU code (the sweep's final scaling) before
// an MFMA or a store reads it.
#define TSQR_DPP " row_newbcast:%c[J] row_mask:0xf bank_mask:0xf\n\t"
#define TSQR_NOP_GUARD "s_nop 7\n\ts_nop 7\n\ts_nop 7\n\t"
#define TSQR_NOP "s_nop 4\n\t"
#define TSQR_DOT4(OP, s) \
    OP " %[a0], %[x" #s "0], %[x" #s "0]" TSQR_DPP OP " %[a1], %[x" #s "1], %[x" #s "1]" TSQR_DPP \
    OP " %[a2], %[x" #s "2], %[x" #s "2]" TSQR_DPP OP " %[a3], %[x" #s "3], %[x" #s "3]" TSQR_DPP
#define TSQR_UPD4(OP, s) \
    OP " %[x" #s "0], %[x" #s "0], %[cf]" TSQR_DPP OP " %[x" #s "1], %[x" #s "1], %[cf]" TSQR_DPP \
    OP " %[x" #s "2], %[x" #s "2], %[cf]" TSQR_DPP OP " %[x" #s "3], %[x" #s "3], %[cf]" TSQR_DPP
#define TSQR_XI(s, L) \
    [x##s##0] "v"(x[s][0][L]), [x##s##1] "v"(x[s][1][L]), [x##s##2] "v"(x[s][2][L]), [x##s##3] "v"(x[s][3][L])
#define TSQR_XO(s, L) \
    [x##s##0] "+v"(x[s][0][L]), [x##s##1] "+v"(x[s][1][L]), [x##s##2] "+v"(x[s][2][L]), [x##s##3] "+v"(x[s][3][L])
#define TSQR_ACC [a0] "+v"(a[0]), [a1] "+v"(a[1]), [a2] "+v"(a[2]), [a3] "+v"(a[3])

#define TSQR_DOT_BODY(OP, NOPS)                                                                                    \
    if constexpr (NS == 1)                                                                                         \
        asm(NOPS TSQR_DOT4(OP, 0) : TSQR_ACC : TSQR_XI(0, L), [J] "n"(J));                                         \
    else if constexpr (NS == 2)                                                                                    \
        asm(NOPS TSQR_DOT4(OP, 0) TSQR_DOT4(OP, 1) : TSQR_ACC : TSQR_XI(0, L), TSQR_XI(1, L), [J] "n"(J));        \
    else if constexpr (NS == 3)                                                                                    \
        asm(NOPS TSQR_DOT4(OP, 0) TSQR_DOT4(OP, 1) TSQR_DOT4(OP, 2)                                               \
            : TSQR_ACC : TSQR_XI(0, L), TSQR_XI(1, L), TSQR_XI(2, L), [J] "n"(J));                                 \
    else                                                                                                           \
        asm(NOPS TSQR_DOT4(OP, 0) TSQR_DOT4(OP, 1) TSQR_DOT4(OP, 2) TSQR_DOT4(OP, 3)                              \
            : TSQR_ACC : TSQR_XI(0, L), TSQR_XI(1, L), TSQR_XI(2, L), TSQR_XI(3, L), [J] "n"(J));
#define TSQR_UPD_BODY(OP)                                                                                          \
    if constexpr (NS == 1)                                                                                         \
        asm(TSQR_NOP TSQR_UPD4(OP, 0) : TSQR_XO(0, L) : [cf] "v"(coef), [J] "n"(J));                               \
    else if constexpr (NS == 2)                                                                                    \
        asm(TSQR_NOP TSQR_UPD4(OP, 0) TSQR_UPD4(OP, 1) : TSQR_XO(0, L), TSQR_XO(1, L) : [cf] "v"(coef), [J] "n"(J)); \
    else if constexpr (NS == 3)                                                                                    \
        asm(TSQR_NOP TSQR_UPD4(OP, 0) TSQR_UPD4(OP, 1) TSQR_UPD4(OP, 2)                                           \
            : TSQR_XO(0, L), TSQR_XO(1, L), TSQR_XO(2, L) : [cf] "v"(coef), [J] "n"(J));                           \
    else                                                                                                           \
        asm(TSQR_NOP TSQR_UPD4(OP, 0) TSQR_UPD4(OP, 1) TSQR_UPD4(OP, 2) TSQR_UPD4(OP, 3)                          \
            : TSQR_XO(0, L), TSQR_XO(1, L), TSQR_XO(2, L), TSQR_XO(3, L) : [cf] "v"(coef), [J] "n"(J));

template <int J, int NS, int L, bool GUARD, int SGX, int NPX>
__device__ __forceinline__ void dot_bc(double (&a)[4], const double (&x)[SGX][4][NPX]) {
    static_assert(NS >= 1 && NS <= SGX && SGX <= 4, "row groups");
    if constexpr (GUARD) {
        TSQR_DOT_BODY("v_fmac_f64_dpp", TSQR_NOP_GUARD)
    } else {
        TSQR_DOT_BODY("v_fmac_f64_dpp", TSQR_NOP)
    }
}
template <int J, int NS, int L, bool GUARD, int SGX, int NPX>
__device__ __forceinline__ void dot_bc(float (&a)[4], const float (&x)[SGX][4][NPX]) {
    static_assert(NS >= 1 && NS <= SGX && SGX <= 4, "row groups");
    if constexpr (GUARD) {
        TSQR_DOT_BODY("v_fmac_f32_dpp", TSQR_NOP_GUARD)
    } else {
        TSQR_DOT_BODY("v_fmac_f32_dpp", TSQR_NOP)
    }
}
template <int J, int NS, int L, int SGX, int NPX>
__device__ __forceinline__ void upd_bc(double (&x)[SGX][4][NPX], double coef) {
    static_assert(NS >= 1 && NS <= SGX && SGX <= 4, "row groups");
    TSQR_UPD_BODY("v_fmac_f64_dpp")
}
template <int J, int NS, int L, int SGX, int NPX>
__device__ __forceinline__ void upd_bc(float (&x)[SGX][4][NPX], float coef) {
    static_assert(NS >= 1 && NS <= SGX && SGX <= 4, "row groups");
    TSQR_UPD_BODY("v_fmac_f32_dpp")
}
// acc += bcast(a)[lane J] * b, one term of a sum whose running sums
// alternate: the leading wait states cover a VALU write of any operand one
// instruction earlier (2) and, for the first term (FIRST), an EXEC write (5).
template <int J, bool FIRST>
__device__ __forceinline__ void fmac_bc(double& acc, double a, double b) {
    if constexpr (FIRST)
        asm("s_nop 4\n\tv_fmac_f64_dpp %0, %1, %2" TSQR_DPP : "+v"(acc) : "v"(a), "v"(b), [J] "n"(J));
    else
        asm("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2" TSQR_DPP : "+v"(acc) : "v"(a), "v"(b), [J] "n"(J));
}
template <int J, bool FIRST>
__device__ __forceinline__ void fmac_bc(float& acc, float a, float b) {
    if constexpr (FIRST)
        asm("s_nop 4\n\tv_fmac_f32_dpp %0, %1, %2" TSQR_DPP : "+v"(acc) : "v"(a), "v"(b), [J] "n"(J));
    else
        asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2" TSQR_DPP : "+v"(acc) : "v"(a), "v"(b), [J] "n"(J));
}
#undef TSQR_DOT_BODY
#undef TSQR_UPD_BODY
#undef TSQR_ACC
#undef TSQR_XO
#undef TSQR_XI
#undef TSQR_UPD4
#undef TSQR_DOT4
#undef TSQR_NOP
#undef TSQR_NOP_GUARD
#undef TSQR_DPP

// Order this wave's LDS (and global) accesses across its lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Householder scalars from alpha and sigma^2 = ||tail||^2 (valid for
// sigma^2 > 0; the caller replaces them when sigma^2 == 0):
// nrm = sqrt(alpha^2 + sigma^2), beta = -sign(alpha) nrm (sign(0) = +1),
// tau = (beta - alpha)/beta = 1 + |alpha|/nrm, scale = 1/(alpha - beta), and
// rbeta = 1/beta = -tau * scale, the factor that takes v^T x to the update
// coefficient of the scaled tail (-tau (v^T x) scale).
// The hardware reciprocal square root and reciprocal are refined by one
// third-order step each, y0 (1 + e/2 + 3e^2/8) with e = 1 - s y0^2 and
// r0 (1 + e + e^2) with e = 1 - d r0 (from about 22 correct bits to full
// precision; fewer dependent operations than two Newton steps, and this
// chain is the latency of every column of the sweep).  alpha - beta never
// cancels: both terms carry the sign of alpha.
__device__ __forceinline__ void hh_scalars(double alpha, double sigma2, double& beta, double& tau, double& scale,
                                           double& rbeta) {
    const double s = fma(alpha, alpha, sigma2);
    const double y0 = __builtin_amdgcn_rsq(s);
    const double e = fma(-s * y0, y0, 1.0);
    const double y = fma(y0, e * fma(e, 0.375, 0.5), y0);
    double nrm = s * y;
    nrm = fma(fma(-nrm, nrm, s), 0.5 * y, nrm);
    const bool pos = alpha >= 0.0;
    beta = pos ? -nrm : nrm;
    rbeta = pos ? -y : y;
    tau = fma(fabs(alpha), y, 1.0);
    const double d = alpha - beta;
    const double r0 = __builtin_amdgcn_rcp(d);
    const double e2 = fma(-d, r0, 1.0);
    scale = fma(r0, fma(e2, e2, e2), r0);
}
__device__ __forceinline__ void hh_scalars(float alpha, float sigma2, float& beta, float& tau, float& scale,
                                           float& rbeta) {
    const float s = fmaf(alpha, alpha, sigma2);
    float y = __builtin_amdgcn_rsqf(s);
    y = fmaf(0.5f * y, fmaf(-s * y, y, 1.0f), y);
    float nrm = s * y;
    nrm = fmaf(fmaf(-nrm, nrm, s), 0.5f * y, nrm);
    const bool pos = alpha >= 0.0f;
    beta = pos ? -nrm : nrm;
    rbeta = pos ? -y : y;
    tau = fmaf(fabsf(alpha), y, 1.0f);
    const float d = alpha - beta;
    float r = __builtin_amdgcn_rcpf(d);
    scale = fmaf(r, fmaf(-d, r, 1.0f), r);
}

// ---- per-wave LDS -------------------------------------------------------------
template <typename T, int NP>
struct WSmem {
    static constexpr int NCP = 16 * NP;
    static constexpr int RP = NCP * (NCP + 1) / 2;
    T R[RP];            // on-chip R, upper triangle packed by rows
    T scr[16][17];      // transposes; the column sweep's sink for stores without a target
    T td[NP][16][17];   // diagonal T blocks of the panels (row l of block p in td[p][l]);
                        // entries below the diagonal stay zero
    T scl[16];          // scales of the current panel's columns
    T zero;             // holds 0
};
// Packed index of R[r][c], c >= r, rows of length NCP.
template <int NCP>
__host__ __device__ constexpr int rpi(int r, int c) {
    return r * NCP - ((r * (r - 1)) >> 1) + (c - r);
}

// Entry of a reflector as a matrix operand when the heads lie in the tile:
// zero above the head row, one on it.
template <typename T>
__device__ __forceinline__ T vmask(T x, int r, int c) {
    return (r > c) ? x : ((r == c) ? T(1) : T(0));
}

// Packed-T index of T[i][j], i <= j (column by column).
__device__ __forceinline__ int64_t tpi(int i, int j) { return (int64_t)j * (j + 1) / 2 + i; }

// ---- the column sweep of one panel -------------------------------------------------
//
// Panel p (columns 16p .. 16p + 15) of a block held in x[.][.][L] (tile
// layout), reduced column by column with one lane reduction per column:
// g_c = sum over the tail rows of x_j x_c for every column c at once gives
// sigma^2 = g_j and v_j^T x_c = head_c + scale_j g_c.  MODE 0: the heads lie
// in the tile (row group p; row groups [p, SG) are live); otherwise the heads
// are rows of the on-chip R (packed rows of NCP columns at R) and row groups
// [0, S1) of the tile are live (a tree node's lower triangle has S1 = p + 1).
// Columns j >= n are not skipped: they are zero, so the arithmetic leaves
// the tile unchanged (sigma^2 = 0, tau = 0, coef = 0) and no value has to be
// merged across a branch.
//
// On return the panel's tails are the scaled reflector tails, td holds the
// panel's diagonal T block on and above its diagonal (entries below it are
// never written and must be zero), scl[k] holds the scale of column k, and
// in MODE != 0 R's rows of the panel hold the panel's columns of the new R.
// sink: 64 entries a lane writes when its store has no target (every lane
// stores, so no store sits behind a branch); zero: an entry holding 0.
//
// Shared by the one- and two-wave engines, so both produce the same bits.
template <typename T, int NCP, int MODE, int SG, int NPX, int L, int p, int S1>
__device__ __forceinline__ void sweep_panel(T (&x)[SG][4][NPX], T* __restrict__ R, T (&td)[16][17],
                                            T* __restrict__ sink, T* __restrict__ scl, const T* __restrict__ zero,
                                            const int n_) {
    typedef Mfma<T> M;
    constexpr int c0 = 16 * p;
    constexpr int S0 = (MODE == 0) ? p : 0;
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    const int c = c0 + l16;
    // Column k of the panel's T: T[a][k] = -tau_k sum_{i<k} T[a][i] P[i][k],
    // T[k][k] = tau_k, with the in-panel Gram entries P[i][k] = v_i^T v_k =
    // scale_i w_i of column k's step (lanes i < k), in two running sums.
    // Formed one column late, inside the next column's step, where it
    // overlaps that column's reduction and Householder scalars.
    T pw_prev = T(0), tau_prev = T(0);
    auto tcol = [&](auto kc_) {
        constexpr int k = decltype(kc_)::value;
        T tk[2] = {T(0), T(0)};
        sfor<0, k>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            fmac_bc<i, i == 0>(tk[i & 1], pw_prev, td[l16][i]);
        });
        const T t = tk[0] + tk[1];
        T* dst = (l16 < opaque_s(k)) ? &td[l16][k] : (sink + lane);
        *dst = -tau_prev * t;
        td[k][k] = tau_prev;
    };
    sfor<0, 16>([&](auto jc) {
        constexpr int jj = decltype(jc)::value;
        constexpr int j = c0 + jj;
        __builtin_amdgcn_sched_barrier(0);
        // lane conditions of this column, not hoisted out of the sweep
        const int n = opaque_s(n_);
        const bool right = c > opaque_s(j);
        constexpr int hreg = M::row_reg(jj), hl4 = M::row_l4(jj);
        T alpha, hc;
        if constexpr (MODE == 0) {
            const T hv = x[p][hreg][L];
            alpha = rdlane<16 * hl4 + jj>(hv);
            hc = sum4((l4 == hl4) ? hv : T(0));
        } else {
            // R[j][c] for the trailing columns (zero beyond n), 0 elsewhere
            alpha = R[rpi<NCP>(j, j)];
            hc = *(right ? (R + rpi<NCP>(j, 0) + c) : zero);
        }
        T xj[SG][4];
        T acc4[4] = {T(0), T(0), T(0), T(0)};
        if constexpr (MODE == 0) {
            // column j, broadcast to the lanes of the other columns (tail rows only)
            sfor<S0, SG>([&](auto sc) {
                constexpr int s = decltype(sc)::value;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    T v = bcast16<jj>(x[s][i][L]);
                    if constexpr (s == p) v = (M::orow(l4, i) > jj) ? v : T(0);
                    xj[s][i] = v;
                    acc4[i] = fma(v, x[s][i][L], acc4[i]);
                }
            });
        } else {
            dot_bc<jj, S1, L, jj == 0>(acc4, x);
        }
        if constexpr (jj > 0) tcol(ic_t<jj - 1>{});
        const T g = sum4((acc4[0] + acc4[1]) + (acc4[2] + acc4[3]));
        const T sigma2 = bcast16<jj>(g);
        T beta, tau, scale, rbeta;
        hh_scalars(alpha, sigma2, beta, tau, scale, rbeta);
        const bool zt = (sigma2 == T(0));
        tau = zt ? T(0) : tau;
        scale = zt ? T(0) : scale;
        beta = zt ? alpha : beta;
        const bool trail = right && (c < n);
        // coef = -tau w scale = w / beta, its factor selected off the critical path
        const T mcoef = (trail && !zt) ? rbeta : T(0);
        const T w = fma(scale, g, hc);
        const T tw = tau * w;
        const T coef = w * mcoef;
        if constexpr (MODE != 0) {
            // R[j][c] -= tau w_c (zero stays zero beyond n); R[j][j] = beta
            T* dst = right ? (R + rpi<NCP>(j, 0) + c) : (sink + lane);
            *dst = hc - tw;
            R[rpi<NCP>(j, j)] = beta;
        }
        if constexpr (MODE == 0) {
            sfor<S0, SG>([&](auto sc) {
                constexpr int s = decltype(sc)::value;
#pragma unroll
                for (int i = 0; i < 4; ++i) x[s][i][L] = fma(xj[s][i], coef, x[s][i][L]);
            });
            T& hv = x[p][hreg][L];
            const T nh = (l16 == jj) ? beta : (trail ? hv - tw : hv);
            hv = (l4 == hl4) ? nh : hv;
        } else {
            upd_bc<jj, S1, L>(x, coef);
        }
        // column j keeps its tail unscaled until the panel ends
        scl[jj] = scale;
        pw_prev = scl[l16] * w;
        tau_prev = tau;
    });
    tcol(ic_t<15>{});
    // reflector tails: scale the panel's columns (delayed from the sweep)
    const T sc_lane = scl[l16];
    constexpr int SE = (MODE == 0) ? SG : S1;
    sfor<S0, SE>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if constexpr (MODE == 0 && s == p)
                x[s][i][L] = (M::orow(l4, i) > l16) ? x[s][i][L] * sc_lane : x[s][i][L];
            else
                x[s][i][L] *= sc_lane;
        }
    });
}

// ---- the block factorisation -----------------------------------------------------
//
// Hooks.  pre(p) runs before panel p and post(p) once panel p's rows of R
// are final (its sweep and its update of the trailing columns are done).
// done(p) runs as soon as column tile p holds its final values (reflector
// tails, and R above them in a chain's first block), so its store overlaps
// the rest of the block instead of all tiles leaving at the end; free(p)
// once tile p's registers are no longer read (the next block may be loaded
// into them): right after panel p when no Q is kept, after the last panel's
// Gram products when it is.  emit() runs after the panels (a tree node
// stores its reflectors there).  Every hook is called for every panel,
// also for panels beyond n (zero columns), in panel order.
struct NoHook {
    template <typename P>
    __device__ void operator()(P) const {}
};

// WQ = false: only R and the reflectors are wanted (no Q is kept), so tau
// and T are neither stored nor, above the panels' diagonal blocks, formed.
template <typename T, int NP, int SG, int MODE, bool WQ = true, typename Emit, typename Pre = NoHook,
          typename Post = NoHook, typename Done = NoHook, typename Free = NoHook>
__device__ __forceinline__ void wave_block(T (&x)[SG][4][NP], WSmem<T, NP>& sm, const int n_, T* __restrict__ Tout,
                                           T* __restrict__ tauout, Emit&& emit, Pre&& pre = Pre{},
                                           Post&& post = Post{}, Done&& done = Done{}, Free&& free_ = Free{}) {
    typedef Mfma<T> M;
    typedef typename M::acc acc_t;
    constexpr int NCP = 16 * NP;
    // Gram blocks P_ac = V_a^T V_c (a < c) for the off-diagonal blocks of T,
    // each formed as soon as panel c is done (MFMA(V_c, V_a) gives P_ac in
    // the A-operand layout); rows where V_c or V_a vanishes are skipped:
    // above panel c's heads in the first block, below panel a's rows in a
    // tree node.
    acc_t P[NP][NP];

    sfor<0, NP>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int c0 = 16 * p;
        const int n = opaque_s(n_);
        if (c0 >= n) {
            if constexpr (WQ && NP > 1 && p > 0)
                sfor<0, p>([&](auto ac_) { P[decltype(ac_)::value][p] = acc_t{0, 0, 0, 0}; });
            done(pc);
            if constexpr (!WQ) free_(pc);
            return;
        }
        pre(pc);
        const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
        // live row groups of this panel
        constexpr int S0 = (MODE == 0) ? p : 0;
        constexpr int S1 = (MODE == 2) ? p + 1 : SG;
        const int c = c0 + l16;
        sweep_panel<T, NCP, MODE, SG, NP, p, p, S1>(x, sm.R, sm.td[p], &sm.scr[0][0], sm.scl, &sm.zero, n_);
        wave_sync();
        if (WQ && l4 == 0 && c < n) tauout[c] = sm.td[p][l16][l16];
        done(pc);
        if constexpr (WQ && NP > 1 && p > 0) {
            sfor<0, p>([&](auto ac_) {
                constexpr int a = decltype(ac_)::value;
                P[a][p] = acc_t{0, 0, 0, 0};
            });
            sfor<0, SG>([&](auto sc) {
                constexpr int s = decltype(sc)::value;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    sfor<0, p>([&](auto ac_) {
                        constexpr int a = decltype(ac_)::value;
                        constexpr bool live = (MODE == 0) ? (s >= p) : ((MODE == 2) ? (s <= a) : true);
                        if constexpr (live) {
                            T vc = x[s][i][p];
                            if constexpr (MODE == 0 && s == p) vc = vmask(vc, M::orow(l4, i), l16);
                            P[a][p] = M::mma(vc, x[s][i][a], P[a][p]);
                        }
                    });
                }
            });
        }

        // diagonal T block in the MFMA D layout; to global
        wave_sync();
        T tpp[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) tpp[r] = sm.td[p][M::orow(l4, r)][l16];
        wave_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = c0 + M::orow(l4, r);
            if (WQ && i <= c && c < n) Tout[tpi(i, c)] = tpp[r];
        }
        if constexpr (p + 1 < NP) {
            {
                // ---------------------------------------------- W = V_p^T X (trailing tiles)
                acc_t w0[NP];
                sfor<p + 1, NP>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    w0[q] = acc_t{0, 0, 0, 0};
                    if constexpr (MODE != 0) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int i = c0 + M::orow(l4, r), cc = 16 * q + l16;
                            const T v = sm.R[rpi<NCP>(i, cc)];
                            w0[q][r] = (i < n && cc < n) ? v : T(0);
                        }
                    }
                });
                sfor<S0, S1>([&](auto sc) {
                    constexpr int s = decltype(sc)::value;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        T a = x[s][i][p];
                        if constexpr (MODE == 0 && s == p) a = vmask(a, M::orow(l4, i), l16);
                        sfor<p + 1, NP>([&](auto qc) {
                            constexpr int q = decltype(qc)::value;
                            w0[q] = M::mma(a, x[s][i][q], w0[q]);
                        });
                    }
                });
                // ---------------------------------------------- -W' = -T_pp^T W; R rows
                T ntpp[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) ntpp[r] = -tpp[r];
                acc_t nw[NP];
                sfor<p + 1, NP>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    nw[q] = acc_t{0, 0, 0, 0};
                });
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) {
                    sfor<p + 1, NP>([&](auto qc) {
                        constexpr int q = decltype(qc)::value;
                        nw[q] = M::mma(ntpp[kc], w0[q][kc], nw[q]);
                    });
                }
                if constexpr (MODE != 0) {
                    sfor<p + 1, NP>([&](auto qc) {
                        constexpr int q = decltype(qc)::value;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int i = c0 + M::orow(l4, r), cc = 16 * q + l16;
                            if (i < n && cc < n) sm.R[rpi<NCP>(i, cc)] += nw[q][r];
                        }
                    });
                }
                // ---------------------------------------------- X -= V_p W'
                sfor<S0, S1>([&](auto sc) {
                    constexpr int s = decltype(sc)::value;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        T v = x[s][i][p];
                        if constexpr (MODE == 0 && s == p) v = vmask(v, M::orow(l4, i), l16);
                        sm.scr[M::orow(l4, i)][l16] = v;
                    }
                    wave_sync();
                    T vt[4];
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc) vt[kc] = sm.scr[l16][M::orow(l4, kc)];
                    wave_sync();
                    acc_t u[NP];
                    sfor<p + 1, NP>([&](auto qc) {
                        constexpr int q = decltype(qc)::value;
                        u[q] = acc_t{x[s][0][q], x[s][1][q], x[s][2][q], x[s][3][q]};
                    });
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc) {
                        sfor<p + 1, NP>([&](auto qc) {
                            constexpr int q = decltype(qc)::value;
                            u[q] = M::mma(vt[kc], nw[q][kc], u[q]);
                        });
                    }
                    sfor<p + 1, NP>([&](auto qc) {
                        constexpr int q = decltype(qc)::value;
#pragma unroll
                        for (int r = 0; r < 4; ++r) x[s][r][q] = u[q][r];
                    });
                });
            }
        }
        if constexpr (MODE == 0 && p < SG) {
            // rows of row group p of the block's R are final: into the on-chip R
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * p + M::orow(l4, i);
                sfor<p, NP>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    const int cc = 16 * q + l16;
                    if (r < n && cc >= r && cc < n) sm.R[rpi<NCP>(r, cc)] = x[p][i][q];
                });
            }
        }
        post(pc);
        if constexpr (!WQ) free_(pc);
    });

    const int n = opaque_s(n_);
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    (void)l4;

    if constexpr (NP == 1 || !WQ) {
        if constexpr (WQ) free_(ic_t<0>{});
        emit();
    } else {
        // ------------------------------------------------------ T blocks above the diagonal
        sfor<0, NP>([&](auto pc) { free_(pc); });
        emit();
        // diagonal blocks from LDS: D layout (tD) and A-operand layout (tA)
        // (entries beyond n and below the diagonal are zero in td)
        T tD[NP][4], tA[NP][4];
        sfor<0, NP>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = M::orow(l4, r);
                tD[b][r] = sm.td[b][o][l16];
                tA[b][r] = sm.td[b][l16][o];
            }
        });
        // T_ab = -T_aa sum_{c=a+1..b} P_ac T_cb, a = b-1 .. 0
        sfor<1, NP>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            {
                acc_t tcb[NP];
                tcb[b] = acc_t{tD[b][0], tD[b][1], tD[b][2], tD[b][3]};
                sfor<0, b>([&](auto ar) {
                    constexpr int a = b - 1 - decltype(ar)::value;
                    acc_t y = acc_t{0, 0, 0, 0};
                    sfor<a + 1, b + 1>([&](auto cc_) {
                        constexpr int cq = decltype(cc_)::value;
#pragma unroll
                        for (int kc = 0; kc < 4; ++kc) y = M::mma(P[a][cq][kc], tcb[cq][kc], y);
                    });
                    acc_t t = acc_t{0, 0, 0, 0};
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc) t = M::mma(tA[a][kc], y[kc], t);
                    tcb[a] = -t;
                    const int jx = 16 * b + l16;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (jx < n) Tout[tpi(16 * a + M::orow(l4, r), jx)] = tcb[a][r];
                });
            }
        });
    }
    wave_sync();
}

// ---- tile I/O -------------------------------------------------------------------
// Row 16s + orow(l4, i) of the tile is the lane's base row orow(l4, 0) plus a
// lane-independent offset, so a full tile needs one per-lane pointer; a
// partial tile (last block of a chain, n < NCP) takes the masked path.
template <typename T, int NP, int SG>
__device__ __forceinline__ void wload(T (&x)[SG][4][NP], const T* __restrict__ A, int64_t lda, int64_t r0, int rows,
                                      int n) {
    typedef Mfma<T> M;
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    if (rows == 16 * SG && n == 16 * NP) {
        const T* __restrict__ pb = A + (r0 + M::orow(l4, 0)) * lda + l16;
#pragma unroll
        for (int s = 0; s < SG; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const T* __restrict__ pr = pb + (int64_t)(16 * s + M::orow(0, i) - M::orow(0, 0)) * lda;
#pragma unroll
                for (int q = 0; q < NP; ++q) x[s][i][q] = pr[16 * q];
            }
        return;
    }
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * s + M::orow(l4, i);
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int cc = 16 * q + l16;
                x[s][i][q] = (r < rows && cc < n) ? A[(r0 + r) * lda + cc] : T(0);
            }
        }
}

// One column tile q (columns 16q..16q+15) of a block.
template <typename T, int NP, int SG, int Q>
__device__ __forceinline__ void wload_tile(T (&x)[SG][4][NP], const T* __restrict__ A, int64_t lda, int64_t r0,
                                           int rows, int n) {
    typedef Mfma<T> M;
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    if (rows == 16 * SG && n == 16 * NP) {
        const T* __restrict__ pb = A + (r0 + M::orow(l4, 0)) * lda + 16 * Q + l16;
#pragma unroll
        for (int s = 0; s < SG; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) x[s][i][Q] = pb[(int64_t)(16 * s + M::orow(0, i) - M::orow(0, 0)) * lda];
        return;
    }
    const int cc = 16 * Q + l16;
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * s + M::orow(l4, i);
            x[s][i][Q] = (r < rows && cc < n) ? A[(r0 + r) * lda + cc] : T(0);
        }
}

template <typename T, int NP, int SG, int Q>
__device__ __forceinline__ void wstore_tile(const T (&x)[SG][4][NP], T* __restrict__ A, int64_t lda, int64_t r0,
                                            int rows, int n) {
    typedef Mfma<T> M;
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    if (rows == 16 * SG && n == 16 * NP) {
        T* __restrict__ pb = A + (r0 + M::orow(l4, 0)) * lda + 16 * Q + l16;
#pragma unroll
        for (int s = 0; s < SG; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) pb[(int64_t)(16 * s + M::orow(0, i) - M::orow(0, 0)) * lda] = x[s][i][Q];
        return;
    }
    const int cc = 16 * Q + l16;
    if (cc >= n) return;
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * s + M::orow(l4, i);
            if (r < rows) A[(r0 + r) * lda + cc] = x[s][i][Q];
        }
}

template <typename T, int NP, int SG>
__device__ __forceinline__ void wstore(const T (&x)[SG][4][NP], T* __restrict__ A, int64_t lda, int64_t r0, int rows,
                                       int n) {
    typedef Mfma<T> M;
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
    if (rows == 16 * SG && n == 16 * NP) {
        T* __restrict__ pb = A + (r0 + M::orow(l4, 0)) * lda + l16;
#pragma unroll
        for (int s = 0; s < SG; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                T* __restrict__ pr = pb + (int64_t)(16 * s + M::orow(0, i) - M::orow(0, 0)) * lda;
#pragma unroll
                for (int q = 0; q < NP; ++q) pr[16 * q] = x[s][i][q];
            }
        return;
    }
#pragma unroll
    for (int s = 0; s < SG; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * s + M::orow(l4, i);
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int cc = 16 * q + l16;
                if (r < rows && cc < n) A[(r0 + r) * lda + cc] = x[s][i][q];
            }
        }
}

// R (LDS, packed) -> row-major n x n with zeros below the diagonal (lane =
// column, one row per step).
template <typename T, int NP>
__device__ __forceinline__ void r_out(const WSmem<T, NP>& sm, int n, T* __restrict__ R, int64_t ldr, bool lower) {
    constexpr int NCP = 16 * NP;
    const int j = lane_id();
    for (int i = 0; i < n; ++i) {
        if (j < n && (j >= i || lower)) R[i * ldr + j] = (j >= i) ? sm.R[rpi<NCP>(i, j >= i ? j : i)] : T(0);
    }
}
// The packed R travels through global memory as is (slot of rslot(n, NP)
// elements); copies are coalesced and independent.
template <int NP>
__host__ __device__ inline int64_t rslot(int64_t n) {
    const int64_t rp = (int64_t)(16 * NP) * (16 * NP + 1) / 2;
    return n * n > rp ? n * n : rp;
}
template <typename T, int NP>
__device__ __forceinline__ void r_pub(const WSmem<T, NP>& sm, T* __restrict__ dst) {
    constexpr int RP = WSmem<T, NP>::RP;
    const int l = lane_id();
#pragma unroll 4
    for (int e = l; e < RP; e += 64) pub_store(dst + e, sm.R[e]);
}
template <typename T, int NP>
__device__ __forceinline__ void r_get(WSmem<T, NP>& sm, const T* __restrict__ src) {
    constexpr int RP = WSmem<T, NP>::RP;
    constexpr int IT = (RP + 63) / 64;
    const int l = lane_id();
    T v[IT];
#pragma unroll
    for (int t = 0; t < IT; ++t) v[t] = (l + 64 * t < RP) ? pub_load(src + l + 64 * t) : T(0);
#pragma unroll
    for (int t = 0; t < IT; ++t)
        if (l + 64 * t < RP) sm.R[l + 64 * t] = v[t];
    wave_sync();
}
// Tile (operand layout) of a packed upper-triangular R, from LDS or (PUB) from
// a copy published by another workgroup.
template <typename T, int NP, bool PUB = false>
__device__ __forceinline__ void tile_of_packed(T (&x)[NP][4][NP], const T* __restrict__ Rp, int n) {
    typedef Mfma<T> M;
    constexpr int NCP = 16 * NP;
    const int lane = lane_id(), l16 = lane & 15, l4 = lane >> 4;
#pragma unroll
    for (int s = 0; s < NP; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * s + M::orow(l4, i);
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int cc = 16 * q + l16;
                const bool ok = cc >= r && cc < n && r < n;
                const T* a = Rp + rpi<NCP>(ok ? r : 0, ok ? cc : 0);
                const T v = PUB ? pub_load(a) : *a;
                x[s][i][q] = ok ? v : T(0);
            }
        }
}

// ---- one chain, then the tree nodes this wave completes -----------------------------
//
// Tree (Sec. 2.1; any tree shape gives a valid QR): level lev has stride
// a^(lev-1); the node at i0 (a multiple of a*stride) folds its children
// i0 + t*stride (t = 1..a-1, < W) into child i0.  Each chain, or node result,
// is published in Rbuf; the wave that completes a node's last child (an
// atomic count per node, zeroed before the launch) performs the node, so no
// wave waits for another and the levels need no separate launches.  The node
// arithmetic does not depend on which child arrived last.
struct TreeArgs {
    int* cnt;        // W * (levels + 1) counters, zero at launch
    void* Rout;      // final R (row-major, ldr), or null
    int64_t ldr;
    int zero_lower;  // also write zeros below R's diagonal
    int max_polls;   // polls of a bounded wait before it gives up (pipelined tree)
    int* status;     // status word: bit 0 set when a bounded wait gave up
    int64_t rstride; // elements between the R factors of a batch's members
};
// Where member `mem` of a batch writes its R.
template <typename T>
__device__ __forceinline__ T* rout_of(const TreeArgs& ta, int mem) {
    return (T*)ta.Rout + (int64_t)mem * ta.rstride;
}

// ---- the panel-pipelined binary tree ----------------------------------------------
//
// When every wave of the launch is resident at once, a node need not wait for
// its children to finish: panel p of the node [R_a; R_b] touches only R_a's
// rows of panel p and R_b's rows of panels <= p, and a node's rows of panel p
// are final as soon as its own panel p is done (a reflector of an earlier
// panel acts on one row of R_a and on rows of R_b above the panel).  So each
// level runs one panel behind the level below rather than one whole node.
// Node (lev, i0) is performed by wave i0 + 2^(lev-1), the chain of its second
// child, once that chain is done (a bijection between the chains 1..W-1 and
// the nodes); it waits for its children's panels through progress counts
// (lev * W + slot, zero at launch), published after the rows themselves.
__device__ __forceinline__ void pub_flag(int* f, int v) {
    __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until *f >= v, polling at most max_polls times.  The producer is
// resident and never waits on this wave, so it gets there; the bound only
// guarantees that the wave ends.  A wave that gives up sets bit 0 of the
// status word (the host reads it with tsqr_check_status) and goes on with
// whatever rows are in memory: that factorisation's R and Q are then invalid,
// but every wave still exits.  The fence after the wait keeps the compiler
// from moving the loads of the published rows above the flag load (the rows
// themselves are read with device-coherent loads, see pub_load).
__device__ __forceinline__ void wait_flag(const int* f, int v, int max_polls, int* status) {
    bool ok = false;
    for (int it = 0; it < max_polls; ++it) {
        const int cur = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (cur >= v) {
            ok = true;
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    if (!ok && (threadIdx.x & 63) == 0)
        __hip_atomic_fetch_or(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
// Level of the node that actually produces the R of tree position (l, idx):
// positions with a single child pass their child's R up unchanged.
__device__ __forceinline__ int producer_level(int W, int l, int idx) {
    while (l > 0) {
        const int st = 1 << (l - 1);
        if ((W - idx + st - 1) / st >= 2) break;
        --l;
    }
    return l;
}

template <typename T, int NP, bool WQ>
__device__ __forceinline__ void wave_tree_pipe(WSmem<T, NP>& sm, const Geom& g, int c, T* __restrict__ Rbuf,
                                               T* __restrict__ Ynode, T* __restrict__ Tnode,
                                               T* __restrict__ tau_node, const TreeArgs& ta, bool in_rbuf) {
    constexpr int NCP = 16 * NP;
    constexpr int RP = WSmem<T, NP>::RP;
    const int n = (int)g.n;
    const int W = g.W;
    const int npl = (n + 15) / 16;  // live panels
    const int64_t rs = rslot<NP>(n);
    const int64_t tri = (int64_t)n * (n + 1) / 2;
    const int64_t nn = (int64_t)n * n;
    int* prog = ta.cnt;
    const int lane = lane_id();
    // publish the chain's R (all panels at once); a chain reduced by an
    // earlier launch left it in its slot already
    if (!in_rbuf) {
        r_pub<T, NP>(sm, Rbuf + (int64_t)c * rs);
        pub_wait();
    }
    if (lane == 0) pub_flag(prog + c, npl);
    if (c % g.cpm == 0) return;  // a member's first chain performs no node
    const int lev = __builtin_ctz((unsigned)c) + 1;
    const int i0 = c - (1 << (lev - 1));
    const int la = producer_level(W, lev - 1, i0), lb = producer_level(W, lev - 1, c);
    const bool own_b = lb == 0;  // the second child is this wave's own chain
    T x[NP][4][NP];
    if (own_b) {
        tile_of_packed<T, NP>(x, in_rbuf ? (const T*)(Rbuf + (int64_t)c * rs) : (const T*)sm.R, n);
        wave_sync();
    }
    const T* Ra = Rbuf + (int64_t)i0 * rs;
    const T* Rb = Rbuf + (int64_t)c * rs;
    T* Rnode = Rbuf + (int64_t)i0 * rs;  // the node's R replaces child a's, panel by panel
    auto pre = [&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int e0 = rpi<NCP>(16 * p, 16 * p);
        constexpr int e1 = (p + 1 < NP) ? rpi<NCP>(16 * (p + 1), 16 * (p + 1)) : RP;
        wait_flag(prog + la * W + i0, p + 1, ta.max_polls, ta.status);
        if (!own_b) wait_flag(prog + lb * W + c, p + 1, ta.max_polls, ta.status);
        // child a's rows of panel p: all loads issued before any is used
        constexpr int IT = (e1 - e0 + 63) / 64;
        T ra[IT];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const int e = e0 + lane + 64 * u;
            ra[u] = (e < e1) ? pub_load(Ra + e) : T(0);
        }
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const int e = e0 + lane + 64 * u;
            if (e < e1) sm.R[e] = ra[u];
        }
        if (!own_b) {
            typedef Mfma<T> M;
            const int l16 = lane & 15, l4 = lane >> 4;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * p + M::orow(l4, i);
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    const int cc = 16 * q + l16;
                    const bool ok = q >= p && cc >= r && cc < n && r < n;
                    const T v = pub_load(Rb + rpi<NCP>(ok ? r : 0, ok ? cc : 0));
                    x[p][i][q] = ok ? v : T(0);
                }
            }
        }
        wave_sync();
    };
    auto post = [&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int e0 = rpi<NCP>(16 * p, 16 * p);
        constexpr int e1 = (p + 1 < NP) ? rpi<NCP>(16 * (p + 1), 16 * (p + 1)) : RP;
        wave_sync();
        for (int e = e0 + lane; e < e1; e += 64) pub_store(Rnode + e, sm.R[e]);
        pub_wait();
        if (lane == 0) pub_flag(prog + lev * W + i0, p + 1);
    };
    auto emit = [&]() {
        if constexpr (WQ) wstore<T, NP, NP>(x, Ynode + (int64_t)c * nn, n, 0, n, n);
    };
    wave_block<T, NP, NP, 2, WQ>(x, sm, n, Tnode + (int64_t)c * tri, tau_node + (int64_t)c * n, emit, pre, post);
    if (lev == g.levels && ta.Rout) r_out<T, NP>(sm, n, rout_of<T>(ta, i0 / g.cpm), ta.ldr, ta.zero_lower != 0);
}

template <typename T, int NP, int SG, bool PIPE = false, bool WQ = true, bool CHAIN = true>
__device__ __forceinline__ void wave_tsqr(WSmem<T, NP>& sm, const Geom& g, int c, T* __restrict__ A, int64_t lda,
                                          T* __restrict__ tau_blk, T* __restrict__ T_blk, T* __restrict__ Rbuf,
                                          T* __restrict__ Ynode, T* __restrict__ Tnode, T* __restrict__ tau_node,
                                          const TreeArgs& ta) {
    const int n = (int)g.n;
    const int64_t tri = (int64_t)n * (n + 1) / 2;
    const int64_t nn = (int64_t)n * n;
    // the sweep writes the diagonal T blocks on and above their diagonals only
    for (int e = lane_id(); e < NP * 16 * 17; e += 64) (&sm.td[0][0][0])[e] = T(0);
    if (lane_id() == 0) sm.zero = T(0);
    wave_sync();
    if constexpr (!CHAIN) {
        // the chain was reduced by another launch: its R is in Rbuf, where
        // the pipelined tree reads it
        if (!PIPE || g.levels == 0) r_get<T, NP>(sm, Rbuf + (int64_t)c * rslot<NP>(n));
    } else {
        // R starts at zero, so its entries beyond column n stay zero
        for (int e = lane_id(); e < (int)(sizeof(sm.R) / sizeof(T)); e += 64) sm.R[e] = T(0);
        wave_sync();
        // ---- the chain (flat tree)
        const int64_t start = chain_start(g, c), end = chain_end(g, c);
        const int nb = chain_nblocks(g, c);
        const int64_t blk0 = chain_blk0(g, c);
        constexpr int H = 16 * SG;
        // Each column tile is stored as soon as its panel is done, and the
        // next block's tile is loaded into its registers as soon as they are
        // free (right after the panel without an implicit Q, else during the
        // T products), so the block's HBM traffic is spread over its work.
        T x[SG][4][NP];
        wload<T, NP, SG>(x, A, lda, start, (int)((end - start) < H ? (end - start) : H), n);
        for (int b = 0; b < nb; ++b) {
            const int64_t r0 = start + (int64_t)b * H;
            const int rows = (int)((end - r0) < H ? (end - r0) : H);
            const int64_t r1 = r0 + H;
            const int rows1 = (int)((end - r1) < H ? (end - r1) : H);
            const bool more = b + 1 < nb;
            auto done = [&](auto pc) { wstore_tile<T, NP, SG, decltype(pc)::value>(x, A, lda, r0, rows, n); };
            auto free_ = [&](auto pc) {
                if (more) wload_tile<T, NP, SG, decltype(pc)::value>(x, A, lda, r1, rows1, n);
            };
            auto emit = [] {};
            if (b == 0)
                wave_block<T, NP, SG, 0, WQ>(x, sm, n, T_blk + (blk0 + b) * tri, tau_blk + (blk0 + b) * n, emit,
                                             NoHook{}, NoHook{}, done, free_);
            else
                wave_block<T, NP, SG, 1, WQ>(x, sm, n, T_blk + (blk0 + b) * tri, tau_blk + (blk0 + b) * n, emit,
                                             NoHook{}, NoHook{}, done, free_);
        }
    }
    // ---- the tree
    if (g.levels == 0) {  // every chain is a whole member
        if (ta.Rout) r_out<T, NP>(sm, n, rout_of<T>(ta, c / g.cpm), ta.ldr, ta.zero_lower != 0);
        return;
    }
    if constexpr (PIPE) {
        wave_tree_pipe<T, NP, WQ>(sm, g, c, Rbuf, Ynode, Tnode, tau_node, ta, !CHAIN);
        return;
    }
    const int64_t rs = rslot<NP>(n);
    int cur = c;
    for (int lev = 1; lev <= g.levels; ++lev) {
        const int64_t stride = ipow(g.arity, lev - 1);
        const int64_t span = stride * g.arity;
        const int i0 = (int)((cur / span) * span);
        int nch = (int)((g.W - i0 + stride - 1) / stride);
        if (nch > g.arity) nch = g.arity;
        if (nch <= 1) continue;  // unpaired: carried up unchanged
        // (a chain reduced by an earlier launch left its R in its slot already)
        if (CHAIN || lev > 1) {
            r_pub<T, NP>(sm, Rbuf + (int64_t)cur * rs);
            pub_wait();
        }
        int old = 0;
        if ((threadIdx.x & 63) == 0) old = atomicAdd(ta.cnt + (int64_t)(lev - 1) * g.W + i0, 1);
        old = __builtin_amdgcn_readfirstlane(old);
        if (old != nch - 1) return;
        // the other children's published rows are read only after the count
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // The node folds children 1..nch-1 into child 0 in order, whichever
        // child arrived last.  This wave's own R is taken from LDS, the others
        // from their published copies.
        T own[NP][4][NP];
        const int tself = (int)((cur - i0) / stride);
        if (tself != 0) {
            tile_of_packed<T, NP>(own, sm.R, n);
            wave_sync();
            r_get<T, NP>(sm, Rbuf + (int64_t)i0 * rs);
        }
        for (int t = 1; t < nch; ++t) {
            const int64_t ch = i0 + t * stride;
            T xc[NP][4][NP];
            if (t == tself) {
#pragma unroll
                for (int a = 0; a < NP; ++a)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int q = 0; q < NP; ++q) xc[a][i][q] = own[a][i][q];
            } else {
                tile_of_packed<T, NP, true>(xc, Rbuf + ch * rs, n);
            }
            auto emit = [&]() {
                if constexpr (WQ) wstore<T, NP, NP>(xc, Ynode + ch * nn, n, 0, n, n);
            };
            wave_block<T, NP, NP, 2, WQ>(xc, sm, n, Tnode + ch * tri, tau_node + ch * n, emit);
        }
        cur = i0;
    }
    if (ta.Rout) r_out<T, NP>(sm, n, rout_of<T>(ta, cur / g.cpm), ta.ldr, ta.zero_lower != 0);
}

}  // namespace tsqr
