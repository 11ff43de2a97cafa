// TSQR factorisation kernels for gfx950 (paper Sec. 2.1).
//
//  * k_chain_factor: one workgroup (4 waves) per chain, a contiguous range of
//    rows.  It runs sequential TSQR on a flat tree (Sec. 2.1): the first block
//    is a plain Householder QR; every later block is factored stacked under the
//    R factor kept on chip, so A is read once and the reflectors are written
//    once (Table 4, Eq. TSQR_seq_runtime: 2mn words).
//  * k_tree_combine: one wave per tree node; folds the R factors of the node's
//    children into the first child's R, one stacked-triangle QR per child
//    (Sec. 2.1, Eqs. TSQR_binarytree_2/3).  Reflector j touches the head row j
//    and only the nonzero rows of the lower triangle, so the stored bottom
//    reflectors stay upper triangular (the zeros of the triangles stay exact).
//
// Local QR of one block (factor_block): blocked Householder QR.  Columns are
// taken in panels of 16; inside a panel each reflector is formed column by
// column (unit topmost entry, Sec. 5.2; beta = -sign(alpha)||x||, sign(0)=+1,
// tau = 0 for a zero tail).  The panel then updates the trailing columns as a
// block reflector I - V T V^T (Schreiber-Van Loan form, cited in Sec. 2.1; the
// trailing update of Sec. 3.1), whose two products run on the FP64/FP32 MFMA
// units.  The same MFMA pass yields the Gram blocks V_q^T V_p that complete the
// block's full T, stored for the later applications of Q.
//
// Register tile: the MFMA operand layout.  Lane l of wave w holds column
// 16p + l%16 of rows w*16*SG + 16s + orow(l/16, i) for s < SG, i < 4, p < NP.
// Hence a column of a panel lives in 4 lanes of each wave: its reductions are
// two lane swaps (v_permlane16/32_swap) plus one LDS exchange across waves,
// and the reflector is broadcast to the other columns of a 16-lane row with
// one DPP row_newbcast per row.
#include "tsqr_engine.hpp"

namespace tsqr {
using namespace dev;

template <typename T, int NC, int NW, int SG>
__global__ __launch_bounds__(64 * NW) void k_chain_factor(Geom g, T* __restrict__ A, int64_t lda,
                                                          T* __restrict__ tau_blk, T* __restrict__ T_blk,
                                                          T* __restrict__ Rbuf) {
    __shared__ FSmem<T, NC, NW> sm;
    chain_body<T, NC, NW, SG>(sm, g, A, lda, tau_blk, T_blk, Rbuf, (int)blockIdx.x);
}

// One node of the reduction tree at level `lev`: fold children
// i + t*stride (t = 1..arity-1) into the R of child i.
template <typename T, int NC>
__global__ __launch_bounds__(64 * CombineShape<NC>::NW) void k_tree_combine(Geom g, int lev, T* __restrict__ Rbuf,
                                                                           T* __restrict__ Ynode,
                                                                           T* __restrict__ Tnode,
                                                                           T* __restrict__ tau_node) {
    constexpr int NW = CombineShape<NC>::NW;
    constexpr int SG = CombineShape<NC>::SG;
    __shared__ FSmem<T, NC, NW> sm;
    const int64_t stride = ipow(g.arity, lev - 1);
    const int64_t i0 = (int64_t)blockIdx.x * g.arity * stride;
    if (i0 + stride >= g.W) return;
    combine_body<T, NC, NW, SG>(sm, g, Rbuf, i0, stride, g.arity, Ynode, Tnode, tau_node);
}

template <typename T>
__global__ void k_copy_r(int64_t n, const T* __restrict__ Rsrc, int64_t lds, T* __restrict__ R, int64_t ldr,
                         int zero_lower) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int64_t i = e / n, j = e - i * n;
    if (j >= i) R[i * ldr + j] = Rsrc[i * lds + j];
    else if (zero_lower) R[i * ldr + j] = T(0);
}

template <typename T, int NC>
static hipError_t factor_nc(const Geom& g, T* A, int64_t lda, const Work& wk, hipStream_t st) {
    T* tau_blk = (T*)wk.tau_blk;
    T* T_blk = (T*)wk.T_blk;
    T* Rbuf = (T*)wk.Rbuf;
    phase_begin(0, st);
    switch (g.h) {
        case 64: k_chain_factor<T, NC, 4, 1><<<g.W, 256, 0, st>>>(g, A, lda, tau_blk, T_blk, Rbuf); break;
        case 128: k_chain_factor<T, NC, 4, 2><<<g.W, 256, 0, st>>>(g, A, lda, tau_blk, T_blk, Rbuf); break;
        case 256: k_chain_factor<T, NC, 4, 4><<<g.W, 256, 0, st>>>(g, A, lda, tau_blk, T_blk, Rbuf); break;
        default: return hipErrorInvalidValue;
    }
    phase_end(0, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int lev = 1; lev <= g.levels; ++lev) {
        const int64_t stride = ipow(g.arity, lev - 1);
        const int64_t span = stride * g.arity;
        const int nodes = (int)((g.W + span - 1) / span);
        constexpr int cthreads = 64 * CombineShape<NC>::NW;
        k_tree_combine<T, NC><<<nodes, cthreads, 0, st>>>(g, lev, Rbuf, (T*)wk.Ynode, (T*)wk.Tnode,
                                                          (T*)wk.tau_node);
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

hipError_t launch_copy_r(bool f64, int64_t n, const void* Rsrc, int64_t lds, void* R, int64_t ldr, bool zero_lower,
                         hipStream_t st) {
    const int64_t tot = n * n;
    const int64_t nb = (tot + 255) / 256;
    if (f64)
        k_copy_r<double><<<(unsigned)nb, 256, 0, st>>>(n, (const double*)Rsrc, lds, (double*)R, ldr, zero_lower ? 1 : 0);
    else
        k_copy_r<float><<<(unsigned)nb, 256, 0, st>>>(n, (const float*)Rsrc, lds, (float*)R, ldr, zero_lower ? 1 : 0);
    return hipGetLastError();
}

}  // namespace tsqr
