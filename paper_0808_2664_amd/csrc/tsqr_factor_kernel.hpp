// The factor kernel k_wave_tsqr and its launcher (paper Sec. 2.1).  Each
// (type, panel count, Q kept or not) instantiation of launch_wave is compiled
// in a translation unit of its own (tsqr_factor_inst.hip, built once per
// instantiation), so the fully unrolled column sweeps compile in parallel.
#pragma once
#include "tsqr_wave.hpp"
#include "tsqr_wave2.hpp"

namespace tsqr {

// Waves per SIMD the factor kernel is compiled for (register budget 512/occ):
// the FP64 tile of a 64 x 64 block takes 128 registers per lane and the
// kernel needs the whole file; the FP32 kernel fits two waves per SIMD.
template <typename T>
struct WaveOcc {
    static constexpr int value = sizeof(T) == 8 ? 1 : 2;
};

// PIPE: the panel-pipelined binary tree, where a node's wave waits for its
// children's panels.  It is launched only when the device can hold all its
// waves at once (one 64-lane workgroup per chain), with an ordinary launch:
// with the device otherwise idle every workgroup is dispatched at once, and
// workgroups held back by other work on the device are dispatched as that
// work retires (it never waits on this kernel), so every wait ends; a wait
// that does not end within TreeArgs::max_polls sets the status word
// (TSQR_ERR_TIMEOUT) instead of hanging.  A cooperative launch would only
// add the runtime's own co-residency check, and in a process that had made
// one, later rocprofv3 exits faulted and CAQR on CU-masked streams ran
// slower.
// CHAIN = false: the chains were reduced by the two-wave chain kernel, whose
// R factors are in Rbuf; this launch runs the tree only.
template <typename T, int NP, int SG, bool PIPE, bool WQ, bool CHAIN>
__global__ __launch_bounds__(64, WaveOcc<T>::value) void k_wave_tsqr(Geom g, T* __restrict__ A, int64_t lda, T* __restrict__ tau_blk,
                                                     T* __restrict__ T_blk, T* __restrict__ Rbuf,
                                                     T* __restrict__ Ynode, T* __restrict__ Tnode,
                                                     T* __restrict__ tau_node, TreeArgs ta) {
    __shared__ WSmem<T, NP> sm;
    wave_tsqr<T, NP, SG, PIPE, WQ, CHAIN>(sm, g, (int)blockIdx.x, A, lda, tau_blk, T_blk, Rbuf, Ynode, Tnode, tau_node,
                                          ta);
}

// Workgroups of k_wave_tsqr<T, NP, SG, true, WQ, CHAIN> the device keeps resident at once.
template <typename T, int NP, int SG, bool WQ, bool CHAIN>
static int64_t pipe_capacity() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    static int64_t cap[64];
    static bool done[64];
    if (dev < 0 || dev >= 64) return 0;
    if (!done[dev]) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_wave_tsqr<T, NP, SG, true, WQ, CHAIN>, 64, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            per_cu = 0;
        }
        cap[dev] = (int64_t)per_cu * cus;
        done[dev] = true;
    }
    return cap[dev];
}

// The tree (and, with CHAIN, the chains) in one launch.
template <typename T, int NP, int SG, bool WQ, bool CHAIN>
static hipError_t launch_tree(const Geom& g, T* A, int64_t lda, const Work& wk, const TreeArgs& ta, hipStream_t st) {
    T *tau_blk = (T*)wk.tau_blk, *T_blk = (T*)wk.T_blk, *Rbuf = (T*)wk.Rbuf;
    T *Ynode = (T*)wk.Ynode, *Tnode = (T*)wk.Tnode, *tau_node = (T*)wk.tau_node;
    // TREE_PIPE_PLAIN: the caller has checked the residency on its own units
    const bool pipe = g.W > 1 && g.arity == 2 &&
                      ((g.flags & TREE_PIPE_PLAIN) ||
                       (!(g.flags & TREE_LEVELWISE) && g.W <= pipe_capacity<T, NP, SG, WQ, CHAIN>()));
    if (pipe) {
        k_wave_tsqr<T, NP, SG, true, WQ, CHAIN><<<g.W, 64, 0, st>>>(g, A, lda, tau_blk, T_blk, Rbuf, Ynode, Tnode,
                                                                    tau_node, ta);
        return hipGetLastError();
    }
    k_wave_tsqr<T, NP, SG, false, WQ, CHAIN><<<g.W, 64, 0, st>>>(g, A, lda, tau_blk, T_blk, Rbuf, Ynode, Tnode,
                                                                 tau_node, ta);
    return hipGetLastError();
}

// FP64 with more than 32 columns: the chains on the two-wave engine
// (tsqr_wave2.hpp), then the tree in a second launch; otherwise (and with
// Geom::flags ONE_WAVE) chains and tree in one launch of the one-wave engine.
template <typename T, int NP, int SG, bool WQ>
hipError_t launch_wave(const Geom& g, T* A, int64_t lda, const Work& wk, const TreeArgs& ta, hipStream_t st) {
    if constexpr (NP == 4 && sizeof(T) == 8) {
        if (!(g.flags & ONE_WAVE)) {
            k_chain2<T, WQ><<<g.W, 128, 0, st>>>(g, A, lda, (T*)wk.tau_blk, (T*)wk.T_blk, (T*)wk.Rbuf);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            return launch_tree<T, NP, SG, WQ, false>(g, A, lda, wk, ta, st);
        }
    }
    return launch_tree<T, NP, SG, WQ, true>(g, A, lda, wk, ta, st);
}

}  // namespace tsqr
