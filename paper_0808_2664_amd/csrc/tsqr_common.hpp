// Shared host/device definitions of the TSQR library (gfx950).
//
// Geometry of one TSQR (paper Sec. 2.1): the m x n matrix is split into W
// contiguous row ranges ("chains").  Each chain is reduced by one workgroup
// with the flat tree of sequential TSQR (Sec. 2.1, flat-tree picture): its
// first block is factored, the R factor stays on chip, and every further block
// is factored stacked under that R.  The W chain R factors are then reduced on
// a tree of arity `arity` (binary by default, Eq. TSQR_binarytree_1..4).
// Any tree gives a valid QR (Sec. 2.1, remark after the flat tree).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsqr {

// ----------------------------------------------------------------- geometry
struct Geom {
    int64_t m = 0, n = 0;
    int h = 0;            // rows per block (tile height of the chain kernel)
    int64_t S = 0;        // rows per chain, a multiple of h (the last chain differs)
    int W = 0;            // number of chains
    int arity = 2;        // tree arity
    int levels = 0;       // tree levels above the chains
    int64_t nblocks = 0;  // blocks over all chains
    int NC = 0;           // padded column count: 8, 16, 32 or 64
    int flags = 0;        // TREE_LEVELWISE
    // A batch of independent matrices of mb rows each, stacked (member b is
    // rows b*mb .. b*mb + mb - 1), is reduced as a forest: each member has
    // its own cpm chains (a power of the arity) and its own tree of `levels`
    // levels, rooted at chain b*cpm.  One matrix: mb = m, cpm = W.
    int64_t mb = 0;       // rows per member
    int cpm = 0;          // chains per member
    int64_t bpm = 0;      // blocks per member
};

// Geom::flags: reduce the tree node by node as children complete, never with
// the panel-pipelined tree (the tsqr_opts flag of the same meaning).
constexpr int TREE_LEVELWISE = 1;
// Geom::flags: reduce every chain with the one-wave engine, also where the
// two-wave chain engine applies (FP64, more than 32 columns).
constexpr int ONE_WAVE = 2;
// Geom::flags (set by the library only): the panel-pipelined tree with an
// ordinary launch, its waves' residency guaranteed by the caller (CAQR's
// panels on a CU-masked stream of their own, with at most one wave per SIMD
// of its units); takes precedence over TREE_LEVELWISE.
constexpr int TREE_PIPE_PLAIN = 4;

// Chain c is chain c % cpm of member c / cpm; a member's last chain takes
// the member's remaining rows.
__host__ __device__ inline int64_t chain_start(const Geom& g, int c) {
    const int mem = c / g.cpm, loc = c - mem * g.cpm;
    return (int64_t)mem * g.mb + (int64_t)loc * g.S;
}
__host__ __device__ inline int64_t chain_end(const Geom& g, int c) {
    const int mem = c / g.cpm, loc = c - mem * g.cpm;
    return (loc == g.cpm - 1) ? (int64_t)(mem + 1) * g.mb : (int64_t)mem * g.mb + (int64_t)(loc + 1) * g.S;
}
__host__ __device__ inline int chain_nblocks(const Geom& g, int c) {
    int64_t len = chain_end(g, c) - chain_start(g, c);
    return (int)((len + g.h - 1) / g.h);
}
__host__ __device__ inline int64_t chain_blk0(const Geom& g, int c) {
    const int mem = c / g.cpm, loc = c - mem * g.cpm;
    return (int64_t)mem * g.bpm + (int64_t)loc * (g.S / g.h);
}

// Tree level `lev` (1-based) with arity a: stride = a^(lev-1).  Nodes start at
// multiples of a*stride; their children are i + t*stride, t = 1..a-1, < W.
// The step that folds child c into its node is stored in slot c (1 <= c < W).
__host__ __device__ inline int64_t ipow(int64_t a, int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= a;
    return r;
}

inline int packed_tri(int n) { return n * (n + 1) / 2; }

// Workspace carried by an implicit Q (the "tree of Q factors", Sec. 2.1).
struct Work {
    void* base = nullptr;
    size_t bytes = 0;
    void* tau_blk = nullptr;   // nblocks x n
    void* T_blk = nullptr;     // nblocks x n(n+1)/2, packed upper, column by column
    void* Rbuf = nullptr;      // W slots: each chain's packed R, published for the tree
    void* Ynode = nullptr;     // W x n x n  (slot c holds the step folding chain c)
    void* Tnode = nullptr;     // W x n(n+1)/2
    void* tau_node = nullptr;  // W x n
    int* cnt = nullptr;        // W x levels node arrival counters
    // explicit Q with signs: when set, the root slab of member b starts as
    // D_b = diag(sign of R_b's diagonal) instead of I_n (R_b at sgnR + b*sgn_sr)
    const void* sgnR = nullptr;
    int64_t sgn_ldr = 0, sgn_sr = 0;
};

enum ApplyMode { MODE_QT = 0, MODE_Q = 1, MODE_FORMQ = 2 };

// Profiling hook: when set, events are recorded on the launch stream right
// before and after the chain (leaf) kernel of a phase:
// 0 factor, 1 apply Q^T, 2 apply Q, 3 form Q.
constexpr int NPHASE = 4;
struct PhaseEvents {
    hipEvent_t start[NPHASE] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t stop[NPHASE] = {nullptr, nullptr, nullptr, nullptr};
};
extern PhaseEvents g_phase;
inline void phase_begin(int p, hipStream_t st) {
    if (g_phase.start[p]) (void)hipEventRecord(g_phase.start[p], st);
}
inline void phase_end(int p, hipStream_t st) {
    if (g_phase.stop[p]) (void)hipEventRecord(g_phase.stop[p], st);
}

// Launchers (defined in the .hip files).  Return a hipError_t.
// TSQR of A into the reflectors (in A), the tree of Q factors (wk) and R
// (row-major, ldr; zeros below the diagonal when zero_lower; R may be null).
// want_q = false: only R and the leaf reflectors are produced (no implicit Q
// is kept, so tau, T and the tree's reflectors are not formed or stored).
// rstride: elements between the R factors of a batch's members (0 for one matrix).
hipError_t launch_factor(bool f64, const Geom& g, void* A, int64_t lda, const Work& wk, void* R, int64_t ldr,
                         int64_t rstride, bool zero_lower, bool want_q, int max_polls, hipStream_t st);
// Host-side geometry and workspace layout (tsqr_capi.hip).
struct GeomOpts {
    int block_rows = 0, chains = 0, arity = 0, flags = 0;
};
// Polls of a bounded wait in the panel-pipelined tree before it gives up.
constexpr int kDefaultMaxPolls = 1 << 22;
// Device address of the library's status word on the current device (bit 0:
// a bounded wait gave up), or null if it could not be obtained.
int* status_word();
// Stream-ordered workspace allocation from the library's memory pool on the
// current device, which keeps up to kPoolKeepBytes of freed memory cached
// across synchronisations (the default pool returns it at every one, so each
// call would map its workspace again on the host).  Free with hipFreeAsync.
constexpr uint64_t kPoolKeepBytes = 2ull << 30;
hipError_t ws_malloc(void** p, size_t bytes, hipStream_t st);
int make_geom_opts(int64_t m, int64_t n, const GeomOpts& o, Geom* g);
size_t work_bytes(const Geom& g, bool f64);
void work_carve(Work* w, const Geom& g, bool f64);

// Block shapes of the factor kernel: rows per block h for NC padded columns.
bool wave_shape_ok(int NC, int h);
int wave_default_h(int NC);
hipError_t launch_copy_r(bool f64, int64_t n, const void* Rsrc, int64_t lds, void* R, int64_t ldr, bool zero_lower,
                         hipStream_t st);
hipError_t launch_apply(bool store_f64, bool compute_f64, const Geom& g, const void* Y, int64_t ldy,
                        const Work& wk, void* B, int64_t ldb, int64_t k, int mode, hipStream_t st);
// [I_n; 0] at the top of every member's thin Q (the slab of each member's root chain).
hipError_t launch_init_formq(bool f64, int64_t members, int64_t mb, int64_t n, void* Q, int64_t ldq, const void* sgnR,
                             int64_t sgn_ldr, int64_t sgn_sr, hipStream_t st);
// Whether launch_apply takes the wide kernels (a 16-column tile of B over all
// 64 rows of a block per wave) for k columns on geometry g.
bool apply_wide(const Geom& g, int64_t k);
hipError_t launch_fill_identity(bool f64, int64_t m, int64_t n, void* Q, int64_t ldq, hipStream_t st);
// Least squares steps after Q^T B (tsqr_lstsq.hip): X = R^{-1} B(0:n, :) in
// place, and the 2-norms of rows [r0, m) of each of the k columns of B.
hipError_t launch_trsm_upper(bool f64, int64_t n, const void* R, int64_t ldr, void* B, int64_t ldb, int64_t k,
                             hipStream_t st);
hipError_t launch_colnorm(bool f64, int64_t r0, int64_t m, const void* B, int64_t ldb, int64_t k, void* rnorm,
                          hipStream_t st);
// CholeskyQR (passes = 1) or CholeskyQR2 (passes = 2) of A into Q and R.
hipError_t launch_cholqr(bool f64, int64_t m, int64_t n, const void* A, int64_t lda, void* Q, int64_t ldq, void* R,
                         int64_t ldr, int passes, hipStream_t st);
// Modified Gram-Schmidt of A into Q and R (n + 1 passes over the rows).
hipError_t launch_mgs(bool f64, int64_t m, int64_t n, const void* A, int64_t lda, void* Q, int64_t ldq, void* R,
                      int64_t ldr, hipStream_t st);
hipError_t launch_backward(bool f64, int64_t batch, int64_t m, int64_t n, const void* Q, int64_t ldq, int64_t sq,
                           const void* R, int64_t ldr, int64_t sr, const void* dQ, int64_t lddq, int64_t sdq,
                           const void* dR, int64_t lddr, int64_t sdr, void* dA, int64_t ldda, int64_t sda,
                           hipStream_t st);

}  // namespace tsqr

#ifdef __HIP_DEVICE_COMPILE__
#define TSQR_DEVICE 1
#endif

namespace tsqr {
namespace dev {

// ---- cross-lane helpers (wave64) ----
// DPP controls: quad_perm [1,0,3,2] (xor 1), quad_perm [2,3,0,1] (xor 2),
// row_half_mirror (lane i <-> 7-i within each group of 8).
constexpr int DPP_XOR1 = 0xB1;
constexpr int DPP_XOR2 = 0x4E;
constexpr int DPP_HMIRROR = 0x141;

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    int x = __builtin_bit_cast(int, v);
    x = __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(float, x);
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    struct P { int lo, hi; };
    P p = __builtin_bit_cast(P, v);
    p.lo = __builtin_amdgcn_update_dpp(0, p.lo, CTRL, 0xF, 0xF, false);
    p.hi = __builtin_amdgcn_update_dpp(0, p.hi, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, p);
}

// Sum over the 8 consecutive lanes of a group; every lane of the group gets the
// same (bitwise) result because each step adds the same two operands.
template <typename T>
__device__ __forceinline__ T sum8(T v) {
    v += dpp<DPP_XOR1>(v);
    v += dpp<DPP_XOR2>(v);
    v += dpp<DPP_HMIRROR>(v);
    return v;
}

__device__ __forceinline__ double shfl(double v, int src) {
    struct P { int lo, hi; };
    P p = __builtin_bit_cast(P, v);
    p.lo = __builtin_amdgcn_ds_bpermute(src << 2, p.lo);
    p.hi = __builtin_amdgcn_ds_bpermute(src << 2, p.hi);
    return __builtin_bit_cast(double, p);
}
__device__ __forceinline__ float shfl(float v, int src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, v)));
}

// ---- MFMA 16x16x4 (one block) in FP64 and FP32 ----
// Operand layout (lane l of a wave64):
//   A (16x4):  A[l % 16][l / 16]
//   B (4x16):  B[l / 16][l % 16]
//   D (16x16): FP32: D[4*(l/16) + r][l % 16];  FP64: D[4*r + l/16][l % 16]
//   (r = 0..3; the FP64 form was confirmed on gfx950 by a lane-layout probe)
// orow(l/16, r) gives the output row of register r.
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename C>
struct Mfma;
template <>
struct Mfma<double> {
    typedef d4 acc;
    __device__ __forceinline__ static acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __host__ __device__ static constexpr int orow(int l4, int r) { return 4 * r + l4; }
    // register and 16-lane row holding output row rho (inverse of orow)
    __host__ __device__ static constexpr int row_reg(int rho) { return rho >> 2; }
    __host__ __device__ static constexpr int row_l4(int rho) { return rho & 3; }
};
template <>
struct Mfma<float> {
    typedef f4 acc;
    __device__ __forceinline__ static acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __host__ __device__ static constexpr int orow(int l4, int r) { return 4 * l4 + r; }
    __host__ __device__ static constexpr int row_reg(int rho) { return rho & 3; }
    __host__ __device__ static constexpr int row_l4(int rho) { return rho >> 2; }
};

// ---- hand-over between workgroups of one launch ----
// The L2 caches of the chip's XCDs are not coherent with one another for
// ordinary stores, so a device-scope fence has to write a whole L2 back to
// memory; with many workgroups fencing while others stream output, those
// write-backs serialise.  Data handed from one workgroup to another inside a
// launch (a published R factor or slab) therefore uses device-coherent
// accesses instead: written through to memory (pub_store), awaited before the
// arrival is counted (pub_wait), and read past any non-coherent cached copy
// (pub_load).  No other memory needs to be visible at that point.
template <typename T>
struct PubBits;
template <>
struct PubBits<double> { typedef unsigned long long U; };
template <>
struct PubBits<float> { typedef unsigned int U; };

template <typename T>
__device__ __forceinline__ void pub_store(T* p, T v) {
    typedef typename PubBits<T>::U U;
    __hip_atomic_store((U*)p, __builtin_bit_cast(U, v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T pub_load(const T* p) {
    typedef typename PubBits<T>::U U;
    return __builtin_bit_cast(T, __hip_atomic_load((U*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
// every vector memory access of this wave has completed (stores acknowledged)
__device__ __forceinline__ void pub_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

}  // namespace dev
}  // namespace tsqr
