// TSQR factorisation kernel for gfx950 (paper Sec. 2.1).
//
// k_wave_tsqr: one wave (one workgroup of 64 lanes) per chain.  The wave runs
// sequential TSQR over its chain's row blocks (flat tree: block 0 is a plain
// Householder QR, every later block is factored stacked under the R kept on
// chip), so A is read once and the reflectors are written once (Table 4,
// Eq. TSQR_seq_runtime: 2mn words).  The chain R factors are then reduced on
// the tree inside the same launch: a node is performed by the wave that
// finishes its last child (see tsqr_wave.hpp for the engine and the tree).
#include "tsqr_wave.hpp"

namespace tsqr {

__global__ void k_zero_i32(int* __restrict__ p, int64_t count) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = 0;
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

// Block height of the factor kernel: 64 rows (SG = 4 row groups of 16), so a
// lane holds at most 64 entries of the tile and the first block of a chain
// holds its n <= 64 heads.
bool wave_shape_ok(int NC, int h) {
    (void)NC;
    return h == 64;
}

int wave_default_h(int NC) {
    (void)NC;
    return 64;
}

template <typename T, int NP, int SG, bool WQ>
hipError_t launch_wave(const Geom& g, T* A, int64_t lda, const Work& wk, const TreeArgs& ta, hipStream_t st);
// defined in tsqr_factor_inst.hip, one object per instantiation
#define TSQR_FACTOR_EXTERN(T, NP, WQ) \
    extern template hipError_t launch_wave<T, NP, 4, WQ>(const Geom&, T*, int64_t, const Work&, const TreeArgs&, hipStream_t);
TSQR_FACTOR_EXTERN(double, 1, true)
TSQR_FACTOR_EXTERN(double, 2, true)
TSQR_FACTOR_EXTERN(double, 4, true)
TSQR_FACTOR_EXTERN(double, 1, false)
TSQR_FACTOR_EXTERN(double, 2, false)
TSQR_FACTOR_EXTERN(double, 4, false)
TSQR_FACTOR_EXTERN(float, 1, true)
TSQR_FACTOR_EXTERN(float, 2, true)
TSQR_FACTOR_EXTERN(float, 4, true)
TSQR_FACTOR_EXTERN(float, 1, false)
TSQR_FACTOR_EXTERN(float, 2, false)
TSQR_FACTOR_EXTERN(float, 4, false)
#undef TSQR_FACTOR_EXTERN

template <typename T, bool WQ>
static hipError_t factor_t(const Geom& g, T* A, int64_t lda, const Work& wk, const TreeArgs& ta, hipStream_t st) {
    const int NP = g.NC <= 16 ? 1 : g.NC / 16;
    const int SG = g.h / 16;
    if (SG != 4) return hipErrorInvalidValue;
    switch (NP) {
        case 4: return launch_wave<T, 4, 4, WQ>(g, A, lda, wk, ta, st);
        case 2: return launch_wave<T, 2, 4, WQ>(g, A, lda, wk, ta, st);
        case 1: return launch_wave<T, 1, 4, WQ>(g, A, lda, wk, ta, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_factor(bool f64, const Geom& g, void* A, int64_t lda, const Work& wk, void* R, int64_t ldr,
                         int64_t rstride, bool zero_lower, bool want_q, int max_polls, hipStream_t st) {
    int* status = status_word();
    if (!status) return hipErrorInvalidDevice;
    const int64_t ncnt = (int64_t)g.W * (g.levels + 1);
    k_zero_i32<<<(unsigned)((ncnt + 255) / 256), 256, 0, st>>>(wk.cnt, ncnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    TreeArgs ta{wk.cnt, R, ldr, zero_lower ? 1 : 0, max_polls > 0 ? max_polls : kDefaultMaxPolls, status, rstride};
    phase_begin(0, st);
    if (want_q)
        e = f64 ? factor_t<double, true>(g, (double*)A, lda, wk, ta, st)
                : factor_t<float, true>(g, (float*)A, lda, wk, ta, st);
    else
        e = f64 ? factor_t<double, false>(g, (double*)A, lda, wk, ta, st)
                : factor_t<float, false>(g, (float*)A, lda, wk, ta, st);
    phase_end(0, st);
    return e;
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
