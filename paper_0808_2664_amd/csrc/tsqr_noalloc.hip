// R-only TSQR that allocates nothing (tsqr_factor_noalloc), for callers that
// cannot allocate device memory: code under stream capture, tight serving
// loops, harnesses that forbid allocation.
//
// It runs the same kernels as tsqr_factor with q_out = NULL (chains, then the
// tree; no implicit Q is formed), with the factor's scratch memory -- the
// chains' published R factors and the tree's counters -- taken from a fixed
// device array instead of a stream-ordered allocation.  The array is a
// file-scope __device__ variable: each device the library runs on holds its
// own copy for the life of the process.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol); the
// device address is obtained once per device with hipGetSymbolAddress and
// used everywhere after that.
//
// Every call on a device shares that device's array and leaves its contents
// behind; the counters that must start at zero are cleared by a fill kernel
// at the start of each call.  Calls that overlap on one device (two streams,
// or two host threads) race on the array: the caller serialises them.
#include "../../include/tsqr.h"
#include "tsqr_common.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)40 << 20;  // 40 MiB per device

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices];
bool g_scratch_done[kMaxDevices];

// Device address of this device's scratch array, or null (HIP error kept).
void* scratch_ptr(hipError_t* err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *err = e != hipSuccess ? e : hipErrorInvalidDevice;
        return nullptr;
    }
    if (!g_scratch_done[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
        g_scratch_done[dev] = true;
    }
    return g_scratch_ptr[dev];
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

namespace tsqr {
int make_geom(int64_t m, int64_t n, const tsqr_opts* o, Geom* g);
int record_hip_error(hipError_t e);
}

extern "C" {

size_t tsqr_factor_noalloc_scratch_bytes(void) { return kScratchBytes; }

int tsqr_factor_noalloc(int dtype, int64_t m, int64_t n, void* A, int64_t lda, void* R, int64_t ldr,
                        const tsqr_opts* opts, void* stream) {
    if (dtype != TSQR_F32 && dtype != TSQR_F64) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return n > m ? -2 : -3;
    if (n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!R) return -6;
    if (ldr < n) return -7;
    if (opts && (opts->flags & ~TSQR_FLAGS_ALL)) return -8;
    tsqr::Geom g;
    int rc = tsqr::make_geom(m, n, opts, &g);
    if (rc != 0) return rc == -1 ? -2 : rc;
    const bool f64 = dtype == TSQR_F64;
    const size_t es = f64 ? 8 : 4;
    // scratch: each chain's published R (slots as the factor kernel indexes
    // them), then the W x (levels + 1) counters
    const size_t ncp = g.NC <= 16 ? 16 : (size_t)g.NC;
    const size_t rp = ncp * (ncp + 1) / 2, nn = (size_t)n * (size_t)n;
    const size_t slot = nn > rp ? nn : rp;
    const size_t rbuf = al256((size_t)g.W * slot * es);
    const size_t ncnt = (size_t)g.W * (size_t)(g.levels + 1);
    if (rbuf + al256(ncnt * sizeof(int)) > kScratchBytes) return TSQR_ERR_SCRATCH;
    hipError_t e = hipSuccess;
    char* base = (char*)scratch_ptr(&e);
    if (!base) return tsqr::record_hip_error(e);
    tsqr::Work wk;
    wk.base = base;
    wk.bytes = kScratchBytes;
    wk.Rbuf = base;
    wk.cnt = (int*)(base + rbuf);
    // tau, T and the tree's reflectors are neither formed nor stored without
    // an implicit Q (the kernel is instantiated without them); their pointers
    // are set to valid memory all the same
    wk.tau_blk = wk.T_blk = wk.Ynode = wk.Tnode = wk.tau_node = base;
    e = tsqr::launch_factor(f64, g, A, lda, wk, R, ldr, 0, true, false, opts ? opts->max_polls : 0,
                            (hipStream_t)stream);
    return e == hipSuccess ? 0 : tsqr::record_hip_error(e);
}

}  // extern "C"
