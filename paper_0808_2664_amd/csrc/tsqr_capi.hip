// C ABI of libtsqr.so: argument checks, tree geometry, workspace and the
// launch sequences of TSQR (Sec. 2.1) and its implicit Q.
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/tsqr.h"
#include "tsqr_common.hpp"

using tsqr::Geom;
using tsqr::Work;

struct tsqr_qtree_s {
    int kind = 0;  // 0 TSQR, 1 CAQR
    bool f64 = true;
    Geom g;
    void* A = nullptr;  // borrowed reflector storage
    int64_t lda = 0;
    Work wk;
    hipStream_t stream = nullptr;
    // CAQR: one TSQR tree per panel, panel p acting on rows/cols p*panel..
    std::vector<tsqr_qtree_s*> panels;
    int64_t m = 0, n = 0, panel = 0;
    int64_t members = 1;  // batched TSQR: independent stacked matrices of m / members rows
};

static thread_local int g_last_hip = 0;

namespace tsqr {
PhaseEvents g_phase;

// One workspace pool per device, made on first use; if the pool cannot be
// made, the device's default pool serves.
static std::mutex g_pool_mu;
static hipMemPool_t g_pool[64];
static bool g_pool_tried[64];

static hipMemPool_t device_pool(int dev) {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (!g_pool_tried[dev]) {
        g_pool_tried[dev] = true;
        hipMemPoolProps props;
        memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        if (hipMemPoolCreate(&pool, &props) == hipSuccess) {
            uint64_t keep = kPoolKeepBytes;
            if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) == hipSuccess) {
                g_pool[dev] = pool;
            } else {
                (void)hipMemPoolDestroy(pool);
            }
        }
        (void)hipGetLastError();
    }
    return g_pool[dev];
}

hipError_t ws_malloc(void** p, size_t bytes, hipStream_t st) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipMemPool_t pool = (dev >= 0 && dev < 64) ? device_pool(dev) : nullptr;
    return pool ? hipMallocFromPoolAsync(p, bytes, pool, st) : hipMallocAsync(p, bytes, st);
}
}

extern "C" int tsqr_release_workspace_pools(void) {
    std::lock_guard<std::mutex> lock(tsqr::g_pool_mu);
    hipError_t first = hipSuccess;
    for (int dev = 0; dev < 64; ++dev)
        if (tsqr::g_pool[dev]) {
            hipError_t e = hipMemPoolTrimTo(tsqr::g_pool[dev], 0);
            if (e != hipSuccess && first == hipSuccess) first = e;
        }
    if (first != hipSuccess) {
        g_last_hip = (int)first;
        return TSQR_ERR_HIP;
    }
    return 0;
}

static int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return e == hipErrorOutOfMemory ? TSQR_ERR_NOMEM : TSQR_ERR_HIP;
}

// The library's status word (bit 0: a bounded wait of the pipelined tree
// gave up); each device holds its own copy.  Kernels receive its device
// address as an argument; the host side obtains that address once per device.
static __device__ __align__(256) int g_status;

namespace tsqr {

int record_hip_error(hipError_t e) { return hip_fail(e); }

int* status_word() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    static int* addr[64];
    static bool done[64];
    if (!done[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_status)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        addr[dev] = (int*)p;
        done[dev] = true;
    }
    return addr[dev];
}

int padded_nc(int64_t n) { return n <= 8 ? 8 : n <= 16 ? 16 : n <= 32 ? 32 : 64; }

// Chains by default: one one-wave chain per SIMD (4 per CU on 256 CUs), the
// number the factor kernel keeps resident at once.
constexpr int64_t kDefaultChains = 1024;

// Tree geometry for (m, n): chains of whole blocks, the last chain absorbing
// a remainder too short to hold an n x n leaf (a chain's first block must hold
// n rows: its R is an n x n triangle).
int make_geom(int64_t m, int64_t n, const tsqr_opts* o, Geom* g);

int make_geom_opts(int64_t m, int64_t n, const GeomOpts& go, Geom* g) {
    tsqr_opts o{go.block_rows, go.chains, go.arity, go.flags, 0};
    return make_geom(m, n, &o, g);
}

int make_geom(int64_t m, int64_t n, const tsqr_opts* o, Geom* g) {
    if (n < 1 || n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    if (m < n) return -1;
    const int NC = padded_nc(n);
    int h = (o && o->block_rows) ? o->block_rows : wave_default_h(NC);
    int chains = (o && o->chains) ? o->chains : 0;
    int arity = (o && o->arity) ? o->arity : 2;
    const int flags = o ? o->flags : 0;
    if (flags & ~TSQR_FLAGS_ALL) return TSQR_ERR_UNSUPPORTED;
    if (!wave_shape_ok(NC, h)) return TSQR_ERR_UNSUPPORTED;
    if (arity < 2 || chains < 0) return TSQR_ERR_UNSUPPORTED;
    const int64_t blocks_total = (m + h - 1) / h;
    int64_t W0 = chains > 0 ? chains : (blocks_total < kDefaultChains ? blocks_total : kDefaultChains);
    if (W0 < 1) W0 = 1;
    if (W0 > blocks_total) W0 = blocks_total;
    int64_t per = (m + W0 - 1) / W0;               // rows per chain before rounding
    int64_t S = ((per + h - 1) / h) * h;           // whole blocks
    int64_t W = (m + S - 1) / S;
    if (W > 1 && m - (W - 1) * S < n) W -= 1;      // merge a too-short last chain
    if (W > 0x7fffffff) return TSQR_ERR_UNSUPPORTED;
    g->m = m;
    g->n = n;
    g->h = h;
    g->S = S;
    g->W = (int)W;
    g->arity = arity;
    int levels = 0;
    int64_t stride = 1;
    while (stride < W) {
        stride *= arity;
        ++levels;
    }
    g->levels = levels;
    const int64_t last = m - (W - 1) * S;
    g->nblocks = (W - 1) * (S / h) + (last + h - 1) / h;
    g->NC = padded_nc(n);
    g->flags = ((flags & TSQR_FLAG_TREE_LEVELWISE) ? TREE_LEVELWISE : 0) | ((flags & TSQR_FLAG_ONE_WAVE) ? ONE_WAVE : 0);
    g->mb = m;
    g->cpm = (int)W;
    g->bpm = g->nblocks;
    return 0;
}

// Forest geometry of `batch` stacked matrices of mb rows (Geom::mb): each
// member is cut into the same cpm chains and reduced by its own tree of
// arity a, so cpm must be a power of a and the one-member geometry must have
// exactly cpm chains.  chains (opts) = chains per member; 0 picks the largest
// such power of a that gives about `target` chains in all.
int make_geom_batch(int64_t batch, int64_t mb, int64_t n, const tsqr_opts* o, int64_t target, Geom* g) {
    if (batch < 1) return -2;
    const int arity = (o && o->arity) ? o->arity : 2;
    if (arity < 2) return TSQR_ERR_UNSUPPORTED;
    int64_t cpm = 1;
    if (o && o->chains) {
        cpm = o->chains;
    } else {
        while (cpm * arity * batch <= target) cpm *= arity;
    }
    for (;;) {
        int64_t p = 1;
        while (p < cpm) p *= arity;
        if (p != cpm) return TSQR_ERR_UNSUPPORTED;  // not a power of the arity
        tsqr_opts o1 = o ? *o : tsqr_opts{0, 0, 0, 0, 0};
        o1.chains = (int32_t)cpm;
        o1.arity = arity;
        Geom g1;
        int rc = make_geom(mb, n, &o1, &g1);
        if (rc != 0) return rc;
        if (g1.W == cpm) {
            if (batch * cpm > 0x7fffffff || batch * mb < mb) return TSQR_ERR_UNSUPPORTED;
            *g = g1;
            g->m = batch * mb;
            g->W = (int)(batch * cpm);
            g->nblocks = batch * g1.nblocks;
            g->mb = mb;
            g->cpm = (int)cpm;
            g->bpm = g1.nblocks;
            return 0;
        }
        // fewer chains than asked for (short member): a smaller power
        if ((o && o->chains) || cpm == 1) return TSQR_ERR_UNSUPPORTED;
        cpm /= arity;
    }
}

// Elements of one chain's published R: its packed upper triangle (rows of
// length 16 * panels), or n * n if larger.
static size_t rslot_elems(const Geom& g) {
    const size_t ncp = g.NC <= 16 ? 16 : (size_t)g.NC;
    const size_t rp = ncp * (ncp + 1) / 2, nn = (size_t)g.n * g.n;
    return nn > rp ? nn : rp;
}

size_t work_bytes(const Geom& g, bool f64) {
    const size_t es = f64 ? 8 : 4;
    const size_t n = (size_t)g.n, tri = n * (n + 1) / 2;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t ncnt = (size_t)g.W * (g.levels + 1);
    return al(g.nblocks * n * es) + al(g.nblocks * tri * es) + al((size_t)g.W * rslot_elems(g) * es) +
           al((size_t)g.W * n * n * es) + al((size_t)g.W * tri * es) + al((size_t)g.W * n * es) + al(ncnt * 4);
}

void work_carve(Work* w, const Geom& g, bool f64) {
    const size_t es = f64 ? 8 : 4;
    const size_t n = (size_t)g.n, tri = n * (n + 1) / 2;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char* p = (char*)w->base;
    w->tau_blk = p;
    p += al(g.nblocks * n * es);
    w->T_blk = p;
    p += al(g.nblocks * tri * es);
    w->Rbuf = p;
    p += al((size_t)g.W * rslot_elems(g) * es);
    w->Ynode = p;
    p += al((size_t)g.W * n * n * es);
    w->Tnode = p;
    p += al((size_t)g.W * tri * es);
    w->tau_node = p;
    p += al((size_t)g.W * n * es);
    w->cnt = (int*)p;
}

}  // namespace tsqr

// ------------------------------------------------------------------ helpers

static int check_dtype(int dtype) { return dtype == TSQR_F32 || dtype == TSQR_F64; }

// TSQR of a device matrix into a fresh handle (shared by tsqr_factor and the
// CAQR panels).  R: optional; r_upper_only keeps what is below R's diagonal.
static int factor_geom(int dtype, const Geom& g, void* A, int64_t lda, void* R, int64_t ldr, int64_t rstride,
                       bool r_upper_only, const tsqr_opts* opts, tsqr_qtree_s** out, hipStream_t st, bool want_q);

static int factor_impl(int dtype, int64_t m, int64_t n, void* A, int64_t lda, void* R, int64_t ldr,
                       bool r_upper_only, const tsqr_opts* opts, tsqr_qtree_s** out, hipStream_t st,
                       bool want_q = true, int extra_gflags = 0) {
    Geom g;
    int rc = tsqr::make_geom(m, n, opts, &g);
    if (rc != 0) return rc;
    g.flags |= extra_gflags;
    return factor_geom(dtype, g, A, lda, R, ldr, 0, r_upper_only, opts, out, st, want_q);
}

static int factor_geom(int dtype, const Geom& g, void* A, int64_t lda, void* R, int64_t ldr, int64_t rstride,
                       bool r_upper_only, const tsqr_opts* opts, tsqr_qtree_s** out, hipStream_t st, bool want_q) {
    const int64_t m = g.m, n = g.n;
    const bool f64 = dtype == TSQR_F64;
    tsqr_qtree_s* q = new tsqr_qtree_s();
    q->kind = 0;
    q->f64 = f64;
    q->g = g;
    q->A = A;
    q->lda = lda;
    q->stream = st;
    q->m = m;
    q->n = n;
    q->members = g.m / g.mb;
    q->wk.bytes = tsqr::work_bytes(g, f64);
    hipError_t e = tsqr::ws_malloc(&q->wk.base, q->wk.bytes, st);
    if (e != hipSuccess) {
        delete q;
        return hip_fail(e);
    }
    tsqr::work_carve(&q->wk, g, f64);
    e = tsqr::launch_factor(f64, g, A, lda, q->wk, R, ldr, rstride, !r_upper_only, want_q, opts ? opts->max_polls : 0,
                            st);
    if (e != hipSuccess) {
        (void)hipFreeAsync(q->wk.base, st);
        delete q;
        return hip_fail(e);
    }
    *out = q;
    return 0;
}

static void destroy_impl(tsqr_qtree_s* q) {
    if (!q) return;
    for (auto* p : q->panels) destroy_impl(p);
    if (q->wk.base) (void)hipFreeAsync(q->wk.base, q->stream);
    delete q;
}

// ------------------------------------------------------------------ C ABI

extern "C" {

int tsqr_factor(int dtype, int64_t m, int64_t n, void* A, int64_t lda, void* R, int64_t ldr,
                const tsqr_opts* opts, tsqr_qtree* q_out, void* stream) {
    if (!check_dtype(dtype)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return n > m ? -2 : -3;
    if (n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    if (!A) return -4;
    if (lda < n) return -5;
    if (R && ldr < n) return -7;
    if (opts && (opts->flags & ~TSQR_FLAGS_ALL)) return -8;
    if (!R && !q_out) return -9;
    tsqr_qtree_s* q = nullptr;
    int rc = factor_impl(dtype, m, n, A, lda, R, ldr, false, opts, &q, (hipStream_t)stream, q_out != nullptr);
    if (rc != 0) return rc == -1 ? -2 : rc;
    if (q_out) *q_out = q;
    else destroy_impl(q);
    return 0;
}

int tsqr_factor_batched(int dtype, int64_t batch, int64_t m, int64_t n, void* A, int64_t lda, void* R, int64_t ldr,
                        int64_t strideR, const tsqr_opts* opts, tsqr_qtree* q_out, void* stream) {
    if (!check_dtype(dtype)) return -1;
    if (batch < 1 || batch > 65535) return -2;
    if (m < 1) return -3;
    if (n < 1 || n > m) return n > m ? -3 : -4;
    if (n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    if (!A) return -5;
    if (lda < n) return -6;
    if (R && ldr < n) return -8;
    if (R && batch > 1 && strideR < n * ldr) return -9;
    if (opts && (opts->flags & ~TSQR_FLAGS_ALL)) return -10;
    if (!R && !q_out) return -11;
    Geom g;
    // about one chain per SIMD (two for FP32, whose factor kernel fits two waves)
    int rc = tsqr::make_geom_batch(batch, m, n, opts, dtype == TSQR_F64 ? 1024 : 2048, &g);
    if (rc != 0) return rc == -1 ? -3 : rc;
    tsqr_qtree_s* q = nullptr;
    rc = factor_geom(dtype, g, A, lda, R, ldr, strideR, false, opts, &q, (hipStream_t)stream, q_out != nullptr);
    if (rc != 0) return rc;
    if (q_out) *q_out = q;
    else destroy_impl(q);
    return 0;
}

static int apply_impl(tsqr_qtree_s* q, int64_t k, void* B, int64_t ldb, int mode, hipStream_t st);

static int apply_one(tsqr_qtree_s* q, int64_t k, void* B, int64_t ldb, int mode, bool compute_f64,
                     hipStream_t st) {
    hipError_t e = tsqr::launch_apply(q->f64, compute_f64, q->g, q->A, q->lda, q->wk, B, ldb, k, mode, st);
    return e == hipSuccess ? 0 : hip_fail(e);
}

// CAQR: Q = Q_0 Q_1 ... Q_{P-1}, panel p acting on rows p*b .. m-1.
static int apply_impl(tsqr_qtree_s* q, int64_t k, void* B, int64_t ldb, int mode, hipStream_t st) {
    if (q->kind == 0) return apply_one(q, k, B, ldb, mode, q->f64, st);
    const size_t es = q->f64 ? 8 : 4;
    const int P = (int)q->panels.size();
    for (int i = 0; i < P; ++i) {
        const int p = (mode == tsqr::MODE_QT) ? i : P - 1 - i;
        char* Bp = (char*)B + (size_t)p * q->panel * ldb * es;
        int rc = apply_one(q->panels[p], k, Bp, ldb, mode == tsqr::MODE_FORMQ ? tsqr::MODE_Q : mode, q->f64, st);
        if (rc) return rc;
    }
    return 0;
}

int tsqr_apply_qt(tsqr_qtree q, int64_t k, void* B, int64_t ldb, void* stream) {
    if (!q) return -1;
    if (k < 0) return -2;
    if (k == 0) return 0;
    if (!B) return -3;
    if (ldb < k) return -4;
    return apply_impl(q, k, B, ldb, tsqr::MODE_QT, (hipStream_t)stream);
}

int tsqr_lstsq(int dtype, int64_t m, int64_t n, void* A, int64_t lda, int64_t k, void* B, int64_t ldb, void* rnorm,
               const tsqr_opts* opts, void* stream) {
    if (!check_dtype(dtype)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return n > m ? -2 : -3;
    if (n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    if (!A) return -4;
    if (lda < n) return -5;
    if (k < 0) return -6;
    if (k > 0 && !B) return -7;
    if (k > 0 && ldb < k) return -8;
    if (opts && (opts->flags & ~TSQR_FLAGS_ALL)) return -10;
    if (k > ((int64_t)1 << 36)) return TSQR_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = dtype == TSQR_F64;
    void* R = nullptr;
    hipError_t e = tsqr::ws_malloc(&R, (size_t)(n * n) * (f64 ? 8 : 4), st);
    if (e != hipSuccess) return hip_fail(e);
    tsqr_qtree_s* q = nullptr;
    // without right-hand sides only R is needed (no implicit Q is formed)
    int rc = factor_impl(dtype, m, n, A, lda, R, n, false, opts, &q, st, k > 0);
    if (rc == -1) rc = -2;
    if (rc == 0 && k > 0) {
        rc = apply_one(q, k, B, ldb, tsqr::MODE_QT, f64, st);
        if (rc == 0) {
            e = tsqr::launch_trsm_upper(f64, n, R, n, B, ldb, k, st);
            if (e != hipSuccess) rc = hip_fail(e);
        }
        if (rc == 0 && rnorm) {
            e = tsqr::launch_colnorm(f64, n, m, B, ldb, k, rnorm, st);
            if (e != hipSuccess) rc = hip_fail(e);
        }
    }
    if (q) destroy_impl(q);
    (void)hipFreeAsync(R, st);
    return rc;
}

int tsqr_cholqr(int dtype, int64_t m, int64_t n, const void* A, int64_t lda, void* Q, int64_t ldq, void* R,
                int64_t ldr, int passes, void* stream) {
    if (!check_dtype(dtype)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return n > m ? -2 : -3;
    if (n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!Q) return -6;
    if (ldq < n) return -7;
    if (!R) return -8;
    if (ldr < n) return -9;
    if (passes != 1 && passes != 2) return -10;
    hipError_t e = tsqr::launch_cholqr(dtype == TSQR_F64, m, n, A, lda, Q, ldq, R, ldr, passes, (hipStream_t)stream);
    return e == hipSuccess ? 0 : hip_fail(e);
}

int tsqr_mgs(int dtype, int64_t m, int64_t n, const void* A, int64_t lda, void* Q, int64_t ldq, void* R,
             int64_t ldr, void* stream) {
    if (!check_dtype(dtype)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return n > m ? -2 : -3;
    if (n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!Q) return -6;
    if (ldq < n || (Q == A && ldq != lda)) return -7;
    if (!R) return -8;
    if (ldr < n) return -9;
    hipError_t e = tsqr::launch_mgs(dtype == TSQR_F64, m, n, A, lda, Q, ldq, R, ldr, (hipStream_t)stream);
    return e == hipSuccess ? 0 : hip_fail(e);
}

int tsqr_apply_q(tsqr_qtree q, int64_t k, void* B, int64_t ldb, void* stream) {
    if (!q) return -1;
    if (k < 0) return -2;
    if (k == 0) return 0;
    if (!B) return -3;
    if (ldb < k) return -4;
    return apply_impl(q, k, B, ldb, tsqr::MODE_Q, (hipStream_t)stream);
}

int tsqr_form_q(tsqr_qtree q, void* Q, int64_t ldq, void* stream) {
    if (!q) return -1;
    if (!Q) return -2;
    if (ldq < q->n) return -3;
    hipStream_t st = (hipStream_t)stream;
    if (q->kind != 0) {
        // CAQR: Q [I_n; 0] by applying the panel trees in reverse order
        hipError_t e = tsqr::launch_fill_identity(q->f64, q->m, q->n, Q, ldq, st);
        if (e != hipSuccess) return hip_fail(e);
        return apply_impl(q, q->n, Q, ldq, tsqr::MODE_Q, st);
    }
    hipError_t e = tsqr::launch_init_formq(q->f64, q->members, q->m / q->members, q->n, Q, ldq, nullptr, 0, 0, st);
    if (e != hipSuccess) return hip_fail(e);
    return apply_one(q, q->n, Q, ldq, tsqr::MODE_FORMQ, q->f64, st);
}

int tsqr_form_q_signed(tsqr_qtree q, void* Q, int64_t ldq, void* R, int64_t ldr, int64_t strideR, void* stream) {
    if (!q) return -1;
    if (!Q) return -2;
    if (ldq < q->n) return -3;
    if (!R) return -4;
    if (ldr < q->n) return -5;
    if (q->members > 1 && strideR < q->n * ldr) return -6;
    hipStream_t st = (hipStream_t)stream;
    const int dt = q->f64 ? TSQR_F64 : TSQR_F32;
    if (q->kind != 0) {
        // CAQR: the explicit Q, then the signs in a pass of their own
        int rc = tsqr_form_q(q, Q, ldq, stream);
        return rc != 0 ? rc : tsqr_sign_normalize(dt, q->m, q->n, Q, ldq, R, ldr, stream);
    }
    // the root slab of each member starts as D = diag(sign R_jj): Q D in the
    // explicit-Q pass itself (D is +-1, so the bits are those of Q, column j
    // negated where d_j = -1); R's rows afterwards, in stream order
    tsqr::Work wk = q->wk;
    wk.sgnR = R;
    wk.sgn_ldr = ldr;
    wk.sgn_sr = strideR;
    hipError_t e = tsqr::launch_init_formq(q->f64, q->members, q->m / q->members, q->n, Q, ldq, R, ldr, strideR, st);
    if (e == hipSuccess) e = tsqr::launch_apply(q->f64, q->f64, q->g, q->A, q->lda, wk, Q, ldq, q->n, tsqr::MODE_FORMQ, st);
    if (e != hipSuccess) return hip_fail(e);
    return tsqr_sign_normalize_batched(dt, q->members, 0, q->n, nullptr, q->n, R, ldr, strideR, stream);
}

// CAQR's split of the device between its two streams: the panel
// factorisations (a few dozen latency-bound workgroups, on the critical path
// whenever the trailing update is short) run on r compute units of every XCD
// and the trailing updates on the others, so that a panel kernel never waits
// for CU slots held by update workgroups nor shares a SIMD with their MFMA
// work.  Only on a whole MI355X (256 CUs in 8 XCDs), where bit i of a
// stream's CU mask selects a CU of XCD i mod 8 (read back from the XCC_ID
// register of the workgroups of masked streams): bits 0 .. 8r - 1 give r CUs
// on every XCD, and every XCD keeps CUs in both masks.  The streams are made
// once per device and r and kept until the process ends (or
// tsqr_release_streams).
constexpr int kSplitMaxR = 4;
static std::mutex g_split_mu;
static hipStream_t g_split_cache[64][kSplitMaxR][2];
static bool g_split_tried[64][kSplitMaxR];

static bool caqr_split_streams(int r, hipStream_t* upd, hipStream_t* fac) {
    constexpr int kCUs = 256, kXCDs = 8, kMaxR = kSplitMaxR;
    if (r < 1 || r > kMaxR) return false;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    auto& cache = g_split_cache;
    auto& tried = g_split_tried;
    std::lock_guard<std::mutex> lock(g_split_mu);
    if (!tried[dev][r - 1]) {
        tried[dev][r - 1] = true;
        int cus = 0;
        hipDeviceProp_t prop;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        if (cus != kCUs || strncmp(prop.gcnArchName, "gfx950", 6) != 0) return false;
        uint32_t mask_f[kCUs / 32], mask_u[kCUs / 32];
        for (int w = 0; w < kCUs / 32; ++w) mask_f[w] = mask_u[w] = 0;
        for (int i = 0; i < kCUs; ++i) {
            uint32_t* m = (i < kXCDs * r) ? mask_f : mask_u;
            m[i / 32] |= 1u << (i % 32);
        }
        hipStream_t su = nullptr, sf = nullptr;
        if (hipExtStreamCreateWithCUMask(&su, kCUs / 32, mask_u) != hipSuccess ||
            hipExtStreamCreateWithCUMask(&sf, kCUs / 32, mask_f) != hipSuccess) {
            (void)hipGetLastError();
            if (su) (void)hipStreamDestroy(su);
            return false;
        }
        cache[dev][r - 1][0] = su;
        cache[dev][r - 1][1] = sf;
    }
    *upd = cache[dev][r - 1][0];
    *fac = cache[dev][r - 1][1];
    return *upd != nullptr && *fac != nullptr;
}

int tsqr_release_streams(void) {
    std::lock_guard<std::mutex> lock(g_split_mu);
    bool any = false;  // no HIP call at all when none was made
    for (int dev = 0; dev < 64 && !any; ++dev)
        for (int r = 0; r < kSplitMaxR; ++r) any = any || g_split_cache[dev][r][0] || g_split_cache[dev][r][1];
    if (!any) return 0;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return hip_fail(hipGetLastError());
    hipError_t first = hipSuccess;
    for (int dev = 0; dev < 64; ++dev)
        for (int r = 0; r < kSplitMaxR; ++r) {
            hipStream_t* p = g_split_cache[dev][r];
            if (!p[0] && !p[1]) continue;
            hipError_t e = hipSetDevice(dev);
            for (int k = 0; k < 2 && e == hipSuccess; ++k)
                if (p[k]) {
                    e = hipStreamSynchronize(p[k]);
                    if (e == hipSuccess) e = hipStreamDestroy(p[k]);
                    p[k] = nullptr;
                }
            if (e != hipSuccess && first == hipSuccess) first = e;
            g_split_tried[dev][r] = false;
        }
    hipError_t e = hipSetDevice(cur);
    if (first == hipSuccess) first = e;
    return first == hipSuccess ? 0 : hip_fail(first);
}

int caqr_factor(int dtype, int64_t m, int64_t n, void* A, int64_t lda, int64_t panel, int update_dtype,
                const tsqr_opts* opts, tsqr_qtree* q_out, void* stream) {
    if (!check_dtype(dtype)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return n > m ? -2 : -3;
    if (!A) return -4;
    if (lda < n) return -5;
    if (panel == 0) panel = 64;
    if (panel < 1 || panel > TSQR_MAX_N) return -6;
    if (!check_dtype(update_dtype)) return -7;
    if (update_dtype == TSQR_F64 && dtype == TSQR_F32) return -7;
    if (opts && (opts->flags & ~TSQR_FLAGS_ALL)) return -8;
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = dtype == TSQR_F64;
    const bool cf64 = update_dtype == TSQR_F64;
    const size_t es = f64 ? 8 : 4;
    tsqr_qtree_s* q = new tsqr_qtree_s();
    q->kind = 1;
    q->f64 = f64;
    q->A = A;
    q->lda = lda;
    q->stream = st;
    q->m = m;
    q->n = n;
    q->panel = panel;
    // Right-looking QR with TSQR panels (Sec. 3): factor panel k, then apply
    // its implicit Q^T to the trailing columns (Sec. 3.1, leaves then tree).
    // Look-ahead: once panel k's update has reached the next panel's columns,
    // panel k+1 is factored on a second stream while the rest of panel k's
    // update proceeds; panel k+1's update waits for both.
    // Panel trees: chains of a few blocks (the tree's node steps add to the
    // trailing update what the leaves cost, so one-block chains double it;
    // longer chains lengthen the panel factorisation, which the look-ahead
    // hides only behind a long enough update): eight blocks for panels of
    // 12288 rows or more, four below (measured on 8192^2 and 16384^2), node
    // by node (no waiting on a stream shared with the update).
    // the switch point to the split device (below), in trailing columns
    // (16384^2: 8192 with the FP64 update, 12288 with FP32 products; the
    // whole run split loses 4 ms and gains 8, none split loses 7 and 8;
    // 8192^2: split throughout is best; with the pipelined panel trees on
    // the masked stream, 6144 / 10240 (FP64) and 10240 / 14336 (FP32) were
    // slower again)
    const int64_t split_cols = cf64 ? 8192 : 12288;
    // early: a panel factored before the switch point (whether or not the
    // device is then split, so that both schedules factor the same trees)
    auto early_panel = [&](int64_t r1) {
        return r1 == 0 ? (n - (n < panel ? n : panel) > split_cols) : (n - r1 > split_cols);
    };
    auto panel_opts = [&](int64_t rows, bool early) {
        tsqr_opts o = opts ? *opts : tsqr_opts{0, 0, 0, 0, 0};
        if (o.chains == 0) {
            const int64_t blocks = (rows + 63) / 64;
            // eight-block chains halve the update's tree steps against four;
            // shorter panels take four so that their factor (on the critical
            // path near the end) stays short.  The switch: 6144 rows with the
            // FP64 update (against 12288: 16384^2 255.7 -> 247.1 ms, 12288^2
            // 140.7 -> 132.1 ms, 8192^2 61.0 -> 60.6 ms); with FP32 products
            // 12288 rows, or 8192 on matrices of 12288 columns or more
            // (12288^2: 121.6 -> 118.1 ms, 16384^2: 206.2 -> 203.7 ms against
            // eight for every panel; 8192 on 8192^2 was slower).
            // Before the switch point, where the update is long, panels of
            // 12288 rows or more take sixteen: half the update's tree steps again,
            // the longer panel factor hidden behind the update (16384^2: FP64
            // 261.1 -> 257.1 ms, FP32 products 215.4 -> 207.2 ms; twelve and
            // twenty, trees that are not powers of two, were slower)
            const bool eight = cf64 ? rows >= 6144 : (rows >= 12288 || (n >= 12288 && rows >= 8192));
            int chain_blocks = eight ? 8 : 4;
            if (early && rows >= 12288) chain_blocks = 16;
            const int64_t w = (blocks + chain_blocks - 1) / chain_blocks;
            o.chains = (int32_t)(w < 1 ? 1 : (w > 1024 ? 1024 : w));
        }
        o.flags |= TSQR_FLAG_TREE_LEVELWISE;
        return o;
    };
    // The update stream su and the panel stream s2: the caller's stream and a
    // second stream while the trailing updates are long (they need every
    // unit; the panel hides behind them), then the CU-masked pair that splits
    // the device (two workgroups of the first panel's chain kernel per
    // reserved unit) once the trailing columns are few enough for the panel
    // factorisation to be on the critical path.
    hipStream_t su = st, s2 = nullptr, mu = nullptr, mf = nullptr;
    bool masked = false;
    int split_r = 0;  // reserved CUs per XCD
    if (!(opts && (opts->flags & TSQR_FLAG_SHARED_CUS)) && n > panel) {
        Geom g0;
        const tsqr_opts o0 = panel_opts(m, early_panel(0));
        if (tsqr::make_geom(m, n < panel ? n : panel, &o0, &g0) == 0) {
            const int r = (g0.W + 15) / 16;
            split_r = r < 1 ? 1 : (r > 4 ? 4 : r);
            masked = caqr_split_streams(split_r, &mu, &mf);
        }
    }
    hipEvent_t ev_head = nullptr, ev_fact = nullptr, ev_in = nullptr, ev_sw = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
    hipStream_t s2_own = s2;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_head, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_fact, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_sw, hipEventDisableTiming);
    auto cleanup = [&]() {
        if (ev_head) (void)hipEventDestroy(ev_head);
        if (ev_fact) (void)hipEventDestroy(ev_fact);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_sw) (void)hipEventDestroy(ev_sw);
        if (s2_own) (void)hipStreamDestroy(s2_own);
    };
    auto factor_panel = [&](int64_t r0, hipStream_t fs) -> int {
        const int64_t cols = (n - r0) < panel ? (n - r0) : panel;
        const int64_t rows = m - r0;
        char* P = (char*)A + ((size_t)r0 * lda + r0) * es;
        tsqr_opts po = panel_opts(rows, early_panel(r0));
        // on the masked panel stream (its 8r units alone run the panel's
        // kernels, in order) the tree is panel-pipelined with an ordinary
        // launch when its waves fit one per SIMD there
        int gflags = 0;
        if (fs != s2_own && su != st && po.chains <= 32 * split_r) gflags = tsqr::TREE_PIPE_PLAIN;
        tsqr_qtree_s* pq = nullptr;
        int rc = factor_impl(dtype, rows, cols, P, lda, P, lda, true, &po, &pq, fs, true, gflags);
        if (rc != 0) return rc == -1 ? -2 : rc;
        pq->stream = st;  // later applies and the release run on the caller's stream
        q->panels.push_back(pq);
        return 0;
    };
    // switch to the masked pair: it starts after everything issued so far
    // (su has already waited for the last panel factorisation on s2)
    auto go_masked = [&]() -> hipError_t {
        hipError_t err = hipEventRecord(ev_sw, su);
        if (err == hipSuccess) err = hipStreamWaitEvent(mu, ev_sw, 0);
        if (err == hipSuccess) err = hipStreamWaitEvent(mf, ev_sw, 0);
        su = mu;
        s2 = mf;
        return err;
    };
    if (e == hipSuccess && masked && n - (n < panel ? n : panel) <= split_cols) e = go_masked();
    // the first panel is factored on s2 after the caller's earlier work
    if (e == hipSuccess && su == st) {
        e = hipEventRecord(ev_in, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(s2, ev_in, 0);
    }
    int rc = (e == hipSuccess) ? factor_panel(0, s2) : hip_fail(e);
    if (rc == 0) {
        e = hipEventRecord(ev_fact, s2);
        if (e == hipSuccess) e = hipStreamWaitEvent(su, ev_fact, 0);
        if (e != hipSuccess) rc = hip_fail(e);
    }
    for (int64_t r0 = 0; rc == 0 && r0 < n; r0 += panel) {
        const int64_t cols = (n - r0) < panel ? (n - r0) : panel;
        const int64_t tc = n - r0 - cols;
        if (tc <= 0) break;
        if (masked && su == st && tc <= split_cols) {
            e = go_masked();
            if (e != hipSuccess) { rc = hip_fail(e); break; }
        }
        tsqr_qtree_s* pq = q->panels.back();
        char* P = (char*)A + ((size_t)r0 * lda + r0) * es;
        char* Bt = P + (size_t)cols * es;
        const int64_t head = tc < panel ? tc : panel;  // the next panel's columns
        e = tsqr::launch_apply(f64, cf64, pq->g, pq->A, pq->lda, pq->wk, Bt, lda, head, tsqr::MODE_QT, su);
        if (e == hipSuccess) e = hipEventRecord(ev_head, su);
        if (e == hipSuccess) e = hipStreamWaitEvent(s2, ev_head, 0);
        if (e != hipSuccess) { rc = hip_fail(e); break; }
        rc = factor_panel(r0 + cols, s2);
        if (rc != 0) break;
        e = hipEventRecord(ev_fact, s2);
        if (e == hipSuccess && tc > head)
            e = tsqr::launch_apply(f64, cf64, pq->g, pq->A, pq->lda, pq->wk, Bt + (size_t)head * es, lda, tc - head,
                                   tsqr::MODE_QT, su);
        if (e == hipSuccess) e = hipStreamWaitEvent(su, ev_fact, 0);
        if (e != hipSuccess) rc = hip_fail(e);
    }
    // the caller's stream resumes after every panel and update
    if (su != st) {
        e = hipEventRecord(ev_sw, su);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, ev_sw, 0);
        if (e != hipSuccess && rc == 0) rc = hip_fail(e);
    }
    cleanup();
    if (rc != 0) {
        destroy_impl(q);
        return rc;
    }
    if (q_out) *q_out = q;
    else destroy_impl(q);
    return 0;
}

// Left-looking CAQR over column blocks (Sec. 3.2: left-looking QR with TSQR
// panels has the costs of the right-looking form).  Column block k (w
// columns) first receives the implicit Q^T of every panel factored before
// it, oldest first (each application: the panel's leaves, then its tree);
// inside the block the panels are right-looking.  Every column thus sees the
// same panel transformations in the same order as in caqr_factor; w = panel
// is plain left-looking, w >= n plain right-looking without look-ahead.
// Everything runs on the caller's stream.
int caqr_factor_left(int dtype, int64_t m, int64_t n, void* A, int64_t lda, int64_t panel, int64_t block_cols,
                     int update_dtype, const tsqr_opts* opts, tsqr_qtree* q_out, void* stream) {
    if (!check_dtype(dtype)) return -1;
    if (m < 1) return -2;
    if (n < 1 || n > m) return n > m ? -2 : -3;
    if (!A) return -4;
    if (lda < n) return -5;
    if (panel == 0) panel = 64;
    if (panel < 1 || panel > TSQR_MAX_N) return -6;
    if (block_cols == 0) block_cols = panel;
    if (block_cols < panel || block_cols % panel != 0) return -7;
    if (!check_dtype(update_dtype)) return -8;
    if (update_dtype == TSQR_F64 && dtype == TSQR_F32) return -8;
    if (opts && (opts->flags & ~TSQR_FLAGS_ALL)) return -9;
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = dtype == TSQR_F64;
    const bool cf64 = update_dtype == TSQR_F64;
    const size_t es = f64 ? 8 : 4;
    tsqr_qtree_s* q = new tsqr_qtree_s();
    q->kind = 1;
    q->f64 = f64;
    q->A = A;
    q->lda = lda;
    q->stream = st;
    q->m = m;
    q->n = n;
    q->panel = panel;
    // panel trees node by node (no wave waits on another), chains of eight
    // 64-row blocks unless opts sets the chain count
    auto factor_panel = [&](int64_t r0) -> int {
        const int64_t cols = (n - r0) < panel ? (n - r0) : panel;
        const int64_t rows = m - r0;
        char* P = (char*)A + ((size_t)r0 * lda + r0) * es;
        tsqr_opts po = opts ? *opts : tsqr_opts{0, 0, 0, 0, 0};
        if (po.chains == 0) {
            const int64_t w = ((rows + 63) / 64 + 7) / 8;
            po.chains = (int32_t)(w < 1 ? 1 : (w > 1024 ? 1024 : w));
        }
        po.flags |= TSQR_FLAG_TREE_LEVELWISE;
        tsqr_qtree_s* pq = nullptr;
        int rc = factor_impl(dtype, rows, cols, P, lda, P, lda, true, &po, &pq, st, true, 0);
        if (rc != 0) return rc == -1 ? -2 : rc;
        q->panels.push_back(pq);
        return 0;
    };
    // Q^T of panel j (rows j*panel .. m-1) on `cols` columns from column c0
    auto apply_panel = [&](size_t j, int64_t c0, int64_t cols) -> int {
        tsqr_qtree_s* pq = q->panels[j];
        char* B = (char*)A + ((size_t)j * panel * lda + c0) * es;
        hipError_t e = tsqr::launch_apply(f64, cf64, pq->g, pq->A, pq->lda, pq->wk, B, lda, cols, tsqr::MODE_QT, st);
        return e == hipSuccess ? 0 : hip_fail(e);
    };
    int rc = 0;
    for (int64_t c0 = 0; rc == 0 && c0 < n; c0 += block_cols) {
        const int64_t wc = (n - c0) < block_cols ? (n - c0) : block_cols;
        const size_t before = q->panels.size();
        for (size_t j = 0; rc == 0 && j < before; ++j) rc = apply_panel(j, c0, wc);
        for (int64_t r0 = c0; rc == 0 && r0 < c0 + wc; r0 += panel) {
            rc = factor_panel(r0);
            const int64_t cols = (n - r0) < panel ? (n - r0) : panel;
            const int64_t tc = c0 + wc - r0 - cols;
            if (rc == 0 && tc > 0) rc = apply_panel(q->panels.size() - 1, r0 + cols, tc);
        }
    }
    if (rc != 0) {
        destroy_impl(q);
        return rc;
    }
    if (q_out) *q_out = q;
    else destroy_impl(q);
    return 0;
}

int tsqr_qtree_destroy(tsqr_qtree q) {
    destroy_impl(q);
    return 0;
}

int tsqr_qtree_info(tsqr_qtree q, int64_t* info) {
    if (!q) return -1;
    if (!info) return -2;
    info[0] = q->m;
    info[1] = q->n;
    info[2] = q->g.h;
    info[3] = q->g.W;
    info[4] = q->g.arity;
    info[5] = q->g.levels;
    info[6] = q->g.nblocks;
    info[7] = q->f64 ? TSQR_F64 : TSQR_F32;
    info[8] = q->kind;
    info[9] = q->panel;
    return 0;
}

int tsqr_qtree_members(tsqr_qtree q, int64_t* members) {
    if (!q) return -1;
    if (!members) return -2;
    *members = q->members;
    return 0;
}

int tsqr_apply_layout(tsqr_qtree q, int64_t panel, int64_t k) {
    if (!q) return -1;
    const tsqr_qtree_s* t = q;
    if (q->kind == 1) {
        if (panel < 0 || panel >= (int64_t)q->panels.size()) return -2;
        t = q->panels[(size_t)panel];
    } else if (panel != 0) {
        return -2;
    }
    if (k < 1) return -3;
    return tsqr::apply_wide(t->g, k) ? 1 : 0;
}

int tsqr_plan_geometry(int64_t m, int64_t n, const tsqr_opts* opts, int64_t* out) {
    if (m < 1) return -1;
    if (n < 1 || n > m) return n > m ? -1 : -2;
    if (!out) return -4;
    Geom g;
    int rc = tsqr::make_geom(m, n, opts, &g);
    if (rc == -1) return -1;
    if (rc != 0) return rc;
    out[0] = g.h;
    out[1] = g.S;
    out[2] = g.W;
    out[3] = g.arity;
    out[4] = g.levels;
    out[5] = g.nblocks;
    out[6] = g.NC;
    return 0;
}

int tsqr_copy_r(int dtype, int64_t n, const void* src, int64_t lds, void* dst, int64_t ldd, void* stream) {
    if (!check_dtype(dtype)) return -1;
    if (n < 0) return -2;
    if (!src) return -3;
    if (lds < n) return -4;
    if (!dst) return -5;
    if (ldd < n) return -6;
    if (n == 0) return 0;
    hipError_t e = tsqr::launch_copy_r(dtype == TSQR_F64, n, src, lds, dst, ldd, true, (hipStream_t)stream);
    return e == hipSuccess ? 0 : hip_fail(e);
}

int tsqr_backward(int dtype, int64_t batch, int64_t m, int64_t n, const void* Q, int64_t ldq, int64_t strideQ,
                  const void* R, int64_t ldr, int64_t strideR, const void* dQ, int64_t lddq, int64_t stridedQ,
                  const void* dR, int64_t lddr, int64_t stridedR, void* dA, int64_t ldda, int64_t stridedA,
                  void* stream) {
    if (!check_dtype(dtype)) return -1;
    if (batch < 1) return -2;
    if (m < 1) return -3;
    if (n < 1 || n > m) return n > m ? -3 : -4;
    if (n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    if (!Q) return -5;
    if (ldq < n) return -6;
    if (!R) return -8;
    if (ldr < n) return -9;
    if (dQ && lddq < n) return -12;
    if (dR && lddr < n) return -15;
    if (!dA) return -17;
    if (ldda < n) return -18;
    if (batch > 65535) return -2;
    hipError_t e = tsqr::launch_backward(dtype == TSQR_F64, batch, m, n, Q, ldq, strideQ, R, ldr, strideR, dQ, lddq,
                                         stridedQ, dR, lddr, stridedR, dA, ldda, stridedA, (hipStream_t)stream);
    return e == hipSuccess ? 0 : hip_fail(e);
}

int tsqr_last_hip_error(void) { return g_last_hip; }

int tsqr_check_status(void* stream) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    int* w = tsqr::status_word();
    if (!w) return hip_fail(hipErrorInvalidSymbol);
    int v = 0;
    e = hipMemcpy(&v, w, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e);
    if (v != 0) {
        e = hipMemset(w, 0, sizeof(int));
        if (e != hipSuccess) return hip_fail(e);
    }
    return (v & 1) ? TSQR_ERR_TIMEOUT : 0;
}

int tsqr_set_phase_events(int phase, void* start, void* stop) {
    if (phase < 0 || phase >= tsqr::NPHASE) return -1;
    tsqr::g_phase.start[phase] = (hipEvent_t)start;
    tsqr::g_phase.stop[phase] = (hipEvent_t)stop;
    return 0;
}

const char* tsqr_status_string(int status) {
    switch (status) {
        case TSQR_SUCCESS: return "success";
        case TSQR_ERR_HIP: return "HIP runtime error";
        case TSQR_ERR_NOMEM: return "device memory allocation failed";
        case TSQR_ERR_PLAN: return "handle or shape mismatch";
        case TSQR_ERR_UNSUPPORTED: return "unsupported size or option";
        case TSQR_ERR_TIMEOUT: return "a bounded wait inside a factorisation gave up; its results are invalid";
        case TSQR_ERR_SCRATCH: return "the problem needs more scratch memory than the fixed buffer holds";
        default: return status < 0 ? "invalid argument" : "unknown status";
    }
}

}  // extern "C"

// ------------------------------------------------------------------ sign normalisation

template <typename T>
__global__ void k_sign_normalize(int64_t m, int64_t n, T* __restrict__ Q, int64_t ldq, T* __restrict__ R,
                                 int64_t ldr) {
    // one pass over R (rows) and Q (all rows); d_j = -1 if R_jj < 0 else +1
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t totq = Q ? m * n : 0;
    if (e < totq) {
        const int64_t i = e / n, j = e - i * n;
        if (R[j * ldr + j] < T(0)) Q[i * ldq + j] = -Q[i * ldq + j];
    }
}

template <typename T>
__global__ void k_sign_normalize_r(int64_t n, T* __restrict__ R, int64_t ldr) {
    // row i of R scaled by d_i; each workgroup owns one row and reads R_ii first
    const int64_t i = blockIdx.x;
    const T d = (R[i * ldr + i] < T(0)) ? T(-1) : T(1);
    __syncthreads();
    for (int64_t j = i + threadIdx.x; j < n; j += blockDim.x) R[i * ldr + j] *= d;
}

template <typename T>
__global__ void k_sign_normalize_b(int64_t mb, int64_t n, T* __restrict__ Q, int64_t ldq, const T* __restrict__ R,
                                   int64_t ldr, int64_t sr) {
    // Q of member blockIdx.y: column j scaled by the sign of its R_jj
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= mb * n) return;
    const int64_t i = e / n, j = e - i * n, b = blockIdx.y;
    const T* Rb = R + b * sr;
    if (Rb[j * ldr + j] < T(0)) Q[(b * mb + i) * ldq + j] = -Q[(b * mb + i) * ldq + j];
}

template <typename T>
__global__ void k_sign_normalize_rb(int64_t n, T* __restrict__ R, int64_t ldr, int64_t sr) {
    // row blockIdx.x of member blockIdx.y's R scaled by the sign of its diagonal entry
    T* Rb = R + (int64_t)blockIdx.y * sr;
    const int64_t i = blockIdx.x;
    const T d = (Rb[i * ldr + i] < T(0)) ? T(-1) : T(1);
    __syncthreads();
    for (int64_t j = i + threadIdx.x; j < n; j += blockDim.x) Rb[i * ldr + j] *= d;
}

extern "C" int tsqr_sign_normalize_batched(int dtype, int64_t batch, int64_t m, int64_t n, void* Q, int64_t ldq,
                                           void* R, int64_t ldr, int64_t strideR, void* stream) {
    if (!check_dtype(dtype)) return -1;
    if (batch < 1 || batch > 65535) return -2;
    if (m < 0) return -3;
    if (n < 0 || (Q && n > m)) return -4;
    if (Q && ldq < n) return -6;
    if (!R) return -7;
    if (ldr < n) return -8;
    if (batch > 1 && strideR < n * ldr) return -9;
    if (n == 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    if (Q && m > 0) {
        const dim3 grid((unsigned)((m * n + 255) / 256), (unsigned)batch);
        if (dtype == TSQR_F64)
            k_sign_normalize_b<double><<<grid, 256, 0, st>>>(m, n, (double*)Q, ldq, (const double*)R, ldr, strideR);
        else
            k_sign_normalize_b<float><<<grid, 256, 0, st>>>(m, n, (float*)Q, ldq, (const float*)R, ldr, strideR);
    }
    const dim3 gr((unsigned)n, (unsigned)batch);
    if (dtype == TSQR_F64)
        k_sign_normalize_rb<double><<<gr, 64, 0, st>>>(n, (double*)R, ldr, strideR);
    else
        k_sign_normalize_rb<float><<<gr, 64, 0, st>>>(n, (float*)R, ldr, strideR);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : hip_fail(e);
}

extern "C" int tsqr_sign_normalize(int dtype, int64_t m, int64_t n, void* Q, int64_t ldq, void* R, int64_t ldr,
                                   void* stream) {
    if (!check_dtype(dtype)) return -1;
    if (m < 0) return -2;
    if (n < 0 || (Q && n > m)) return -3;
    if (Q && ldq < n) return -5;
    if (!R) return -6;
    if (ldr < n) return -7;
    if (n == 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    const int64_t totq = Q ? m * n : 0;
    if (totq > 0) {
        const int64_t nb = (totq + 255) / 256;
        if (dtype == TSQR_F64)
            k_sign_normalize<double><<<(unsigned)nb, 256, 0, st>>>(m, n, (double*)Q, ldq, (double*)R, ldr);
        else
            k_sign_normalize<float><<<(unsigned)nb, 256, 0, st>>>(m, n, (float*)Q, ldq, (float*)R, ldr);
    }
    if (dtype == TSQR_F64)
        k_sign_normalize_r<double><<<(unsigned)n, 64, 0, st>>>(n, (double*)R, ldr);
    else
        k_sign_normalize_r<float><<<(unsigned)n, 64, 0, st>>>(n, (float*)R, ldr);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : hip_fail(e);
}
