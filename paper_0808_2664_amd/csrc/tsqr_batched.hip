// Batched TSQR of many uneven matrices in one graph launch (Sec. 2.1 per
// matrix; the tree shape of each matrix is a per-matrix choice, as the
// paper's tuning discussion allows).
//
// Work decomposition: every chain of every matrix is one work item.  Items
// are sorted longest first and served by persistent one-wave workers through
// an atomic counter; a worker factors its chain with the one-wave engine and
// then performs the tree nodes of that matrix it completes last (atomic node
// arrival counts), so no worker waits for another and one launch covers the
// leaves and the trees of all matrices.  Matrices are grouped by column class
// (1..16, 17..32, 33..64 columns -> 1, 2, 4 panels): one persistent kernel
// per class, the classes on parallel branches of the captured graph.
//
// Graph safety: the work counter and the node counters are cleared by a fill
// kernel inside the graph (no memset node), and the matrix pointers and
// leading dimensions are read from device arrays at run time, so a captured
// graph can be replayed with new matrices at the same array addresses.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/tsqr.h"
#include "tsqr_wave.hpp"

namespace tsqr {

struct BMat {
    Geom g;
    void* tau_blk;
    void* T_blk;
    void* Rbuf;
    void* Ynode;
    void* Tnode;
    void* tau_node;
    int* cnt;
};

struct BItem {
    int32_t mat, chain;
};

template <typename T, int NP, int OCC>
__global__ __launch_bounds__(64, OCC) void k_batch_tsqr(const BMat* __restrict__ mats, const BItem* __restrict__ items,
                                                        int nitems, int* __restrict__ next, T* const* __restrict__ A,
                                                        const int64_t* __restrict__ lda, T* const* __restrict__ R,
                                                        const int64_t* __restrict__ ldr) {
    __shared__ WSmem<T, NP> sm;
    for (;;) {
        int it = 0;
        if ((threadIdx.x & 63) == 0) it = atomicAdd(next, 1);
        it = __builtin_amdgcn_readfirstlane(it);
        if (it >= nitems) break;
        const BItem bi = items[it];
        const BMat bm = mats[bi.mat];
        TreeArgs ta{bm.cnt, (void*)R[bi.mat], ldr[bi.mat], 1, 0, nullptr, 0};  // no bounded waits (node by node)
        wave_tsqr<T, NP, 4, false, false>(sm, bm.g, bi.chain, A[bi.mat], lda[bi.mat], (T*)bm.tau_blk, (T*)bm.T_blk, (T*)bm.Rbuf,
                            (T*)bm.Ynode, (T*)bm.Tnode, (T*)bm.tau_node, ta);
    }
}

__global__ void k_batch_zero(int* __restrict__ p, int64_t count) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = 0;
}

constexpr int kClasses = 3;  // 1, 2, 4 panels
inline int class_of(int64_t n) { return n <= 16 ? 0 : (n <= 32 ? 1 : 2); }

template <typename T>
static const void* batch_kernel(int cls) {
    switch (cls) {
        case 0: return (const void*)&k_batch_tsqr<T, 1, 2>;
        case 1: return (const void*)&k_batch_tsqr<T, 2, 2>;
        default: return (const void*)&k_batch_tsqr<T, 4, (sizeof(T) == 8 ? 1 : 2)>;
    }
}

template <typename T>
static hipError_t launch_batch_class(int cls, int grid, hipStream_t st, const BMat* mats, const BItem* items,
                                     int nitems, int* next, void* const* A, const int64_t* lda, void* const* R,
                                     const int64_t* ldr) {
    T* const* a = (T* const*)A;
    T* const* r = (T* const*)R;
    switch (cls) {
        case 0: k_batch_tsqr<T, 1, 2><<<grid, 64, 0, st>>>(mats, items, nitems, next, a, lda, r, ldr); break;
        case 1: k_batch_tsqr<T, 2, 2><<<grid, 64, 0, st>>>(mats, items, nitems, next, a, lda, r, ldr); break;
        default:
            k_batch_tsqr<T, 4, (sizeof(T) == 8 ? 1 : 2)><<<grid, 64, 0, st>>>(mats, items, nitems, next, a, lda, r, ldr);
            break;
    }
    return hipGetLastError();
}

// Default tree shape of a matrix in a batch: chains of about 4096 rows (the
// batch supplies the parallelism, so trees stay shallow), binary tree.
inline int batch_default_chains(int64_t m) {
    int64_t c = (m + 4095) / 4096;
    return (int)(c < 1 ? 1 : (c > 1024 ? 1024 : c));
}

}  // namespace tsqr

using tsqr::BItem;
using tsqr::BMat;
using tsqr::Geom;

struct tsqr_batch_s {
    bool f64 = true;
    int count = 0;
    std::vector<Geom> geoms;
    void* dmem = nullptr;
    size_t bytes = 0;
    BMat* mats = nullptr;
    BItem* items = nullptr;
    int* cnt = nullptr;  // [next per class][node counters of every matrix]
    int64_t ncnt = 0;
    int64_t total_chains = 0;
    int nitems[tsqr::kClasses] = {0, 0, 0};
    int64_t item0[tsqr::kClasses] = {0, 0, 0};
    int grid[tsqr::kClasses] = {0, 0, 0};
    hipStream_t cap[tsqr::kClasses] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[tsqr::kClasses] = {nullptr, nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
};

static thread_local int g_batch_hip = 0;

static int bfail(hipError_t e) {
    g_batch_hip = (int)e;
    return e == hipErrorOutOfMemory ? TSQR_ERR_NOMEM : TSQR_ERR_HIP;
}

static void batch_release(tsqr_batch_s* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (int c = 0; c < tsqr::kClasses; ++c) {
        if (b->join[c]) (void)hipEventDestroy(b->join[c]);
        if (b->cap[c]) (void)hipStreamDestroy(b->cap[c]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->dmem) (void)hipFree(b->dmem);
    delete b;
}

extern "C" {

int tsqr_batch_plan_create(int dtype, int32_t count, const int64_t* m, const int64_t* n, const tsqr_opts* opts,
                           tsqr_batch* plan_out) {
    if (dtype != TSQR_F32 && dtype != TSQR_F64) return -1;
    if (count < 1) return -2;
    if (!m) return -3;
    if (!n) return -4;
    if (!plan_out) return -6;
    for (int i = 0; i < count; ++i) {
        if (n[i] < 1 || m[i] < n[i]) return n[i] < 1 ? -4 : -3;
        if (n[i] > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
        if (opts && opts[i].flags != 0) return -5;
    }
    const bool f64 = dtype == TSQR_F64;
    const size_t es = f64 ? 8 : 4;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    tsqr_batch_s* b = new tsqr_batch_s();
    b->f64 = f64;
    b->count = count;
    b->geoms.resize(count);
    // geometry and byte layout
    std::vector<size_t> off(count), cnt_off(count);
    size_t wbytes = 0;
    int64_t ncnt = tsqr::kClasses;  // one work counter per class first
    for (int i = 0; i < count; ++i) {
        tsqr::GeomOpts go;
        if (opts) {
            go.block_rows = opts[i].block_rows;
            go.chains = opts[i].chains;
            go.arity = opts[i].arity;
        }
        if (go.chains == 0) go.chains = tsqr::batch_default_chains(m[i]);
        if (go.arity == 0) go.arity = 2;
        int rc = tsqr::make_geom_opts(m[i], n[i], go, &b->geoms[i]);
        if (rc != 0) {
            delete b;
            return rc == -1 ? -3 : rc;
        }
        off[i] = wbytes;
        wbytes += al(tsqr::work_bytes(b->geoms[i], f64));
        cnt_off[i] = (size_t)ncnt;
        const Geom& g = b->geoms[i];
        ncnt += (int64_t)g.W * (g.levels > 0 ? g.levels : 1);
        b->total_chains += g.W;
    }
    // work items per class, longest chain first (ties: matrix, chain order)
    std::vector<BItem> items;
    items.reserve((size_t)b->total_chains);
    for (int c = 0; c < tsqr::kClasses; ++c) {
        std::vector<BItem> ci;
        for (int i = 0; i < count; ++i) {
            if (tsqr::class_of(n[i]) != c) continue;
            for (int w = 0; w < b->geoms[i].W; ++w) ci.push_back(BItem{i, w});
        }
        std::stable_sort(ci.begin(), ci.end(), [&](const BItem& x, const BItem& y) {
            const int64_t lx = tsqr::chain_end(b->geoms[x.mat], x.chain) - tsqr::chain_start(b->geoms[x.mat], x.chain);
            const int64_t ly = tsqr::chain_end(b->geoms[y.mat], y.chain) - tsqr::chain_start(b->geoms[y.mat], y.chain);
            return lx * b->geoms[x.mat].n > ly * b->geoms[y.mat].n;
        });
        b->item0[c] = (int64_t)items.size();
        b->nitems[c] = (int)ci.size();
        items.insert(items.end(), ci.begin(), ci.end());
    }
    b->ncnt = ncnt;
    const size_t mats_b = al(sizeof(BMat) * count), items_b = al(sizeof(BItem) * items.size()),
                 cnt_b = al(sizeof(int) * (size_t)ncnt);
    b->bytes = wbytes + mats_b + items_b + cnt_b;
    hipError_t e = hipMalloc(&b->dmem, b->bytes);
    if (e != hipSuccess) {
        delete b;
        return bfail(e);
    }
    char* base = (char*)b->dmem;
    b->mats = (BMat*)(base + wbytes);
    b->items = (BItem*)(base + wbytes + mats_b);
    b->cnt = (int*)(base + wbytes + mats_b + items_b);
    std::vector<BMat> hm(count);
    for (int i = 0; i < count; ++i) {
        tsqr::Work w;
        w.base = base + off[i];
        tsqr::work_carve(&w, b->geoms[i], f64);
        hm[i].g = b->geoms[i];
        hm[i].tau_blk = w.tau_blk;
        hm[i].T_blk = w.T_blk;
        hm[i].Rbuf = w.Rbuf;
        hm[i].Ynode = w.Ynode;
        hm[i].Tnode = w.Tnode;
        hm[i].tau_node = w.tau_node;
        hm[i].cnt = b->cnt + cnt_off[i];
    }
    (void)es;
    e = hipMemcpy(b->mats, hm.data(), sizeof(BMat) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(b->items, items.data(), sizeof(BItem) * items.size(), hipMemcpyHostToDevice);
    // persistent workers: as many one-wave workgroups as stay resident
    int dev = 0, cus = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (int c = 0; c < tsqr::kClasses && e == hipSuccess; ++c) {
        if (b->nitems[c] == 0) continue;
        int per_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, f64 ? tsqr::batch_kernel<double>(c) : tsqr::batch_kernel<float>(c), 64, 0);
        if (e != hipSuccess) break;
        int64_t gsz = (int64_t)(per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
        if (gsz > b->nitems[c]) gsz = b->nitems[c];
        b->grid[c] = (int)gsz;
    }
    for (int c = 0; c < tsqr::kClasses && e == hipSuccess; ++c) {
        e = hipStreamCreateWithFlags(&b->cap[c], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[c], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e != hipSuccess) {
        batch_release(b);
        return bfail(e);
    }
    *plan_out = b;
    return 0;
}

static hipError_t batch_capture(tsqr_batch_s* b, void* const* A, const int64_t* lda, void* const* R,
                                const int64_t* ldr) {
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    hipStream_t s0 = b->cap[0];
    hipError_t e = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const unsigned zb = (unsigned)((b->ncnt + 255) / 256);
    tsqr::k_batch_zero<<<zb, 256, 0, s0>>>(b->cnt, b->ncnt);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(b->fork, s0);
    for (int c = 0; c < tsqr::kClasses && e == hipSuccess; ++c) {
        if (b->nitems[c] == 0) continue;
        hipStream_t sc = b->cap[c];
        if (c != 0) e = hipStreamWaitEvent(sc, b->fork, 0);
        if (e != hipSuccess) break;
        const BItem* it = b->items + b->item0[c];
        e = b->f64 ? tsqr::launch_batch_class<double>(c, b->grid[c], sc, b->mats, it, b->nitems[c], b->cnt + c, A,
                                                      lda, R, ldr)
                   : tsqr::launch_batch_class<float>(c, b->grid[c], sc, b->mats, it, b->nitems[c], b->cnt + c, A,
                                                     lda, R, ldr);
        if (e == hipSuccess && c != 0) e = hipEventRecord(b->join[c], sc);
        if (e == hipSuccess && c != 0) e = hipStreamWaitEvent(s0, b->join[c], 0);
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s0, &g);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return e;
    b->key[0] = A;
    b->key[1] = lda;
    b->key[2] = R;
    b->key[3] = ldr;
    return hipSuccess;
}

int tsqr_batch_factor(tsqr_batch b, void* const* A, const int64_t* lda, void* const* R, const int64_t* ldr,
                      void* stream) {
    if (!b) return -1;
    if (!A) return -2;
    if (!lda) return -3;
    if (!R) return -4;
    if (!ldr) return -5;
    hipError_t e = hipSuccess;
    if (!b->exec || b->key[0] != (const void*)A || b->key[1] != (const void*)lda || b->key[2] != (const void*)R ||
        b->key[3] != (const void*)ldr)
        e = batch_capture(b, A, lda, R, ldr);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    return e == hipSuccess ? 0 : bfail(e);
}

int tsqr_batch_plan_info(tsqr_batch b, int64_t* out) {
    if (!b) return -1;
    if (!out) return -2;
    int classes = 0, workers = 0;
    for (int c = 0; c < tsqr::kClasses; ++c) {
        if (b->nitems[c] > 0) ++classes;
        workers += b->grid[c];
    }
    out[0] = b->count;
    out[1] = b->total_chains;
    out[2] = classes;
    out[3] = (int64_t)b->bytes;
    out[4] = b->exec ? 1 : 0;
    out[5] = workers;
    return 0;
}

int tsqr_batch_plan_destroy(tsqr_batch b) {
    batch_release(b);
    return 0;
}

}  // extern "C"
