// C ABI of the batched solver (batch.hip): a handle with `capacity` slots of
// workspace for problems up to max_m x max_n, rank up to max_r; one call
// solves up to `capacity` independent problems with one kernel launch.
#include "engine.hpp"
#include "sfr.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

namespace sfr {

// items with n up to this many columns run in the narrow kernel variant
constexpr int64_t kBatchNarrowN = 128;

static const int kBatchBuckets[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
constexpr int kNumBatchBuckets = 10;

static int batch_bucket(int r)
{
    for (int R : kBatchBuckets)
        if (R >= r) return R;
    return -1;
}

static int bucket_index(int R)
{
    for (int i = 0; i < kNumBatchBuckets; ++i)
        if (kBatchBuckets[i] == R) return i;
    return -1;
}

static bool item_valid(const sfr_ctx* h, const sfr_batch_item& it)
{
    if (it.m < 1 || it.m > h->max_m || it.n < 1 || it.n > h->max_n) return false;
    if (it.r < 1 || it.r > h->max_r || it.r > it.m || it.r > it.n) return false;
    if (!(it.lambda > 0.0) || it.lambda > 1e300 || !(it.mu > 0.0) || it.mu > 1e300) return false;
    if (!(it.tol >= 0.0) || it.tol > 1e300) return false;
    if (!it.M || !it.U || !it.B || !it.V || it.ldm < it.n || (it.S && it.lds < it.n)) return false;
    return true;
}

// descriptor of the caller's item `it` for workspace slot `pos`
static void build_desc(const sfr_ctx* h, const sfr_batch_item& it, int32_t pos, BatchItemDev& d)
{
    memset(&d, 0, sizeof(d));
    d.m = (int32_t)it.m; d.n = (int32_t)it.n; d.r = it.r; d.ldy = (int32_t)h->ldy;
    d.lambda = it.lambda; d.mu0 = it.mu; d.tol = it.tol;
    d.M = static_cast<const float*>(it.M); d.ldm = it.ldm;
    d.U = static_cast<float*>(it.U); d.B = it.B; d.V = static_cast<float*>(it.V);
    d.S = static_cast<float*>(it.S); d.lds = it.lds;
    float* const* w = &h->slot_ws[(size_t)pos * 6];
    d.Y0 = w[0]; d.Y1 = w[1]; d.P0 = w[2]; d.P1 = w[3]; d.Q0 = w[4]; d.Q1 = w[5];
}

// descriptor of the caller's item `it` in launch position `pos` (workspace slot pos)
static void fill_desc(sfr_ctx* h, const sfr_batch_item& it, int32_t pos)
{
    build_desc(h, it, pos, h->items_h[pos]);
}

}  // namespace sfr

using namespace sfr;

extern "C" {

sfr_status sfr_create_batch(sfr_handle* out, int32_t capacity, int64_t max_m, int64_t max_n, int32_t max_r,
                            const sfr_options* opt)
{
    if (!out) return SFR_ERR_ARG;
    *out = nullptr;
    if (!opt || opt->struct_size != sizeof(sfr_options)) return SFR_ERR_ARG;
    sfr_options o = *opt;
    if (o.precision != SFR_F32 || o.nystrom_l != 0) return SFR_ERR_ARG;
    // BF16 operands for the p and Q products of the matrix-core form (rank
    // buckets 8 to 16) in the leading iterations; FP32 iterations after
    if (o.bf16_iters < 0 || o.bf16_iters > 100000 || !(o.bf16_tol >= 0.0) || o.bf16_tol > 1e300) return SFR_ERR_ARG;
    if (o.bf16 == 0 && (o.bf16_iters != 0 || o.bf16_tol != 0.0)) return SFR_ERR_ARG;
    if (capacity < 1 || capacity > 65536) return SFR_ERR_ARG;
    if (max_m < 1 || max_m > (1 << 22) || max_n < 1 || max_n > 512) return SFR_ERR_ARG;
    if (max_r < 1 || max_r > 16 || max_r > max_m || max_r > max_n) return SFR_ERR_ARG;
    if (o.rho == 0.0) o.rho = 1.5;
    if (o.mu_bar == 0.0) o.mu_bar = 1e9;
    if (o.max_iter == 0) o.max_iter = 300;
    if (!(o.rho > 1.0) || !(o.mu_bar > 0.0) || o.rho > 1e300 || o.mu_bar > 1e300) return SFR_ERR_ARG;
    if (o.max_iter < 1 || o.max_iter > 100000 || o.fixed_iters < 0 || o.fixed_iters > 100000) return SFR_ERR_ARG;
    sfr_ctx* h = new (std::nothrow) sfr_ctx();
    if (!h) return SFR_ERR_NOMEM;
    h->batch = true;
    h->capacity = capacity;
    h->max_m = max_m;
    h->max_n = max_n;
    h->max_r = max_r;
    h->prm.rho = o.rho;
    h->prm.mu_bar = o.mu_bar;
    h->prm.max_iter = o.max_iter;
    h->prm.fixed_iters = o.fixed_iters;
    h->prm.bf16 = o.bf16 != 0;
    h->prm.bf16_iters = o.bf16_iters;
    h->prm.bf16_tol = o.bf16_tol;
    h->ldy = (max_n + 3) / 4 * 4;
    const size_t ny = (size_t)max_m * h->ldy, np = (size_t)max_m * 16, nq = (size_t)max_n * 16;
    bool ok = dev_alloc(h->allocs, h->batch_bytes, (void**)&h->items_d, sizeof(BatchItemDev) * (size_t)capacity);
    h->slot_ws.assign((size_t)capacity * 6, nullptr);
    for (int s = 0; s < capacity && ok; ++s) {
        float** w = &h->slot_ws[(size_t)s * 6];
        ok = ok && dev_alloc(h->allocs, h->batch_bytes, (void**)&w[0], ny * sizeof(float));
        ok = ok && dev_alloc(h->allocs, h->batch_bytes, (void**)&w[1], ny * sizeof(float));
        ok = ok && dev_alloc(h->allocs, h->batch_bytes, (void**)&w[2], np * sizeof(float));
        ok = ok && dev_alloc(h->allocs, h->batch_bytes, (void**)&w[3], np * sizeof(float));
        ok = ok && dev_alloc(h->allocs, h->batch_bytes, (void**)&w[4], nq * sizeof(float));
        ok = ok && dev_alloc(h->allocs, h->batch_bytes, (void**)&w[5], nq * sizeof(float));
    }
    if (ok && hipHostMalloc((void**)&h->items_h, sizeof(BatchItemDev) * (size_t)capacity, hipHostMallocDefault) !=
                  hipSuccess) {
        h->items_h = nullptr;
        ok = false;
    }
    // the narrow items' launch runs on a side stream of default priority,
    // forked from and joined to the caller's stream with events
    if (ok && (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
               hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
               hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess))
        ok = false;
    if (!ok) {
        free_all(h->allocs);
        if (h->items_h) (void)hipHostFree(h->items_h);
        if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
        if (h->ev_join) (void)hipEventDestroy(h->ev_join);
        if (h->side) (void)hipStreamDestroy(h->side);
        (void)hipGetLastError();
        delete h;
        return SFR_ERR_NOMEM;
    }
    h->order.assign((size_t)capacity, 0);
    *out = h;
    return SFR_OK;
}

sfr_status sfr_solve_batch(sfr_handle h, const sfr_batch_item* items, int32_t count, sfr_info* infos,
                           int32_t* statuses, void* hip_stream)
{
    if (!h || h->magic != 0x53465221u || !h->batch || h->qactive) return SFR_ERR_HANDLE;
    if (count < 0 || count > h->capacity || (count > 0 && !items)) return SFR_ERR_ARG;
    if (count == 0) return SFR_OK;
    // validate every item before any device work
    int Rw = 1, Rn = 1, nw = 0;
    for (int32_t i = 0; i < count; ++i) {
        const sfr_batch_item& it = items[i];
        if (!item_valid(h, it)) return SFR_ERR_ARG;
        if (it.n > kBatchNarrowN) {
            Rw = std::max(Rw, batch_bucket(it.r));
            ++nw;
        } else {
            Rn = std::max(Rn, batch_bucket(it.r));
        }
    }
    // wide items (n > 128) first, then the narrow ones, each in call order
    {
        int32_t a = 0, b = nw;
        for (int32_t i = 0; i < count; ++i) h->order[(items[i].n > kBatchNarrowN) ? a++ : b++] = i;
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    for (int32_t pos = 0; pos < count; ++pos) fill_desc(h, items[h->order[pos]], pos);
    BatchParams bp;
    bp.rho = h->prm.rho;
    bp.mu_bar = h->prm.mu_bar;
    bp.max_iter = h->prm.max_iter;
    bp.fixed_iters = h->prm.fixed_iters;
    bp.bf16 = h->prm.bf16 ? 1 : 0;
    bp.bf16_iters = h->prm.bf16_iters;
    bp.bf16_tol = h->prm.bf16_tol;
    const size_t bytes = sizeof(BatchItemDev) * (size_t)count;
    const int nn = count - nw;
    bool ok = hipMemcpyAsync(h->items_d, h->items_h, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    if (ok && nn > 0) {
        // fork: the side stream waits for the descriptors, runs the narrow
        // items, and the caller's stream waits for it before the copy back
        ok = hipEventRecord(h->ev_fork, s) == hipSuccess && hipStreamWaitEvent(h->side, h->ev_fork, 0) == hipSuccess &&
             launch_batch(h->items_d + nw, nn, Rn, true, h->variant[1][bucket_index(Rn)], bp, h->side) == hipSuccess &&
             hipEventRecord(h->ev_join, h->side) == hipSuccess;
    }
    if (ok && nw > 0) ok = launch_batch(h->items_d, nw, Rw, false, h->variant[0][bucket_index(Rw)], bp, s) == hipSuccess;
    if (ok && nn > 0) ok = hipStreamWaitEvent(s, h->ev_join, 0) == hipSuccess;
    if (ok) ok = launch_batch_orth(h->items_d, count, s) == hipSuccess;
    if (!ok || hipMemcpyAsync(h->items_h, h->items_d, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(h->side);
        return SFR_ERR_DEVICE;
    }
    sfr_status worst = SFR_OK;
    int32_t worst_i = count;      // the first failing item in call order
    for (int32_t pos = 0; pos < count; ++pos) {
        const int32_t i = h->order[pos];
        const BatchItemDev& d = h->items_h[pos];
        sfr_status st = (sfr_status)d.status;
        if (st == SFR_OK && !(d.min_eig_B > 0.0)) st = SFR_WARN_NOT_SPD;
        if (d.status == 1) st = SFR_WARN_MAXITER;
        if (statuses) statuses[i] = st;
        if (infos) {
            sfr_info& f = infos[i];
            memset(&f, 0, sizeof(f));
            if (st >= 0) {
                f.iters = d.iters;
                f.converged = (d.status == SFR_OK) ? 1 : 0;
                f.rel_residual = d.res;
                f.min_eig_B = d.min_eig_B;
                f.mu_final = d.mu_final;
                f.mu0 = items[i].mu;
                f.orth_err = d.orth_err;
            }
        }
        if (st < 0 && i < worst_i) {
            worst = st;
            worst_i = i;
        }
    }
    return worst;
}

sfr_status sfr_tune_batch(sfr_handle h, const sfr_batch_item* items, int32_t count, int32_t* table,
                          void* hip_stream)
{
    if (!h || h->magic != 0x53465221u || !h->batch || h->qactive) return SFR_ERR_HANDLE;
    if (count < 0 || count > h->capacity || (count > 0 && !items)) return SFR_ERR_ARG;
    for (int32_t i = 0; i < count; ++i)
        if (!item_valid(h, items[i])) return SFR_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    constexpr int kTuneIters = 4;
    BatchParams bp;
    bp.rho = h->prm.rho;
    bp.mu_bar = h->prm.mu_bar;
    bp.max_iter = h->prm.max_iter;
    bp.fixed_iters = kTuneIters;
    bp.bf16 = 0;
    bp.bf16_iters = 0;
    bp.bf16_tol = 0.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return SFR_ERR_DEVICE;
    }
    sfr_status st = SFR_OK;
    // one group per (class, rank bucket) present among the items
    for (int cls = 0; cls < 2 && st == SFR_OK; ++cls) {
        for (int bi = 0; bi < kNumBatchBuckets && st == SFR_OK; ++bi) {
            const int R = kBatchBuckets[bi];
            int32_t g = 0;
            for (int32_t i = 0; i < count; ++i) {
                const bool narrow = items[i].n <= kBatchNarrowN;
                if ((narrow ? 1 : 0) == cls && batch_bucket(items[i].r) == R) fill_desc(h, items[i], g++);
            }
            if (g == 0) continue;
            const size_t bytes = sizeof(BatchItemDev) * (size_t)g;
            int best = kBVAuto;
            float best_ms = 0.f;
            const int cands[] = {kBVNarrow, kBVRow1, kBVRow2, kBVMfma};
            for (int v : cands) {
                if (!batch_variant_valid(R, v) || (v == kBVNarrow && cls == 0)) continue;
                float ms = 0.f;
                for (int rep = 0; rep < 2 && st == SFR_OK; ++rep) {   // the first run warms up
                    if (hipMemcpyAsync(h->items_d, h->items_h, bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
                        hipEventRecord(e0, s) != hipSuccess ||
                        launch_batch(h->items_d, g, R, cls == 1, v, bp, s) != hipSuccess ||
                        hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                        st = SFR_ERR_DEVICE;
                }
                if (st != SFR_OK) break;
                if (best == kBVAuto || ms < best_ms) {
                    best = v;
                    best_ms = ms;
                }
            }
            if (st == SFR_OK) h->variant[cls][bi] = (int8_t)best;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SFR_OK) {
        (void)hipGetLastError();
        return st;
    }
    if (table) {
        for (int cls = 0; cls < 2; ++cls)
            for (int bi = 0; bi < kNumBatchBuckets; ++bi) table[cls * kNumBatchBuckets + bi] = h->variant[cls][bi];
    }
    return SFR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Queue form: persistent kernels fed while they run.
namespace sfr {

static bool queue_launch(sfr_ctx* h, int q)
{
    BatchParams bp;
    bp.rho = h->prm.rho;
    bp.mu_bar = h->prm.mu_bar;
    bp.max_iter = h->prm.max_iter;
    bp.fixed_iters = h->prm.fixed_iters;
    bp.bf16 = h->prm.bf16 ? 1 : 0;
    bp.bf16_iters = h->prm.bf16_iters;
    bp.bf16_tol = h->prm.bf16_tol;
    return launch_batch_queue(h->qitems, bp, h->qdev + q, h->qhost[q], h->qdone, h->capacity, q, h->qgrid[q],
                              h->qstream[q]) == hipSuccess;
}

// A persistent kernel leaves after a long idle spell; relaunch it when work
// for it is pending and it has ended.
static bool queue_keepalive(sfr_ctx* h, int q)
{
    if (h->qpending[q] == 0) return true;
    const hipError_t e = hipStreamQuery(h->qstream[q]);
    if (e == hipErrorNotReady) return true;
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return queue_launch(h, q);
}

void batch_queue_release(sfr_ctx* h)
{
    if (h->qactive) {
        for (int q = 0; q < 2; ++q) __atomic_store_n(&h->qhost[q]->closed, 1, __ATOMIC_RELEASE);
        for (int q = 0; q < 2; ++q) (void)hipStreamSynchronize(h->qstream[q]);
        h->qactive = false;
    }
    if (h->qitems) (void)hipHostFree(h->qitems);
    if (h->qdone) (void)hipHostFree(h->qdone);
    for (int q = 0; q < 2; ++q) {
        if (h->qhost[q]) (void)hipHostFree(h->qhost[q]);
        if (h->qstream[q]) (void)hipStreamDestroy(h->qstream[q]);
        h->qhost[q] = nullptr;
        h->qstream[q] = nullptr;
    }
    h->qitems = nullptr;
    h->qdone = nullptr;
}

static void queue_free_host(sfr_ctx* h)
{
    if (h->qitems) (void)hipHostFree(h->qitems);
    if (h->qdone) (void)hipHostFree(h->qdone);
    for (int q = 0; q < 2; ++q) {
        if (h->qhost[q]) (void)hipHostFree(h->qhost[q]);
        if (h->qstream[q]) (void)hipStreamDestroy(h->qstream[q]);
        h->qhost[q] = nullptr;
        h->qstream[q] = nullptr;
    }
    h->qitems = nullptr;
    h->qdone = nullptr;
}

}  // namespace sfr

extern "C" {

sfr_status sfr_queue_start(sfr_handle h, int32_t grid_large, int32_t grid_small)
{
    if (!h || h->magic != 0x53465221u || !h->batch || h->qactive) return SFR_ERR_HANDLE;
    if (grid_large < 0 || grid_small < 0 || grid_large > 65536 || grid_small > 65536) return SFR_ERR_ARG;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return SFR_ERR_DEVICE;
    }
    const int cap = h->capacity;
    if (!h->qitems) {
        bool ok = hipHostMalloc((void**)&h->qitems, sizeof(BatchItemDev) * (size_t)cap, hipHostMallocCoherent) ==
                      hipSuccess &&
                  hipHostMalloc((void**)&h->qdone, sizeof(int32_t) * (size_t)cap, hipHostMallocCoherent) == hipSuccess;
        for (int q = 0; q < 2 && ok; ++q)
            ok = hipHostMalloc((void**)&h->qhost[q], sizeof(BatchQueueHost), hipHostMallocCoherent) == hipSuccess &&
                 hipStreamCreateWithFlags(&h->qstream[q], hipStreamNonBlocking) == hipSuccess;
        if (ok && !h->qdev) ok = dev_alloc(h->allocs, h->batch_bytes, (void**)&h->qdev, 2 * sizeof(BatchQueueDev));
        if (!ok) {
            (void)hipGetLastError();
            queue_free_host(h);
            return SFR_ERR_NOMEM;
        }
    }
    memset(h->qitems, 0, sizeof(BatchItemDev) * (size_t)cap);
    memset(h->qdone, 0, sizeof(int32_t) * (size_t)cap);
    for (int q = 0; q < 2; ++q) memset(h->qhost[q], 0, sizeof(BatchQueueHost));
    BatchQueueDev zero[2];
    memset(zero, 0, sizeof(zero));
    if (hipMemcpy(h->qdev, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return SFR_ERR_DEVICE;
    }
    h->qgrid[0] = grid_large > 0 ? grid_large : std::max(1, cus * 3 / 4);
    h->qgrid[1] = grid_small > 0 ? grid_small : std::max(1, cus / 4);
    h->qfree.clear();
    for (int32_t s = cap - 1; s >= 0; --s) h->qfree.push_back(s);
    h->qseq.assign((size_t)cap, 0);
    h->qwhich.assign((size_t)cap, 0);
    h->qpending[0] = h->qpending[1] = 0;
    for (int q = 0; q < 2; ++q)
        if (!queue_launch(h, q)) {
            (void)hipGetLastError();
            h->qhost[0]->closed = 1;
            h->qhost[1]->closed = 1;
            (void)hipStreamSynchronize(h->qstream[0]);
            (void)hipStreamSynchronize(h->qstream[1]);
            return SFR_ERR_DEVICE;
        }
    h->qactive = true;
    return SFR_OK;
}

sfr_status sfr_queue_submit(sfr_handle h, const sfr_batch_item* item, int32_t* ticket)
{
    if (!h || h->magic != 0x53465221u || !h->batch || !h->qactive) return SFR_ERR_HANDLE;
    if (!item || !ticket || !item_valid(h, *item)) return SFR_ERR_ARG;
    if (h->qfree.empty()) return SFR_ERR_BUSY;
    const int32_t slot = h->qfree.back();
    h->qfree.pop_back();
    const int q = (item->r <= 6) ? 1 : 0;
    BatchItemDev d;
    build_desc(h, *item, slot, d);
    if (++h->qnext_seq <= 0) h->qnext_seq = 1;
    d.seq = h->qnext_seq;
    h->qitems[slot] = d;
    h->qseq[slot] = d.seq;
    h->qwhich[slot] = (int8_t)q;
    BatchQueueHost* hq = h->qhost[q];
    const int32_t t = __atomic_load_n(&hq->tail, __ATOMIC_RELAXED);
    __atomic_store_n(&hq->order[t % h->capacity], slot, __ATOMIC_RELAXED);
    __atomic_store_n(&hq->tail, t + 1, __ATOMIC_RELEASE);   // descriptor and entry before the tail
    ++h->qpending[q];
    *ticket = slot;
    if (!queue_keepalive(h, q)) return SFR_ERR_DEVICE;
    return SFR_OK;
}

sfr_status sfr_queue_poll(sfr_handle h, int32_t ticket, int32_t* done, sfr_info* info, int32_t* status)
{
    if (!h || h->magic != 0x53465221u || !h->batch || !h->qactive) return SFR_ERR_HANDLE;
    if (!done || ticket < 0 || ticket >= h->capacity || h->qseq[ticket] == 0) return SFR_ERR_ARG;
    *done = 0;
    const int32_t seq = h->qseq[ticket];
    if (__atomic_load_n(&h->qdone[ticket], __ATOMIC_ACQUIRE) != seq) {
        if (!queue_keepalive(h, h->qwhich[ticket])) return SFR_ERR_DEVICE;
        return SFR_OK;
    }
    const BatchItemDev& d = h->qitems[ticket];
    sfr_status st = (sfr_status)d.status;
    if (st == SFR_OK && !(d.min_eig_B > 0.0)) st = SFR_WARN_NOT_SPD;
    if (d.status == 1) st = SFR_WARN_MAXITER;
    if (status) *status = st;
    if (info) {
        memset(info, 0, sizeof(*info));
        if (st >= 0) {
            info->iters = d.iters;
            info->converged = (d.status == SFR_OK) ? 1 : 0;
            info->rel_residual = d.res;
            info->min_eig_B = d.min_eig_B;
            info->mu_final = d.mu_final;
            info->mu0 = d.mu0;
            info->orth_err = d.orth_err;
        }
    }
    *done = 1;
    --h->qpending[(int)h->qwhich[ticket]];
    h->qseq[ticket] = 0;
    h->qfree.push_back(ticket);
    return SFR_OK;
}

sfr_status sfr_queue_stop(sfr_handle h)
{
    if (!h || h->magic != 0x53465221u || !h->batch || !h->qactive) return SFR_ERR_HANDLE;
    // pending work is drained first (a kernel that left idle is relaunched)
    bool ok = queue_keepalive(h, 0) && queue_keepalive(h, 1);
    for (int q = 0; q < 2; ++q) __atomic_store_n(&h->qhost[q]->closed, 1, __ATOMIC_RELEASE);
    for (int q = 0; q < 2; ++q) ok = (hipStreamSynchronize(h->qstream[q]) == hipSuccess) && ok;
    h->qactive = false;
    if (!ok) {
        (void)hipGetLastError();
        return SFR_ERR_DEVICE;
    }
    return SFR_OK;
}

}  // extern "C"
