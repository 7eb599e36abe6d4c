// Host-side engine and handle layout shared by api.hip and nys.hip.
#pragma once

#include "sfr_internal.hpp"
#include "sfr.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace sfr {

// Host forecast of where a tolerance-driven solve stops, from the state
// snapshots the host reads between batches of queued iterations.  Once mu
// grows by rho per iteration the residual falls about geometrically, so the
// last two snapshots give its rate and the iteration at which it reaches
// tol.  The forecast only sizes the batches queued ahead of the host's
// checks, so that few iterations run after the stop (they return at once
// but still cost their launches); the device decides the stop, and a full
// batch is queued again whenever none is in flight and it has not stopped.
struct StopForecast {
    int idx = 0;        // iteration of the last snapshot's residual (0: none)
    double res = 0.0;
    int last = 0;       // forecast: last iteration to queue (0: no forecast)

    void observe(const DevState& ph)
    {
        // FR-ADM tests iteration k - 1 in step k, Alg. 4 iteration k;
        // ph.k is the next step's index
        const int i = ph.tsvd ? ph.k - 1 : ph.k - 2;
        const double r = ph.res;
        if (i < 1 || !(r > 0.0) || !std::isfinite(r)) {
            idx = 0;
            last = 0;
            return;
        }
        last = 0;
        if (idx >= 1 && i > idx && r < res && ph.tol > 0.0) {
            const double rate = std::log(r / res) / (double)(i - idx);   // < 0
            const double more = std::ceil(std::log(ph.tol / r) / rate);
            if (std::isfinite(more) && more < 1e6)
                last = i + (int)std::max(0.0, more) + (ph.tsvd ? 0 : 1);
        }
        idx = i;
        res = r;
    }
    // iterations to queue from k on, at most `batch`; idle: none in flight
    int size(int k, int batch, bool idle) const
    {
        if (last == 0) return batch;
        if (last >= k) return std::min(batch, last - k + 1);
        return idle ? batch : 0;
    }
};

// Launch shape of one sweep kernel on the engine's problem.
struct SweepCfg {
    int mfma = 0;   // 1: the matrix-core sweep (sweep_mfma.hip), else sweep.hip
    int tiles = 0;  // matrix-core sweep: 16-column tiles per wavefront (0: the bucket's default form)
    int rb = 0;     // matrix-core sweep: reduce-then-broadcast cluster exchange (else all-gather)
    int lpr = 64, nv = 1, W = 0, c = 1, cpx = 1, xcd_local = 1, ncl = 8, grid = 8, H = 4, nbands = 0, nbl_max = 0;
    size_t lds = 0;
};

struct LrEngine;   // large-rank FR-ADM engine (lr.hip)

// Launch shape of the first sweep (first.hip): column slices gx, row groups gy
// of `rows` rows (gy column partials of Q, gx gy partials of ||M||^2).
struct FirstPlan {
    bool ok = false;
    bool narrow = false;   // fewer than 256 vectors a row: rows packed into a workgroup
    int gx = 0, gy = 0, rows = 0;
};

// Residual history entries every engine holds at least: the mu_0 estimate
// (Alg. 4 on M) runs up to 60 steps whatever the handle's max_iter.
constexpr int kResHistMin = 64;

struct Engine {
    int m = 0, n = 0, ne = 0, r = 0, R = 0;   // ne: column count the kernels see (padded)
    bool f64 = false;
    size_t esz = 4;
    int vec = 4;
    // launch configurations: cfg[0] for the FR-ADM general sweeps (modes 1,
    // 2), cfg[1] for the sweeps on X = M (mode 0); tag_stride, the larger
    // band count per cluster, keeps exchange tags increasing across sweeps
    SweepCfg cfg[2];
    int tag_stride = 0;
    int max_grid = 0, max_ncl = 0;
    int rows_q = 0, nqb = 0, rows_p = 0, npb = 0, E = 0;
    bool gram_reduce = false;   // the Gram partials are summed before the step kernel
    FirstPlan first;            // the first sweep's shape (first.hip), if it applies
    int hist_len = 0;
    // workspace
    void* Y[2] = {nullptr, nullptr};
    int64_t ldy = 0;
    void* P[2] = {nullptr, nullptr};
    void* Q[2] = {nullptr, nullptr};
    void* Qpart = nullptr;
    double* dy2part = nullptr;
    double* rpart = nullptr;     // residual partials of the S pass (fixed-count solves)
    unsigned long long* exch = nullptr;
    size_t exch_words = 0;
    double* GQpart = nullptr;
    double* GPpart = nullptr;
    DevState* st = nullptr;
    double* res_hist = nullptr;
    void* Mpad = nullptr;             // padded copy of M when the kernels need it
    int64_t ldmpad = 0;
    std::vector<void*> allocs;
    size_t bytes = 0;
    DevState* host_state = nullptr;   // pinned mirror used for init / readback
    DevState* host_poll = nullptr;    // pinned: two header snapshots, one per batch in flight
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> prof_ev;  // start/stop pairs of timed sweeps
    double sweep_ms = 0.0;
    int sweeps_timed = 0;
};

struct Params {
    double lambda = 0, mu0 = 0, tol = 0, rho = 1.5, mu_bar = 1e9;
    int max_iter = 300, fixed_iters = 0;
    bool profile = false;
    // BF16-operand contractions (FP32 storage; matrix-core sweep) for the
    // leading iterations: until bf16_iters iterations or a residual <=
    // bf16_tol (either 0: not used); FP32 iterations then continue from that
    // iterate under the rule above.  Both 0: every iteration in BF16.
    bool bf16 = false;
    int bf16_iters = 0;
    double bf16_tol = 0.0;
};

// What a solve writes once the iteration has stopped: the factors U, B, V
// (U NULL: no factors, e.g. the mu_0 estimate, which reads only the state),
// the sparse part S of M (optional), the smallest eigenvalue of B and the
// factors' orthogonality error (into the state).  The kernels are queued behind the iteration and
// write nothing if it ended with an error.
template <typename T>
struct OutputSpec {
    T* U = nullptr;
    double* B = nullptr;
    T* V = nullptr;
    const T* M = nullptr;
    int64_t ldm = 0;
    T* S = nullptr;
    int64_t lds = 0;
    bool min_eig = false;
};

}  // namespace sfr

struct sfr_ctx {
    uint32_t magic = 0x53465221u;
    int64_t m = 0, n = 0;
    int32_t r = 0;
    bool f64 = false;
    bool nys = false;
    int32_t l = 0;
    sfr::Params prm;
    bool mu_auto = false;   // mu <= 0 at creation: mu_0 = 1.25 / ||M||_2 per solve
    double mu_left = 0, mu_top = 0;
    sfr::Engine main;       // FR-ADM engine (m x n)
    sfr::Engine left, top;  // FR-Nys sub-engines (m x l, l x n)
    sfr::LrEngine* lr = nullptr;  // large-rank engine (r > 32)
    // FR-Nys workspace
    void* C = nullptr;
    void* Rb = nullptr;
    int64_t* perm_d = nullptr;
    void* UL = nullptr; double* BL = nullptr; void* VL = nullptr;
    void* UT = nullptr; double* BT = nullptr; void* VT = nullptr;
    double* core = nullptr;  // r x r workspace of the combine (several blocks)
    void* Ucomb = nullptr;   // m x R combined row factor
    void* Vcomb = nullptr;   // n x R combined column factor
    // batched handle (sfr_create_batch)
    bool batch = false;
    int32_t capacity = 0, max_r = 0;
    int64_t max_m = 0, max_n = 0, ldy = 0;
    sfr::BatchItemDev* items_d = nullptr;   // device descriptors (capacity)
    sfr::BatchItemDev* items_h = nullptr;   // pinned mirror
    std::vector<float*> slot_ws;            // per slot: Y0, Y1, P0, P1, Q0, Q1
    std::vector<int32_t> order;             // launch position -> caller's item index
    int8_t variant[2][16] = {};             // [narrow][bucket index]: tuned band-loop form (0: default)
    hipStream_t side = nullptr;             // second launch of a batch (narrow items)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    size_t batch_bytes = 0;
    // queue form (sfr_queue_*): two persistent kernels (queue 0: r > 6 on
    // the R = 16 matrix-core form; queue 1: r <= 6 on the R = 6 form)
    bool qactive = false;
    sfr::BatchItemDev* qitems = nullptr;         // pinned coherent: descriptors and results, per slot
    int32_t* qdone = nullptr;                    // pinned coherent: per slot, the sequence number of the last solve
    sfr::BatchQueueHost* qhost[2] = {nullptr, nullptr};   // pinned coherent
    sfr::BatchQueueDev* qdev = nullptr;          // device: claim counters of the two queues
    hipStream_t qstream[2] = {nullptr, nullptr};
    int qgrid[2] = {0, 0};
    std::vector<int32_t> qfree;                  // free slots
    std::vector<int32_t> qseq;                   // per slot: sequence number in flight (0: free)
    std::vector<int8_t> qwhich;                  // per slot: its queue
    int32_t qnext_seq = 0;
    int64_t qpending[2] = {0, 0};                // submitted and not yet retired, per queue
    std::vector<void*> allocs;
};


namespace sfr {
// Large-rank FR-ADM engine (kMaxR < r <= kMaxRLarge, FP32; lr.hip).
struct LrEngine;
sfr_status lr_create(LrEngine** out, int m, int n, int r, int hist_len);
void lr_destroy(LrEngine* e);
size_t lr_bytes(const LrEngine* e);
sfr_status lr_solve(LrEngine* e, const Params& prm, bool mu_auto, const float* M, int64_t ldm, float* U, double* B,
                    float* V, float* S, int64_t lds, sfr_info* info, hipStream_t s);
sfr_status lr_tsvd(LrEngine* e, const Params& prm, const float* M, int64_t ldm, float* U, double* B, float* V,
                   sfr_info* info, hipStream_t s);

FirstPlan first_sweep_plan(const Engine& e);
template <typename T>
hipError_t launch_first_sweep(const SweepArgs<T>& a, int R, const FirstPlan& f, hipStream_t s);

// Shape of an engine (sizes, rank bucket, launch configurations); no
// device memory is touched.
sfr_status engine_plan(Engine& e, int m, int n, int r, bool f64, int hist_len);
// engine_plan, then the device workspace (hipMalloc) and the pinned host
// mirrors and poll events.
sfr_status engine_create(Engine& e, int m, int n, int r, bool f64, int hist_len);

// Assign the planned engine's device buffers in a fixed order, each from
// get(bytes) (nullptr: failure).  pad: also a padded copy of M (m x ne).
template <typename Get>
bool engine_buffers(Engine& e, bool pad, Get&& get)
{
    const size_t mn = (size_t)e.m * (size_t)e.ldy;
    for (int b = 0; b < 2; ++b)
        if (!(e.Y[b] = get(mn * e.esz))) return false;
    for (int b = 0; b < 2; ++b)
        if (!(e.P[b] = get((size_t)e.m * e.R * e.esz))) return false;
    for (int b = 0; b < 2; ++b)
        if (!(e.Q[b] = get((size_t)e.ne * e.R * e.esz))) return false;
    const int nqp = std::max(e.max_ncl, e.first.ok ? e.first.gy : 0);
    const int ndy = std::max(e.max_grid, e.first.ok ? e.first.gx * e.first.gy : 0);
    if (!(e.Qpart = get((size_t)nqp * e.ne * e.R * e.esz))) return false;
    if (!(e.dy2part = static_cast<double*>(get(sizeof(double) * (size_t)ndy)))) return false;
    if (!(e.rpart = static_cast<double*>(get(sizeof(double) * (size_t)lowrank_res_parts(e.m, e.n))))) return false;
    if (e.exch_words && !(e.exch = static_cast<unsigned long long*>(get(8 * e.exch_words)))) return false;
    if (!(e.GQpart = static_cast<double*>(get(sizeof(double) * (size_t)e.nqb * e.E)))) return false;
    if (!(e.GPpart = static_cast<double*>(get(sizeof(double) * (size_t)e.npb * e.E)))) return false;
    if (!(e.st = static_cast<DevState*>(get(sizeof(DevState))))) return false;
    if (!(e.res_hist = static_cast<double*>(get(sizeof(double) * (size_t)(std::max(e.hist_len, kResHistMin) + 2)))))
        return false;
    if (pad) {
        e.ldmpad = e.ne;
        if (!(e.Mpad = get((size_t)e.m * e.ldmpad * e.esz))) return false;
    }
    return true;
}

// sfr_create's host-side argument checks; o receives the options with the
// defaults filled in.
sfr_status validate_create(int64_t m, int64_t n, int32_t r, double lambda, double mu, double tol,
                           const sfr_options* opt, sfr_options& o);
void params_from(const sfr_options& o, double lambda, double mu, double tol, Params& p);
// FR-ADM on an engine (sfr_solve): the mu_0 estimate if mu_auto, the
// iteration, the outputs and the report.
sfr_status engine_solve(Engine& e, const Params& prm, bool mu_auto, const void* M, int64_t ldm, void* U, double* B,
                        void* V, void* S, int64_t lds, sfr_info* info, hipStream_t s);
void engine_destroy(Engine& e);
bool dev_alloc(std::vector<void*>& list, size_t& bytes, void** p, size_t sz);
void free_all(std::vector<void*>& list);
// tsvd: FixedRankOptFull (Alg. 4) on X = M instead of FR-ADM.
template <typename T>
sfr_status engine_iterate(Engine& e, const Params& p, double mu0, const T* M, int64_t ldm,
                          const OutputSpec<T>& out, hipStream_t s, bool tsvd = false);
sfr_status nys_setup(sfr_ctx* h);
// Stop a batched handle's queue form (if running) and free its host buffers.
void batch_queue_release(sfr_ctx* h);
}  // namespace sfr
