// Host side of the C ABI declared in include/sfr.h.
//
// One Engine owns the device workspace of one m x n FR-ADM solve shape and
// drives the device-resident iteration: per iteration k it enqueues
//   sweep(k)  fused pass over M / Y                       (sweep.hip)
//   gram(k)   Q = sum of column partials, G_Q, G_P         (sweep.hip)
//   step(k)   FP64 r x r projectors, mu, convergence test  (small.hip)
// in batches; every kernel returns at once after the step kernel has set
// the device `done` flag, so the host only reads the flag between batches
// and the stopping iteration equals the one the test selects.
#include "engine.hpp"

#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

namespace sfr {

bool dev_alloc(std::vector<void*>& list, size_t& bytes, void** p, size_t sz)
{
    *p = nullptr;
    if (sz == 0) sz = 16;
    if (hipMalloc(p, sz) != hipSuccess) { *p = nullptr; return false; }
    list.push_back(*p);
    bytes += sz;
    return true;
}

void free_all(std::vector<void*>& list)
{
    for (void* p : list) (void)hipFree(p);
    list.clear();
}

static int bucket_rank(int r)
{
    static const int Rs[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32};
    for (int R : Rs)
        if (R >= r) return R;
    return -1;
}

template <typename T>
static size_t lds_of(int R, int lpr, int W, int c) { return sweep_lds_bytes_c<T>(R, lpr, W, c); }

// Pick the row-pass shape (lanes per row, vectors per lane), the cluster
// size and the grid of one sweep kernel for an m x ne problem.
static sfr_status configure_grid(const Engine& e, SweepCfg& sc);

static sfr_status configure_sweep(const Engine& e, SweepCfg& sc, bool mfma)
{
    bool rb_forced = false;
    const int vec = e.vec;
    sc.mfma = mfma ? 1 : 0;
    const int nvec = (e.ne + vec - 1) / vec;
    const size_t ldsmax = 160 * 1024;
    int best_lpr = -1, best_nv = -1;
    long best_waste = -1;
    // single-slice shapes (c = 1): choose the least lane waste
    const int wmax = e.f64 ? sweep_max_width<double>(e.R) : sweep_max_width<float>(e.R);
    for (int lpr = 4; lpr <= 64; lpr *= 2) {
        const int nv = (nvec + lpr - 1) / lpr;
        if (nv > 4) continue;
        const int W = lpr * vec * nv;
        if (W > wmax) continue;
        const size_t L = e.f64 ? lds_of<double>(e.R, lpr, W, 1) : lds_of<float>(e.R, lpr, W, 1);
        if (L > ldsmax) continue;
        const long waste = (long)lpr * nv - nvec;
        if (best_waste < 0 || waste < best_waste || (waste == best_waste && lpr > best_lpr)) {
            best_waste = waste; best_lpr = lpr; best_nv = nv;
        }
    }
    if (sc.mfma) {
        // the R = 16 bucket takes its wide form (8 tiles per wavefront,
        // 1024-column slices) where n holds one such slice
        sc.tiles = (e.R == 16 && e.ne >= sweep_mfma_width(16, 8)) ? 8 : 0;
        const int mw = sweep_mfma_width(e.R, sc.tiles);
        sc.lpr = 64; sc.nv = 4; sc.c = (e.ne + mw - 1) / mw;
        // wide clusters of the 4-tile forms exchange by reduce-then-broadcast
        // (SFR_EXCH=gather or =reduce in the environment forces one form
        // where both exist; they give bitwise the same result)
        const char* ex = getenv("SFR_EXCH");
        const bool rb_ok = sweep_mfma_rb_supported(e.R, sc.tiles) && sc.c > 1;
        bool rb = rb_ok && sc.c >= kRbMinMembers;
        if (ex && strcmp(ex, "gather") == 0) rb = false;
        if (ex && strcmp(ex, "reduce") == 0) rb = rb_ok;
        rb_forced = ex && (strcmp(ex, "gather") == 0 || strcmp(ex, "reduce") == 0);
        sc.rb = rb ? 1 : 0;
    } else if (best_lpr > 0) {
        sc.lpr = best_lpr; sc.nv = best_nv; sc.c = 1;
    } else {
        // wide rows: one row per wave, slices of W columns exchanged in clusters
        sc.lpr = 64;
        sc.nv = 4;
        while (sc.nv > 1 && 64 * vec * sc.nv > wmax) --sc.nv;
        for (;;) {
            const int W = 64 * vec * sc.nv;
            const size_t L = e.f64 ? lds_of<double>(e.R, 64, W, 2) : lds_of<float>(e.R, 64, W, 2);
            if (L <= ldsmax || sc.nv == 1) break;
            --sc.nv;
        }
        sc.c = (e.ne + 64 * vec * sc.nv - 1) / (64 * vec * sc.nv);
    }
    sfr_status fs = configure_grid(e, sc);
    // Reduce-then-broadcast puts two dependent waits on each band; with few
    // bands per cluster (the l x n blocks of FR-Nys) the pipeline never
    // fills and all-gather is the faster form.
    if (fs == SFR_OK && sc.rb && !rb_forced && sc.nbl_max < kRbMinBands) {
        sc.rb = 0;
        fs = configure_grid(e, sc);
    }
    return fs;
}

// Slice width, band height, LDS size and grid of a sweep whose kernel form
// (vector or matrix-core, lanes per row, tiles, exchange form) and cluster
// width are chosen.
static sfr_status configure_grid(const Engine& e, SweepCfg& sc)
{
    const int vec = e.vec;
    sc.W = sc.mfma ? sweep_mfma_width(e.R, sc.tiles) : sc.lpr * vec * sc.nv;
    const int tpb = e.f64 ? sweep_threads<double>(e.R) : sweep_threads<float>(e.R);
    sc.H = sc.mfma ? 16 : (tpb / 64) * (64 / sc.lpr);
    sc.nbands = (e.m + sc.H - 1) / sc.H;
    if (sc.mfma) sc.lds = sweep_mfma_lds_bytes(e.R, sc.tiles, sc.rb != 0);
    else sc.lds = e.f64 ? lds_of<double>(e.R, sc.lpr, sc.W, sc.c) : lds_of<float>(e.R, sc.lpr, sc.W, sc.c);

    int bpc = 0;
    hipError_t herr = sc.mfma ? sweep_mfma_prepare(e.R, sc.tiles, sc.rb != 0, sc.lds, &bpc)
                              : (e.f64 ? sweep_prepare<double>(e.R, sc.lpr, sc.W, sc.lds, &bpc)
                                       : sweep_prepare<float>(e.R, sc.lpr, sc.W, sc.lds, &bpc));
    if (herr != hipSuccess || bpc < 1) return SFR_ERR_DEVICE;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SFR_ERR_DEVICE;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return SFR_ERR_DEVICE;
    bpc = std::min(bpc, 2);
    const int maxres = cus * bpc;
    // Every member of a cluster must be resident at once (they wait on each
    // other), so the grid never exceeds what the device holds in one wave.
    if (sc.c == 1) {
        int want = std::min(((sc.nbands + kXCD - 1) / kXCD) * kXCD, (maxres / kXCD) * kXCD);
        if (want < kXCD) want = kXCD;
        sc.cpx = want / kXCD;
        sc.xcd_local = 1;
        sc.ncl = kXCD * sc.cpx;
    } else if (kXCD * sc.c <= maxres) {
        sc.cpx = std::max(1, maxres / (kXCD * sc.c));
        while (sc.cpx > 1 && kXCD * (sc.cpx - 1) >= sc.nbands) --sc.cpx;  // no more clusters than bands
        sc.xcd_local = 1;
        sc.ncl = kXCD * sc.cpx;
    } else if (sc.c <= maxres) {
        sc.xcd_local = 0;
        sc.cpx = 0;
        sc.ncl = std::max(1, std::min(maxres / sc.c, sc.nbands));
    } else {
        return SFR_ERR_ARG;  // more column slices than resident workgroups
    }
    sc.grid = sc.ncl * sc.c;
    sc.nbl_max = (sc.nbands + sc.ncl - 1) / sc.ncl;
    return SFR_OK;
}

static size_t exch_words_of(const Engine& e, const SweepCfg& sc)
{
    if (sc.c <= 1) return 0;
    const size_t partial = (size_t)sc.ncl * kExchSlots * sc.c * sc.H * e.R * (e.esz / 4);
    // reduce-then-broadcast: the owners' sums follow the partials
    const size_t reduced = sc.rb ? (size_t)sc.ncl * kExchSlots * sc.H * e.R : 0;
    return partial + reduced;
}

// The matrix-core sweep takes FP32 problems with at least one full member
// slice (1024 columns for R <= 12, 512 above).  It runs the sweeps of mode 0
// (X = M: the first FR-ADM sweep and every Alg. 4 step) and, for R >= 12,
// every sweep: there it is the faster kernel (at R = 12 the vector kernel's
// per-lane state takes the whole register file, one wave per SIMD).  For
// R <= 10 the FR-ADM general sweeps stay on the vector kernel, whose
// row-contiguous loads stream better.
// SFR_SWEEP=vector or =mfma in the environment forces one kernel for every
// sweep (both are exact; used to test both).
static sfr_status configure(Engine& e)
{
    const char* pick = getenv("SFR_SWEEP");
    const bool want_vector = pick && strcmp(pick, "vector") == 0;
    const bool want_mfma = pick && strcmp(pick, "mfma") == 0;
    const bool mfma_ok = !e.f64 && sweep_mfma_supported(e.R) && e.ne >= sweep_mfma_width(e.R, 0);
    const bool general_mfma = mfma_ok && !want_vector && (want_mfma || e.R >= 12);
    sfr_status st = configure_sweep(e, e.cfg[0], general_mfma);
    if (st != SFR_OK) return st;
    st = configure_sweep(e, e.cfg[1], mfma_ok && !want_vector);
    if (st != SFR_OK) return st;
    e.tag_stride = std::max(e.cfg[0].nbl_max, e.cfg[1].nbl_max);
    e.max_grid = std::max(e.cfg[0].grid, e.cfg[1].grid);
    e.max_ncl = std::max(e.cfg[0].ncl, e.cfg[1].ncl);
    e.exch_words = std::max(exch_words_of(e, e.cfg[0]), exch_words_of(e, e.cfg[1]));
    // Gram launch shape.  Q: rows per workgroup such that each thread sums
    // about 32 cluster partials, with as many workgroups as that takes.
    // P: one segment of the Gram kernel (kGramU kTPB / R rows) per workgroup.
    const int rows = kTPB / e.R;
    const int qrows = std::max(1, std::min(rows, (kTPB * 32) / (e.R * std::max(1, e.max_ncl))));
    e.nqb = std::max(1, std::min((e.ne + qrows - 1) / qrows, kMaxGramPartials));
    e.rows_q = (e.ne + e.nqb - 1) / e.nqb;
    const int prows = (kGramU * kTPB) / e.R;
    e.npb = std::max(1, std::min((e.m + prows - 1) / prows, kMaxGramPartials));
    e.rows_p = (e.m + e.npb - 1) / e.npb;
    e.E = e.R * (e.R + 1) / 2;
    // the step kernel splits each of the 2E entries over nseg threads
    const int nseg = (2 * e.E >= kStepTPB) ? 1 : kStepTPB / (2 * e.E);
    e.gram_reduce = std::max(e.npb, e.nqb) > kStepPartialLoads * nseg;
    if (step_prepare(e.R) != hipSuccess) return SFR_ERR_DEVICE;
    return SFR_OK;
}

sfr_status engine_plan(Engine& e, int m, int n, int r, bool f64, int hist_len)
{
    e.m = m; e.n = n; e.r = r; e.f64 = f64;
    e.esz = f64 ? 8 : 4;
    e.vec = f64 ? 2 : 4;
    e.ne = ((n + e.vec - 1) / e.vec) * e.vec;
    e.R = bucket_rank(r);
    if (e.R < 0) return SFR_ERR_ARG;
    e.hist_len = hist_len;
    sfr_status cs = configure(e);
    if (cs != SFR_OK) return cs;
    e.ldy = e.ne;
    e.first = first_sweep_plan(e);
    return SFR_OK;
}

sfr_status engine_create(Engine& e, int m, int n, int r, bool f64, int hist_len)
{
    sfr_status ps = engine_plan(e, m, n, r, f64, hist_len);
    if (ps != SFR_OK) return ps;
    bool ok = engine_buffers(e, e.ne != e.n, [&](size_t sz) -> void* {
        void* p = nullptr;
        return dev_alloc(e.allocs, e.bytes, &p, sz) ? p : nullptr;
    });
    if (ok && hipHostMalloc((void**)&e.host_state, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        e.host_state = nullptr;
        ok = false;
    }
    if (ok && hipHostMalloc((void**)&e.host_poll, 2 * sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        e.host_poll = nullptr;
        ok = false;
    }
    for (int b = 0; b < 2 && ok; ++b)
        if (hipEventCreateWithFlags(&e.poll_ev[b], hipEventDisableTiming) != hipSuccess) {
            e.poll_ev[b] = nullptr;
            ok = false;
        }
    if (!ok) {
        engine_destroy(e);
        (void)hipGetLastError();
        return SFR_ERR_NOMEM;
    }
    return SFR_OK;
}

void engine_destroy(Engine& e)
{
    free_all(e.allocs);
    if (e.host_state) { (void)hipHostFree(e.host_state); e.host_state = nullptr; }
    if (e.host_poll) { (void)hipHostFree(e.host_poll); e.host_poll = nullptr; }
    for (int b = 0; b < 2; ++b)
        if (e.poll_ev[b]) { (void)hipEventDestroy(e.poll_ev[b]); e.poll_ev[b] = nullptr; }
    for (hipEvent_t ev : e.prof_ev) (void)hipEventDestroy(ev);
    e.prof_ev.clear();
}

#define HIPCHK(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) {                   \
            (void)hipGetLastError();               \
            return SFR_ERR_DEVICE;                 \
        }                                          \
    } while (0)

// Solves whose sweeps run in clusters (c > 1) hold this lock for their whole
// run.  Cluster members wait on each other's partial row products, so all of
// them must be resident at once; a plain launch gives that while no other
// kernel whose workgroups wait on one another holds compute units, since
// every other kernel drains and frees its slots.  Two such solves of one
// process (handles driven from two host threads on two streams) therefore
// run one after the other; solves without cluster waits run beside them.
// The guard waits for its stream before it lets go, so a solve that returns
// early on an error leaves no cluster kernel queued behind the lock.
static std::mutex g_cluster_solve;

struct ClusterGuard {
    std::unique_lock<std::mutex> lk;
    hipStream_t s;
    ClusterGuard(bool waits, hipStream_t s_) : lk(g_cluster_solve, std::defer_lock), s(s_)
    {
        if (waits) lk.lock();
    }
    ~ClusterGuard()
    {
        if (lk.owns_lock()) (void)hipStreamSynchronize(s);
    }
};

// Iterate Alg. 1 on the engine's shape and write the outputs of the
// returned iterate.  M: device, row-major, ldm.  A fixed iteration count is
// queued in one go; a tolerance-driven solve is queued in batches of 8 with
// one batch running ahead of the host's check of the previous one (kernels
// of a finished solve return at once).  The output kernels follow the last
// batch on the stream; the host waits once, at the end.
template <typename T>
sfr_status engine_iterate(Engine& e, const Params& p, double mu0, const T* M, int64_t ldm,
                          const OutputSpec<T>& out, hipStream_t s, bool tsvd)
{
    ClusterGuard guard(e.cfg[0].c > 1 || e.cfg[1].c > 1, s);
    const bool aligned = ((uintptr_t)M % 16 == 0) && (ldm % e.vec == 0) && (e.ne == e.n);
    const T* Mk = M;
    int64_t ldk = ldm;
    if (!aligned) {
        if (!e.Mpad) {
            e.ldmpad = e.ne;
            void* q = nullptr;
            if (hipMalloc(&q, (size_t)e.m * e.ldmpad * e.esz) != hipSuccess) { (void)hipGetLastError(); return SFR_ERR_NOMEM; }
            e.allocs.push_back(q);
            e.bytes += (size_t)e.m * e.ldmpad * e.esz;
            e.Mpad = q;
        }
        HIPCHK(launch_copy_pad<T>(M, ldm, static_cast<T*>(e.Mpad), e.ldmpad, e.m, e.n, s));
        Mk = static_cast<const T*>(e.Mpad);
        ldk = e.ldmpad;
    }
    // the first phase's stopping rule: the handle's, or for a two-phase BF16
    // solve its bulk phase's (see below)
    const bool two_phase = p.bf16 && !tsvd && (p.bf16_iters > 0 || p.bf16_tol > 0.0);
    const int budget = p.fixed_iters > 0 ? p.fixed_iters : p.max_iter;
    int fixed1 = p.fixed_iters, max1 = p.max_iter;
    double tol1 = p.tol;
    if (two_phase) {
        const int cap = p.bf16_iters > 0 ? std::min(p.bf16_iters, budget) : budget;
        if (p.bf16_tol > 0.0) {
            fixed1 = 0;
            tol1 = p.bf16_tol;
            max1 = cap;
        } else {
            fixed1 = cap;
        }
    }
    DevState& h = *e.host_state;
    memset(&h, 0, sizeof(DevState));
    h.m = e.m; h.n = e.ne; h.r = e.r; h.R = e.R;
    h.max_iter = max1; h.fixed_iters = fixed1;
    h.lambda = p.lambda; h.rho = p.rho; h.mu_bar = p.mu_bar; h.tol = tol1;
    h.M = Mk; h.ldm = ldk;
    h.k = 1; h.done = 0; h.status = 0;
    h.mu = mu0; h.mu_prev = mu0;
    h.tsvd = tsvd ? 1 : 0;
    // A fixed-count FR-ADM solve that returns S stops with the step of its
    // last iteration K: the S pass of the outputs also takes the residual
    // of iteration K, which would otherwise need sweep K + 1 (a pass over
    // M and both Y buffers that the returned iterate does not use).
    const bool stop_in_step = (fixed1 > 0) && !two_phase && !tsvd && (out.S != nullptr);
    h.stop_after = stop_in_step ? fixed1 : 0;
    for (int i = 0; i < kMaxR; ++i) {
        h.E1[i * kMaxR + i] = 1.0;
        h.E2[i * kMaxR + i] = 1.0;
        h.B[i * kMaxR + i] = 1.0;
    }
    for (int i = 0; i < e.r; ++i) {
        h.TV[i * kMaxR + i] = 1.0;
        h.TVf[i * kMaxR + i] = 1.0f;
    }
    HIPCHK(hipMemcpyAsync(e.st, &h, sizeof(DevState), hipMemcpyHostToDevice, s));
    HIPCHK(launch_init_q<T>(static_cast<T*>(e.Q[0]), e.ne, e.r, e.R, s));
    if (e.exch_words) HIPCHK(launch_fill_u64(e.exch, e.exch_words, s));

    // FR-ADM stops at the start of a step (iteration k - 1 converged), Alg. 4
    // at the end of one, so FR-ADM launches one more sweep/step pair.
    //
    // A BF16 solve runs in two phases.  The bulk phase takes the leading
    // iterations with BF16-operand contractions, until bf16_iters iterations
    // or a residual <= bf16_tol, whichever comes first, within the handle's
    // own budget.  FP32 iterations then continue from its returned iterate
    // under the handle's rule.  The switch has to come while the iteration
    // still contracts: late in a solve (large mu) L hardly moves and S
    // absorbs the residual, so FP32 iterations there do not remove an error
    // in L.
    const int limit = (fixed1 > 0 ? fixed1 : max1) + ((tsvd || stop_in_step) ? 0 : 1);
    const int batch = 8;
    // Profiling: start/stop events bound to every general sweep (k >= 3).
    if (p.profile) {
        const size_t need = 2 * (size_t)std::max(0, limit - 2);
        while (e.prof_ev.size() < need) {
            hipEvent_t ev;
            HIPCHK(hipEventCreate(&ev));
            e.prof_ev.push_back(ev);
        }
    }
    // one iteration: sweep k, Gram reduction, FP64 step.  bf: BF16-operand
    // contractions (matrix-core sweep); timed_ok: HIP events bound to the
    // sweep's dispatch when profiling.
    // The first sweep starts from V_0 = I_{n x r}: where its shape allows,
    // first.hip takes it without the row products and the exchange
    // (SFR_FIRST=sweep keeps the general sweep, to test both).
    const char* first_env = getenv("SFR_FIRST");
    const FirstPlan fp = (first_env && strcmp(first_env, "sweep") == 0) ? FirstPlan() : e.first;
    auto enqueue_iter = [&](int k, bool bf, bool timed_ok) -> sfr_status {
        SweepArgs<T> a;
        a.st = e.st;
        a.Yprev = static_cast<const T*>(e.Y[(k - 1) & 1]);
        a.Ynext = static_cast<T*>(e.Y[k & 1]);
        a.ldy = e.ldy;
        a.Pprev = static_cast<const T*>(e.P[(k - 1) & 1]);
        a.Pnext = static_cast<T*>(e.P[k & 1]);
        a.Qprev = static_cast<const T*>(e.Q[(k - 1) & 1]);
        a.Qpart = static_cast<T*>(e.Qpart);
        a.dy2part = e.dy2part;
        a.exch = e.exch;
        a.m = e.m; a.n = e.ne;
        a.mode = (k == 1 || tsvd) ? 0 : (k == 2 ? 1 : 2);
        const SweepCfg& sc = e.cfg[(a.mode == 0 || bf) ? 1 : 0];
        a.lpr = sc.lpr; a.nv = sc.nv; a.W = sc.W; a.c = sc.c; a.cpx = sc.cpx; a.xcd_local = sc.xcd_local;
        a.ncl = sc.ncl; a.nbands = sc.nbands; a.nbl_max = e.tag_stride;
        const bool timed = timed_ok && p.profile && k >= 3 && k <= limit;
        hipEvent_t ev0 = timed ? e.prof_ev[2 * (k - 3)] : nullptr;
        hipEvent_t ev1 = timed ? e.prof_ev[2 * (k - 3) + 1] : nullptr;
        const bool first = (k == 1) && fp.ok;
        int ncl_k = sc.ncl, ndy_k = sc.grid;
        if (first) {
            HIPCHK(launch_first_sweep<T>(a, e.R, fp, s));
            ncl_k = fp.gy;
            ndy_k = fp.gx * fp.gy;
        } else if constexpr (sizeof(T) == 4) {
            if (sc.mfma) HIPCHK(launch_sweep_mfma(a, e.R, sc.tiles, sc.rb != 0, sc.grid, sc.lds, s, ev0, ev1, bf));
            else HIPCHK(launch_sweep<T>(a, e.R, sc.grid, sc.lds, s, ev0, ev1));
        } else {
            HIPCHK(launch_sweep<T>(a, e.R, sc.grid, sc.lds, s, ev0, ev1));
        }
        GramArgs<T> g;
        g.st = e.st;
        g.Qpart = static_cast<const T*>(e.Qpart);
        g.Qnext = static_cast<T*>(e.Q[k & 1]);
        g.Pnext = static_cast<const T*>(e.P[k & 1]);
        g.GQpart = e.GQpart; g.GPpart = e.GPpart;
        g.m = e.m; g.n = e.ne; g.ncl = ncl_k;
        g.rows_q = e.rows_q; g.nqb = e.nqb; g.rows_p = e.rows_p; g.npb = e.npb;
        HIPCHK(launch_gram<T>(g, e.R, s));
        if (e.gram_reduce) HIPCHK(launch_gram_reduce(e.st, e.GQpart, e.nqb, e.GPpart, e.npb, e.E, s));
        StepArgs sa;
        sa.st = e.st;
        sa.GPpart = e.GPpart; sa.npb = e.gram_reduce ? 1 : e.npb;
        sa.GQpart = e.GQpart; sa.nqb = e.gram_reduce ? 1 : e.nqb;
        sa.dy2part = e.dy2part; sa.ndy = ndy_k;
        sa.res_hist = e.res_hist;
        sa.ns_kappa = e.f64 ? kNsKappaF64 : kNsKappaF32;
        sa.dk_tau = e.f64 ? kDkTauF64 : kDkTauF32;
        HIPCHK(launch_step(sa, e.R, s));
        return SFR_OK;
    };
    // One phase: iterations k0 .. lim, queued in one go (fixed rule) or in
    // batches of up to 8 with one batch running ahead of the host's check of
    // the previous one, cut at the forecast stop (StopForecast).  *K
    // receives the returned iterate when the host knows it (fixed rule:
    // lim - 1; polled: from the state), else -1.
    auto run_phase = [&](int k0, int lim, bool bf, bool fixed_rule, bool timed_ok, int* K) -> sfr_status {
        *K = -1;
        int k = k0;
        int launched_batches = 0, checked_batches = 0;   // this phase's poll slots
        auto enqueue_batch = [&](int count) -> sfr_status {
            for (int b = 0; b < count && k <= lim; ++b, ++k) {
                const sfr_status es = enqueue_iter(k, bf, timed_ok);
                if (es != SFR_OK) return es;
            }
            if (!fixed_rule) {
                const int slot = launched_batches & 1;
                HIPCHK(hipMemcpyAsync(&e.host_poll[slot], e.st, offsetof(DevState, B), hipMemcpyDeviceToHost, s));
                if (e.poll_ev[slot]) HIPCHK(hipEventRecord(e.poll_ev[slot], s));
            }
            ++launched_batches;
            return SFR_OK;
        };
        sfr_status es;
        if (fixed_rule) {
            while (k <= lim) {
                es = enqueue_batch(batch);
                if (es != SFR_OK) return es;
            }
            *K = lim - 1;   // if the phase failed instead, what follows returns at once
            return SFR_OK;
        }
        StopForecast fc;
        es = enqueue_batch(batch);
        if (es != SFR_OK) return es;
        for (;;) {
            if (k <= lim) {
                const int count = fc.size(k, batch, checked_batches == launched_batches);
                if (count > 0) {
                    es = enqueue_batch(count);
                    if (es != SFR_OK) return es;
                }
            }
            if (checked_batches == launched_batches) return SFR_OK;   // k > lim: reported below
            const int slot = checked_batches & 1;
            // without poll events (an engine that owns no host objects) the
            // whole stream is waited for, which covers this batch's snapshot
            if (e.poll_ev[slot]) HIPCHK(hipEventSynchronize(e.poll_ev[slot]));
            else HIPCHK(hipStreamSynchronize(s));
            const DevState& ph = e.host_poll[slot];
            ++checked_batches;
            if (ph.done || ph.exch_timeout) {
                if (ph.done && ph.status >= 0 && !ph.exch_timeout) *K = ph.iters;
                return SFR_OK;
            }
            fc.observe(ph);
        }
    };
    int bulk_iters = -1;
    sfr_status es = run_phase(1, limit, p.bf16, fixed1 > 0, true, &bulk_iters);
    if (es != SFR_OK) return es;
    if (two_phase && bulk_iters >= 1 && bulk_iters < budget) {
        // ---- FP32 iterations from the bulk phase's returned iterate K: the
        // state goes back to the handle's rule; sweep K + 1 is run again, so
        // the exchange words of its first run are cleared
        HIPCHK(launch_refine_start(e.st, p.fixed_iters, p.tol, p.max_iter, s));
        if (e.exch_words) HIPCHK(launch_fill_u64(e.exch, e.exch_words, s));
        int K2 = -1;
        es = run_phase(bulk_iters + 1, budget + 1, false, p.fixed_iters > 0, false, &K2);
        if (es != SFR_OK) return es;
    }
    // ---- outputs of the returned iterate, then one wait
    PingPong<T> pp;
    for (int b = 0; b < 2; ++b) {
        pp.P[b] = static_cast<T*>(e.P[b]);
        pp.Q[b] = static_cast<T*>(e.Q[b]);
        pp.Y[b] = static_cast<const T*>(e.Y[b]);
    }
    if (out.U) {
        HIPCHK(launch_factors<T>(e.st, pp, e.m, e.n, e.r, e.R, out.U, out.V, out.B, s));
        HIPCHK(launch_orth<T>(e.st, out.U, e.m, out.V, e.n, e.r, e.GPpart, e.npb, e.GQpart, e.nqb,
                              &e.st->orth_err, s));
    }
    if (out.S) {
        LowrankArgs<T> la;
        memset(&la, 0, sizeof(la));
        la.st = e.st;
        la.pp = pp;
        la.M = out.M;
        la.ldm = out.ldm;
        la.ldy = e.ldy;
        la.S = out.S;
        la.lds = out.lds;
        la.m = e.m;
        la.n = e.n;
        la.mode = 0;
        la.lam = p.lambda;
        la.mu = 1.0;
        la.min_eig = out.min_eig ? 1 : 0;
        la.rpart = stop_in_step ? e.rpart : nullptr;
        int parts = 0;
        HIPCHK(launch_lowrank_pass<T>(la, e.R, s, &parts));
        if (stop_in_step) HIPCHK(launch_res_final(e.st, e.rpart, parts, e.res_hist, s));
    } else if (out.min_eig) {
        HIPCHK(launch_final_small(e.st, e.R, s));
    }
    HIPCHK(hipMemcpyAsync(e.host_state, e.st, offsetof(DevState, B), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    e.sweep_ms = 0.0;
    e.sweeps_timed = 0;
    if (p.profile && h.done) {
        // sweeps that did work (of a two-phase BF16 solve: its bulk phase)
        const int kstop = (two_phase && bulk_iters >= 1) ? bulk_iters : h.iters;
        const int last = std::min(kstop + (tsvd ? 0 : 1), limit);
        for (int kk = 3; kk <= last; ++kk) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e.prof_ev[2 * (kk - 3)], e.prof_ev[2 * (kk - 3) + 1]));
            e.sweep_ms += ms;
            ++e.sweeps_timed;
        }
        if (e.sweeps_timed) e.sweep_ms /= e.sweeps_timed;
    }
    if (h.exch_timeout) return SFR_ERR_DEVICE;
    if (!h.done) return SFR_ERR_DEVICE;  // the step kernel always stops by `limit`
    if (h.status < 0) return (sfr_status)h.status;
    return SFR_OK;
}

template sfr_status engine_iterate<float>(Engine&, const Params&, double, const float*, int64_t,
                                          const OutputSpec<float>&, hipStream_t, bool);
template sfr_status engine_iterate<double>(Engine&, const Params&, double, const double*, int64_t,
                                           const OutputSpec<double>&, hipStream_t, bool);

}  // namespace sfr

using namespace sfr;

static sfr_status fill_info(const Engine& e, sfr_info* info, sfr_status st)
{
    const DevState& h = *e.host_state;
    if (info) {
        info->iters = h.iters;
        info->iters_top = 0;
        info->converged = (h.status == kOK) ? 1 : 0;
        info->rel_residual = h.res;
        info->min_eig_B = h.min_eig_B;
        info->mu_final = h.mu_prev;
        info->sweep_ms = e.sweep_ms;
        info->sweeps_timed = e.sweeps_timed;
        info->mu0 = 0.0;
        info->orth_err = h.orth_err;
    }
    if (st != SFR_OK) return st;
    if (h.status == kWarnMaxIter) return SFR_WARN_MAXITER;
    if (!(h.min_eig_B > 0.0)) return SFR_WARN_NOT_SPD;
    return SFR_OK;
}

// mu_0 = 1.25 / ||M||_2, the initial penalty taken for handles created with
// mu <= 0.  ||M||_2 is the largest eigenvalue of B after Alg. 4 on M (run to
// a change of B of 1e-6 relative, at most 60 steps).  The estimate lives in
// the handle's workspace and state only; no caller buffer is written.
template <typename T>
static sfr_status estimate_mu0(Engine& e, const Params& prm, const T* M, int64_t ldm, hipStream_t s, double* mu0)
{
    Params p = prm;
    p.tol = 1e-6;
    p.fixed_iters = 0;
    p.max_iter = 60;
    p.bf16 = false;
    p.bf16_iters = 0;
    p.bf16_tol = 0.0;
    p.profile = false;
    OutputSpec<T> o;   // no factors: only B in the state is read
    o.min_eig = false;
    const sfr_status st = engine_iterate<T>(e, p, 1.0, M, ldm, o, s, true);
    if (st < 0) return st;
    HIPCHK(launch_max_eig(e.st, e.R, s));
    double smax = 0.0;
    HIPCHK(hipMemcpyAsync(&smax, &e.st->max_eig_B, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!(smax > 0.0) || !std::isfinite(smax)) return SFR_ERR_NONFINITE;
    *mu0 = 1.25 / smax;
    return SFR_OK;
}

namespace sfr {

sfr_status engine_solve(Engine& e, const Params& prm, bool mu_auto, const void* M, int64_t ldm, void* U, double* B,
                        void* V, void* S, int64_t lds, sfr_info* info, hipStream_t s)
{
    sfr_status st = SFR_OK;
    double mu0 = prm.mu0;
    if (e.f64) {
        OutputSpec<double> o;
        o.U = static_cast<double*>(U); o.B = B; o.V = static_cast<double*>(V);
        o.M = static_cast<const double*>(M); o.ldm = ldm; o.S = static_cast<double*>(S); o.lds = lds;
        o.min_eig = true;
        if (mu_auto) st = estimate_mu0<double>(e, prm, o.M, ldm, s, &mu0);
        if (st == SFR_OK) st = engine_iterate<double>(e, prm, mu0, static_cast<const double*>(M), ldm, o, s);
    } else {
        OutputSpec<float> o;
        o.U = static_cast<float*>(U); o.B = B; o.V = static_cast<float*>(V);
        o.M = static_cast<const float*>(M); o.ldm = ldm; o.S = static_cast<float*>(S); o.lds = lds;
        o.min_eig = true;
        if (mu_auto) st = estimate_mu0<float>(e, prm, o.M, ldm, s, &mu0);
        if (st == SFR_OK) st = engine_iterate<float>(e, prm, mu0, static_cast<const float*>(M), ldm, o, s);
    }
    if (st < 0) {
        if (info) memset(info, 0, sizeof(*info));
        return st;
    }
    st = fill_info(e, info, st);
    if (info) info->mu0 = mu0;
    return st;
}

// Host-side validation of sfr_create's arguments; `o` receives the options
// with their defaults filled in.
sfr_status validate_create(int64_t m, int64_t n, int32_t r, double lambda, double mu, double tol,
                           const sfr_options* opt, sfr_options& o)
{
    memset(&o, 0, sizeof(o));
    if (opt) {
        if (opt->struct_size != sizeof(sfr_options)) return SFR_ERR_ARG;
        o = *opt;
    }
    if (m < 1 || n < 1 || r < 1 || r > kMaxRLarge || r > m || r > n) return SFR_ERR_ARG;
    if (m > (int64_t)1 << 30 || n > (int64_t)1 << 30) return SFR_ERR_ARG;
    if (!(lambda > 0.0) || !(tol >= 0.0) || lambda > 1e300 || tol > 1e300) return SFR_ERR_ARG;
    if (o.precision != SFR_F64 && o.precision != SFR_F32) return SFR_ERR_ARG;
    if (o.bf16 != 0 && (o.precision != SFR_F32 || o.nystrom_l != 0)) return SFR_ERR_ARG;
    if (o.bf16_iters < 0 || o.bf16_iters > 100000 || !(o.bf16_tol >= 0.0) || o.bf16_tol > 1e300) return SFR_ERR_ARG;
    if (o.bf16 == 0 && (o.bf16_iters != 0 || o.bf16_tol != 0.0)) return SFR_ERR_ARG;
    if (o.rho == 0.0) o.rho = 1.5;
    if (o.mu_bar == 0.0) o.mu_bar = 1e9;
    if (o.max_iter == 0) o.max_iter = 300;
    if (!(o.rho > 1.0) || !(o.mu_bar > 0.0) || o.rho > 1e300 || o.mu_bar > 1e300) return SFR_ERR_ARG;
    if (o.max_iter < 1 || o.max_iter > 100000 || o.fixed_iters < 0 || o.fixed_iters > 100000) return SFR_ERR_ARG;
    if (o.nystrom_l < 0) return SFR_ERR_ARG;
    // ranks above the fused sweeps' bucket run on the large-rank engine:
    // FP32 FR-ADM (and Alg. 4) only
    if (r > kMaxR && (o.precision != SFR_F32 || o.nystrom_l != 0 || o.bf16 != 0)) return SFR_ERR_ARG;
    if (o.nystrom_l > 0) {
        if (o.nystrom_l < r || o.nystrom_l > m || o.nystrom_l > n) return SFR_ERR_ARG;
        if (!(o.mu_left > 0.0) || !(o.mu_top > 0.0) || o.mu_left > 1e300 || o.mu_top > 1e300) return SFR_ERR_ARG;
    } else {
        if (!std::isfinite(mu) || mu > 1e300) return SFR_ERR_ARG;
    }
    return SFR_OK;
}

void params_from(const sfr_options& o, double lambda, double mu, double tol, Params& p)
{
    p.lambda = lambda; p.mu0 = mu; p.tol = tol;
    p.rho = o.rho; p.mu_bar = o.mu_bar;
    p.max_iter = o.max_iter; p.fixed_iters = o.fixed_iters;
    p.profile = o.profile != 0;
    p.bf16 = o.bf16 != 0;
    p.bf16_iters = o.bf16_iters;
    p.bf16_tol = o.bf16_tol;
}

}  // namespace sfr

extern "C" {

const char* sfr_version(void) { return "0.1.0"; }

const char* sfr_status_string(sfr_status s)
{
    switch (s) {
    case SFR_OK: return "ok";
    case SFR_ERR_ARG: return "invalid argument";
    case SFR_ERR_NOMEM: return "device workspace allocation failed";
    case SFR_ERR_DEVICE: return "HIP runtime error or device wait bound reached";
    case SFR_ERR_RANK: return "rank(X V B) < r: Stiefel projector not unique";
    case SFR_ERR_NONFINITE: return "non-finite value in M or in the iteration";
    case SFR_ERR_HANDLE: return "invalid handle for this call";
    case SFR_ERR_SCRATCH: return "problem needs more device workspace than the static scratch holds";
    case SFR_ERR_BUSY: return "no free slot: every slot of the queue holds a problem in flight";
    case SFR_WARN_MAXITER: return "max_iter reached before the tolerance";
    case SFR_WARN_NOT_SPD: return "returned B is not positive definite";
    }
    return "unknown status";
}

sfr_status sfr_create(sfr_handle* out, int64_t m, int64_t n, int32_t r, double lambda, double mu, double tol,
                      const sfr_options* opt)
{
    if (!out) return SFR_ERR_ARG;
    *out = nullptr;
    sfr_options o;
    const sfr_status vs = validate_create(m, n, r, lambda, mu, tol, opt, o);
    if (vs != SFR_OK) return vs;
    const bool nys = o.nystrom_l > 0;
    sfr_ctx* h = new (std::nothrow) sfr_ctx();
    if (!h) return SFR_ERR_NOMEM;
    h->m = m; h->n = n; h->r = r;
    h->f64 = (o.precision == SFR_F64);
    h->nys = nys;
    h->l = o.nystrom_l;
    params_from(o, lambda, mu, tol, h->prm);
    h->mu_auto = !nys && !(mu > 0.0);
    h->mu_left = o.mu_left; h->mu_top = o.mu_top;
    const int hist = std::max(o.max_iter, o.fixed_iters);
    sfr_status st;
    if (r > kMaxR) {
        st = lr_create(&h->lr, (int)m, (int)n, r, hist);
    } else if (!nys) {
        st = engine_create(h->main, (int)m, (int)n, r, h->f64, hist);
        // the BF16 bulk phase runs on the matrix-core sweep
        if (st == SFR_OK && h->prm.bf16 && !h->main.cfg[1].mfma) st = SFR_ERR_ARG;
    } else {
        st = nys_setup(h);
    }
    if (st != SFR_OK) {
        lr_destroy(h->lr);
        engine_destroy(h->main);
        engine_destroy(h->left);
        engine_destroy(h->top);
        free_all(h->allocs);
        if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
        if (h->ev_join) (void)hipEventDestroy(h->ev_join);
        if (h->side) (void)hipStreamDestroy(h->side);
        delete h;
        return st;
    }
    *out = h;
    return SFR_OK;
}

sfr_status sfr_destroy(sfr_handle h)
{
    if (!h) return SFR_OK;
    if (h->magic != 0x53465221u) return SFR_ERR_HANDLE;
    if (h->batch) batch_queue_release(h);
    lr_destroy(h->lr);
    engine_destroy(h->main);
    engine_destroy(h->left);
    engine_destroy(h->top);
    free_all(h->allocs);
    if (h->items_h) (void)hipHostFree(h->items_h);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->side) (void)hipStreamDestroy(h->side);
    h->magic = 0;
    delete h;
    return SFR_OK;
}

sfr_status sfr_workspace_bytes(sfr_handle h, uint64_t* bytes)
{
    if (!h || h->magic != 0x53465221u) return SFR_ERR_HANDLE;
    if (!bytes) return SFR_ERR_ARG;
    size_t b = h->main.bytes + h->left.bytes + h->top.bytes + h->batch_bytes + lr_bytes(h->lr);
    *bytes = (uint64_t)b;
    return SFR_OK;
}

sfr_status sfr_solve(sfr_handle h, const void* M, int64_t ldm, void* U, double* B, void* V, void* S, int64_t lds,
                     sfr_info* info, void* hip_stream)
{
    if (!h || h->magic != 0x53465221u || h->nys || h->batch) return SFR_ERR_HANDLE;
    if (!M || !U || !B || !V) return SFR_ERR_ARG;
    if (ldm < h->n || (S && lds < h->n)) return SFR_ERR_ARG;
    if (h->lr)
        return lr_solve(h->lr, h->prm, h->mu_auto, static_cast<const float*>(M), ldm, static_cast<float*>(U), B,
                        static_cast<float*>(V), static_cast<float*>(S), lds, info, static_cast<hipStream_t>(hip_stream));
    return engine_solve(h->main, h->prm, h->mu_auto, M, ldm, U, B, V, S, lds, info,
                        static_cast<hipStream_t>(hip_stream));
}

sfr_status sfr_tsvd(sfr_handle h, const void* M, int64_t ldm, void* U, double* B, void* V, sfr_info* info,
                    void* hip_stream)
{
    if (!h || h->magic != 0x53465221u || h->nys || h->batch) return SFR_ERR_HANDLE;
    if (!M || !U || !B || !V) return SFR_ERR_ARG;
    if (ldm < h->n) return SFR_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (h->lr)
        return lr_tsvd(h->lr, h->prm, static_cast<const float*>(M), ldm, static_cast<float*>(U), B,
                       static_cast<float*>(V), info, s);
    Engine& e = h->main;
    sfr_status st;
    if (h->f64) {
        OutputSpec<double> o;
        o.U = static_cast<double*>(U); o.B = B; o.V = static_cast<double*>(V);
        o.min_eig = true;
        st = engine_iterate<double>(e, h->prm, h->prm.mu0, static_cast<const double*>(M), ldm, o, s, true);
    } else {
        OutputSpec<float> o;
        o.U = static_cast<float*>(U); o.B = B; o.V = static_cast<float*>(V);
        o.min_eig = true;
        st = engine_iterate<float>(e, h->prm, h->prm.mu0, static_cast<const float*>(M), ldm, o, s, true);
    }
    if (st < 0) {
        if (info) memset(info, 0, sizeof(*info));
        return st;
    }
    return fill_info(e, info, st);
}

}  // extern "C"
