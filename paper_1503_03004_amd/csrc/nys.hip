// FR-Nys (Alg. 3): random row shuffle, FR-ADM on the m x l left block and
// on the l x n top block, Nystrom combination L = L_L (L_L[1:l,1:l])^+ L_T,
// S = M - L.
//
// The combination is kept factored.  With L_L = U_L B_L V_L^T and
// A = U_L[1:l,:] B_L (l x r, rank r), the intersection block is
// W = L_L[1:l,1:l] = A V_L^T, so W^+ = V_L (A^T A)^{-1} A^T and
//   L = U_L G V_T^T,   G = B_L (A^T A)^{-1} A^T U_T B_T   (r x r).
// The r x r core is then written as G = Wl diag(sig) Zr^T (FP64), so the
// returned factors are U = U_L Wl (rows restored to M's order), B =
// diag(sig) and V = V_T Zr, again in St x SPD x St.  The only dense work
// after the two sub-solves is one pass writing S.
#include "engine.hpp"
#include "small_la.hpp"

#include <string.h>

#include <algorithm>
#include <thread>

namespace sfr {

// Threads of the combine's r x r algebra: one wavefront up to R = 12, a
// workgroup of 512 from R = 16 (as the step kernel: each Jacobi round then
// has >= 128 2 x 2 blocks).
template <int R>
constexpr int nys_combine_threads() { return R >= 16 ? 512 : 64; }

// From U_L (rows 0..l-1 used), B_L, U_T, B_T build G and its SVD, by NT
// threads.  status: 0, or kErrRank if A^T A or G is singular.  The r x r
// matrices are held R x R with an identity block on the padded indices.
template <typename T, int R>
__global__ void __launch_bounds__(nys_combine_threads<R>()) nys_combine_kernel(const T* UL, const double* BL,
                                                                               const T* UT, const double* BT,
                                                                               int l, int r, double* Wl,
                                                                               double* Zr, double* sig,
                                                                               int32_t* status)
{
    constexpr int NT = nys_combine_threads<R>();
    __shared__ double H1[R * LDP], H2[R * LDP], Bl[R * LDP], Bt[R * LDP];
    __shared__ double T1[R * LDP], T2[R * LDP], Ev[R * LDP], G[R * LDP];
    __shared__ __align__(16) double cs[2 * 16];
    __shared__ double wbuf[kMaxR];
    const int lane = lid<NT>();
    // H1 = U_L[0:l]^T U_L[0:l], H2 = U_L[0:l]^T U_T
    for (int e = lane; e < R * R; e += NT) {
        const int a = e / R, b = e % R;
        const bool pad = (a >= r) || (b >= r);
        double s1 = 0.0, s2 = 0.0;
        if (!pad) {
            for (int i = 0; i < l; ++i) {
                const double ua = (double)UL[(int64_t)i * r + a];
                s1 = fma(ua, (double)UL[(int64_t)i * r + b], s1);
                s2 = fma(ua, (double)UT[(int64_t)i * r + b], s2);
            }
        }
        const double id = (a == b) ? 1.0 : 0.0;
        H1[a * LDP + b] = pad ? id : s1;
        H2[a * LDP + b] = pad ? id : s2;
        Bl[a * LDP + b] = pad ? id : BL[a * r + b];
        Bt[a * LDP + b] = pad ? id : BT[a * r + b];
        Ev[a * LDP + b] = id;
    }
    lsync<NT>();
    // A^T A = B_L H1 B_L
    wmm<R, NT>(T1, Bl, H1);
    wmm<R, NT>(T2, T1, Bl);
    wsym<R, NT>(T2);
    wjacobi<R, NT>(T2, Ev, cs);
    for (int i = lane; i < R; i += NT) wbuf[i] = T2[i * LDP + i];
    lsync<NT>();
    // every thread reads the whole diagonal for the rank test
    double wmax = -INFINITY, wmin = INFINITY;
    for (int i = 0; i < r; ++i) {
        wmax = fmax(wmax, wbuf[i]);
        wmin = fmin(wmin, wbuf[i]);
    }
    bool ok = (wmax > 0.0) && (wmin > (double)r * DBL_EPSILON * wmax) && isfinite(wmax);
    // T1 = (A^T A)^{-1}
    for (int e = lane; e < R * R; e += NT) {
        const int i = e / R, j = e % R;
        double s = 0.0;
        for (int t = 0; t < R; ++t) s = fma(Ev[i * LDP + t] / wbuf[t], Ev[j * LDP + t], s);
        T1[i * LDP + j] = s;
    }
    lsync<NT>();
    // G = B_L (A^T A)^{-1} (B_L H2) B_T
    wmm<R, NT>(T2, Bl, T1);      // B_L (A^T A)^{-1}
    wmm<R, NT>(H1, Bl, H2);      // A^T U_T = B_L H2
    wmm<R, NT>(T1, T2, H1);
    wmm<R, NT>(G, T1, Bt);
    // SVD of G from the eigendecomposition of G^T G = Zr diag(sig^2) Zr^T
    wmtm<R, NT>(T2, G, G);
    wsym<R, NT>(T2);
    for (int e = lane; e < R * R; e += NT) Ev[(e / R) * LDP + e % R] = ((e / R) == (e % R)) ? 1.0 : 0.0;
    lsync<NT>();
    wjacobi<R, NT>(T2, Ev, cs);
    for (int i = lane; i < R; i += NT) {
        const double w = T2[i * LDP + i];
        wbuf[i] = w > 0.0 ? sqrt(w) : 0.0;
    }
    lsync<NT>();
    double smax = -INFINITY, smin = INFINITY;
    for (int i = 0; i < r; ++i) {
        smax = fmax(smax, wbuf[i]);
        smin = fmin(smin, wbuf[i]);
    }
    ok = ok && (smax > 0.0) && (smin > (double)r * DBL_EPSILON * smax) && isfinite(smax);
    // Wl = G Zr diag(1/sig)
    wmm<R, NT>(T1, G, Ev);
    for (int e = lane; e < r * r; e += NT) {
        const int i = e / r, j = e % r;
        Wl[i * r + j] = wbuf[j] > 0.0 ? T1[i * LDP + j] / wbuf[j] : 0.0;
        Zr[i * r + j] = Ev[i * LDP + j];
    }
    for (int i = lane; i < r; i += NT) sig[i] = wbuf[i];
    if (lane == 0) *status = ok ? kOK : kErrRank;
}

template <typename T>
static hipError_t launch_nys_combine(int R, const T* UL, const double* BL, const T* UT, const double* BT, int l,
                                     int r, double* Wl, double* Zr, double* sig, int32_t* status, hipStream_t s)
{
    switch (R) {
#define CASE(rr)                                                                                          \
    case rr:                                                                                              \
        hipLaunchKernelGGL((nys_combine_kernel<T, rr>), dim3(1), dim3(nys_combine_threads<rr>()), 0, s, UL, BL, \
                           UT, BT, l, r, Wl, Zr, sig, status);                                            \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(8) CASE(10) CASE(12) CASE(16) CASE(20) CASE(24)
        CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// U[perm[i]] = (U_L Wl)_i,  V = V_T Zr,  B = diag(sig), and the R-wide row
// factors A = U diag(sig), Vc = V of the S pass.
template <typename T>
__global__ void nys_factors_kernel(const T* UL, const T* VT, const int64_t* perm, const double* Wl,
                                   const double* Zr, const double* sig, int m, int n, int r, int R, T* U, T* V,
                                   double* B, T* A, T* Vc)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nu = (int64_t)m * R, nvv = (int64_t)n * R;
    if (e < nu) {
        const int i = (int)(e / R), k = (int)(e % R);
        const int64_t dst = perm[i];
        double u = 0.0;
        if (k < r)
            for (int t = 0; t < r; ++t) u = fma((double)UL[(int64_t)i * r + t], Wl[t * r + k], u);
        if (k < r) U[dst * r + k] = (T)u;
        A[dst * R + k] = (k < r) ? (T)(u * sig[k]) : T(0);
    } else if (e < nu + nvv) {
        const int64_t f = e - nu;
        const int j = (int)(f / R), k = (int)(f % R);
        double v = 0.0;
        if (k < r)
            for (int t = 0; t < r; ++t) v = fma((double)VT[(int64_t)j * r + t], Zr[t * r + k], v);
        if (k < r) V[(int64_t)j * r + k] = (T)v;
        Vc[f] = (k < r) ? (T)v : T(0);
    } else if (e < nu + nvv + (int64_t)r * r) {
        const int64_t f = e - nu - nvv;
        const int i = (int)(f / r), j = (int)(f % r);
        B[f] = (i == j) ? sig[i] : 0.0;
    }
}

#define HIPCHK(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) {                   \
            (void)hipGetLastError();               \
            return SFR_ERR_DEVICE;                 \
        }                                          \
    } while (0)

sfr_status nys_setup(sfr_ctx* h)
{
    const bool f64 = h->f64;
    const size_t esz = f64 ? 8 : 4;
    const int m = (int)h->m, n = (int)h->n, r = h->r, l = h->l;
    const int hist = std::max(h->prm.max_iter, h->prm.fixed_iters);
    sfr_status st = engine_create(h->left, m, l, r, f64, hist);
    if (st != SFR_OK) return st;
    st = engine_create(h->top, l, n, r, f64, hist);
    if (st != SFR_OK) return st;
    const int R = h->left.R;
    size_t bytes = 0;
    bool ok = true;
    ok = ok && dev_alloc(h->allocs, bytes, &h->C, (size_t)m * l * esz);
    ok = ok && dev_alloc(h->allocs, bytes, &h->Rb, (size_t)l * n * esz);
    ok = ok && dev_alloc(h->allocs, bytes, (void**)&h->perm_d, sizeof(int64_t) * (size_t)m);
    ok = ok && dev_alloc(h->allocs, bytes, &h->UL, (size_t)m * r * esz);
    ok = ok && dev_alloc(h->allocs, bytes, &h->VL, (size_t)l * r * esz);
    ok = ok && dev_alloc(h->allocs, bytes, &h->UT, (size_t)l * r * esz);
    ok = ok && dev_alloc(h->allocs, bytes, &h->VT, (size_t)n * r * esz);
    ok = ok && dev_alloc(h->allocs, bytes, (void**)&h->BL, sizeof(double) * (size_t)r * r);
    ok = ok && dev_alloc(h->allocs, bytes, (void**)&h->BT, sizeof(double) * (size_t)r * r);
    // core: Wl, Zr (r x r each), sig (r), status
    ok = ok && dev_alloc(h->allocs, bytes, (void**)&h->core, sizeof(double) * (size_t)(2 * r * r + r + 2));
    ok = ok && dev_alloc(h->allocs, bytes, &h->Ucomb, (size_t)m * R * esz);
    ok = ok && dev_alloc(h->allocs, bytes, &h->Vcomb, (size_t)n * R * esz);
    if (!ok) return SFR_ERR_NOMEM;
    h->left.bytes += bytes;
    // the l x n sub-solve runs on a second stream beside the m x l one
    if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return SFR_ERR_DEVICE;
    }
    return SFR_OK;
}

// Whether any sweep of the engine runs in clusters (c > 1), whose members
// wait on each other's partial row products.
static bool engine_waits(const Engine& e)
{
    return e.cfg[0].c > 1 || e.cfg[1].c > 1;
}

template <typename T>
static sfr_status nys_run(sfr_ctx* h, const T* M, int64_t ldm, T* U, double* B, T* V, T* S, int64_t lds,
                          double* min_sig, double* orth, hipStream_t s)
{
    const int m = (int)h->m, n = (int)h->n, r = h->r, l = h->l;
    const int R = h->left.R;
    HIPCHK(launch_nys_gather<T>(M, ldm, h->perm_d, m, n, l, static_cast<T*>(h->C), static_cast<T*>(h->Rb), s));
    // The two sub-solves are independent: the l x n one runs on the side
    // stream, driven from a host thread, while this thread drives the m x l
    // one on the caller's stream; each engine_iterate waits for its own
    // stream, and the join orders the combine after both.  They overlap
    // only if at most one of them runs cluster sweeps: a kernel without
    // inter-workgroup waits always drains and frees its slots, so the
    // members of the other one's clusters all become resident.  If both
    // wait on cluster members, the l x n sub-solve runs after the m x l one.
    HIPCHK(hipEventRecord(h->ev_fork, s));
    HIPCHK(hipStreamWaitEvent(h->side, h->ev_fork, 0));
    OutputSpec<T> ol;
    ol.U = static_cast<T*>(h->UL); ol.B = h->BL; ol.V = static_cast<T*>(h->VL);
    OutputSpec<T> ot;
    ot.U = static_cast<T*>(h->UT); ot.B = h->BT; ot.V = static_cast<T*>(h->VT);
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    sfr_status st_top = SFR_ERR_DEVICE;
    auto run_top = [&]() {
        if (hipSetDevice(dev) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        st_top = engine_iterate<T>(h->top, h->prm, h->mu_top, static_cast<const T*>(h->Rb), n, ot, h->side);
    };
    std::thread top;
    bool threaded = !(engine_waits(h->left) && engine_waits(h->top));
    if (threaded) {
        try {
            top = std::thread(run_top);
        } catch (...) {   // no thread available: the two sub-solves run one after the other
            threaded = false;
        }
    }
    const sfr_status st_left = engine_iterate<T>(h->left, h->prm, h->mu_left, static_cast<const T*>(h->C), l, ol, s);
    if (threaded) top.join();
    else run_top();
    HIPCHK(hipEventRecord(h->ev_join, h->side));
    HIPCHK(hipStreamWaitEvent(s, h->ev_join, 0));
    if (st_left != SFR_OK) return st_left;
    if (st_top != SFR_OK) return st_top;
    double* Wl = h->core;
    double* Zr = Wl + r * r;
    double* sig = Zr + r * r;
    int32_t* status = reinterpret_cast<int32_t*>(sig + r);
    HIPCHK(launch_nys_combine<T>(R, static_cast<const T*>(h->UL), h->BL, static_cast<const T*>(h->UT), h->BT, l, r,
                                 Wl, Zr, sig, status, s));
    double host_core[kMaxR + 2];
    HIPCHK(hipMemcpyAsync(host_core, sig, sizeof(double) * (size_t)(r + 1), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int32_t cst;
    memcpy(&cst, &host_core[r], sizeof(cst));
    if (cst != kOK) return (sfr_status)cst;
    double ms = INFINITY;
    for (int i = 0; i < r; ++i) ms = std::min(ms, host_core[i]);
    *min_sig = ms;
    const int64_t cnt = (int64_t)m * R + (int64_t)n * R + (int64_t)r * r;
    hipLaunchKernelGGL(nys_factors_kernel<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       static_cast<const T*>(h->UL), static_cast<const T*>(h->VT), h->perm_d, Wl, Zr, sig, m, n,
                       r, R, U, V, B, static_cast<T*>(h->Ucomb), static_cast<T*>(h->Vcomb));
    HIPCHK(hipGetLastError());
    HIPCHK(launch_orth<T>(nullptr, U, m, V, n, r, h->left.GPpart, h->left.npb, h->top.GQpart, h->top.nqb,
                          &h->left.st->orth_err, s));
    HIPCHK(hipMemcpyAsync(orth, &h->left.st->orth_err, sizeof(double), hipMemcpyDeviceToHost, s));
    if (S) {
        LowrankArgs<T> la;
        memset(&la, 0, sizeof(la));
        la.M = M;
        la.ldm = ldm;
        la.A = static_cast<const T*>(h->Ucomb);
        la.Vt = static_cast<const T*>(h->Vcomb);
        la.S = S;
        la.lds = lds;
        la.m = m;
        la.n = n;
        la.mode = 1;
        la.lam = 0.0;
        la.mu = 1.0;
        HIPCHK(launch_lowrank_pass<T>(la, R, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return SFR_OK;
}

}  // namespace sfr

using namespace sfr;

extern "C" sfr_status sfr_solve_nys(sfr_handle h, const void* M, int64_t ldm, const int64_t* perm, void* U,
                                    double* B, void* V, void* S, int64_t lds, sfr_info* info, void* hip_stream)
{
    if (!h || h->magic != 0x53465221u || !h->nys || h->batch) return SFR_ERR_HANDLE;
    if (!M || !perm || !U || !B || !V) return SFR_ERR_ARG;
    if (ldm < h->n || (S && lds < h->n)) return SFR_ERR_ARG;
    // perm must be a permutation of 0..m-1
    {
        std::vector<unsigned char> seen((size_t)h->m, 0);
        for (int64_t i = 0; i < h->m; ++i) {
            const int64_t p = perm[i];
            if (p < 0 || p >= h->m || seen[(size_t)p]) return SFR_ERR_ARG;
            seen[(size_t)p] = 1;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (hipMemcpyAsync(h->perm_d, perm, sizeof(int64_t) * (size_t)h->m, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        return SFR_ERR_DEVICE;
    }
    double min_sig = 0.0, orth = 0.0;
    sfr_status st;
    if (h->f64)
        st = nys_run<double>(h, static_cast<const double*>(M), ldm, static_cast<double*>(U), B,
                             static_cast<double*>(V), static_cast<double*>(S), lds, &min_sig, &orth, s);
    else
        st = nys_run<float>(h, static_cast<const float*>(M), ldm, static_cast<float*>(U), B,
                            static_cast<float*>(V), static_cast<float*>(S), lds, &min_sig, &orth, s);
    if (st < 0) {
        if (info) memset(info, 0, sizeof(*info));
        return st;
    }
    const DevState& hl = *h->left.host_state;
    const DevState& ht = *h->top.host_state;
    if (info) {
        memset(info, 0, sizeof(*info));
        info->iters = hl.iters;
        info->iters_top = ht.iters;
        info->converged = (hl.status == kOK && ht.status == kOK) ? 1 : 0;
        info->rel_residual = std::max(hl.res, ht.res);
        info->min_eig_B = min_sig;
        info->mu_final = hl.mu_prev;
        info->orth_err = orth;
    }
    if (hl.status == kWarnMaxIter || ht.status == kWarnMaxIter) return SFR_WARN_MAXITER;
    return SFR_OK;
}
