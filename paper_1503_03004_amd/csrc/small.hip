// FP64 r x r algebra of one FR-ADM iteration, on the device.
//
// Given the Grams G_P = P^T P, G_Q = Q^T Q of the sweep and the previous
// SPD factor B0, the closed-form projectors of Sec. 4.1 become
//   C1 = (B0 G_P B0)^{-1/2}            U  = P B0 C1          (eq. (7))
//   K  = B0 C1 B0,  C2 = (K G_Q K)^{-1/2}, V = Q K C2         (eq. (7))
//   B  = Sym(C1 B0 G_Q K C2)                                  (eq. (8))
// and the next sweep rebuilds L rows as a_i = P_i (B0 C1 B).
//
// Inverse square roots come from the one-wavefront Jacobi eigendecomposition
// of small_la.hpp, started from the eigenbasis found in the previous
// iteration: the Grams change little from one iteration to the next, so one
// or two sweeps suffice.
#include "small_la.hpp"

namespace sfr {

// Workgroup size of the step kernel: the partial sums are latency bound,
// so as many threads as the r x r algebra's register use allows (1024
// threads leave 128 registers a lane, which buckets 5 and 12 and up exceed).
// Up to R = 4 (2E <= 20 Gram entries) 256 threads already take every
// partial in one round of loads, and the workgroup barriers cost less.
template <int R>
constexpr int step_tpb() { return R <= 4 ? 256 : ((R <= 10 && R != 5) ? 1024 : 512); }

// The r x r matrices are held R x R (R the rank bucket, a compile-time
// size) with an identity block on the padded indices: every product and
// inverse square root below is then block diagonal and exact on the
// leading r x r block, and the padded block is dropped when the transforms
// are stored.
template <int R>
__global__ void __launch_bounds__(step_tpb<R>()) step_kernel(StepArgs a)
{
    DevState* st = a.st;
    if (st->done) return;
    if (st->exch_timeout) {   // a sweep hit its wait bound: stop the solve
        if (threadIdx.x == 0) st->done = 1;
        return;
    }
    constexpr int TPB = step_tpb<R>();
    // threads of the r x r algebra: one wavefront up to R = 12, the whole
    // workgroup above (each Jacobi round then has >= 128 2x2 blocks)
    constexpr int NT = (R >= 16) ? TPB : 64;
    constexpr int E = R * (R + 1) / 2;
    __shared__ double Gp[R * LDP], Gq[R * LDP], Bm[R * LDP], C1[R * LDP];
    __shared__ double C2[R * LDP], Km[R * LDP], T1[R * LDP], T2[R * LDP];
    __shared__ double Ev[R * LDP], Ev2[R * LDP];
    __shared__ double seg[2 * E > TPB ? 2 * E : TPB];
    __shared__ double tri[2][E];
    __shared__ double red[TPB / 64];
    __shared__ __align__(16) double cs[2 * 16];
    __shared__ double wbuf[kMaxR];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = st->r, k = st->k;

    // ---- one round of loads: B0 and the two warm-start bases (wave 0, into
    // registers), the residual partials and the Gram partials.  The Gram
    // partials (upper triangles) are summed in a fixed order: thread w owns
    // entry e of Gram g over the partials b = s, s + nseg, ... (segment s),
    // then the nseg segment sums are added in order.
    // Every load below is unconditional (indices are clamped into range and
    // the surplus masked afterwards), so each thread has all of its loads in
    // flight at once: one memory round trip for the lot.
    constexpr int NPL = (R * R + NT - 1) / NT;
    double rb[NPL], re1[NPL], re2[NPL];
    if (tid < NT) {
#pragma unroll
        for (int u = 0; u < NPL; ++u) {
            const int e = min(tid + NT * u, R * R - 1);
            const int i = e / R, j = e % R;
            rb[u] = st->B[i * kMaxR + j];
            re1[u] = st->E1[i * kMaxR + j];
            re2[u] = st->E2[i * kMaxR + j];
        }
    }
    constexpr int DYU = (kMaxDyPartials + TPB - 1) / TPB;
    double dyv[DYU];
#pragma unroll
    for (int u = 0; u < DYU; ++u) dyv[u] = a.dy2part[min(tid + u * TPB, a.ndy - 1)];
    constexpr int nseg = (2 * E >= TPB) ? 1 : TPB / (2 * E);
    constexpr int PER = (kMaxGramPartials + nseg - 1) / nseg;   // partials per segment
    constexpr int CH = PER < 32 ? PER : 32;                      // loads in flight
    for (int w = tid; w < 2 * E * nseg; w += TPB) {
        const int g = w / (E * nseg), rem = w % (E * nseg);
        const int sg = rem / E, e = rem % E;
        const double* part = g ? a.GQpart : a.GPpart;
        const int count = g ? a.nqb : a.npb;
        double s = 0.0;
        for (int u0 = 0; u0 < PER; u0 += CH) {
            double v[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) v[u] = part[(size_t)min(sg + (u0 + u) * nseg, count - 1) * E + e];
#pragma unroll
            for (int u = 0; u < CH; ++u) s += (sg + (u0 + u) * nseg < count) ? v[u] : 0.0;
        }
        seg[w] = s;
    }

    // ---- convergence test of iteration k-1 (or ||M||_F on the first pass)
    double part = 0.0;
#pragma unroll
    for (int u = 0; u < DYU; ++u) part += (tid + u * TPB < a.ndy) ? dyv[u] : 0.0;
    for (int e = tid + DYU * TPB; e < a.ndy; e += TPB) part += a.dy2part[e];
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    double total = 0.0;
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w) total += red[w];
    if (k == 1) {
        const double nrm = sqrt(total);
        if (!(nrm > 0.0) || !isfinite(nrm)) {
            if (tid == 0) { st->nrmM = nrm; st->status = kErrNonFinite; st->iters = 0; st->done = 1; }
            return;
        }
        if (tid == 0) st->nrmM = nrm;
    } else if (!st->tsvd) {
        const double res = sqrt(total) / (st->mu_prev * st->nrmM);
        const int kdone = k - 1;
        bool stop = false;
        int32_t status = kOK;
        if (!isfinite(res)) { stop = true; status = kErrNonFinite; }
        else if (st->fixed_iters > 0) { stop = kdone >= st->fixed_iters; }
        else if (res <= st->tol) { stop = true; }
        else if (kdone >= st->max_iter) { stop = true; status = kWarnMaxIter; }
        if (tid == 0) {
            a.res_hist[kdone - 1] = res;
            st->res = res;
        }
        if (stop) {
            if (tid == 0) { st->status = status; st->iters = kdone; st->done = 1; }
            return;
        }
    }

    // ---- Grams: add the segment sums
    for (int w = tid; w < 2 * E; w += TPB) {
        const int g = w / E, e = w % E;
        double s = 0.0;
#pragma unroll
        for (int sg = 0; sg < nseg; ++sg) s += seg[(g * nseg + sg) * E + e];
        tri[g][e] = s;
    }
    __syncthreads();
    if (tid >= NT) return;

    // ---- the r x r algebra: NT threads from here on
#pragma unroll
    for (int u = 0; u < NPL; ++u) {
        const int e = tid + NT * u;
        if (e >= R * R) break;
        const int i = e / R, j = e % R;
        const int x = i < j ? i : j, y = i < j ? j : i;
        const int t = x * R - x * (x - 1) / 2 + (y - x);   // upper-triangle index of (x, y)
        const bool pad = (i >= r) || (j >= r);
        Gp[i * LDP + j] = pad ? (i == j ? 1.0 : 0.0) : tri[0][t];
        Gq[i * LDP + j] = pad ? (i == j ? 1.0 : 0.0) : tri[1][t];
        Bm[i * LDP + j] = rb[u];
        Ev[i * LDP + j] = re1[u];
        Ev2[i * LDP + j] = re2[u];
    }
    lsync<NT>();

    if (!lstep_algebra<R, NT>(Gp, Gq, Bm, C1, C2, Km, T1, T2, Ev, Ev2, cs, wbuf, r, a.dk_tau)) {
        if (tid == 0) { st->status = kErrRank; st->iters = k - 1; st->done = 1; }
        return;
    }
    // only the R x R block changes; the rest keeps the values set at the
    // start of the solve (zero, identity on the diagonal of B)
#pragma unroll
    for (int u = 0; u < NPL; ++u) {
        const int e = tid + NT * u;
        if (e >= R * R) break;
        const int i = e / R, j = e % R;
        const int g = i * kMaxR + j;
        const bool in = (i < r) && (j < r);
        const double tu = in ? Km[i * LDP + j] : 0.0;
        const double tv = in ? Gp[i * LDP + j] : 0.0;
        st->B[g] = in ? T2[i * LDP + j] : (i == j ? 1.0 : 0.0);
        st->TU[g] = tu;
        st->TUbar[g] = in ? T1[i * LDP + j] : 0.0;
        st->TV[g] = tv;
        st->TUf[g] = (float)tu;
        st->TVf[g] = (float)tv;
        st->E1[g] = Ev[i * LDP + j];
        st->E2[g] = Ev2[i * LDP + j];
    }
    if (st->tsvd) {
        // Alg. 4 stops after this step once B has settled:
        // ||B_k - B_{k-1}||_F <= tol ||B_k||_F (or after fixed_iters steps)
        double d2 = 0.0, n2 = 0.0;
#pragma unroll
        for (int u = 0; u < NPL; ++u) {
            const int e = tid + NT * u;
            const int i = e / R, j = e % R;
            if (e < R * R && i < r && j < r) {
                const double bn = T2[i * LDP + j], bo = Bm[i * LDP + j];
                d2 = fma(bn - bo, bn - bo, d2);
                n2 = fma(bn, bn, n2);
            }
        }
        d2 = wave_sum(d2);
        n2 = wave_sum(n2);
        if constexpr (NT > 64) {
            // red[] (the residual reduction's, free now) holds the wave sums
            if (lane == 0) { red[wave] = d2; seg[wave] = n2; }
            __syncthreads();
            d2 = 0.0; n2 = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) { d2 += red[w]; n2 += seg[w]; }
        }
        const double res = sqrt(d2 / n2);
        bool stop = false;
        int32_t status = kOK;
        if (!isfinite(res)) { stop = true; status = kErrNonFinite; }
        else if (st->fixed_iters > 0) { stop = k >= st->fixed_iters; }
        else if (res <= st->tol) { stop = true; }
        else if (k >= st->max_iter) { stop = true; status = kWarnMaxIter; }
        if (tid == 0) {
            a.res_hist[k - 1] = res;
            st->res = res;
            st->k = k + 1;
            if (stop) { st->status = status; st->iters = k; st->done = 1; }
        }
        return;
    }
    if (tid == 0) {
        const double mu = st->mu;
        st->mu_prev = mu;
        const double nm = st->rho * mu;
        st->mu = nm < st->mu_bar ? nm : st->mu_bar;
        st->k = k + 1;
    }
}

// Smallest eigenvalue of the returned B (is it in SPD_r?  Appendix, Lemma 2).
template <int R>
__global__ void __launch_bounds__(64) final_small_kernel(DevState* st)
{
    __shared__ double A[R * LDP], Ev[R * LDP];
    __shared__ __align__(16) double cs[2 * 16];
    const double w = wmin_eig<R>(st->B, kMaxR, st->r, A, Ev, cs);
    if (threadIdx.x == 0) st->min_eig_B = w;
}

// Largest eigenvalue of the returned B.  After Alg. 4 on M, B has the r
// leading singular values of M as its eigenvalues (Theorem 2), so this is
// ||M||_2 (full Jacobi convergence from the identity basis).
template <int R>
__global__ void __launch_bounds__(64) max_eig_kernel(DevState* st)
{
    __shared__ double A[R * LDP], Ev[R * LDP];
    __shared__ __align__(16) double cs[2 * 16];
    const int lane = threadIdx.x;
    const int r = st->r;
    for (int e = lane; e < R * R; e += 64) {
        const int i = e / R, j = e % R;
        const bool pad = (i >= r) || (j >= r);
        A[i * LDP + j] = pad ? (i == j ? 1.0 : 0.0) : st->B[i * kMaxR + j];
        Ev[i * LDP + j] = (i == j) ? 1.0 : 0.0;
    }
    lsync<64>();
    wjacobi<R, 64>(A, Ev, cs);
    if (lane == 0) {
        double w = -INFINITY;
        for (int i = 0; i < r; ++i) w = fmax(w, A[i * LDP + i]);
        st->max_eig_B = w;
    }
}

#define SFR_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32)

hipError_t launch_step(const StepArgs& a, int R, hipStream_t s)
{
    switch (R) {
#define CASE(rr) case rr: hipLaunchKernelGGL(step_kernel<rr>, dim3(1), dim3(step_tpb<rr>()), 0, s, a); break;
        SFR_R_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Continue a stopped solve from its returned iterate K (the second phase of
// a BF16 solve): every buffer of iterate K (Y_K, P_K, Q_K) and the state of
// its step (transforms, B, mu, the warm-start bases) are intact, so this only
// installs the new stopping rule, clears the stop and sets the next sweep to
// K + 1.  A solve that stopped with an error, or with no iterations left in
// the new rule, stays stopped.
__global__ void refine_start_kernel(DevState* st, int fixed_iters, double tol, int max_iter)
{
    if (threadIdx.x != 0) return;
    if (!st->done || st->status < 0 || st->exch_timeout) return;
    const int K = st->iters;
    if (K >= (fixed_iters > 0 ? fixed_iters : max_iter)) return;
    st->status = kOK;
    st->fixed_iters = fixed_iters;
    st->tol = tol;
    st->max_iter = max_iter;
    st->k = K + 1;
    st->done = 0;
}

hipError_t launch_refine_start(DevState* st, int fixed_iters, double tol, int max_iter, hipStream_t s)
{
    hipLaunchKernelGGL(refine_start_kernel, dim3(1), dim3(64), 0, s, st, fixed_iters, tol, max_iter);
    return hipGetLastError();
}

hipError_t launch_max_eig(DevState* st, int R, hipStream_t s)
{
    switch (R) {
#define CASE(rr) case rr: hipLaunchKernelGGL(max_eig_kernel<rr>, dim3(1), dim3(64), 0, s, st); break;
        SFR_R_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_final_small(DevState* st, int R, hipStream_t s)
{
    switch (R) {
#define CASE(rr) case rr: hipLaunchKernelGGL(final_small_kernel<rr>, dim3(1), dim3(64), 0, s, st); break;
        SFR_R_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sfr
