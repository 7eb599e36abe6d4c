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

// Sum of `count` FP64 partial vectors of length E (part[b * E + e]) in a
// fixed order, spread over the workgroup: segment sums, then segments.
__device__ void sum_partials(double* out_lds, const double* part, int count, int E, double* seg)
{
    const int tid = threadIdx.x;
    const int nseg = max(1, kTPB / E);
    for (int w = tid; w < E * nseg; w += kTPB) {
        const int e = w / nseg, sg = w % nseg;
        double s = 0.0;
#pragma unroll 8
        for (int b = sg; b < count; b += nseg) s += part[(size_t)b * E + e];
        seg[w] = s;
    }
    __syncthreads();
    for (int e = tid; e < E; e += kTPB) {
        double s = 0.0;
        for (int sg = 0; sg < nseg; ++sg) s += seg[e * nseg + sg];
        out_lds[e] = s;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kTPB) step_kernel(StepArgs a)
{
    DevState* st = a.st;
    if (st->done) return;
    __shared__ double Gp[kMaxR * LDP], Gq[kMaxR * LDP], Bm[kMaxR * LDP], C1[kMaxR * LDP];
    __shared__ double C2[kMaxR * LDP], Km[kMaxR * LDP], T1[kMaxR * LDP], T2[kMaxR * LDP];
    __shared__ double Ev[kMaxR * LDP], Ev2[kMaxR * LDP];
    __shared__ double seg[2 * kMaxR * (kMaxR + 1) / 2 + kTPB];
    __shared__ double tri[2][kMaxR * (kMaxR + 1) / 2];
    __shared__ double red[kTPB / 64];
    __shared__ double cs[4 * 16];
    __shared__ double wbuf[kMaxR];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = st->r, R = st->R, k = st->k;
    const int E = R * (R + 1) / 2;

    // ---- convergence test of iteration k-1 (or ||M||_F on the first pass)
    double part = 0.0;
    for (int e = tid; e < a.ndy; e += kTPB) part += a.dy2part[e];
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    const double total = (red[0] + red[1]) + (red[2] + red[3]);
    if (k == 1) {
        const double nrm = sqrt(total);
        if (!(nrm > 0.0) || !isfinite(nrm)) {
            if (tid == 0) { st->nrmM = nrm; st->status = kErrNonFinite; st->iters = 0; st->done = 1; }
            return;
        }
        if (tid == 0) st->nrmM = nrm;
    } else {
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

    // ---- Grams (upper triangles, fixed summation order)
    sum_partials(tri[0], a.GPpart, a.npb, E, seg);
    sum_partials(tri[1], a.GQpart, a.nqb, E, seg);
    if (wave != 0) return;

    // ---- the r x r algebra: one wavefront from here on
    for (int e = lane; e < E; e += 64) {
        int x = 0, rem = e;
        while (rem >= R - x) { rem -= R - x; ++x; }
        const int y = x + rem;
        if (x < r && y < r) {
            Gp[x * LDP + y] = tri[0][e]; Gp[y * LDP + x] = tri[0][e];
            Gq[x * LDP + y] = tri[1][e]; Gq[y * LDP + x] = tri[1][e];
        }
    }
    for (int e = lane; e < r * r; e += 64) {
        const int i = e / r, j = e % r;
        Bm[i * LDP + j] = st->B[i * kMaxR + j];
        Ev[i * LDP + j] = st->E1[i * kMaxR + j];
        Ev2[i * LDP + j] = st->E2[i * kMaxR + j];
    }
    wsync();

    // ---- U-step: C1 = (B0 G_P B0)^{-1/2}
    wmm(T1, Bm, Gp, r);
    wmm(T2, T1, Bm, r);
    wsym(T2, r);
    const bool ok1 = winv_sqrt(C1, T2, Ev, T1, r, cs, wbuf);
    // ---- V-step: K = B0 C1 B0, C2 = (K G_Q K)^{-1/2}
    wmm(T1, Bm, C1, r);          // T1 = B0 C1  (the U transform)
    wmm(Km, T1, Bm, r);
    wsym(Km, r);
    wmm(T2, Km, Gq, r);
    wmm(C2, T2, Km, r);          // K G_Q K (C2 as scratch)
    wsym(C2, r);
    wcopy(T2, C2, r);
    const bool ok2 = winv_sqrt(C2, T2, Ev2, Gp, r, cs, wbuf);   // Gp free now
    if (!ok1 || !ok2) {
        if (lane == 0) { st->status = kErrRank; st->iters = k - 1; st->done = 1; }
        return;
    }
    // TV = K C2 -> Gp ; B = Sym(C1 B0 G_Q K C2) -> T2 ; TU = B0 C1 B -> Km
    wmm(Gp, Km, C2, r);               // TV
    wmm(T2, C1, Bm, r);               // C1 B0
    wmm(C2, T2, Gq, r);               // C1 B0 G_Q
    wmm(T2, C2, Gp, r);               // C1 B0 G_Q K C2
    wsym(T2, r);                      // new B
    wmm(Km, T1, T2, r);               // TU
    for (int e = lane; e < kMaxR * kMaxR; e += 64) {
        const int i = e / kMaxR, j = e % kMaxR;
        const bool in = (i < r) && (j < r);
        const double b = in ? T2[i * LDP + j] : 0.0;
        const double tu = in ? Km[i * LDP + j] : 0.0;
        const double tub = in ? T1[i * LDP + j] : 0.0;
        const double tv = in ? Gp[i * LDP + j] : 0.0;
        st->B[e] = b;
        st->TU[e] = tu;
        st->TUbar[e] = tub;
        st->TV[e] = tv;
        st->TUf[e] = (float)tu;
        st->TVf[e] = (float)tv;
        if (in) {
            st->E1[e] = Ev[i * LDP + j];
            st->E2[e] = Ev2[i * LDP + j];
        }
    }
    if (lane == 0) {
        const double mu = st->mu;
        st->mu_prev = mu;
        const double nm = st->rho * mu;
        st->mu = nm < st->mu_bar ? nm : st->mu_bar;
        st->k = k + 1;
    }
}

// Smallest eigenvalue of the returned B (is it in SPD_r?  Appendix, Lemma 2).
__global__ void __launch_bounds__(64) final_small_kernel(DevState* st)
{
    __shared__ double A[kMaxR * LDP], Ev[kMaxR * LDP];
    __shared__ double cs[4 * 16];
    const int r = st->r;
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < r * r; e += 64) {
        const int i = e / r, j = e % r;
        A[i * LDP + j] = st->B[i * kMaxR + j];
        Ev[i * LDP + j] = (i == j) ? 1.0 : 0.0;
    }
    wsync();
    wjacobi(A, Ev, r, cs);
    double w = INFINITY;
    for (int i = lane; i < r; i += 64) w = fmin(w, A[i * LDP + i]);
    w = wave_min(w);
    if (lane == 0) st->min_eig_B = w;
}

hipError_t launch_step(const StepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(step_kernel, dim3(1), dim3(kTPB), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_final_small(DevState* st, hipStream_t s)
{
    hipLaunchKernelGGL(final_small_kernel, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

}  // namespace sfr
