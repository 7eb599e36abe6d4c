// FP64 r x r algebra of one FR-ADM iteration, on the device (one workgroup).
//
// Given the Grams G_P = P^T P, G_Q = Q^T Q of the sweep and the previous
// SPD factor B0, the closed-form projectors of Sec. 4.1 become
//   C1 = (B0 G_P B0)^{-1/2}            U  = P B0 C1          (eq. (7))
//   K  = B0 C1 B0,  C2 = (K G_Q K)^{-1/2}, V = Q K C2         (eq. (7))
//   B  = Sym(C1 B0 G_Q K C2)                                  (eq. (8))
// and the next sweep rebuilds L rows as a_i = P_i (B0 C1 B).
// Inverse square roots come from a cyclic Jacobi eigendecomposition
// (Golub & Van Loan, Matrix Computations, Sec. 8.5) with the parallel
// round-robin ordering: r/2 disjoint rotations per round.
#include "sfr_internal.hpp"

#include <float.h>

namespace sfr {

constexpr int LDP = kMaxR + 1;  // LDS pitch of an r x r matrix (doubles)

__device__ double block_sum(double v, double* red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = kTPB / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    double out = red[0];
    __syncthreads();
    return out;
}

__device__ double block_max(double v, double* red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = kTPB / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    double out = red[0];
    __syncthreads();
    return out;
}

__device__ double block_min(double v, double* red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = kTPB / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmin(red[tid], red[tid + s]);
        __syncthreads();
    }
    double out = red[0];
    __syncthreads();
    return out;
}

// C = A B (r x r, pitch LDP).  C must not alias A or B.
__device__ void mm(double* C, const double* A, const double* B, int r)
{
    for (int e = threadIdx.x; e < r * r; e += kTPB) {
        const int i = e / r, j = e % r;
        double s = 0.0;
        for (int t = 0; t < r; ++t) s = fma(A[i * LDP + t], B[t * LDP + j], s);
        C[i * LDP + j] = s;
    }
    __syncthreads();
}

__device__ void symmetrize(double* A, int r)
{
    for (int e = threadIdx.x; e < r * r; e += kTPB) {
        const int i = e / r, j = e % r;
        if (i < j) {
            const double s = 0.5 * (A[i * LDP + j] + A[j * LDP + i]);
            A[i * LDP + j] = s;
            A[j * LDP + i] = s;
        }
    }
    __syncthreads();
}

// Round-robin pairing: position 0 holds player 0, positions 1..N-1 rotate.
__device__ inline int rr_player(int pos, int round, int N)
{
    return pos == 0 ? 0 : ((pos - 1 + round) % (N - 1)) + 1;
}

// A (r x r symmetric, LDS) -> diag(eigenvalues) in place; E = eigenvectors
// (columns).  cs: LDS scratch of 4 * 16 doubles; red: 256 doubles.
__device__ void jacobi_eig(double* A, double* E, int r, double* cs, double* red)
{
    const int tid = threadIdx.x;
    for (int e = tid; e < r * r; e += kTPB) {
        const int i = e / r, j = e % r;
        E[i * LDP + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (r == 1) return;
    const int N = r + (r & 1);
    const int npair = N / 2;
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int e = tid; e < r * r; e += kTPB) {
            const int i = e / r, j = e % r;
            const double v = A[i * LDP + j];
            if (i == j) dia += v * v; else off += v * v;
        }
        off = block_sum(off, red);
        dia = block_sum(dia, red);
        if (!(off > 1e-30 * dia)) break;
        for (int round = 0; round < N - 1; ++round) {
            if (tid < npair) {
                int p = rr_player(tid, round, N);
                int q = rr_player(N - 1 - tid, round, N);
                if (p > q) { int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < r) {
                    const double apq = A[p * LDP + q];
                    if (apq != 0.0) {
                        const double tau = (A[q * LDP + q] - A[p * LDP + p]) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                cs[4 * tid + 0] = c;
                cs[4 * tid + 1] = s;
                cs[4 * tid + 2] = (double)p;
                cs[4 * tid + 3] = (double)q;
            }
            __syncthreads();
            // A <- A J and E <- E J  (columns p, q of every row)
            for (int it = tid; it < npair * r; it += kTPB) {
                const int pi = it / r, x = it % r;
                const int p = (int)cs[4 * pi + 2], q = (int)cs[4 * pi + 3];
                if (q >= r) continue;
                const double c = cs[4 * pi + 0], s = cs[4 * pi + 1];
                const double ap = A[x * LDP + p], aq = A[x * LDP + q];
                A[x * LDP + p] = c * ap - s * aq;
                A[x * LDP + q] = s * ap + c * aq;
                const double ep = E[x * LDP + p], eq = E[x * LDP + q];
                E[x * LDP + p] = c * ep - s * eq;
                E[x * LDP + q] = s * ep + c * eq;
            }
            __syncthreads();
            // A <- J^T A  (rows p, q of every column)
            for (int it = tid; it < npair * r; it += kTPB) {
                const int pi = it / r, x = it % r;
                const int p = (int)cs[4 * pi + 2], q = (int)cs[4 * pi + 3];
                if (q >= r) continue;
                const double c = cs[4 * pi + 0], s = cs[4 * pi + 1];
                const double ap = A[p * LDP + x], aq = A[q * LDP + x];
                A[p * LDP + x] = c * ap - s * aq;
                A[q * LDP + x] = s * ap + c * aq;
            }
            __syncthreads();
        }
    }
}

// Out = A^{-1/2} for symmetric A (destroyed).  Returns false if A is not
// positive definite to working precision (the Stiefel projector of eq. (7)
// needs rank r).
__device__ bool inv_sqrt(double* Out, double* A, double* E, int r, double* cs, double* red,
                         double* wbuf)
{
    jacobi_eig(A, E, r, cs, red);
    const int tid = threadIdx.x;
    double wmax = -INFINITY, wmin = INFINITY;
    for (int i = tid; i < r; i += kTPB) {
        wbuf[i] = A[i * LDP + i];
        wmax = fmax(wmax, wbuf[i]);
        wmin = fmin(wmin, wbuf[i]);
    }
    wmax = block_max(wmax, red);
    wmin = block_min(wmin, red);
    const bool ok = (wmax > 0.0) && (wmin > (double)r * DBL_EPSILON * wmax) && isfinite(wmax);
    for (int e = tid; e < r * r; e += kTPB) {
        const int i = e / r, j = e % r;
        double s = 0.0;
        for (int t = 0; t < r; ++t) {
            const double wt = wbuf[t] > 0.0 ? 1.0 / sqrt(wbuf[t]) : 0.0;
            s = fma(E[i * LDP + t] * wt, E[j * LDP + t], s);
        }
        Out[i * LDP + j] = s;
    }
    __syncthreads();
    return ok;
}

__global__ void __launch_bounds__(kTPB) step_kernel(StepArgs a)
{
    DevState* st = a.st;
    if (st->done) return;
    __shared__ double Gp[kMaxR * LDP], Gq[kMaxR * LDP], Bm[kMaxR * LDP], C1[kMaxR * LDP];
    __shared__ double C2[kMaxR * LDP], Km[kMaxR * LDP], T1[kMaxR * LDP], T2[kMaxR * LDP];
    __shared__ double Ev[kMaxR * LDP];
    __shared__ double red[kTPB];
    __shared__ double cs[4 * 16];
    __shared__ double wbuf[kMaxR];
    const int tid = threadIdx.x;
    const int r = st->r, R = st->R, k = st->k;
    const int E = R * (R + 1) / 2;

    // ---- convergence test of iteration k-1 (or ||M||_F on the first pass)
    double part = 0.0;
    for (int e = tid; e < a.ndy; e += kTPB) part += a.dy2part[e];
    const double total = block_sum(part, red);
    if (k == 1) {
        const double nrm = sqrt(total);
        if (tid == 0) st->nrmM = nrm;
        if (!(nrm > 0.0) || !isfinite(nrm)) {
            if (tid == 0) { st->status = kErrNonFinite; st->iters = 0; st->done = 1; }
            return;
        }
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
    for (int e = tid; e < E; e += kTPB) {
        int x = 0, rem = e;
        while (rem >= R - x) { rem -= R - x; ++x; }
        const int y = x + rem;
        double sp = 0.0, sq = 0.0;
        for (int b = 0; b < a.npb; ++b) sp += a.GPpart[(size_t)b * E + e];
        for (int b = 0; b < a.nqb; ++b) sq += a.GQpart[(size_t)b * E + e];
        if (x < r && y < r) {
            Gp[x * LDP + y] = sp; Gp[y * LDP + x] = sp;
            Gq[x * LDP + y] = sq; Gq[y * LDP + x] = sq;
        }
    }
    for (int e = tid; e < r * r; e += kTPB) {
        const int i = e / r, j = e % r;
        Bm[i * LDP + j] = st->B[i * kMaxR + j];
    }
    __syncthreads();

    // ---- U-step: C1 = (B0 G_P B0)^{-1/2}
    mm(T1, Bm, Gp, r);
    mm(T2, T1, Bm, r);
    symmetrize(T2, r);
    const bool ok1 = inv_sqrt(C1, T2, Ev, r, cs, red, wbuf);
    // ---- V-step: K = B0 C1 B0, C2 = (K G_Q K)^{-1/2}
    mm(T1, Bm, C1, r);          // T1 = B0 C1  (the U transform)
    mm(Km, T1, Bm, r);
    symmetrize(Km, r);
    mm(T2, Km, Gq, r);
    mm(Ev, T2, Km, r);          // Ev used as scratch for K G_Q K
    symmetrize(Ev, r);
    for (int e = tid; e < r * r; e += kTPB) T2[(e / r) * LDP + e % r] = Ev[(e / r) * LDP + e % r];
    __syncthreads();
    const bool ok2 = inv_sqrt(C2, T2, Ev, r, cs, red, wbuf);
    if (!ok1 || !ok2) {
        if (tid == 0) { st->status = kErrRank; st->iters = k - 1; st->done = 1; }
        return;
    }
    // TV = K C2 -> Ev ; B = Sym(C1 B0 G_Q K C2) -> Gp (reused)
    mm(Ev, Km, C2, r);                // TV
    mm(T2, C1, Bm, r);                // C1 B0
    mm(Gp, T2, Gq, r);                // C1 B0 G_Q
    mm(T2, Gp, Ev, r);                // C1 B0 G_Q K C2
    symmetrize(T2, r);                // T2 = new B
    mm(Gq, T1, T2, r);                // TU = B0 C1 B
    for (int e = tid; e < kMaxR * kMaxR; e += kTPB) {
        const int i = e / kMaxR, j = e % kMaxR;
        const bool in = (i < r) && (j < r);
        const double b = in ? T2[i * LDP + j] : 0.0;
        const double tu = in ? Gq[i * LDP + j] : 0.0;
        const double tub = in ? T1[i * LDP + j] : 0.0;
        const double tv = in ? Ev[i * LDP + j] : 0.0;
        st->B[e] = b;
        st->TU[e] = tu;
        st->TUbar[e] = tub;
        st->TV[e] = tv;
        st->TUf[e] = (float)tu;
        st->TVf[e] = (float)tv;
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
__global__ void __launch_bounds__(kTPB) final_small_kernel(DevState* st)
{
    __shared__ double A[kMaxR * LDP], Ev[kMaxR * LDP];
    __shared__ double red[kTPB];
    __shared__ double cs[4 * 16];
    const int r = st->r;
    const int tid = threadIdx.x;
    for (int e = tid; e < r * r; e += kTPB) A[(e / r) * LDP + e % r] = st->B[(e / r) * kMaxR + e % r];
    __syncthreads();
    jacobi_eig(A, Ev, r, cs, red);
    double w = INFINITY;
    for (int i = tid; i < r; i += kTPB) w = fmin(w, A[i * LDP + i]);
    w = block_min(w, red);
    if (tid == 0) st->min_eig_B = w;
}

hipError_t launch_step(const StepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(step_kernel, dim3(1), dim3(kTPB), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_final_small(DevState* st, hipStream_t s)
{
    hipLaunchKernelGGL(final_small_kernel, dim3(1), dim3(kTPB), 0, s, st);
    return hipGetLastError();
}

}  // namespace sfr
