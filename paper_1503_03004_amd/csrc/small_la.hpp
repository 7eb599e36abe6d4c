// One-wavefront FP64 dense linear algebra on r x r matrices in LDS (r <= 32):
// products, symmetrisation and a cyclic Jacobi eigendecomposition
// (Golub & Van Loan, Matrix Computations, Sec. 8.5) with the parallel
// round-robin ordering.  Every routine is executed by all 64 lanes of one
// wavefront and orders its LDS phases with wavefront fences only.
#pragma once

#include "sfr_internal.hpp"

#include <float.h>

namespace sfr {

constexpr int LDP = kMaxR + 1;  // LDS pitch of an r x r matrix (doubles)

// Orders the LDS accesses of the lanes of one wavefront.
__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// C = A B (r x r, pitch LDP), one wavefront.  C must not alias A or B.
template <int N>
__device__ inline void wmm(double* C, const double* A, const double* B)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int e0 = 0; e0 < N * N; e0 += 64) {
        const int e = e0 + lane;
        if (e >= N * N) break;
        const int i = e / N, j = e % N;
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < N; ++t) s = fma(A[i * LDP + t], B[t * LDP + j], s);
        C[i * LDP + j] = s;
    }
    wsync();
}

// C = A^T B
template <int N>
__device__ inline void wmtm(double* C, const double* A, const double* B)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int e0 = 0; e0 < N * N; e0 += 64) {
        const int e = e0 + lane;
        if (e >= N * N) break;
        const int i = e / N, j = e % N;
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < N; ++t) s = fma(A[t * LDP + i], B[t * LDP + j], s);
        C[i * LDP + j] = s;
    }
    wsync();
}

template <int N>
__device__ inline void wsym(double* A)
{
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < N * N; e += 64) {
        const int i = e / N, j = e % N;
        if (i < j) {
            const double s = 0.5 * (A[i * LDP + j] + A[j * LDP + i]);
            A[i * LDP + j] = s;
            A[j * LDP + i] = s;
        }
    }
    wsync();
}

template <int N>
__device__ inline void wcopy(double* D, const double* A)
{
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < N * N; e += 64) D[(e / N) * LDP + e % N] = A[(e / N) * LDP + e % N];
    wsync();
}

// Round-robin pairing: position 0 holds player 0, positions 1..N-1 rotate.
__device__ inline int rr_player(int pos, int round, int N)
{
    return pos == 0 ? 0 : ((pos - 1 + round) % (N - 1)) + 1;
}

// One wavefront.  A (r x r symmetric, LDS) -> diag(eigenvalues) in place;
// E holds on entry an orthogonal starting basis E0 and on exit the
// eigenvectors, with A_in = E diag E^T.  On entry A must already be
// expressed in the basis E0 (A = E0^T A_in E0).  cs: LDS scratch 8 * 16.
//
// Each rotation sets its pair exactly (a_pq = 0, a_pp -= t a_pq,
// a_qq += t a_pq), so off-diagonal entries shrink without a rounding floor
// and the relative test |a_pq| <= eps sqrt(|a_pp a_qq|) is reached also for
// graded matrices; the test is made for all pairs before each sweep.
template <int r>
__device__ inline void wjacobi(double* A, double* E, double* cs)
{
    const int lane = threadIdx.x & 63;
    if (r == 1) return;
    constexpr int N = r + (r & 1);
    constexpr int npair = N / 2;
    for (int sweep = 0; sweep < 16; ++sweep) {
        int big = 0;
        for (int e = lane; e < r * r; e += 64) {
            const int i = e / r, j = e % r;
            if (i < j) {
                const double apq = A[i * LDP + j];
                if (fabs(apq) > DBL_EPSILON * sqrt(fabs(A[i * LDP + i] * A[j * LDP + j])) && apq != 0.0) big = 1;
            }
        }
        if (!__any(big)) break;
        for (int round = 0; round < N - 1; ++round) {
            if (lane < npair) {
                int p = rr_player(lane, round, N);
                int q = rr_player(N - 1 - lane, round, N);
                if (p > q) { int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0, t = 0.0, app = 0.0, aqq = 0.0, apq = 0.0;
                if (q < r) {
                    apq = A[p * LDP + q];
                    app = A[p * LDP + p];
                    aqq = A[q * LDP + q];
                    if (fabs(apq) > DBL_EPSILON * sqrt(fabs(app * aqq)) && apq != 0.0) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                double* w = cs + 8 * lane;
                w[0] = c; w[1] = s; w[2] = (double)p; w[3] = (double)q;
                w[4] = app - t * apq;   // new a_pp
                w[5] = aqq + t * apq;   // new a_qq
                w[6] = (s != 0.0) ? 1.0 : 0.0;
            }
            wsync();
            // A <- A J and E <- E J  (columns p, q of every row)
            for (int it = lane; it < npair * r; it += 64) {
                const int pi = it / r, x = it % r;
                const double* w = cs + 8 * pi;
                if (w[6] == 0.0) continue;
                const int p = (int)w[2], q = (int)w[3];
                const double c = w[0], s = w[1];
                const double ap = A[x * LDP + p], aq = A[x * LDP + q];
                A[x * LDP + p] = c * ap - s * aq;
                A[x * LDP + q] = s * ap + c * aq;
                const double ep = E[x * LDP + p], eq = E[x * LDP + q];
                E[x * LDP + p] = c * ep - s * eq;
                E[x * LDP + q] = s * ep + c * eq;
            }
            wsync();
            // A <- J^T A  (rows p, q of every column); the 2 x 2 block of
            // the pair takes its exact rotated values
            for (int it = lane; it < npair * r; it += 64) {
                const int pi = it / r, x = it % r;
                const double* w = cs + 8 * pi;
                if (w[6] == 0.0) continue;
                const int p = (int)w[2], q = (int)w[3];
                const double c = w[0], s = w[1];
                if (x == p) {
                    A[p * LDP + p] = w[4];
                    A[q * LDP + p] = 0.0;
                } else if (x == q) {
                    A[q * LDP + q] = w[5];
                    A[p * LDP + q] = 0.0;
                } else {
                    const double ap = A[p * LDP + x], aq = A[q * LDP + x];
                    A[p * LDP + x] = c * ap - s * aq;
                    A[q * LDP + x] = s * ap + c * aq;
                }
            }
            wsync();
        }
    }
}

// Out = A^{-1/2} for symmetric A (destroyed), one wavefront.  E: on entry
// the warm-start basis, on exit the eigenvectors of A.  T: scratch.  Only
// the leading `nreal` eigenvalues are tested (the rest belong to an
// identity padding block).  Returns false if A is not positive definite to
// working precision (the Stiefel projector of eq. (7) needs rank r).
template <int N>
__device__ inline bool winv_sqrt(double* Out, double* A, double* E, double* T, int nreal, double* cs, double* wbuf)
{
    const int lane = threadIdx.x & 63;
    // A <- E^T A E
    wmm<N>(T, A, E);
    wmtm<N>(A, E, T);
    wsym<N>(A);
    wjacobi<N>(A, E, cs);
    double wmax = -INFINITY, wmin = INFINITY;
    for (int i = lane; i < N; i += 64) {
        wbuf[i] = A[i * LDP + i];
        if (i < nreal) {
            wmax = fmax(wmax, wbuf[i]);
            wmin = fmin(wmin, wbuf[i]);
        }
    }
    wmax = wave_max(wmax);
    wmin = wave_min(wmin);
    wsync();
    const bool ok = (wmax > 0.0) && (wmin > (double)nreal * DBL_EPSILON * wmax) && isfinite(wmax);
#pragma unroll
    for (int e0 = 0; e0 < N * N; e0 += 64) {
        const int e = e0 + lane;
        if (e >= N * N) break;
        const int i = e / N, j = e % N;
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < N; ++t) {
            const double wt = wbuf[t] > 0.0 ? 1.0 / sqrt(wbuf[t]) : 0.0;
            s = fma(E[i * LDP + t] * wt, E[j * LDP + t], s);
        }
        Out[i * LDP + j] = s;
    }
    wsync();
    return ok;
}

}  // namespace sfr
