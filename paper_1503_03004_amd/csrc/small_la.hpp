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
__device__ inline void wmm(double* C, const double* A, const double* B, int r)
{
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < r * r; e += 64) {
        const int i = e / r, j = e % r;
        double s = 0.0;
        for (int t = 0; t < r; ++t) s = fma(A[i * LDP + t], B[t * LDP + j], s);
        C[i * LDP + j] = s;
    }
    wsync();
}

// C = A^T B
__device__ inline void wmtm(double* C, const double* A, const double* B, int r)
{
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < r * r; e += 64) {
        const int i = e / r, j = e % r;
        double s = 0.0;
        for (int t = 0; t < r; ++t) s = fma(A[t * LDP + i], B[t * LDP + j], s);
        C[i * LDP + j] = s;
    }
    wsync();
}

__device__ inline void wsym(double* A, int r)
{
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < r * r; e += 64) {
        const int i = e / r, j = e % r;
        if (i < j) {
            const double s = 0.5 * (A[i * LDP + j] + A[j * LDP + i]);
            A[i * LDP + j] = s;
            A[j * LDP + i] = s;
        }
    }
    wsync();
}

__device__ inline void wcopy(double* D, const double* A, int r)
{
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < r * r; e += 64) D[(e / r) * LDP + e % r] = A[(e / r) * LDP + e % r];
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
// expressed in the basis E0 (A = E0^T A_in E0).  cs: LDS scratch 4 * 16.
__device__ inline void wjacobi(double* A, double* E, int r, double* cs)
{
    const int lane = threadIdx.x & 63;
    if (r == 1) return;
    const int N = r + (r & 1);
    const int npair = N / 2;
    for (int sweep = 0; sweep < 40; ++sweep) {
        int rotated = 0;
        for (int round = 0; round < N - 1; ++round) {
            if (lane < npair) {
                int p = rr_player(lane, round, N);
                int q = rr_player(N - 1 - lane, round, N);
                if (p > q) { int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < r) {
                    const double apq = A[p * LDP + q];
                    const double app = A[p * LDP + p], aqq = A[q * LDP + q];
                    // rotate unless a_pq is negligible next to its diagonal pair
                    if (fabs(apq) > DBL_EPSILON * sqrt(fabs(app * aqq)) && apq != 0.0) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                        rotated = 1;
                    }
                }
                cs[4 * lane + 0] = c;
                cs[4 * lane + 1] = s;
                cs[4 * lane + 2] = (double)p;
                cs[4 * lane + 3] = (double)q;
            }
            wsync();
            // A <- A J and E <- E J  (columns p, q of every row)
            for (int it = lane; it < npair * r; it += 64) {
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
            wsync();
            // A <- J^T A  (rows p, q of every column)
            for (int it = lane; it < npair * r; it += 64) {
                const int pi = it / r, x = it % r;
                const int p = (int)cs[4 * pi + 2], q = (int)cs[4 * pi + 3];
                if (q >= r) continue;
                const double c = cs[4 * pi + 0], s = cs[4 * pi + 1];
                const double ap = A[p * LDP + x], aq = A[q * LDP + x];
                A[p * LDP + x] = c * ap - s * aq;
                A[q * LDP + x] = s * ap + c * aq;
            }
            wsync();
        }
        // stop after a sweep in which no pair needed a rotation
        if (!__any(rotated)) break;
    }
}

// Out = A^{-1/2} for symmetric A (destroyed), one wavefront.  E: on entry
// the warm-start basis, on exit the eigenvectors of A.  T: scratch.
// Returns false if A is not positive definite to working precision (the
// Stiefel projector of eq. (7) needs rank r).
__device__ inline bool winv_sqrt(double* Out, double* A, double* E, double* T, int r, double* cs, double* wbuf)
{
    const int lane = threadIdx.x & 63;
    // A <- E^T A E
    wmm(T, A, E, r);
    wmtm(A, E, T, r);
    wsym(A, r);
    wjacobi(A, E, r, cs);
    double wmax = -INFINITY, wmin = INFINITY;
    for (int i = lane; i < r; i += 64) {
        wbuf[i] = A[i * LDP + i];
        wmax = fmax(wmax, wbuf[i]);
        wmin = fmin(wmin, wbuf[i]);
    }
    wmax = wave_max(wmax);
    wmin = wave_min(wmin);
    wsync();
    const bool ok = (wmax > 0.0) && (wmin > (double)r * DBL_EPSILON * wmax) && isfinite(wmax);
    for (int e = lane; e < r * r; e += 64) {
        const int i = e / r, j = e % r;
        double s = 0.0;
        for (int t = 0; t < r; ++t) {
            const double wt = wbuf[t] > 0.0 ? 1.0 / sqrt(wbuf[t]) : 0.0;
            s = fma(E[i * LDP + t] * wt, E[j * LDP + t], s);
        }
        Out[i * LDP + j] = s;
    }
    wsync();
    return ok;
}

}  // namespace sfr
