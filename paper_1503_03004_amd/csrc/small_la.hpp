// FP64 dense linear algebra on r x r matrices in LDS (r <= 32): products,
// symmetrisation and a cyclic Jacobi eigendecomposition (Golub & Van Loan,
// Matrix Computations, Sec. 8.5) with the parallel round-robin ordering.
// Every routine is executed by NT threads: one wavefront (NT = 64, the
// default; LDS phases ordered with wavefront fences) or a whole workgroup of
// NT threads (phases ordered with workgroup barriers, which every thread of
// the workgroup must reach).
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

// Ordering and agreement among the NT threads of the algebra.
template <int NT>
__device__ __forceinline__ void lsync()
{
    if constexpr (NT == 64) wsync();
    else __syncthreads();
}
template <int NT>
__device__ __forceinline__ bool l_any(bool p)
{
    if constexpr (NT == 64) return __any(p);
    else return __syncthreads_or(p) != 0;
}
template <int NT>
__device__ __forceinline__ int lid()
{
    return NT == 64 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
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

// C = A B (r x r, pitch LDP).  C must not alias A or B.
template <int N, int NT = 64>
__device__ inline void wmm(double* C, const double* A, const double* B)
{
    const int lane = lid<NT>();
#pragma unroll
    for (int e0 = 0; e0 < N * N; e0 += NT) {
        const int e = e0 + lane;
        if (e >= N * N) break;
        const int i = e / N, j = e % N;
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < N; ++t) s = fma(A[i * LDP + t], B[t * LDP + j], s);
        C[i * LDP + j] = s;
    }
    lsync<NT>();
}

// C = A^T B
template <int N, int NT = 64>
__device__ inline void wmtm(double* C, const double* A, const double* B)
{
    const int lane = lid<NT>();
#pragma unroll
    for (int e0 = 0; e0 < N * N; e0 += NT) {
        const int e = e0 + lane;
        if (e >= N * N) break;
        const int i = e / N, j = e % N;
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < N; ++t) s = fma(A[t * LDP + i], B[t * LDP + j], s);
        C[i * LDP + j] = s;
    }
    lsync<NT>();
}

template <int N, int NT = 64>
__device__ inline void wsym(double* A)
{
    const int lane = lid<NT>();
    for (int e = lane; e < N * N; e += NT) {
        const int i = e / N, j = e % N;
        if (i < j) {
            const double s = 0.5 * (A[i * LDP + j] + A[j * LDP + i]);
            A[i * LDP + j] = s;
            A[j * LDP + i] = s;
        }
    }
    lsync<NT>();
}

template <int N, int NT = 64>
__device__ inline void wcopy(double* D, const double* A)
{
    const int lane = lid<NT>();
    for (int e = lane; e < N * N; e += NT) D[(e / N) * LDP + e % N] = A[(e / N) * LDP + e % N];
    lsync<NT>();
}

// Round-robin pairing: position 0 holds player 0, positions 1..N-1 rotate.
__device__ inline int rr_player(int pos, int round, int N)
{
    return pos == 0 ? 0 : ((pos - 1 + round) % (N - 1)) + 1;
}

// One wavefront.  A (r x r symmetric, LDS) -> diag(eigenvalues) in place;
// E holds on entry an orthogonal starting basis E0 and on exit the
// eigenvectors, with A_in = E diag E^T.  On entry A must already be
// expressed in the basis E0 (A = E0^T A_in E0).  cs: LDS scratch of 2 * 16
// doubles, 16-byte aligned.
//
// Cyclic Jacobi in the round-robin parallel order: each round rotates
// N / 2 disjoint pairs at once.  Each rotation sets its pair exactly
// (a_pq = 0, a_pp -= t a_pq, a_qq += t a_pq), so off-diagonal entries shrink
// without a rounding floor and the relative test
// |a_pq| <= eps sqrt(|a_pp a_qq|) is reached also for graded matrices; the
// test is made for all pairs before each sweep.
//
// A round is two phases.  Pair phase: lane b < N / 2 computes the rotation
// of pair b, t = sign(d) 2 a_pq / (|d| + sqrt(d^2 + 4 a_pq^2)) with
// d = a_qq - a_pp (the smaller root of t^2 + 2 tau t - 1 = 0, tau = d / 2a_pq),
// c = 1 / sqrt(1 + t^2), s = t c, and writes the pair's own 2 x 2 block.
// Update phase: one lane per 2 x 2 block (rows of pair i, columns of pair
// j, i != j) applies J_i^T . J_j, and one lane per 2 x 2 block of E (two
// rows, the columns of one pair) applies . J.  Pair indices are recomputed
// from the round number, so the only data passed between the phases is
// (c, s).  Squares of entries above ~1e150 would overflow d^2 + 4 a_pq^2.
template <int r, int NT = 64>
__device__ inline void wjacobi(double* A, double* E, double* cs, double tau = 0.0)
{
    const int lane = lid<NT>();
    if (r == 1) return;
    constexpr int N = r + (r & 1);
    constexpr int npair = N / 2;
    constexpr int nrp = (r + 1) / 2;              // row pairs of E
    constexpr int nblk = npair * npair;           // 2 x 2 blocks of A
    constexpr int nitem = nblk + nrp * npair;     // + 2 x 2 blocks of E
    for (int sweep = 0; sweep < 16; ++sweep) {
        int big = 0, far = 0;
        for (int e = lane; e < r * r; e += NT) {
            const int i = e / r, j = e % r;
            if (i < j) {
                const double apq = A[i * LDP + j];
                const double app = A[i * LDP + i], aqq = A[j * LDP + j];
                if (apq != 0.0 && apq * apq > DBL_EPSILON * DBL_EPSILON * fabs(app * aqq)) big = 1;
                if (!(fabs(apq) <= tau * fmin(fabs(app), fabs(aqq)))) far = 1;
            }
        }
        const bool any_big = l_any<NT>(big != 0);
        const bool any_far = l_any<NT>(far != 0);
        if (!any_big || !any_far) break;
        for (int round = 0; round < N - 1; ++round) {
            if (lane < npair) {
                int p = rr_player(lane, round, N);
                int q = rr_player(N - 1 - lane, round, N);
                if (p > q) { int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < r) {
                    const double apq = A[p * LDP + q];
                    const double app = A[p * LDP + p];
                    const double aqq = A[q * LDP + q];
                    if (apq != 0.0 && apq * apq > DBL_EPSILON * DBL_EPSILON * fabs(app * aqq)) {
                        const double d = aqq - app;
                        const double h = sqrt(fma(d, d, 4.0 * apq * apq));
                        const double t = (d >= 0.0 ? 2.0 * apq : -2.0 * apq) / (fabs(d) + h);
                        c = rsqrt(fma(t, t, 1.0));
                        s = t * c;
                        A[p * LDP + p] = fma(-t, apq, app);
                        A[q * LDP + q] = fma(t, apq, aqq);
                        A[p * LDP + q] = 0.0;
                        A[q * LDP + p] = 0.0;
                    }
                }
                cs[2 * lane] = c;
                cs[2 * lane + 1] = s;
            }
            lsync<NT>();
            for (int it = lane; it < nitem; it += NT) {
                if (it < nblk) {
                    const int bi = it / npair, bj = it % npair;
                    if (bi == bj) continue;
                    int pi = rr_player(bi, round, N), qi = rr_player(N - 1 - bi, round, N);
                    int pj = rr_player(bj, round, N), qj = rr_player(N - 1 - bj, round, N);
                    if (pi > qi) { int t = pi; pi = qi; qi = t; }
                    if (pj > qj) { int t = pj; pj = qj; qj = t; }
                    const bool hq_i = qi < r, hq_j = qj < r;
                    const double a00 = A[pi * LDP + pj];
                    const double a01 = hq_j ? A[pi * LDP + qj] : 0.0;
                    const double a10 = hq_i ? A[qi * LDP + pj] : 0.0;
                    const double a11 = (hq_i && hq_j) ? A[qi * LDP + qj] : 0.0;
                    const double ci = cs[2 * bi], si = cs[2 * bi + 1];
                    const double cj = cs[2 * bj], sj = cs[2 * bj + 1];
                    const double b00 = cj * a00 - sj * a01, b01 = sj * a00 + cj * a01;
                    const double b10 = cj * a10 - sj * a11, b11 = sj * a10 + cj * a11;
                    A[pi * LDP + pj] = ci * b00 - si * b10;
                    if (hq_j) A[pi * LDP + qj] = ci * b01 - si * b11;
                    if (hq_i) A[qi * LDP + pj] = si * b00 + ci * b10;
                    if (hq_i && hq_j) A[qi * LDP + qj] = si * b01 + ci * b11;
                } else {
                    const int e2 = it - nblk;
                    const int x = e2 / npair, bi = e2 % npair;
                    int p = rr_player(bi, round, N), q = rr_player(N - 1 - bi, round, N);
                    if (p > q) { int t = p; p = q; q = t; }
                    if (q >= r) continue;                 // the idle pair of odd r
                    const int x0 = 2 * x, x1 = 2 * x + 1;
                    const bool h1 = x1 < r;
                    const double e0p = E[x0 * LDP + p], e0q = E[x0 * LDP + q];
                    const double e1p = h1 ? E[x1 * LDP + p] : 0.0, e1q = h1 ? E[x1 * LDP + q] : 0.0;
                    const double c = cs[2 * bi], s = cs[2 * bi + 1];
                    E[x0 * LDP + p] = c * e0p - s * e0q;
                    E[x0 * LDP + q] = s * e0p + c * e0q;
                    if (h1) {
                        E[x1 * LDP + p] = c * e1p - s * e1q;
                        E[x1 * LDP + q] = s * e1p + c * e1q;
                    }
                }
            }
            lsync<NT>();
        }
    }
}

// Out = A^{-1/2} for symmetric A (destroyed), one wavefront.  The Jacobi
// sweeps stop once |a_ij| <= tau min(a_ii, a_jj) in the current basis; the
// rest of the way is the second-order expansion of t^{-1/2} about the
// diagonal, whose error is O(tau^3 r^2) relative (tau: kDkTauF64 or
// kDkTauF32).  Across FR-ADM iterations the Grams move less and less, so the
// previous iteration's basis soon meets this bound with no sweep at all.
// E: on entry the warm-start basis, on exit a basis in which A is diagonal
// to within tau (updated only by the sweeps that were needed).  T, cs, wbuf:
// scratch.  Only the leading `nreal` eigenvalues are tested (the rest belong
// to an identity padding block).  Returns false if A is not positive
// definite to working precision (the Stiefel projector of eq. (7) needs
// rank r).
template <int N, int NT = 64>
__device__ inline bool winv_sqrt(double* Out, double* A, double* E, double* T, int nreal, double* cs, double* wbuf,
                                 double tau)
{
    const int lane = lid<NT>();
    // A <- E^T A E
    wmm<N, NT>(T, A, E);
    wmtm<N, NT>(A, E, T);
    wsym<N, NT>(A);
    wjacobi<N, NT>(A, E, cs, tau);
    // A = D + F, D = diag(d), F off-diagonal with |F_ij| <= tau min(d_i, d_j)
    // (or at the strict Jacobi test).  x = sqrt(d) -> wbuf, y = 1 / x -> cs.
    // Every thread reads the whole diagonal for the positivity test.
    double wmax = -INFINITY, wmin = INFINITY;
    for (int i = 0; i < nreal; ++i) {
        const double d = A[i * LDP + i];
        wmax = fmax(wmax, d);
        wmin = fmin(wmin, d);
    }
    for (int i = lane; i < N; i += NT) {
        const double d = A[i * LDP + i];
        const double x = d > 0.0 ? sqrt(d) : 0.0;
        wbuf[i] = x;
        cs[i] = d > 0.0 ? 1.0 / x : 0.0;
    }
    lsync<NT>();
    const bool ok = (wmax > 0.0) && (wmin > (double)nreal * DBL_EPSILON * wmax) && isfinite(wmax);
    // W_ij = 1 / (x_i + x_j) -> Out, Phi = F o W -> T
    for (int e = lane; e < N * N; e += NT) {
        const int i = e / N, j = e % N;
        const double den = wbuf[i] + wbuf[j];
        const double w = den > 0.0 ? 1.0 / den : 0.0;
        Out[i * LDP + j] = w;
        T[i * LDP + j] = (i == j) ? 0.0 : A[i * LDP + j] * w;
    }
    lsync<NT>();
    // Z = f(D + F) to second order, f(t) = t^{-1/2}:
    //   Z_ij = delta_ij y_i + F_ij f[d_i, d_j] + sum_k F_ik F_kj f[d_i, d_k, d_j],
    //   f[d_i, d_j] = -W_ij y_i y_j,
    //   f[d_i, d_k, d_j] = (x_i + x_k + x_j) y_i y_k y_j W_ik W_kj W_ij,
    // so the sum is W_ij y_i y_j ((x_i + x_j) (Phi Y Phi)_ij + (Phi Phi)_ij).
    // The dropped terms are O(|F|^3) relative.  Z -> A.
#pragma unroll
    for (int e0 = 0; e0 < N * N; e0 += NT) {
        const int e = e0 + lane;
        if (e >= N * N) break;
        const int i = e / N, j = e % N;
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double pp = T[i * LDP + k] * T[k * LDP + j];
            s1 = fma(pp, cs[k], s1);
            s2 += pp;
        }
        const double yy = cs[i] * cs[j];
        const double w = Out[i * LDP + j];
        double z = yy * (w * fma(wbuf[i] + wbuf[j], s1, s2) - T[i * LDP + j]);
        if (i == j) z += cs[i];
        A[i * LDP + j] = z;
    }
    lsync<NT>();
    // Out = E Z E^T
    wmm<N, NT>(T, E, A);
#pragma unroll
    for (int e0 = 0; e0 < N * N; e0 += NT) {
        const int e = e0 + lane;
        if (e >= N * N) break;
        const int i = e / N, j = e % N;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) s = fma(T[i * LDP + k], E[j * LDP + k], s);
        Out[i * LDP + j] = s;
    }
    lsync<NT>();
    return ok;
}

// The r x r algebra of one FixedRankOptStep (Alg. 2) in its one-pass form
// (Sec. 4.1, eqs. (7), (8)), from the Grams G_P = P^T P, G_Q = Q^T Q of the
// products P = X V_0, Q = X^T P and the previous SPD factor B_0:
//   C1 = (B_0 G_P B_0)^{-1/2}            U = P B_0 C1
//   K  = B_0 C1 B_0, C2 = (K G_Q K)^{-1/2}  V = Q K C2
//   B  = Sym(C1 B_0 G_Q K C2)             a_i = P_i (B_0 C1 B)
// Matrices are R x R in LDS with an identity block on the padded indices.
// On entry Gp, Gq, Bm (= B_0), Ev, Ev2 (warm-start eigenbases); on exit
// T1 = B_0 C1 (U transform), Km = B_0 C1 B (row factor transform),
// Gp = K C2 (V transform), T2 = B, and Ev, Ev2 updated.  Returns false if a
// Gram is not positive definite (rank loss, eq. (7)).  tau: the Jacobi stop
// of the two inverse square roots (winv_sqrt).
template <int R, int NT>
__device__ inline bool lstep_algebra(double* Gp, double* Gq, double* Bm, double* C1, double* C2, double* Km,
                                     double* T1, double* T2, double* Ev, double* Ev2, double* cs, double* wbuf,
                                     int r, double tau)
{
    // U-step: C1 = (B0 G_P B0)^{-1/2}
    wmm<R, NT>(T1, Bm, Gp);
    wmm<R, NT>(T2, T1, Bm);
    wsym<R, NT>(T2);
    const bool ok1 = winv_sqrt<R, NT>(C1, T2, Ev, T1, r, cs, wbuf, tau);
    // V-step: K = B0 C1 B0, C2 = (K G_Q K)^{-1/2}
    wmm<R, NT>(T1, Bm, C1);          // T1 = B0 C1  (the U transform)
    wmm<R, NT>(Km, T1, Bm);
    wsym<R, NT>(Km);
    wmm<R, NT>(T2, Km, Gq);
    wmm<R, NT>(C2, T2, Km);          // K G_Q K (C2 as scratch)
    wsym<R, NT>(C2);
    wcopy<R, NT>(T2, C2);
    const bool ok2 = winv_sqrt<R, NT>(C2, T2, Ev2, Gp, r, cs, wbuf, tau);   // Gp free now
    if (!ok1 || !ok2) return false;
    // TV = K C2 -> Gp ; B = Sym(C1 B0 G_Q K C2) -> T2 ; TU = B0 C1 B -> Km
    wmm<R, NT>(Gp, Km, C2);               // TV
    wmm<R, NT>(T2, C1, Bm);               // C1 B0
    wmm<R, NT>(C2, T2, Gq);               // C1 B0 G_Q
    wmm<R, NT>(T2, C2, Gp);               // C1 B0 G_Q K C2
    wsym<R, NT>(T2);                      // new B
    wmm<R, NT>(Km, T1, T2);               // TU
    return true;
}

// Smallest eigenvalue of the leading r x r block of B (row pitch ldb), by NT
// threads; A, Ev: LDS scratch R x LDP, cs: 2 * 16.  Full Jacobi convergence
// from the identity basis.
template <int R, int NT = 64>
__device__ inline double wmin_eig(const double* B, int ldb, int r, double* A, double* Ev, double* cs)
{
    const int lane = lid<NT>();
    for (int e = lane; e < R * R; e += NT) {
        const int i = e / R, j = e % R;
        const bool pad = (i >= r) || (j >= r);
        A[i * LDP + j] = pad ? (i == j ? 1.0 : 0.0) : B[i * ldb + j];
        Ev[i * LDP + j] = (i == j) ? 1.0 : 0.0;
    }
    lsync<NT>();
    wjacobi<R, NT>(A, Ev, cs);
    double w = INFINITY;
    for (int i = 0; i < r; ++i) w = fmin(w, A[i * LDP + i]);
    return w;
}

}  // namespace sfr
