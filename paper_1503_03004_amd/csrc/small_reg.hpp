// FP64 r x r algebra of one FR-ADM step for the smallest rank buckets
// (R <= 4), held in registers.  Every lane of the wavefront computes the whole
// step on its own copy of the matrices, so its phases need no LDS round trip
// and no wavefront fence; at these sizes those, not the arithmetic, set the
// time of the LDS form (small_la.hpp).  The operations are those of
// lstep_algebra / winv_sqrt / wjacobi in the same order, except that the
// Jacobi sweeps rotate the pairs (p, q) one at a time in cyclic row order
// (Golub & Van Loan, Matrix Computations, Sec. 8.5) instead of in parallel
// rounds; both converge to the same eigendecomposition up to rounding.
#pragma once

#include "small_la.hpp"

namespace sfr {

template <int R>
struct RMat {
    double v[R][R];
};

// C = A B
template <int R>
__device__ __forceinline__ RMat<R> rm_mul(const RMat<R>& A, const RMat<R>& B)
{
    RMat<R> C;
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < R; ++t) s = fma(A.v[i][t], B.v[t][j], s);
            C.v[i][j] = s;
        }
    return C;
}

// C = A^T B
template <int R>
__device__ __forceinline__ RMat<R> rm_tmul(const RMat<R>& A, const RMat<R>& B)
{
    RMat<R> C;
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < R; ++t) s = fma(A.v[t][i], B.v[t][j], s);
            C.v[i][j] = s;
        }
    return C;
}

template <int R>
__device__ __forceinline__ void rm_sym(RMat<R>& A)
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = i + 1; j < R; ++j) {
            const double s = 0.5 * (A.v[i][j] + A.v[j][i]);
            A.v[i][j] = s;
            A.v[j][i] = s;
        }
}

// A (symmetric, expressed in the basis E0 held in E) -> diag(eigenvalues);
// E -> E0 times the rotations, so that A_in = E diag E^T.  Sweeps stop as in
// wjacobi: once no off-diagonal entry is above the relative rounding test,
// or all are within tau of the smaller diagonal entry.
template <int R>
__device__ __forceinline__ void rm_jacobi(RMat<R>& A, RMat<R>& E, double tau)
{
    if constexpr (R == 1) return;
    for (int sweep = 0; sweep < 16; ++sweep) {
        bool big = false, far = false;
#pragma unroll
        for (int p = 0; p < R; ++p)
#pragma unroll
            for (int q = p + 1; q < R; ++q) {
                const double apq = A.v[p][q], app = A.v[p][p], aqq = A.v[q][q];
                if (apq != 0.0 && apq * apq > DBL_EPSILON * DBL_EPSILON * fabs(app * aqq)) big = true;
                if (!(fabs(apq) <= tau * fmin(fabs(app), fabs(aqq)))) far = true;
            }
        if (!big || !far) break;
#pragma unroll
        for (int p = 0; p < R; ++p)
#pragma unroll
            for (int q = p + 1; q < R; ++q) {
                const double apq = A.v[p][q], app = A.v[p][p], aqq = A.v[q][q];
                if (!(apq != 0.0 && apq * apq > DBL_EPSILON * DBL_EPSILON * fabs(app * aqq))) continue;
                // the smaller root t of t^2 + (d / a_pq) t - 1 = 0, d = a_qq - a_pp
                const double d = aqq - app;
                const double h = sqrt(fma(d, d, 4.0 * apq * apq));
                const double t = (d >= 0.0 ? 2.0 * apq : -2.0 * apq) / (fabs(d) + h);
                const double c = rsqrt(fma(t, t, 1.0));
                const double s = t * c;
                // columns p, q (and by symmetry rows p, q) rotated
#pragma unroll
                for (int x = 0; x < R; ++x) {
                    if (x == p || x == q) continue;
                    const double axp = A.v[x][p], axq = A.v[x][q];
                    const double np = c * axp - s * axq, nq = s * axp + c * axq;
                    A.v[x][p] = np; A.v[p][x] = np;
                    A.v[x][q] = nq; A.v[q][x] = nq;
                }
                A.v[p][p] = fma(-t, apq, app);
                A.v[q][q] = fma(t, apq, aqq);
                A.v[p][q] = 0.0;
                A.v[q][p] = 0.0;
#pragma unroll
                for (int x = 0; x < R; ++x) {
                    const double ep = E.v[x][p], eq = E.v[x][q];
                    E.v[x][p] = c * ep - s * eq;
                    E.v[x][q] = s * ep + c * eq;
                }
            }
    }
}

// Out = A^{-1/2} (A symmetric positive definite), warm-started from the
// basis E (updated), as winv_sqrt: Jacobi sweeps until A is diagonal to
// within tau in the current basis, then the second-order expansion of
// t^{-1/2} about the diagonal.  Returns false if A is not positive definite
// to working precision (nreal leading eigenvalues tested).
template <int R>
__device__ __forceinline__ bool rm_inv_sqrt(RMat<R>& Out, RMat<R> A, RMat<R>& E, int nreal, double tau)
{
    A = rm_tmul<R>(E, rm_mul<R>(A, E));
    rm_sym<R>(A);
    rm_jacobi<R>(A, E, tau);
    double wmax = -INFINITY, wmin = INFINITY;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        if (i >= nreal) break;
        wmax = fmax(wmax, A.v[i][i]);
        wmin = fmin(wmin, A.v[i][i]);
    }
    double x[R], y[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const double d = A.v[i][i];
        x[i] = d > 0.0 ? sqrt(d) : 0.0;
        y[i] = d > 0.0 ? 1.0 / x[i] : 0.0;
    }
    const bool ok = (wmax > 0.0) && (wmin > (double)nreal * DBL_EPSILON * wmax) && isfinite(wmax);
    // W_ij = 1 / (x_i + x_j), Phi = F o W (F: the off-diagonal part of A)
    RMat<R> W, Phi;
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const double den = x[i] + x[j];
            const double w = den > 0.0 ? 1.0 / den : 0.0;
            W.v[i][j] = w;
            Phi.v[i][j] = (i == j) ? 0.0 : A.v[i][j] * w;
        }
    // Z_ij = delta_ij y_i + y_i y_j (W_ij ((x_i + x_j) (Phi Y Phi)_ij + (Phi Phi)_ij) - Phi_ij)
    RMat<R> Z;
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            double s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const double pp = Phi.v[i][k] * Phi.v[k][j];
                s1 = fma(pp, y[k], s1);
                s2 += pp;
            }
            double z = (y[i] * y[j]) * (W.v[i][j] * fma(x[i] + x[j], s1, s2) - Phi.v[i][j]);
            if (i == j) z += y[i];
            Z.v[i][j] = z;
        }
    // Out = E Z E^T
    const RMat<R> T = rm_mul<R>(E, Z);
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < R; ++k) s = fma(T.v[i][k], E.v[j][k], s);
            Out.v[i][j] = s;
        }
    return ok;
}

// The r x r algebra of one FixedRankOptStep (Alg. 2) in its one-pass form
// (Sec. 4.1, eqs. (7), (8)), as lstep_algebra:
//   C1 = (B0 G_P B0)^{-1/2},  TUbar = B0 C1           (U = P TUbar)
//   K = Sym(B0 C1 B0),  C2 = (K G_Q K)^{-1/2},  TV = K C2   (V = Q TV)
//   B = Sym(C1 B0 G_Q TV),  TU = TUbar B             (a_i = P_i TU)
// E1, E2: the warm-start eigenbases of the two inverse square roots
// (updated).  Returns false on rank loss (either Gram product not positive
// definite to working precision); the outputs are then undefined.
template <int R>
__device__ __forceinline__ bool rm_lstep(const RMat<R>& Gp, const RMat<R>& Gq, const RMat<R>& B0, RMat<R>& E1,
                                         RMat<R>& E2, int r, double tau, RMat<R>& Bn, RMat<R>& TU,
                                         RMat<R>& TUbar, RMat<R>& TV)
{
    RMat<R> A1 = rm_mul<R>(rm_mul<R>(B0, Gp), B0);
    rm_sym<R>(A1);
    RMat<R> C1;
    const bool ok1 = rm_inv_sqrt<R>(C1, A1, E1, r, tau);
    TUbar = rm_mul<R>(B0, C1);
    RMat<R> K = rm_mul<R>(TUbar, B0);
    rm_sym<R>(K);
    RMat<R> A2 = rm_mul<R>(rm_mul<R>(K, Gq), K);
    rm_sym<R>(A2);
    RMat<R> C2;
    const bool ok2 = rm_inv_sqrt<R>(C2, A2, E2, r, tau);
    if (!ok1 || !ok2) return false;
    TV = rm_mul<R>(K, C2);
    Bn = rm_mul<R>(rm_mul<R>(rm_mul<R>(C1, B0), Gq), TV);
    rm_sym<R>(Bn);
    TU = rm_mul<R>(TUbar, Bn);
    return true;
}

}  // namespace sfr
