/*
 * sfr_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, slow, FP64 CPU reference of the sparse fixed-rank (S-FR)
 * decomposition of Ros et al., "Fast and Robust Fixed-Rank Matrix Recovery":
 *
 *   FR-ADM            Alg. 1 (augmented Lagrangian of eq. (4), ADM with
 *                     continuation of the penalty mu)
 *   FixedRankOptStep  Alg. 2 (one alternating pass over St x SPD x St,
 *                     projectors of eq. (7) and eq. (8))
 *   FR-Nys            Alg. 3 (row shuffle, two sub-solves, Nystrom combine)
 *   FixedRankOptFull  Alg. 4 (Appendix; repeated Alg. 2 on a fixed matrix)
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this library.  It shares no code, header, table or helper with the
 * HIP library: every routine here is written from the paper's definitions,
 * in the paper's order, with no blocking or fusion.  Built with
 * -O2 -ffp-contract=off: round-to-nearest FP64, fixed loop order, one thread.
 *
 * Readings of the paper taken here (each is also listed in the design notes):
 *  - lambda: the S-step threshold is lambda/mu_k, i.e. eq. (4) with
 *    lambda*||S||_1; lambda = 1 is the literal Alg. 1.
 *  - V_0 = I_{n x r} (the first r columns of I_n); Alg. 1 prints I_{r x n},
 *    which contradicts V in St_{n,r} of Alg. 2.
 *  - "not converged": res_k = ||M - L_{k+1} - S_{k+1}||_F / ||M||_F <= tol,
 *    tested after the dual update, or k = max_iter.
 *  - The "M" inside Alg. 2 is the L-step input X = M - S_k + Y_k/mu_k.
 *  - P_O is the thin-SVD form of eq. (7) (Q S^T), computed by one-sided
 *    (Hestenes) Jacobi; a singular value below r*eps*sigma_max means
 *    rank < r and P_O is not unique: reported as ORC_RANK.
 *  - FR-Nys: the intersection block pseudo-inverse is pinv(L_L[1:l,1:l])
 *    truncated at rank r; the shuffle permutation is an input.
 *
 * Storage: every matrix is dense row-major double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#define ORC_OK 0
#define ORC_RANK 1      /* P_O undefined: rank(A) < r (eq. (7) needs rank r) */
#define ORC_MAXITER 2   /* stopped by max_iter, outputs valid */
#define ORC_EARG (-1)
#define ORC_ENOMEM (-2)

/* ------------------------------------------------------------------ */
/* Elementwise operators of the notation section                       */
/* ------------------------------------------------------------------ */

/* Soft threshold P_ST[x] = max(0, x - t) + min(0, x + t)  (notation, Sec. 2). */
static double soft(double x, double t)
{
    double a = x - t;
    double b = x + t;
    return (a > 0.0 ? a : 0.0) + (b < 0.0 ? b : 0.0);
}

void orc_soft_threshold(const double* x, int64_t count, double t, double* y)
{
    for (int64_t i = 0; i < count; ++i) y[i] = soft(x[i], t);
}

/* Sym(A) = (A + A^T)/2 of a k x k matrix  (notation, Sec. 2). */
void orc_sym(const double* A, int64_t k, double* out)
{
    for (int64_t i = 0; i < k; ++i)
        for (int64_t j = 0; j < k; ++j) out[i * k + j] = 0.5 * (A[i * k + j] + A[j * k + i]);
}

/* ------------------------------------------------------------------ */
/* Dense products (plain triple loops)                                 */
/* ------------------------------------------------------------------ */

/* C (a x c) = A (a x b) * B (b x c) */
static void mm(const double* A, const double* B, double* C, int64_t a, int64_t b, int64_t c)
{
    for (int64_t i = 0; i < a; ++i) {
        double* Ci = C + i * c;
        for (int64_t j = 0; j < c; ++j) Ci[j] = 0.0;
        for (int64_t k = 0; k < b; ++k) {
            double aik = A[i * b + k];
            const double* Bk = B + k * c;
            for (int64_t j = 0; j < c; ++j) Ci[j] += aik * Bk[j];
        }
    }
}

/* C (b x c) = A^T * B with A (a x b), B (a x c) */
static void mtm(const double* A, const double* B, double* C, int64_t a, int64_t b, int64_t c)
{
    for (int64_t i = 0; i < b * c; ++i) C[i] = 0.0;
    for (int64_t k = 0; k < a; ++k) {
        const double* Ak = A + k * b;
        const double* Bk = B + k * c;
        for (int64_t i = 0; i < b; ++i) {
            double aki = Ak[i];
            double* Ci = C + i * c;
            for (int64_t j = 0; j < c; ++j) Ci[j] += aki * Bk[j];
        }
    }
}

/* C (a x c) = A (a x b) * B^T with B (c x b) */
static void mmt(const double* A, const double* B, double* C, int64_t a, int64_t b, int64_t c)
{
    for (int64_t i = 0; i < a; ++i)
        for (int64_t j = 0; j < c; ++j) {
            double s = 0.0;
            for (int64_t k = 0; k < b; ++k) s += A[i * b + k] * B[j * b + k];
            C[i * c + j] = s;
        }
}

static double frob2(const double* A, int64_t count)
{
    double s = 0.0;
    for (int64_t i = 0; i < count; ++i) s += A[i] * A[i];
    return s;
}

/* ------------------------------------------------------------------ */
/* Thin SVD by one-sided (Hestenes) Jacobi                             */
/* ------------------------------------------------------------------ */

/*
 * A (m x k, m >= k) = W diag(sig) Z^T with W in St_{m,k}, Z in O_k.
 * Pairs of columns of a working copy are rotated until every pair is
 * orthogonal to working precision; Z accumulates the rotations; then
 * sig_j = ||column j|| and W_j = column j / sig_j (zero column -> W_j = 0).
 * Singular values come out unsorted.  Returns the number of sweeps, or -1
 * if 80 sweeps did not converge.
 */
int orc_svd_jacobi(const double* A, int64_t m, int64_t k, double* W, double* sig, double* Z)
{
    double* G = (double*)malloc(sizeof(double) * (size_t)(m * k));
    if (!G) return -2;
    memcpy(G, A, sizeof(double) * (size_t)(m * k));
    for (int64_t i = 0; i < k; ++i)
        for (int64_t j = 0; j < k; ++j) Z[i * k + j] = (i == j) ? 1.0 : 0.0;
    int sweeps = 0, converged = 0;
    while (sweeps < 80 && !converged) {
        converged = 1;
        ++sweeps;
        for (int64_t p = 0; p + 1 < k; ++p) {
            for (int64_t q = p + 1; q < k; ++q) {
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int64_t i = 0; i < m; ++i) {
                    double gp = G[i * k + p], gq = G[i * k + q];
                    alpha += gp * gp;
                    beta += gq * gq;
                    gamma += gp * gq;
                }
                if (gamma == 0.0 || fabs(gamma) <= DBL_EPSILON * sqrt(alpha * beta)) continue;
                converged = 0;
                /* rotation that makes the new columns p, q orthogonal:
                   t solves t^2 + 2 zeta t - 1 = 0, smaller root */
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = c * t;
                for (int64_t i = 0; i < m; ++i) {
                    double gp = G[i * k + p], gq = G[i * k + q];
                    G[i * k + p] = c * gp - s * gq;
                    G[i * k + q] = s * gp + c * gq;
                }
                for (int64_t i = 0; i < k; ++i) {
                    double zp = Z[i * k + p], zq = Z[i * k + q];
                    Z[i * k + p] = c * zp - s * zq;
                    Z[i * k + q] = s * zp + c * zq;
                }
            }
        }
    }
    for (int64_t j = 0; j < k; ++j) {
        double s2 = 0.0;
        for (int64_t i = 0; i < m; ++i) s2 += G[i * k + j] * G[i * k + j];
        double s = sqrt(s2);
        sig[j] = s;
        for (int64_t i = 0; i < m; ++i) W[i * k + j] = (s > 0.0) ? G[i * k + j] / s : 0.0;
    }
    free(G);
    return converged ? sweeps : -1;
}

/*
 * Stiefel projector of eq. (7): P_O[A] = W Z^T from the thin SVD
 * A = W Sigma Z^T (A is m x k, m >= k).  Returns ORC_RANK when
 * sigma_min <= k * eps * sigma_max, where the projector is not unique.
 */
int orc_polar(const double* A, int64_t m, int64_t k, double* out)
{
    if (m < k || k < 1) return ORC_EARG;
    double* W = (double*)malloc(sizeof(double) * (size_t)(m * k));
    double* Z = (double*)malloc(sizeof(double) * (size_t)(k * k));
    double* sig = (double*)malloc(sizeof(double) * (size_t)k);
    if (!W || !Z || !sig) { free(W); free(Z); free(sig); return ORC_ENOMEM; }
    int sw = orc_svd_jacobi(A, m, k, W, sig, Z);
    int rc = ORC_OK;
    double smax = 0.0, smin = INFINITY;
    for (int64_t j = 0; j < k; ++j) {
        if (sig[j] > smax) smax = sig[j];
        if (sig[j] < smin) smin = sig[j];
    }
    if (sw < 0 || !(smax > 0.0) || smin <= (double)k * DBL_EPSILON * smax) rc = ORC_RANK;
    mmt(W, Z, out, m, k, k); /* W (m x k) * Z^T */
    free(W); free(Z); free(sig);
    return rc;
}

/* ------------------------------------------------------------------ */
/* FixedRankOptStep (Alg. 2)                                           */
/* ------------------------------------------------------------------ */

/*
 * One alternating pass on X (m x n) from (B0, V0); U0 is not read by the
 * algorithm (its first line only uses V0 and B0):
 *   U = P_O[X V0 B0]          (U-step, eq. (7))
 *   V = P_O[X^T U B0]         (V-step, eq. (7) transposed, with the new U)
 *   B = Sym(U^T X V)          (SPD step, eq. (8))
 * U (m x r), B (r x r), V (n x r) are outputs; B0, V0 are read first, so
 * B/V may alias B0/V0.
 */
int orc_fr_step(const double* X, int64_t m, int64_t n, int64_t r,
                const double* B0, const double* V0, double* U, double* B, double* V)
{
    if (r < 1 || r > m || r > n) return ORC_EARG;
    double* XV = (double*)malloc(sizeof(double) * (size_t)(m * r));
    double* XtU = (double*)malloc(sizeof(double) * (size_t)(n * r));
    double* T = (double*)malloc(sizeof(double) * (size_t)((m > n ? m : n) * r));
    double* Bc = (double*)malloc(sizeof(double) * (size_t)(r * r));
    double* C = (double*)malloc(sizeof(double) * (size_t)(r * r));
    if (!XV || !XtU || !T || !Bc || !C) { free(XV); free(XtU); free(T); free(Bc); free(C); return ORC_ENOMEM; }
    memcpy(Bc, B0, sizeof(double) * (size_t)(r * r));
    int rc = ORC_OK, rc2;

    /* U-step: A = (X V0) B0 */
    mm(X, V0, XV, m, n, r);
    mm(XV, Bc, T, m, r, r);
    rc2 = orc_polar(T, m, r, U);
    if (rc2 != ORC_OK) rc = rc2;

    /* V-step: A = (X^T U) B0 */
    mtm(X, U, XtU, m, n, r);
    mm(XtU, Bc, T, n, r, r);
    rc2 = orc_polar(T, n, r, V);
    if (rc2 != ORC_OK && rc == ORC_OK) rc = rc2;

    /* SPD step: B = Sym(U^T X V) */
    mm(X, V, XV, m, n, r);
    mtm(U, XV, C, m, r, r);
    orc_sym(C, r, B);

    free(XV); free(XtU); free(T); free(Bc); free(C);
    return rc;
}

/* FixedRankOptFull (Alg. 4): `iters` repetitions of Alg. 2 on a fixed X,
   starting from (B, V) and overwriting (U, B, V). */
int orc_fr_full(const double* X, int64_t m, int64_t n, int64_t r, int32_t iters,
                double* U, double* B, double* V)
{
    int rc = ORC_OK;
    for (int32_t i = 0; i < iters; ++i) {
        rc = orc_fr_step(X, m, n, r, B, V, U, B, V);
        if (rc < 0) return rc;
    }
    return rc;
}

/* ------------------------------------------------------------------ */
/* FR-ADM (Alg. 1)                                                     */
/* ------------------------------------------------------------------ */

/* Initial state of Alg. 1: S = Y = 0, U0 = I_{m x r}, B0 = I_r,
   V0 = I_{n x r}. */
void orc_fradm_init(int64_t m, int64_t n, int64_t r, double* S, double* Y,
                    double* U, double* B, double* V)
{
    if (S) memset(S, 0, sizeof(double) * (size_t)(m * n));
    if (Y) memset(Y, 0, sizeof(double) * (size_t)(m * n));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < r; ++j) U[i * r + j] = (i == j) ? 1.0 : 0.0;
    for (int64_t i = 0; i < r; ++i)
        for (int64_t j = 0; j < r; ++j) B[i * r + j] = (i == j) ? 1.0 : 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < r; ++j) V[i * r + j] = (i == j) ? 1.0 : 0.0;
}

/*
 * One iteration k of Alg. 1 on the state (S_k, Y_k, U_k, B_k, V_k, mu_k):
 *   X        = M - S_k + Y_k / mu_k                       (L-step input)
 *   (U,B,V)  = FixedRankOptStep(X, U_k, B_k, V_k)          (L_{k+1} = U B V^T)
 *   S_{k+1}  = P_ST_{lambda/mu_k}(M - L_{k+1} + Y_k/mu_k)  (S-step)
 *   Y_{k+1}  = Y_k + mu_k (M - L_{k+1} - S_{k+1})          (dual step)
 *   res      = ||M - L_{k+1} - S_{k+1}||_F / nrmM
 *   mu_{k+1} = min(mu_bar, rho mu_k)                       (continuation)
 * X and L are caller scratch (m x n each); L holds L_{k+1} on return.
 */
static int fradm_iter_ws(const double* M, int64_t m, int64_t n, int64_t r, double lambda,
                         double* mu, double rho, double mu_bar, double nrmM,
                         double* S, double* Y, double* U, double* B, double* V,
                         double* X, double* L, double* res)
{
    const int64_t mn = m * n;
    const double mk = *mu;
    for (int64_t i = 0; i < mn; ++i) X[i] = M[i] - S[i] + Y[i] / mk;
    int rc = orc_fr_step(X, m, n, r, B, V, U, B, V);
    if (rc < 0) return rc;
    /* L = U B V^T */
    double* UB = (double*)malloc(sizeof(double) * (size_t)(m * r));
    if (!UB) return ORC_ENOMEM;
    mm(U, B, UB, m, r, r);
    mmt(UB, V, L, m, r, n);
    free(UB);
    const double t = lambda / mk;
    double e2 = 0.0;
    for (int64_t i = 0; i < mn; ++i) {
        double R = M[i] - L[i] + Y[i] / mk;
        S[i] = soft(R, t);
        double E = M[i] - L[i] - S[i];
        Y[i] = Y[i] + mk * E;
        e2 += E * E;
    }
    *res = sqrt(e2) / nrmM;
    double nm = rho * mk;
    *mu = (nm < mu_bar) ? nm : mu_bar;
    return rc;
}

int orc_fradm_iter(const double* M, int64_t m, int64_t n, int64_t r, double lambda,
                   double* mu, double rho, double mu_bar, double nrmM,
                   double* S, double* Y, double* U, double* B, double* V,
                   double* L, double* res)
{
    double* X = (double*)malloc(sizeof(double) * (size_t)(m * n));
    double* Lw = L ? L : (double*)malloc(sizeof(double) * (size_t)(m * n));
    if (!X || !Lw) { free(X); if (!L) free(Lw); return ORC_ENOMEM; }
    int rc = fradm_iter_ws(M, m, n, r, lambda, mu, rho, mu_bar, nrmM, S, Y, U, B, V, X, Lw, res);
    free(X);
    if (!L) free(Lw);
    return rc;
}

/*
 * Full FR-ADM solve (Alg. 1).
 *   fixed_iters > 0: run exactly that many iterations (no residual test);
 *   otherwise stop at the first k with res_k <= tol, or at k = max_iter
 *   (then ORC_MAXITER).
 * Outputs: the last iterate L = U B V^T (U m x r, B r x r, V n x r),
 * S (m x n), Y (m x n, may be NULL), iteration count, final residual and
 * (if res_hist != NULL, sized max(max_iter, fixed_iters)) every residual.
 */
int orc_fradm(const double* M, int64_t m, int64_t n, int64_t r, double lambda, double mu0,
              double rho, double mu_bar, double tol, int32_t max_iter, int32_t fixed_iters,
              double* U, double* B, double* V, double* S, double* Y,
              int32_t* iters, double* res, double* res_hist)
{
    if (m < 1 || n < 1 || r < 1 || r > m || r > n || !(lambda > 0.0) || !(mu0 > 0.0) ||
        !(rho > 0.0) || !M || !U || !B || !V || !S)
        return ORC_EARG;
    const int64_t mn = m * n;
    double* X = (double*)malloc(sizeof(double) * (size_t)mn);
    double* L = (double*)malloc(sizeof(double) * (size_t)mn);
    double* Yw = Y ? Y : (double*)malloc(sizeof(double) * (size_t)mn);
    if (!X || !L || !Yw) { free(X); free(L); if (!Y) free(Yw); return ORC_ENOMEM; }
    orc_fradm_init(m, n, r, S, Yw, U, B, V);
    const double nrmM = sqrt(frob2(M, mn));
    double mu = mu0, rk = INFINITY;
    int32_t k = 0;
    int rc = ORC_OK, status = ORC_OK;
    const int32_t limit = fixed_iters > 0 ? fixed_iters : max_iter;
    while (k < limit) {
        rc = fradm_iter_ws(M, m, n, r, lambda, &mu, rho, mu_bar, nrmM, S, Yw, U, B, V, X, L, &rk);
        ++k;
        if (res_hist) res_hist[k - 1] = rk;
        if (rc != ORC_OK) { status = rc; break; }
        if (fixed_iters <= 0 && rk <= tol) break;
    }
    if (status == ORC_OK && fixed_iters <= 0 && !(rk <= tol)) status = ORC_MAXITER;
    if (iters) *iters = k;
    if (res) *res = rk;
    free(X); free(L);
    if (!Y) free(Yw);
    return status;
}

/* ------------------------------------------------------------------ */
/* FR-Nys (Alg. 3)                                                     */
/* ------------------------------------------------------------------ */

/*
 * Rank-r pseudo-inverse of a k x k matrix W from its SVD, keeping the r
 * largest singular values: W+ = Z_r diag(1/sig_r) W_r^T.
 */
int orc_pinv_rank(const double* Wm, int64_t k, int64_t r, double* out)
{
    double* Wl = (double*)malloc(sizeof(double) * (size_t)(k * k));
    double* Z = (double*)malloc(sizeof(double) * (size_t)(k * k));
    double* sig = (double*)malloc(sizeof(double) * (size_t)k);
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
    if (!Wl || !Z || !sig || !idx) { free(Wl); free(Z); free(sig); free(idx); return ORC_ENOMEM; }
    int sw = orc_svd_jacobi(Wm, k, k, Wl, sig, Z);
    for (int64_t i = 0; i < k; ++i) idx[i] = i;
    /* order singular values, largest first (selection by simple insertion) */
    for (int64_t i = 1; i < k; ++i) {
        int64_t v = idx[i], j = i;
        while (j > 0 && sig[idx[j - 1]] < sig[v]) { idx[j] = idx[j - 1]; --j; }
        idx[j] = v;
    }
    for (int64_t i = 0; i < k * k; ++i) out[i] = 0.0;
    int rc = (sw < 0) ? ORC_RANK : ORC_OK;
    for (int64_t t = 0; t < r && t < k; ++t) {
        int64_t c = idx[t];
        if (!(sig[c] > 0.0)) { rc = ORC_RANK; continue; }
        double inv = 1.0 / sig[c];
        for (int64_t i = 0; i < k; ++i)
            for (int64_t j = 0; j < k; ++j) out[i * k + j] += Z[i * k + c] * inv * Wl[j * k + c];
    }
    free(Wl); free(Z); free(sig); free(idx);
    return rc;
}

/*
 * Alg. 3 with the shuffle given: row i of the shuffled matrix is row
 * perm[i] of M.
 *   C   = Mt[:, 0:l]  (m x l)   -> FR-ADM -> L_L = U_L B_L V_L^T
 *   Rb  = Mt[0:l, :]  (l x n)   -> FR-ADM -> L_T = U_T B_T V_T^T
 *   Wp  = pinv_r(L_L[0:l, 0:l])
 *   L   = L_L Wp L_T (shuffled row order);  S = Mt - L
 * Outputs (all optional except LL, Wp, LT): L_L (m x l), Wp (l x l),
 * L_T (l x n); dense L and S (m x n) returned in M's own row order.
 * Both sub-solves use the same (lambda, rho, mu_bar, tol, max_iter,
 * fixed_iters); mu0_left / mu0_top are their initial penalties.
 */
int orc_frnys(const double* M, int64_t m, int64_t n, int64_t r, int64_t l, const int64_t* perm,
              double lambda, double mu0_left, double mu0_top, double rho, double mu_bar,
              double tol, int32_t max_iter, int32_t fixed_iters,
              double* LL, double* Wp, double* LT, double* L, double* S,
              int32_t* iters_left, int32_t* iters_top)
{
    if (l < r || l > m || l > n || !perm || !LL || !Wp || !LT) return ORC_EARG;
    double* C = (double*)malloc(sizeof(double) * (size_t)(m * l));
    double* Rb = (double*)malloc(sizeof(double) * (size_t)(l * n));
    double* Sc = (double*)malloc(sizeof(double) * (size_t)(m * l));
    double* Sr = (double*)malloc(sizeof(double) * (size_t)(l * n));
    double* UL = (double*)malloc(sizeof(double) * (size_t)(m * r));
    double* VL = (double*)malloc(sizeof(double) * (size_t)(l * r));
    double* UT = (double*)malloc(sizeof(double) * (size_t)(l * r));
    double* VT = (double*)malloc(sizeof(double) * (size_t)(n * r));
    double* BL = (double*)malloc(sizeof(double) * (size_t)(r * r));
    double* BT = (double*)malloc(sizeof(double) * (size_t)(r * r));
    double* T = (double*)malloc(sizeof(double) * (size_t)((m > n ? m : n) * r));
    double* Wb = (double*)malloc(sizeof(double) * (size_t)(l * l));
    int rc = ORC_OK;
    if (!C || !Rb || !Sc || !Sr || !UL || !VL || !UT || !VT || !BL || !BT || !T || !Wb) { rc = ORC_ENOMEM; goto done; }
    for (int64_t i = 0; i < m; ++i) {
        int64_t src = perm[i];
        if (src < 0 || src >= m) { rc = ORC_EARG; goto done; }
        for (int64_t j = 0; j < l; ++j) C[i * l + j] = M[src * n + j];
    }
    for (int64_t i = 0; i < l; ++i)
        for (int64_t j = 0; j < n; ++j) Rb[i * n + j] = M[perm[i] * n + j];
    {
        int32_t kl = 0, kt = 0;
        double rl, rt;
        int a = orc_fradm(C, m, l, r, lambda, mu0_left, rho, mu_bar, tol, max_iter, fixed_iters,
                          UL, BL, VL, Sc, NULL, &kl, &rl, NULL);
        int b = orc_fradm(Rb, l, n, r, lambda, mu0_top, rho, mu_bar, tol, max_iter, fixed_iters,
                          UT, BT, VT, Sr, NULL, &kt, &rt, NULL);
        if (iters_left) *iters_left = kl;
        if (iters_top) *iters_top = kt;
        if (a < 0) { rc = a; goto done; }
        if (b < 0) { rc = b; goto done; }
        if (a == ORC_RANK || b == ORC_RANK) rc = ORC_RANK;
        else if (a == ORC_MAXITER || b == ORC_MAXITER) rc = ORC_MAXITER;
    }
    /* L_L = U_L B_L V_L^T (m x l), L_T = U_T B_T V_T^T (l x n) */
    mm(UL, BL, T, m, r, r);
    mmt(T, VL, LL, m, r, l);
    mm(UT, BT, T, l, r, r);
    mmt(T, VT, LT, l, r, n);
    /* intersection block and its rank-r pseudo-inverse */
    for (int64_t i = 0; i < l; ++i)
        for (int64_t j = 0; j < l; ++j) Wb[i * l + j] = LL[i * l + j];
    {
        int p = orc_pinv_rank(Wb, l, r, Wp);
        if (p < 0) { rc = p; goto done; }
        if (p == ORC_RANK) rc = ORC_RANK;
    }
    if (L || S) {
        double* LW = (double*)malloc(sizeof(double) * (size_t)(m * l));
        double* row = (double*)malloc(sizeof(double) * (size_t)n);
        if (!LW || !row) { free(LW); free(row); rc = ORC_ENOMEM; goto done; }
        mm(LL, Wp, LW, m, l, l);
        for (int64_t i = 0; i < m; ++i) {
            /* shuffled row i is original row perm[i] */
            for (int64_t j = 0; j < n; ++j) {
                double s = 0.0;
                for (int64_t t = 0; t < l; ++t) s += LW[i * l + t] * LT[t * n + j];
                row[j] = s;
            }
            int64_t dst = perm[i];
            for (int64_t j = 0; j < n; ++j) {
                if (L) L[dst * n + j] = row[j];
                if (S) S[dst * n + j] = M[dst * n + j] - row[j];
            }
        }
        free(LW); free(row);
    }
done:
    free(C); free(Rb); free(Sc); free(Sr); free(UL); free(VL); free(UT); free(VT);
    free(BL); free(BT); free(T); free(Wb);
    return rc;
}

/*
 * Same combine as orc_frnys, from already solved blocks, for matrices too
 * large to hold densely: given the two gathered blocks C (m x l) and
 * Rb (l x n), returns L_L, Wp, L_T; entries of L are then
 * L[perm[i], j] = sum_{a,b} L_L[i,a] Wp[a,b] L_T[b,j]  (orc_nys_entries).
 */
int orc_frnys_blocks(const double* C, const double* Rb, int64_t m, int64_t n, int64_t r, int64_t l,
                     double lambda, double mu0_left, double mu0_top, double rho, double mu_bar,
                     double tol, int32_t max_iter, int32_t fixed_iters,
                     double* LL, double* Wp, double* LT, int32_t* iters_left, int32_t* iters_top)
{
    if (l < r || l > m || l > n || !C || !Rb || !LL || !Wp || !LT) return ORC_EARG;
    double* Sc = (double*)malloc(sizeof(double) * (size_t)(m * l));
    double* Sr = (double*)malloc(sizeof(double) * (size_t)(l * n));
    double* UL = (double*)malloc(sizeof(double) * (size_t)(m * r));
    double* VL = (double*)malloc(sizeof(double) * (size_t)(l * r));
    double* UT = (double*)malloc(sizeof(double) * (size_t)(l * r));
    double* VT = (double*)malloc(sizeof(double) * (size_t)(n * r));
    double* BL = (double*)malloc(sizeof(double) * (size_t)(r * r));
    double* BT = (double*)malloc(sizeof(double) * (size_t)(r * r));
    double* T = (double*)malloc(sizeof(double) * (size_t)((m > n ? m : n) * r));
    double* Wb = (double*)malloc(sizeof(double) * (size_t)(l * l));
    int rc = ORC_OK;
    if (!Sc || !Sr || !UL || !VL || !UT || !VT || !BL || !BT || !T || !Wb) { rc = ORC_ENOMEM; goto done2; }
    {
        int32_t kl = 0, kt = 0;
        double rl, rt;
        int a = orc_fradm(C, m, l, r, lambda, mu0_left, rho, mu_bar, tol, max_iter, fixed_iters,
                          UL, BL, VL, Sc, NULL, &kl, &rl, NULL);
        int b = orc_fradm(Rb, l, n, r, lambda, mu0_top, rho, mu_bar, tol, max_iter, fixed_iters,
                          UT, BT, VT, Sr, NULL, &kt, &rt, NULL);
        if (iters_left) *iters_left = kl;
        if (iters_top) *iters_top = kt;
        if (a < 0) { rc = a; goto done2; }
        if (b < 0) { rc = b; goto done2; }
        if (a == ORC_RANK || b == ORC_RANK) rc = ORC_RANK;
        else if (a == ORC_MAXITER || b == ORC_MAXITER) rc = ORC_MAXITER;
    }
    mm(UL, BL, T, m, r, r);
    mmt(T, VL, LL, m, r, l);
    mm(UT, BT, T, l, r, r);
    mmt(T, VT, LT, l, r, n);
    for (int64_t i = 0; i < l; ++i)
        for (int64_t j = 0; j < l; ++j) Wb[i * l + j] = LL[i * l + j];
    {
        int p = orc_pinv_rank(Wb, l, r, Wp);
        if (p < 0) { rc = p; goto done2; }
        if (p == ORC_RANK) rc = ORC_RANK;
    }
done2:
    free(Sc); free(Sr); free(UL); free(VL); free(UT); free(VT); free(BL); free(BT); free(T); free(Wb);
    return rc;
}

/* Entries (si[t], sj[t]) of the shuffled-order Nystrom L = L_L Wp L_T. */
void orc_nys_entries(const double* LL, const double* Wp, const double* LT, int64_t n, int64_t l,
                     const int64_t* si, const int64_t* sj, int64_t count, double* out)
{
    for (int64_t t = 0; t < count; ++t) {
        const double* a = LL + si[t] * l;
        double s = 0.0;
        for (int64_t p = 0; p < l; ++p) {
            double w = 0.0;
            for (int64_t q = 0; q < l; ++q) w += Wp[p * l + q] * LT[q * n + sj[t]];
            s += a[p] * w;
        }
        out[t] = s;
    }
}
