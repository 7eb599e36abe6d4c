"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check is a closed form,
a library routine for a special case, an invariant the paper proves
(Lemma 1, Lemma 2, Theorem 1, Theorem 2), brute force on tiny inputs, or a
hand-derived fixture in tests/golden/.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def orthonormal(rng, m, k):
    q, _ = np.linalg.qr(rng.standard_normal((m, k)))
    return q


# --------------------------------------------------------------------------
# Golden closed forms (hand-derived fixture)
# --------------------------------------------------------------------------

def test_golden_closed_forms():
    g = json.load(open(GOLD))
    st = g["soft_threshold"]
    np.testing.assert_array_equal(oracle.soft_threshold(np.array(st["x"]), st["t"]), np.array(st["y"]))
    sy = g["sym"]
    np.testing.assert_array_equal(oracle.sym(np.array(sy["A"])), np.array(sy["out"]))
    po = g["polar"]
    out, rc = oracle.polar(np.array(po["A"]))
    assert rc == oracle.ORC_OK
    np.testing.assert_allclose(out, np.array(po["out"]), atol=1e-15)


# --------------------------------------------------------------------------
# P1: soft threshold = proximal map of t|.|  (Sec. 2, S-step of Alg. 1)
# --------------------------------------------------------------------------

def test_soft_threshold_is_prox_bruteforce():
    rng = np.random.default_rng(0)
    x = rng.uniform(-5, 5, size=200)
    t = 0.7
    y = oracle.soft_threshold(x, t)
    grid = np.linspace(-6, 6, 240001)  # spacing 5e-5
    for xi, yi in zip(x[:40], y[:40]):
        f = 0.5 * (grid - xi) ** 2 + t * np.abs(grid)
        assert abs(grid[np.argmin(f)] - yi) <= 5e-5
    # exact closed form branches
    assert np.all(y[np.abs(x) <= t] == 0.0)
    big = np.abs(x) > t
    np.testing.assert_allclose(y[big], x[big] - t * np.sign(x[big]), rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# P2: Stiefel projector, eq. (7)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m,k,seed", [(7, 3, 0), (12, 12, 1), (40, 5, 2), (9, 1, 3)])
def test_polar_matches_lapack_svd_and_gram_form(m, k, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, k))
    out, rc = oracle.polar(A)
    assert rc == oracle.ORC_OK
    Q, s, Zt = np.linalg.svd(A, full_matrices=False)
    np.testing.assert_allclose(out, Q @ Zt, atol=1e-13)
    # second form of eq. (7): A (A^T A)^{-1/2}
    w, E = scipy.linalg.eigh(A.T @ A)
    np.testing.assert_allclose(out, A @ (E @ np.diag(w ** -0.5) @ E.T), atol=1e-11)
    # Lemma 1 ingredient: P_O[A]^T A = S Sigma S^T is SPD
    G = out.T @ A
    np.testing.assert_allclose(G, G.T, atol=1e-12)
    assert np.linalg.eigvalsh(0.5 * (G + G.T)).min() > 0


def test_polar_is_procrustes_minimizer():
    """U = P_O[M V B] minimizes ||M - U B V^T|| over St_{m,r} (eq. (7))."""
    rng = np.random.default_rng(5)
    m, n, r = 15, 11, 3
    M = rng.standard_normal((m, n))
    V = orthonormal(rng, n, r)
    B = rng.standard_normal((r, r)); B = B @ B.T + r * np.eye(r)
    U, rc = oracle.polar(M @ V @ B)
    f0 = np.linalg.norm(M - U @ B @ V.T)
    for _ in range(200):
        Up, _ = np.linalg.qr(U + 0.05 * rng.standard_normal(U.shape))
        assert np.linalg.norm(M - Up @ B @ V.T) >= f0 - 1e-12
    for _ in range(50):
        Ur = orthonormal(rng, m, r)
        assert np.linalg.norm(M - Ur @ B @ V.T) >= f0 - 1e-12


def test_polar_rank_deficient_flagged():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((8, 3))
    A[:, 2] = A[:, 0] * 2.0 - A[:, 1]
    _, rc = oracle.polar(A)
    assert rc == oracle.ORC_RANK
    _, rc = oracle.polar(np.zeros((5, 2)))
    assert rc == oracle.ORC_RANK


def test_svd_jacobi_reconstructs():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 6)) @ np.diag([1e3, 10, 1, 0.1, 1e-2, 1e-4])
    W, sig, Z, sw = oracle.svd_jacobi(A)
    assert sw > 0
    np.testing.assert_allclose(W @ np.diag(sig) @ Z.T, A, atol=1e-12)
    np.testing.assert_allclose(np.sort(sig)[::-1], np.linalg.svd(A, compute_uv=False), rtol=1e-12)
    np.testing.assert_allclose(W.T @ W, np.eye(6), atol=1e-12)
    np.testing.assert_allclose(Z.T @ Z, np.eye(6), atol=1e-14)


# --------------------------------------------------------------------------
# P3: SPD step, eq. (8): Sym(U^T X V) is the least-squares minimizer over
# symmetric B, and equals the eigenvalue-clipped projection when SPD
# --------------------------------------------------------------------------

def test_sym_is_least_squares_over_symmetric_B():
    rng = np.random.default_rng(7)
    m, n, r = 10, 9, 3
    X = rng.standard_normal((m, n))
    U = orthonormal(rng, m, r)
    V = orthonormal(rng, n, r)
    Bs = oracle.sym(U.T @ X @ V)
    # brute force: parametrise symmetric B by its upper triangle, solve the
    # linear least-squares problem min ||X - U B V^T||_F
    idx = [(i, j) for i in range(r) for j in range(i, r)]
    cols = []
    for (i, j) in idx:
        E = np.zeros((r, r)); E[i, j] = 1; E[j, i] = 1
        cols.append((U @ E @ V.T).ravel())
    coef, *_ = np.linalg.lstsq(np.stack(cols, 1), X.ravel(), rcond=None)
    Bls = np.zeros((r, r))
    for c, (i, j) in zip(coef, idx):
        Bls[i, j] = c; Bls[j, i] = c
    np.testing.assert_allclose(Bs, Bls, atol=1e-12)


def test_sym_equals_eigenvalue_clipping_when_spd():
    """Nearest SPSD matrix (Higham: clip the eigenvalues of the symmetric
    part) coincides with Sym whenever Sym is already SPD."""
    rng = np.random.default_rng(8)
    r = 5
    for _ in range(20):
        A = rng.standard_normal((r, r)) + 4 * np.eye(r)
        S = oracle.sym(A)
        w, E = np.linalg.eigh(0.5 * (A + A.T))
        clipped = E @ np.diag(np.maximum(w, 0)) @ E.T
        if w.min() > 0:
            np.testing.assert_allclose(S, clipped, atol=1e-12)


# --------------------------------------------------------------------------
# P4/P5: FixedRankOptStep invariants (Alg. 2, Lemma 1, Theorem 2 proof)
# --------------------------------------------------------------------------

def test_fr_step_invariants_and_lemma1():
    rng = np.random.default_rng(11)
    m, n, r = 40, 30, 4
    X = rng.standard_normal((m, r)) @ rng.standard_normal((r, n)) + 0.3 * rng.standard_normal((m, n))
    B0 = rng.standard_normal((r, r)); B0 = B0 @ B0.T + np.eye(r)
    V0 = orthonormal(rng, n, r)
    U, B, V, rc = oracle.fr_step(X, B0, V0)
    assert rc == oracle.ORC_OK
    np.testing.assert_allclose(U.T @ U, np.eye(r), atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(r), atol=1e-12)
    np.testing.assert_array_equal(B, B.T)
    # Lemma 1: U^T X V0 B0 and B0 U^T X V are SPD (B0 only invertible)
    for G in (U.T @ X @ V0 @ B0, B0 @ U.T @ X @ V):
        np.testing.assert_allclose(G, G.T, atol=1e-10 * np.abs(G).max())
        assert np.linalg.eigvalsh(0.5 * (G + G.T)).min() > 0
    # the individual steps are the closed forms of eq. (7) and eq. (8)
    Uq, s, Zt = np.linalg.svd(X @ V0 @ B0, full_matrices=False)
    np.testing.assert_allclose(U, Uq @ Zt, atol=1e-12)
    Vq, s, Zt = np.linalg.svd(X.T @ U @ B0, full_matrices=False)
    np.testing.assert_allclose(V, Vq @ Zt, atol=1e-12)
    C = U.T @ X @ V
    np.testing.assert_allclose(B, 0.5 * (C + C.T), atol=1e-12)


def test_fr_step_identity_B0_gives_symmetric_product():
    """With B0 = I, Lemma 1 makes U^T X V itself SPD, so Sym changes nothing."""
    rng = np.random.default_rng(12)
    m, n, r = 25, 20, 3
    X = rng.standard_normal((m, n))
    U, B, V, rc = oracle.fr_step(X, np.eye(r), orthonormal(rng, n, r))
    C = U.T @ X @ V
    np.testing.assert_allclose(C, C.T, atol=1e-12)
    np.testing.assert_allclose(B, C, atol=1e-12)
    assert np.linalg.eigvalsh(B).min() > 0


def test_fr_step_is_orthogonal_iteration():
    """Theorem 2 proof: span(U_{i+1}) = span(X X^T U_i)."""
    rng = np.random.default_rng(13)
    m, n, r = 30, 25, 4
    X = rng.standard_normal((m, n))
    U1, B1, V1, _ = oracle.fr_step(X, np.eye(r), orthonormal(rng, n, r))
    U2, B2, V2, _ = oracle.fr_step(X, B1, V1)
    Q, _ = np.linalg.qr(X @ X.T @ U1)
    np.testing.assert_allclose(U2 @ U2.T, Q @ Q.T, atol=1e-12)


def test_fr_full_converges_to_tsvd_at_theorem2_rate():
    """Alg. 4 reaches the TSVD (Eckart-Young, eq. (5)) to 1e-12; the
    subspace error contracts like (sigma_{r+1}/sigma_r)^2 per step."""
    rng = np.random.default_rng(14)
    m, n, r = 40, 30, 3
    sig = np.array([10.0, 8.0, 6.0, 3.0, 1.0, 0.5, 0.2])
    Uq = orthonormal(rng, m, sig.size); Vq = orthonormal(rng, n, sig.size)
    X = Uq @ np.diag(sig) @ Vq.T
    T = Uq[:, :r] @ np.diag(sig[:r]) @ Vq[:, :r].T
    Pstar = Uq[:, :r] @ Uq[:, :r].T
    U = np.zeros((m, r)); B = np.eye(r); V = orthonormal(rng, n, r)
    errs = []
    for i in range(60):
        U, B, V, rc = oracle.fr_full(X, U, B, V, 1)
        errs.append(np.linalg.norm(U @ U.T - Pstar, 2))
    assert rel(U @ B @ V.T, T) <= 1e-12
    ratio = (sig[r] / sig[r - 1]) ** 2  # 0.25
    seq = np.array(errs[3:14])
    rates = seq[1:] / seq[:-1]
    assert np.all(rates < ratio * 1.15), rates
    assert np.median(rates) > ratio * 0.85, rates
    # Lemma 2: B at the fixed point is SPD
    assert np.linalg.eigvalsh(B).min() > 0
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(B))[::-1], sig[:r], rtol=1e-12)


# --------------------------------------------------------------------------
# Alg. 1 per-iteration identities and invariants (P4, P7)
# --------------------------------------------------------------------------

def _np_polar(A):
    """P_O[A] of eq. (7) from LAPACK's thin SVD A = Q diag(s) Z^T: Q Z^T."""
    Q, _, Zt = np.linalg.svd(A, full_matrices=False)
    return Q @ Zt


def _np_fixed_rank_step(X, B0, V0):
    """Alg. 2 on X written with numpy: U = P_O[X V0 B0], V = P_O[X^T U B0]
    (eq. (7)), B = Sym(U^T X V) (eq. (8))."""
    U = _np_polar(X @ V0 @ B0)
    V = _np_polar(X.T @ U @ B0)
    C = U.T @ X @ V
    return U, 0.5 * (C + C.T), V


def test_fradm_iteration_identities():
    inst = workloads.plain_fp64(seed=1, m=60, n=50, r=3)
    mu0 = workloads.default_mu0(inst.M)
    st = oracle.FradmState(inst.M, inst.r, inst.lam, mu0)
    M = st.M
    for k in range(12):
        Y_old = st.Y.copy()
        S_old = st.S.copy()
        B_old = st.B.copy()
        V_old = st.V.copy()
        mu_k = st.mu.value
        res, rc = st.step()
        mk = st.mu_used
        assert rc == oracle.ORC_OK
        assert mk == mu_k
        # The L-step (Alg. 1) is FixedRankOptStep (Alg. 2) on
        # X = M - S_k + Y_k / mu_k with the previous (B_k, V_k): compare the
        # returned factors with the SVD closed forms of eqs. (7), (8).
        X = M - S_old + Y_old / mu_k
        Ue, Be, Ve = _np_fixed_rank_step(X, B_old, V_old)
        np.testing.assert_allclose(st.U, Ue, atol=1e-10)
        np.testing.assert_allclose(st.V, Ve, atol=1e-10)
        np.testing.assert_allclose(st.B, Be, atol=1e-10 * np.abs(Be).max())
        L = st.U @ st.B @ st.V.T
        np.testing.assert_allclose(L, st.L, atol=1e-12 * np.abs(L).max())
        # Stiefel factors, symmetric B, rank r
        np.testing.assert_allclose(st.U.T @ st.U, np.eye(3), atol=1e-12)
        np.testing.assert_allclose(st.V.T @ st.V, np.eye(3), atol=1e-12)
        np.testing.assert_array_equal(st.B, st.B.T)
        assert np.linalg.matrix_rank(L) == 3
        # dual bound and the clamp identity: Y_{k+1} = clip(mu_k R, -lam, lam)
        R = M - L + Y_old / mk
        assert np.abs(st.Y).max() <= inst.lam * (1 + 1e-12)
        np.testing.assert_allclose(st.Y, np.clip(mk * R, -inst.lam, inst.lam), atol=1e-12)
        # S_{k+1} = R - Y_{k+1}/mu_k ; residual = (Y_{k+1} - Y_k)/mu_k
        np.testing.assert_allclose(st.S, R - st.Y / mk, atol=1e-11)
        E = M - L - st.S
        np.testing.assert_allclose(E, (st.Y - Y_old) / mk, atol=1e-11)
        assert abs(res - np.linalg.norm(E) / np.linalg.norm(M)) <= 1e-14
        # S = P_ST(S + Y/mu_k) with the same mu (third KKT line, eq. (9))
        np.testing.assert_allclose(st.S, np.sign(R) * np.maximum(np.abs(R) - inst.lam / mk, 0), atol=1e-12)
        # continuation
        assert st.mu.value == min(1e9, 1.5 * mk)


def test_fradm_starts_from_identity_factors():
    """Alg. 1 starts from S = Y = 0, B_0 = I_r and V_0 = I_{n x r} (the
    first r columns of I_n, reading of the transposed initialisation), so
    the first L-step input is M itself and iteration 1 returns
    U = P_O[M I_{n x r}], V = P_O[M^T U], B = Sym(U^T M V) (eqs. (7), (8)).
    The identity factors are built here, independently of the oracle's own
    initialisation."""
    inst = workloads.plain_fp64(seed=4, m=40, n=30, r=4)
    mu0 = workloads.default_mu0(inst.M)
    M, r = inst.M, inst.r
    I_nr = np.eye(M.shape[1], r)
    U1 = _np_polar(M @ I_nr)
    V1 = _np_polar(M.T @ U1)
    C = U1.T @ M @ V1
    B1 = 0.5 * (C + C.T)
    one = oracle.fradm(M, r, inst.lam, mu0, fixed_iters=1)
    np.testing.assert_allclose(one["U"], U1, atol=1e-11)
    np.testing.assert_allclose(one["V"], V1, atol=1e-11)
    np.testing.assert_allclose(one["B"], B1, atol=1e-11 * np.abs(B1).max())
    # the S- and dual steps of iteration 1 with S_1 = Y_1 = 0 and mu_0
    L1 = U1 @ B1 @ V1.T
    R = M - L1
    t = inst.lam / mu0
    S1 = np.sign(R) * np.maximum(np.abs(R) - t, 0.0)
    np.testing.assert_allclose(one["S"], S1, atol=1e-11 * np.abs(M).max())
    # the stepping interface starts from the same state
    st = oracle.FradmState(M, r, inst.lam, mu0)
    np.testing.assert_array_equal(st.V, I_nr)
    np.testing.assert_array_equal(st.B, np.eye(r))
    assert not st.S.any() and not st.Y.any()


def test_fradm_kkt_at_convergence():
    """Theorem 1 / eq. (9): U^T Y ~ 0, Y V ~ 0, M ~ L + S at the stop."""
    inst = workloads.plain_fp64(seed=0)
    mu0 = workloads.default_mu0(inst.M)
    out = oracle.fradm(inst.M, inst.r, inst.lam, mu0, tol=1e-7, want_Y=True)
    assert out["rc"] == oracle.ORC_OK
    Y = out["Y"]
    L = out["U"] @ out["B"] @ out["V"].T
    assert np.linalg.norm(out["U"].T @ Y) / np.linalg.norm(Y) <= 1e-3
    assert np.linalg.norm(Y @ out["V"]) / np.linalg.norm(Y) <= 1e-3
    assert rel(L + out["S"], inst.M) <= 1e-7
    assert np.linalg.eigvalsh(out["B"]).min() > 0


# --------------------------------------------------------------------------
# P9: lambda only rescales mu (substitute Y' = Y/lam, mu' = mu/lam)
# --------------------------------------------------------------------------

def test_lambda_mu_equivalence():
    inst = workloads.plain_fp64(seed=2, m=80, n=70, r=4)
    mu0 = workloads.default_mu0(inst.M)
    lam = inst.lam
    a = oracle.fradm(inst.M, inst.r, lam, mu0, mu_bar=1e9, tol=1e-9)
    b = oracle.fradm(inst.M, inst.r, 1.0, mu0 / lam, mu_bar=1e9 / lam, tol=1e-9)
    assert a["iters"] == b["iters"]
    La = a["U"] @ a["B"] @ a["V"].T
    Lb = b["U"] @ b["B"] @ b["V"].T
    assert rel(La, Lb) <= 1e-11
    assert rel(a["S"], b["S"]) <= 1e-10


# --------------------------------------------------------------------------
# P10: special cases that reduce to exact answers
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,r", [(30, 20, 3), (20, 30, 5), (12, 12, 12)])
def test_no_outliers_exact_in_one_iteration(m, n, r):
    """S0 = 0 (or r = min(m, n)): with B0 = I, Lemma 1 makes the first
    L-step reproduce M exactly, so S = 0 and the residual is 0 after one
    iteration."""
    rng = np.random.default_rng(m * 100 + n + r)
    M = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    out = oracle.fradm(M, r, 1.0 / math.sqrt(max(m, n)), 0.3, tol=1e-12)
    assert out["iters"] == 1
    L = out["U"] @ out["B"] @ out["V"].T
    assert rel(L, M) <= 1e-13
    assert np.abs(out["S"]).max() <= 1e-12 * np.abs(M).max()


# --------------------------------------------------------------------------
# P11: Nystrom combine (Alg. 3) reproduces a rank-r L exactly; only the
# pinv-of-the-intersection-block reading does
# --------------------------------------------------------------------------

def test_nystrom_exact_on_rank_r_and_reading():
    rng = np.random.default_rng(21)
    m, n, r, l = 60, 50, 4, 12
    M = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    perm = workloads.row_permutation(m, seed=3)
    out = oracle.frnys(M, r, l, perm, 1.0 / math.sqrt(max(m, n)), 0.2, 0.2, tol=1e-12)
    assert out["rc"] == oracle.ORC_OK
    assert out["iters_left"] == 1 and out["iters_top"] == 1
    assert rel(out["L"], M) <= 1e-12
    assert np.abs(out["S"]).max() <= 1e-11 * np.abs(M).max()
    # the other reading, (L_L^+)[1:l,1:l], does not reproduce M
    Mt = M[perm]
    alt = out["LL"] @ np.linalg.pinv(out["LL"])[:l, :l] @ out["LT"]
    assert rel(alt, Mt) > 1e-2
    # rank-r pinv of the oracle matches numpy's pinv of the exact rank-r block
    W = out["LL"][:l, :l]
    np.testing.assert_allclose(out["Wp"], np.linalg.pinv(W, rcond=1e-10), atol=1e-9 * np.abs(out["Wp"]).max())
    # entry evaluation agrees with the dense product
    si = np.array([0, 5, 59]); sj = np.array([0, 7, 49])
    np.testing.assert_allclose(oracle.nys_entries(out["LL"], out["Wp"], out["LT"], si, sj),
                               (out["LL"] @ out["Wp"] @ out["LT"])[si, sj], rtol=1e-12)


def test_nystrom_blocks_matches_full():
    inst = workloads.planted(90, 70, 3, seed=4, frac=0.05, kind="uniform", scale=20.0)
    perm = workloads.row_permutation(90, seed=9)
    l = 15
    Mt = inst.M[perm]
    mu_l = workloads.default_mu0(Mt[:, :l]); mu_t = workloads.default_mu0(Mt[:l, :])
    full = oracle.frnys(inst.M, 3, l, perm, inst.lam, mu_l, mu_t, fixed_iters=15)
    blk = oracle.frnys_blocks(Mt[:, :l], Mt[:l, :], 3, inst.lam, mu_l, mu_t, fixed_iters=15)
    np.testing.assert_array_equal(full["LL"], blk["LL"])
    np.testing.assert_array_equal(full["Wp"], blk["Wp"])
    Lsh = blk["LL"] @ blk["Wp"] @ blk["LT"]
    np.testing.assert_allclose(full["L"][perm], Lsh, atol=1e-10 * np.abs(Lsh).max())
    np.testing.assert_allclose(full["S"], inst.M - full["L"], atol=1e-12)


# --------------------------------------------------------------------------
# P12: planted recovery (Sec. 5.1 set-up, 400 x 400, r = 5, FP64)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(10))
def test_planted_recovery_plain(seed):
    inst = workloads.plain_fp64(seed=seed)
    mu0 = workloads.default_mu0(inst.M)
    out = oracle.fradm(inst.M, inst.r, inst.lam, mu0, tol=1e-7, max_iter=300)
    assert out["rc"] == oracle.ORC_OK
    L = out["U"] @ out["B"] @ out["V"].T
    assert rel(L, inst.L0) <= 1e-5
    # support recovered: every planted outlier above 1e-3 is found, and off
    # the planted support S stays at rounding level
    big = np.abs(inst.S0) > 1e-3
    assert np.all(np.abs(out["S"][big]) > 1e-4)
    assert np.all(np.abs(out["S"][inst.S0 == 0]) <= 1e-4)
    assert rel(out["S"], inst.S0) <= 1e-5


# --------------------------------------------------------------------------
# P13: brute force on a tiny instance (eq. (1))
# --------------------------------------------------------------------------

def _rank1_completion(M, omega):
    """Rank-1 L agreeing with M off the support omega, or None."""
    m, n = M.shape
    rows = [i for i in range(m) if all(p[0] != i for p in omega)]
    cols = [j for j in range(n) if all(p[1] != j for p in omega)]
    i0, j0 = rows[0], cols[0]
    if abs(M[i0, j0]) < 1e-12:
        return None
    L = np.outer(M[:, j0], M[i0, :]) / M[i0, j0]
    mask = np.ones_like(M, dtype=bool)
    for p in omega:
        mask[p] = False
    if np.abs(L - M)[mask].max() > 1e-9:
        return None
    return L


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bruteforce_tiny_rank1(seed):
    """8 x 8, rank 1, two planted outliers: enumerate every support of size
    <= 2, complete the rest to rank 1, keep the feasible S of least l1 norm
    (eq. (1)); the converged FR-ADM answer must be that S."""
    n = 8
    rng = np.random.default_rng(seed)
    a = rng.uniform(1, 2, n) * rng.choice([-1, 1], n)
    b = rng.uniform(1, 2, n) * rng.choice([-1, 1], n)
    L0 = np.outer(a, b)
    S0 = np.zeros((n, n))
    S0.flat[rng.choice(n * n, 2, replace=False)] = 3.0 * rng.choice([-1, 1], 2)
    M = L0 + S0
    best = None
    cells = [(i, j) for i in range(n) for j in range(n)]
    for k in range(0, 3):
        for omega in itertools.combinations(cells, k):
            L = _rank1_completion(M, omega)
            if L is None:
                continue
            l1 = np.abs(M - L).sum()
            if best is None or l1 < best[0] - 1e-12:
                best = (l1, L)
    assert best is not None
    out = oracle.fradm(M, 1, 1.0 / math.sqrt(n), 1.25 / np.linalg.norm(M, 2), tol=1e-10, max_iter=300)
    L = out["U"] @ out["B"] @ out["V"].T
    assert np.abs(out["S"]).sum() <= best[0] + 1e-6
    assert np.abs(out["S"]).sum() <= np.abs(S0).sum() + 1e-6
    assert rel(L, best[1]) <= 1e-6
    assert np.linalg.matrix_rank(L, tol=1e-8) == 1
