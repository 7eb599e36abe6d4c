"""GPU parity of FixedRankOptFull (Appendix, Alg. 4) -- sfr_tsvd -- through
the C ABI.

Two references:
  * the FP64 oracle's FixedRankOptFull at the same step count, from the same
    start (B_0 = I, V_0 = I_{n x r}); same tolerances as FR-ADM (FP64 1e-9,
    FP32 1e-5);
  * at convergence, the rank-r truncated SVD of M (Eckart-Young, eq. (5);
    Appendix, Theorem 2), taken from numpy's SVD.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1503_03004_amd as sfr

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-9, "f32": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    sfr.lib()
    yield


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def spectrum_matrix(m, n, sig, seed):
    """M = Q1 diag(sig) Q2^T with Haar-random orthonormal factors."""
    rng = np.random.default_rng(seed)
    k = len(sig)
    Q1, _ = np.linalg.qr(rng.standard_normal((m, k)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, k)))
    return (Q1 * np.asarray(sig)) @ Q2.T


def gpu_tsvd(M, r, precision, tol=1e-12, **opts):
    dt = torch.float64 if precision == "f64" else torch.float32
    Mt = torch.from_numpy(np.ascontiguousarray(M)).to(device="cuda", dtype=dt)
    with sfr.Solver(M.shape[0], M.shape[1], r, 1.0, 1.0, tol, precision=precision, **opts) as s:
        U, B, V, info = s.tsvd(Mt)
        torch.cuda.synchronize()
        return U.double().cpu().numpy(), B.cpu().numpy(), V.double().cpu().numpy(), info


def oracle_full(M, r, steps):
    m, n = M.shape
    U0 = np.eye(m, r)
    V0 = np.eye(n, r)
    U, B, V, rc = oracle.fr_full(M.astype(np.float64), U0, np.eye(r), V0, steps)
    assert rc >= 0
    return U, B, V


@pytest.mark.parametrize("m,n,r,precision,steps", [
    (120, 90, 4, "f64", 6),
    (257, 130, 5, "f64", 4),
    (64, 3000, 3, "f64", 5),      # wide: clusters of column slices
    (3000, 64, 6, "f64", 5),      # tall: several rows per wavefront
    (1500, 2100, 10, "f32", 6),
    (333, 5000, 8, "f32", 3),
])
def test_parity_with_oracle_fixed_steps(m, n, r, precision, steps):
    rng = np.random.default_rng(m * 7 + n)
    M = rng.standard_normal((m, n))
    if precision == "f32":
        M = M.astype(np.float32)
    U, B, V, info = gpu_tsvd(M, r, precision, fixed_iters=steps)
    assert info.iters == steps
    Uo, Bo, Vo = oracle_full(M, r, steps)
    e = rel(U @ B @ V.T, Uo @ Bo @ Vo.T)
    print(f"{m}x{n} r={r} {precision} {steps} steps: rel err L {e:.2e}")
    assert e <= TOL[precision]
    # Stiefel factors
    assert np.abs(U.T @ U - np.eye(r)).max() <= (1e-12 if precision == "f64" else 1e-5)
    assert np.abs(V.T @ V - np.eye(r)).max() <= (1e-12 if precision == "f64" else 1e-5)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tolerance_driven_reaches_the_truncated_svd(precision):
    m, n, r = 400, 300, 5
    sig = np.array([50.0, 40.0, 30.0, 20.0, 10.0, 2.0, 1.5, 1.0, 0.5])   # gap sigma_6 / sigma_5 = 0.2
    M = spectrum_matrix(m, n, sig, seed=3)
    if precision == "f32":
        M = M.astype(np.float32)
    tol = 1e-13 if precision == "f64" else 1e-7
    U, B, V, info = gpu_tsvd(M, r, precision, tol=tol, max_iter=200)
    assert info.converged and info.iters < 200, info
    W, s, Zt = np.linalg.svd(M.astype(np.float64), full_matrices=False)
    T = (W[:, :r] * s[:r]) @ Zt[:r]
    e = rel(U @ B @ V.T, T)
    print(f"{precision}: {info.iters} steps, rel change of B {info.rel_residual:.1e}, rel err vs TSVD {e:.2e}")
    assert e <= (1e-10 if precision == "f64" else 1e-5)
    # Lemma 2: B is SPD at the limit, with the r leading singular values as eigenvalues
    ev = np.sort(np.linalg.eigvalsh(B))[::-1]
    np.testing.assert_allclose(ev, s[:r], rtol=1e-10 if precision == "f64" else 1e-5)
    assert info.min_eig_B > 0


def test_full_size_8000_fp32_steps():
    """8000 x 8000, r = 10, FP32 (the FR-ADM bench shape) against the oracle
    after 3 steps, on the whole L."""
    m = n = 8000
    r = 10
    rng = np.random.default_rng(21)
    A = rng.standard_normal((m, r)).astype(np.float32)
    Bf = rng.standard_normal((n, r)).astype(np.float32)
    M = A @ Bf.T + 0.1 * rng.standard_normal((m, n)).astype(np.float32)
    U, B, V, info = gpu_tsvd(M, r, "f32", fixed_iters=3)
    assert info.iters == 3
    Uo, Bo, Vo = oracle_full(M, r, 3)
    rows = rng.choice(m, 256, replace=False)
    e = rel((U[rows] @ B) @ V.T, (Uo[rows] @ Bo) @ Vo.T)
    print(f"8000^2 r=10 f32, 3 steps: rel err L (256 rows) {e:.2e}")
    assert e <= TOL["f32"]


def test_rank_deficient_input_reports_rank_error():
    """rank(M V_0) < r: the Stiefel projector of eq. (7) is not unique."""
    m, n, r = 50, 40, 3
    M = np.outer(np.arange(1.0, m + 1), np.ones(n))     # rank 1
    Mt = torch.from_numpy(M).cuda()
    U0 = torch.full((m, r), 7.0, dtype=torch.float64, device="cuda")
    B0 = torch.full((r, r), 7.0, dtype=torch.float64, device="cuda")
    V0 = torch.full((n, r), 7.0, dtype=torch.float64, device="cuda")
    with sfr.Solver(m, n, r, 1.0, 1.0, 1e-12) as s:
        _, _, _, info = s.tsvd(Mt, out=(U0, B0, V0), raise_on_error=False)
    torch.cuda.synchronize()
    assert info.status == sfr.SFR_ERR_RANK
    # outputs untouched on error
    assert bool((U0 == 7.0).all()) and bool((B0 == 7.0).all()) and bool((V0 == 7.0).all())


def test_nonfinite_input():
    M = np.random.default_rng(5).standard_normal((60, 40))
    M[3, 7] = np.nan
    Mt = torch.from_numpy(M).cuda()
    with sfr.Solver(60, 40, 2, 1.0, 1.0, 1e-12) as s:
        _, _, _, info = s.tsvd(Mt, raise_on_error=False)
    assert info.status == sfr.SFR_ERR_NONFINITE


def test_handle_serves_solve_and_tsvd():
    """The same handle runs FR-ADM and Alg. 4 in turn with unchanged results."""
    rng = np.random.default_rng(9)
    m, n, r = 200, 150, 4
    M = rng.standard_normal((m, n))
    Mt = torch.from_numpy(M).cuda()
    with sfr.Solver(m, n, r, 0.05, 0.01, 1e-12, fixed_iters=4) as s:
        U1, B1, V1, _ = s.tsvd(Mt)
        L1 = (U1 @ B1 @ V1.T).cpu().numpy()
        s.solve(Mt)
        U2, B2, V2, _ = s.tsvd(Mt)
        L2 = (U2 @ B2 @ V2.T).cpu().numpy()
    assert np.array_equal(L1, L2)
