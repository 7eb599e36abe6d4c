"""GPU parity of the FP64 r x r step's two paths against the FP64 oracle.

The step forms the inverse square roots of the Gram products B0 G_P B0 and
K G_Q K (eq. (7)) by Newton-Schulz on the matrix cores when their condition
number is below a bound set by the solve's precision, and by warm-started
Jacobi eigendecompositions otherwise.  The Gram products scale like B^4, so
cond(L) = sigma_1 / sigma_r of 60 puts them near 1e7, above the FP64 bound
(Jacobi path); at cond(L) = 10 (about 1e4) both precisions take the
Newton-Schulz path.  (FP32 solves at cond(L) = 60 miss the 1e-5 bar on
either path alike, about 3e-5 on L: the FP32 rounding of the m x n work,
amplified by the conditioning, not the r x r algebra.)  Ranks 20 and 32 run
the four-wavefront form of the algebra (32 x 32 blocks).

Bars: FP64 1e-9, FP32 1e-5 relative Frobenius error of L and S against the
oracle run to the GPU's own iteration count.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_1503_03004_amd as sfr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    sfr.lib()
    yield


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def graded(m, n, r, top, seed, frac=0.05, scale=20.0):
    """L0 = U diag(sigma) V^T with sigma geometric from top down to 1 (times
    sqrt(m n) / r), plus Bernoulli(frac) outliers U[-scale, scale]."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    sig = np.geomspace(top, 1.0, r) * np.sqrt(m * n) / r
    L0 = (U * sig) @ V.T
    mask = rng.random((m, n)) < frac
    S0 = np.where(mask, rng.uniform(-scale, scale, (m, n)), 0.0)
    return L0 + S0


def solve(M, r, lam, mu, precision, **kw):
    Mt = torch.from_numpy(M).cuda()
    with sfr.Solver(M.shape[0], M.shape[1], r, lam, mu, kw.pop("tol", 1e-7), precision=precision, **kw) as s:
        U, B, V, S, info = s.solve(Mt)
    torch.cuda.synchronize()
    L = (U.double() @ B @ V.double().T).cpu().numpy()
    return L, S.double().cpu().numpy(), info


@pytest.mark.parametrize("precision,top,bar", [("f64", 60.0, 1e-9), ("f64", 10.0, 1e-9), ("f32", 10.0, 1e-5)])
def test_graded_spectrum(precision, top, bar):
    m, n, r = 700, 600, 8
    Md = graded(m, n, r, top, seed=3)
    M = Md.astype(np.float64 if precision == "f64" else np.float32)
    Mo = M.astype(np.float64)
    lam = 1.0 / np.sqrt(max(m, n))
    mu0 = workloads.default_mu0(Mo)
    tol = 1e-7 if precision == "f64" else 1e-6   # FP32 residuals level off near 1e-7
    L, S, info = solve(M, r, lam, mu0, precision, tol=tol)
    assert info.status == sfr.SFR_OK and info.converged
    o = oracle.fradm(Mo, r, lam, mu0, fixed_iters=info.iters)
    eL, eS = rel(L, o["U"] @ o["B"] @ o["V"].T), rel(S, o["S"])
    print(f"{precision} cond(L) {top}: {info.iters} iterations, L {eL:.2e} S {eS:.2e}, orth {info.orth_err:.1e}")
    assert eL <= bar and eS <= bar
    # the same stop as the oracle at the same tolerance
    ot = oracle.fradm(Mo, r, lam, mu0, tol=tol)
    assert abs(info.iters - ot["iters"]) <= 1


@pytest.mark.parametrize("r", [20, 32])
def test_four_wavefront_algebra_fp64(r):
    m, n = 500, 420
    inst = workloads.planted(m, n, r, seed=r, frac=0.06, kind="uniform", scale=30.0)
    mu0 = workloads.default_mu0(inst.M)
    L, S, info = solve(inst.M, r, inst.lam, mu0, "f64", fixed_iters=12)
    assert info.iters == 12
    o = oracle.fradm(inst.M, r, inst.lam, mu0, fixed_iters=12)
    eL, eS = rel(L, o["U"] @ o["B"] @ o["V"].T), rel(S, o["S"])
    print(f"r={r} FP64: L {eL:.2e} S {eS:.2e}, orth {info.orth_err:.1e}")
    assert eL <= 1e-9 and eS <= 1e-9
    assert info.orth_err <= 1e-12


def test_graded_rank_20_fp64_jacobi_path():
    """r = 20 (four-wavefront form) with cond(L) = 40: the Gram products are
    beyond the FP64 Newton-Schulz bound, so every step takes the Jacobi path
    with the whole workgroup."""
    m, n, r = 520, 480, 20
    M = graded(m, n, r, 40.0, seed=11)
    lam = 1.0 / np.sqrt(max(m, n))
    mu0 = workloads.default_mu0(M)
    L, S, info = solve(M, r, lam, mu0, "f64", fixed_iters=10)
    o = oracle.fradm(M, r, lam, mu0, fixed_iters=10)
    eL, eS = rel(L, o["U"] @ o["B"] @ o["V"].T), rel(S, o["S"])
    print(f"r=20 cond(L) 40 FP64: L {eL:.2e} S {eS:.2e}")
    assert eL <= 1e-9 and eS <= 1e-9


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5, 7, 9, 11, 14, 16])
def test_each_rank_bucket_fp64(r):
    """Every route of the one-wavefront step against the oracle in FP64: the
    register Jacobi form (r <= 3), the LDS Jacobi form (r = 4) and the
    register Newton-Schulz form (5 <= r <= 16), including ranks below their
    bucket (7 -> 8, 9 -> 10, 11 -> 12, 14 -> 16: an identity block pads the
    16 x 16 matrices inside the bucket too)."""
    m, n = 260, 230
    Md = graded(m, n, r, 8.0, seed=40 + r)
    lam = 1.0 / np.sqrt(max(m, n))
    mu0 = workloads.default_mu0(Md)
    L, S, info = solve(Md, r, lam, mu0, "f64", fixed_iters=10)
    assert info.iters == 10
    o = oracle.fradm(Md, r, lam, mu0, fixed_iters=10)
    eL, eS = rel(L, o["U"] @ o["B"] @ o["V"].T), rel(S, o["S"])
    print(f"r={r} FP64: L {eL:.2e} S {eS:.2e}, orth {info.orth_err:.1e}")
    assert eL <= 1e-9 and eS <= 1e-9
    assert info.orth_err <= 1e-12
