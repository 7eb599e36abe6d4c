"""GPU parity of the large-rank engine (32 < r <= 1024, FP32): FR-ADM with
the m x n contractions as matrix-core GEMM tiles and the r x r algebra in
FP64 through Newton-Schulz inverse square roots, against the FP64 oracle.

Shapes: Table 2's regime r = 0.1 m (Sec. 5.1) at 500^2 / r = 50 and
1000^2 / r = 100, and the clustering shapes of Sec. 5.3 (16128 x 5760 r = 38,
4000 x 5760 r = 126, 3755 x 5760 r = 625) scaled down so the oracle
finishes in seconds, with a ragged tail against the 128-row and 64-column
tiles.  Bars as for every FP32 solve: L and S within 1e-5 relative Frobenius
error of the oracle at the same iteration count; U, B, V elementwise within
1e-5 ||L||_F / sigma_r(L).
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


def solve(M32, r, lam, mu, tol=1e-6, **opts):
    Mt = torch.from_numpy(M32).cuda()
    with sfr.Solver(M32.shape[0], M32.shape[1], r, lam, mu, tol, precision="f32", **opts) as s:
        U, B, V, S, info = s.solve(Mt)
    torch.cuda.synchronize()
    return U.double().cpu().numpy(), B.cpu().numpy(), V.double().cpu().numpy(), S.double().cpu().numpy(), info


def check(g, o, what):
    U, B, V, S, info = g
    L = U @ B @ V.T
    Lo = o["U"] @ o["B"] @ o["V"].T
    eL, eS = rel(L, Lo), rel(S, o["S"])
    w = np.linalg.eigvalsh(o["B"])
    bar = 1e-5 * np.linalg.norm(o["B"]) / w.min()
    eU, eV, eB = float(np.abs(U - o["U"]).max()), float(np.abs(V - o["V"]).max()), rel(B, o["B"])
    print(f"{what}: {info.iters} it, L {eL:.1e} S {eS:.1e} U {eU:.1e} V {eV:.1e} B {eB:.1e} (bar {bar:.1e}), "
          f"orth {info.orth_err:.1e}, min eig B {info.min_eig_B:.4e}")
    assert eL <= 1e-5 and eS <= 1e-5, (what, eL, eS)
    assert eU <= bar and eV <= bar and eB <= bar, (what, eU, eV, eB, bar)
    # returned factors and report
    r = B.shape[0]
    assert info.orth_err <= 1e-4
    np.testing.assert_allclose(B, B.T, atol=0)
    assert abs(info.min_eig_B - np.linalg.eigvalsh(B).min()) <= 1e-9 * np.abs(B).max()


SHAPES = [
    (500, 500, 50, 2),        # Table 2, 500^2, r = 0.1 m
    (1000, 1000, 100, 3),     # Table 2, 1000^2, r = 0.1 m
    (1613, 576, 38, 5),       # Yale-B shape 16128 x 5760 / 10, r = 38
    (1000, 1440, 126, 7),     # AR shape 4000 x 5760 / 4, r = 126
    (751, 1152, 125, 11),     # MUCT shape 3755 x 5760 / 5, r = 625 / 5
]


@pytest.mark.parametrize("m,n,r,seed", SHAPES)
def test_large_rank_fixed_iterations(m, n, r, seed):
    inst = workloads.planted(m, n, r, seed=seed, frac=0.10, kind="uniform", scale=50.0, dtype=np.float32)
    Md = inst.M.astype(np.float64)
    mu0 = workloads.default_mu0(Md)
    o = oracle.fradm(Md, r, inst.lam, mu0, fixed_iters=8)
    g = solve(inst.M, r, inst.lam, mu0, fixed_iters=8)
    assert g[4].iters == 8
    check(g, o, f"{m}x{n} r={r} 8 iterations")


def test_large_rank_tolerance_driven():
    """Tolerance-driven (tol 1e-6): the stop is within one iteration of the
    oracle's at the same tolerance, and the result matches the oracle run
    to the GPU's count."""
    m, n, r = 700, 700, 70
    inst = workloads.planted(m, n, r, seed=13, frac=0.10, kind="uniform", scale=50.0, dtype=np.float32)
    Md = inst.M.astype(np.float64)
    mu0 = workloads.default_mu0(Md)
    g = solve(inst.M, r, inst.lam, mu0, tol=1e-6)
    assert g[4].status == sfr.SFR_OK and g[4].converged
    ot = oracle.fradm(Md, r, inst.lam, mu0, tol=1e-6)
    assert abs(g[4].iters - ot["iters"]) <= 1, (g[4].iters, ot["iters"])
    o = oracle.fradm(Md, r, inst.lam, mu0, fixed_iters=g[4].iters)
    check(g, o, f"{m}x{n} r={r} tol 1e-6")
    # planted recovery in this regime (r = 0.1 m, 10 % outliers)
    L = g[0] @ g[1] @ g[2].T
    assert rel(L, inst.L0) <= 1e-4


def test_large_rank_sizes_span_tiles():
    """Both dimensions below one tile, and just above multiples of it."""
    for (m, n, r) in ((60, 50, 33), (129, 65, 40), (257, 130, 64)):
        inst = workloads.planted(m, n, r, seed=m + n, frac=0.05, kind="uniform", scale=20.0, dtype=np.float32)
        Md = inst.M.astype(np.float64)
        mu0 = workloads.default_mu0(Md)
        o = oracle.fradm(Md, r, inst.lam, mu0, fixed_iters=5)
        g = solve(inst.M, r, inst.lam, mu0, fixed_iters=5)
        U, B, V, S, info = g
        L = U @ B @ V.T
        Lo = o["U"] @ o["B"] @ o["V"].T
        print(f"{m}x{n} r={r}: L {rel(L, Lo):.1e} S {rel(S, o['S']):.1e}")
        assert rel(L, Lo) <= 1e-5 and rel(S, o["S"]) <= 1e-5


def test_large_rank_full_rank_special_case():
    """r = min(m, n): with B_0 = I the first L-step reproduces M (Lemma 1),
    so S = 0 and L = M after one iteration (the oracle's special-case pin).
    In FP32 L = M holds to the rounding of the r x r algebra times the
    conditioning of the square Gram (kappa(M)^2 ~ 4e2 here), so the residual
    test would not stop at 1e-6 there: one iteration is run."""
    rng = np.random.default_rng(8)
    M = rng.standard_normal((40, 33)).astype(np.float32)
    U, B, V, S, info = solve(M, 33, 0.1, 0.5, fixed_iters=1)
    assert info.iters == 1
    assert np.abs(S).max() == 0.0      # |M - L| stays far below the threshold lambda / mu_0
    assert rel(U @ B @ V.T, M.astype(np.float64)) <= 1e-4


def test_large_rank_tsvd_and_default_mu0():
    """Alg. 4 at r = 60 reaches numpy's rank-r truncated SVD (Eckart-Young),
    and a handle created with mu <= 0 takes mu_0 = 1.25 / ||M||_2."""
    m, n, r = 600, 500, 60
    rng = np.random.default_rng(4)
    sig = np.concatenate([np.linspace(100, 50, r), np.linspace(10, 1, min(m, n) - r)])
    Uq, _ = np.linalg.qr(rng.standard_normal((m, min(m, n))))
    Vq, _ = np.linalg.qr(rng.standard_normal((n, min(m, n))))
    M = (Uq * sig) @ Vq.T
    M32 = M.astype(np.float32)
    Mt = torch.from_numpy(M32).cuda()
    with sfr.Solver(m, n, r, 1.0, 1.0, 1e-9, precision="f32", max_iter=200) as s:
        U, B, V, info = s.tsvd(Mt)
    L = (U.double() @ B @ V.double().T).cpu().numpy()
    Md = M32.astype(np.float64)
    W, sv, Zt = np.linalg.svd(Md, full_matrices=False)
    T = (W[:, :r] * sv[:r]) @ Zt[:r]
    print(f"tsvd r={r}: {info.iters} steps, rel err vs TSVD {rel(L, T):.2e}")
    assert rel(L, T) <= 2e-6
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(B.cpu().numpy()))[::-1], sv[:r], rtol=2e-6)
    inst = workloads.planted(800, 700, 48, seed=9, frac=0.08, kind="uniform", scale=30.0, dtype=np.float32)
    Md = inst.M.astype(np.float64)
    g = solve(inst.M, 48, inst.lam, 0.0, tol=1e-6)
    exact = 1.25 / np.linalg.norm(Md, 2)
    assert abs(g[4].mu0 / exact - 1.0) <= 1e-6
    o = oracle.fradm(Md, 48, inst.lam, g[4].mu0, fixed_iters=g[4].iters)
    check(g, o, "800x700 r=48, default mu0")


def test_large_rank_rank_deficient_input():
    """rank(M) = 20 < r = 40: the first Gram is singular, so the Stiefel
    projector of eq. (7) is not unique: SFR_ERR_RANK, outputs untouched."""
    rng = np.random.default_rng(6)
    M = (rng.standard_normal((300, 20)) @ rng.standard_normal((20, 250))).astype(np.float32)
    Mt = torch.from_numpy(M).cuda()
    with sfr.Solver(300, 250, 40, 0.05, 0.01, 1e-6, precision="f32") as s:
        out = (torch.full((300, 40), 7.0, device="cuda"), torch.full((40, 40), 7.0, dtype=torch.float64, device="cuda"),
               torch.full((250, 40), 7.0, device="cuda"), torch.full((300, 250), 7.0, device="cuda"))
        info = s.solve(Mt, out=out, raise_on_error=False)[4]
    assert info.status == sfr.SFR_ERR_RANK
    for t in out:
        assert bool((t == 7.0).all())


def test_large_rank_needs_fp32_fradm():
    for kw in (dict(precision="f64"), dict(precision="f32", bf16=True),
               dict(precision="f32", nystrom_l=60, mu_left=1.0, mu_top=1.0)):
        with pytest.raises(sfr.SFRError) as e:
            sfr.Solver(2000, 1500, 40, 0.1, 1.0, 1e-6, **kw)
        assert e.value.code == sfr.SFR_ERR_ARG
