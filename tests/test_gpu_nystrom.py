"""GPU parity of FR-Nys (Alg. 3) against the FP64 oracle through the C ABI.

Both sides take the same row shuffle (drawn by workloads.row_permutation),
the same sub-solve penalties and the same iteration counts.  Tolerances as
for FR-ADM: 1e-9 in FP64, 1e-5 in FP32 (relative Frobenius error of L and
S; the combination adds an r x r FP64 solve and one SVD).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
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


def mus(M, perm, l):
    Mt = M[perm]
    return workloads.default_mu0(Mt[:, :l]), workloads.default_mu0(Mt[:l, :])


def gpu_nys(M, r, l, perm, lam, mu_l, mu_t, precision, **opts):
    dt = torch.float64 if precision == "f64" else torch.float32
    Mt = torch.from_numpy(np.ascontiguousarray(M)).to(device="cuda", dtype=dt)
    with sfr.Solver(M.shape[0], M.shape[1], r, lam, 1.0, opts.pop("tol", 1e-7), precision=precision,
                    nystrom_l=l, mu_left=mu_l, mu_top=mu_t, **opts) as s:
        U, B, V, S, info = s.solve_nys(Mt, perm)
        torch.cuda.synchronize()
        return dict(U=U.double().cpu().numpy(), B=B.cpu().numpy(), V=V.double().cpu().numpy(),
                    S=S.double().cpu().numpy(), info=info)


@pytest.mark.parametrize("m,n,r,l,precision,spass", [
    (600, 500, 5, 40, "f64", "mfma"),
    (2000, 1500, 10, 40, "f32", "mfma"),
    (2000, 1500, 10, 40, "f32", "vector"),   # the dense S = M - L pass on the vector ALU
    (900, 1300, 4, 30, "f32", "mfma"),     # l not a multiple of the vector width
    (300, 2600, 6, 24, "f32", "mfma"),     # wide top block: clusters of column slices
    (1100, 1300, 20, 80, "f32", "mfma"),   # the r = 20 bucket of the dense S pass on the matrix cores
    (1100, 1300, 20, 80, "f32", "vector"),
])
def test_nystrom_parity(monkeypatch, m, n, r, l, precision, spass):
    monkeypatch.setenv("SFR_SPASS", spass)
    inst = workloads.planted(m, n, r, seed=m + n, frac=0.07, kind="laplace", scale=20.0)
    M = inst.M.astype(np.float64 if precision == "f64" else np.float32)
    Md = M.astype(np.float64)
    perm = workloads.row_permutation(m, seed=7)
    mu_l, mu_t = mus(Md, perm, l)
    o = oracle.frnys(Md, r, l, perm, inst.lam, mu_l, mu_t, fixed_iters=12)
    g = gpu_nys(M, r, l, perm, inst.lam, mu_l, mu_t, precision, fixed_iters=12)
    assert g["info"].iters == 12 and g["info"].iters_top == 12
    Lg = g["U"] @ g["B"] @ g["V"].T
    eL, eS = rel(Lg, o["L"]), rel(g["S"], o["S"])
    print(f"nys {m}x{n} r{r} l{l} {precision}: errL {eL:.2e} errS {eS:.2e}")
    assert eL <= TOL[precision] and eS <= TOL[precision], (eL, eS)
    # returned factors are in St x SPD x St with B diagonal
    tol_o = 1e-12 if precision == "f64" else 1e-5
    np.testing.assert_allclose(g["U"].T @ g["U"], np.eye(r), atol=tol_o)
    np.testing.assert_allclose(g["V"].T @ g["V"], np.eye(r), atol=tol_o)
    assert np.all(np.diag(g["B"]) > 0) and np.count_nonzero(g["B"] - np.diag(np.diag(g["B"]))) == 0


def test_nystrom_tolerance_driven_fp64():
    inst = workloads.planted(800, 700, 4, seed=3, frac=0.05, kind="uniform", scale=30.0)
    perm = workloads.row_permutation(800, seed=1)
    l = 80   # this instance is recovered from l = 80 sampled rows/columns (not from l = 32)
    mu_l, mu_t = mus(inst.M, perm, l)
    o = oracle.frnys(inst.M, 4, l, perm, inst.lam, mu_l, mu_t, tol=1e-7)
    g = gpu_nys(inst.M, 4, l, perm, inst.lam, mu_l, mu_t, "f64", tol=1e-7)
    assert (g["info"].iters, g["info"].iters_top) == (o["iters_left"], o["iters_top"])
    assert rel(g["U"] @ g["B"] @ g["V"].T, o["L"]) <= 1e-9
    assert rel(g["S"], o["S"]) <= 1e-9
    assert rel(g["U"] @ g["B"] @ g["V"].T, inst.L0) <= 1e-5


def test_nystrom_exact_without_outliers():
    rng = np.random.default_rng(4)
    M = rng.standard_normal((500, 6)) @ rng.standard_normal((6, 400))
    perm = workloads.row_permutation(500, seed=2)
    g = gpu_nys(M, 6, 24, perm, 0.05, 0.1, 0.1, "f64", tol=1e-12)
    assert g["info"].iters == 1 and g["info"].iters_top == 1
    assert rel(g["U"] @ g["B"] @ g["V"].T, M) <= 1e-12
    assert np.abs(g["S"]).max() <= 1e-10


def test_nystrom_argument_errors():
    M = torch.zeros((50, 40), dtype=torch.float64, device="cuda")
    with sfr.Solver(50, 40, 2, 0.1, 1.0, 1e-7, precision="f64", nystrom_l=8, mu_left=0.1, mu_top=0.1) as s:
        bad = np.arange(50); bad[3] = 4
        with pytest.raises(sfr.SFRError) as e:
            s.solve_nys(M, bad)
        assert e.value.code == sfr.SFR_ERR_ARG
        with pytest.raises(sfr.SFRError) as e:
            s.solve(M)
        assert e.value.code == sfr.SFR_ERR_HANDLE
    with sfr.Solver(50, 40, 2, 0.1, 1.0, 1e-7, precision="f64") as s:
        with pytest.raises(sfr.SFRError) as e:
            s.solve_nys(M, np.arange(50))
        assert e.value.code == sfr.SFR_ERR_HANDLE


@pytest.mark.parametrize("block", ["top", "left"])
def test_nystrom_sub_solve_error_reported(block):
    """An error in either sub-solve (they run concurrently, the l x n one on
    a second stream) is returned, and the outputs are left untouched.  With
    V_0 = I_{n x r}, zero columns 0..r-1 in a block make X V_0 rank-deficient
    (SFR_ERR_RANK): rows perm[:l] of M for the l x n block; every row of M
    for the m x l block, whose columns 0..l-1 are M's."""
    rng = np.random.default_rng(12)
    m, n, r, l = 300, 200, 3, 12
    M = rng.standard_normal((m, n))
    perm = workloads.row_permutation(m, seed=2)
    if block == "top":
        M[perm[:l], :r] = 0.0
    else:
        M[:, :r] = 0.0
    Mt = torch.from_numpy(M).cuda()
    U = torch.full((m, r), 7.0, dtype=torch.float64, device="cuda")
    V = torch.full((n, r), 7.0, dtype=torch.float64, device="cuda")
    B = torch.full((r, r), 7.0, dtype=torch.float64, device="cuda")
    S = torch.full((m, n), 7.0, dtype=torch.float64, device="cuda")
    with sfr.Solver(m, n, r, 0.1, 1.0, 1e-7, precision="f64", nystrom_l=l, mu_left=0.1, mu_top=0.1) as s:
        out = s.solve_nys(Mt, perm, out=(U, B, V, S), raise_on_error=False)
        torch.cuda.synchronize()
    assert out[4].status == sfr.SFR_ERR_RANK, out[4].status
    for t in (U, V, B, S):
        assert bool((t == 7.0).all())


def test_nystrom_full_size_40000():
    """The 40000 x 40000, r = 20, l = 80 FP32 workload, drawn on the device:
    the oracle solves the two gathered blocks in FP64 and evaluates 20000
    sampled entries of S one by one."""
    m = n = 40000
    r, l, iters = 20, 80, 25
    M, A, B, lam = workloads.nystrom_large_device(seed=0)
    assert bool(torch.isfinite(M).all())
    perm = workloads.row_permutation(m, seed=11)
    pt = torch.from_numpy(perm).cuda()
    C = M[pt, :l].double().cpu().numpy()
    Rb = M[pt[:l]].double().cpu().numpy()
    mu_l, mu_t = workloads.default_mu0(C), workloads.default_mu0(Rb)
    o = oracle.frnys_blocks(C, Rb, r, lam, mu_l, mu_t, fixed_iters=iters)
    with sfr.Solver(m, n, r, lam, 1.0, 1e-6, precision="f32", nystrom_l=l, mu_left=mu_l, mu_top=mu_t,
                    fixed_iters=iters) as s:
        U, Bc, V, S, info = s.solve_nys(M, perm)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    t = rng.integers(0, m, 20000)       # shuffled row index
    j = rng.integers(0, n, 20000)
    rows = perm[t]
    Lo = oracle.nys_entries(o["LL"], o["Wp"], o["LT"], t, j)
    rows_t = torch.from_numpy(rows).cuda(); j_t = torch.from_numpy(j).cuda()
    Mv = M[rows_t, j_t].double().cpu().numpy()
    Sg = S[rows_t, j_t].double().cpu().numpy()
    Lg = ((U[rows_t].double() @ Bc) * V[j_t].double()).sum(1).cpu().numpy()
    So = Mv - Lo
    eL, eS = rel(Lg, Lo), rel(Sg, So)
    L0 = (A[rows_t].double() * B[j_t].double()).sum(1).cpu().numpy()
    print(f"nystrom 40000^2: errL {eL:.2e} errS {eS:.2e} recovery {rel(Lg, L0):.2e}")
    assert eL <= 1e-5 and eS <= 1e-5
