"""GPU parity of FR-ADM (Alg. 1 with the Alg. 2 L-step) against the FP64
oracle, through the C ABI (Python binding = argument marshalling only).

Tolerances (relative Frobenius error against the oracle at the same
iteration count):
  FP64: 1e-9.  The GPU forms the Stiefel projections of eq. (7) through the
        Gram inverse square root and the oracle through a Jacobi thin SVD;
        both are exact in real arithmetic, so only rounding differs
        (observed ~1e-14; the margin covers the conditioning of the r x r
        Grams, which squares kappa(X V)).
  FP32: 1e-5, the target accuracy of the FP32 solve; FP32 rounding of the
        m x n work sets a floor of a few 1e-7.
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


def gpu_solve(M, r, lam, mu0, precision, **opts):
    dt = torch.float64 if precision == "f64" else torch.float32
    Mt = torch.from_numpy(np.ascontiguousarray(M)).to(device="cuda", dtype=dt)
    with sfr.Solver(M.shape[0], M.shape[1], r, lam, mu0, opts.pop("tol", 1e-7), precision=precision,
                    **opts) as s:
        U, B, V, S, info = s.solve(Mt)
        torch.cuda.synchronize()
        return dict(U=U.double().cpu().numpy(), B=B.cpu().numpy(), V=V.double().cpu().numpy(),
                    S=S.double().cpu().numpy(), info=info)


def compare(g, o, precision, what=""):
    Lg = g["U"] @ g["B"] @ g["V"].T
    Lo = o["U"] @ o["B"] @ o["V"].T
    eL, eS = rel(Lg, Lo), rel(g["S"], o["S"])
    tol = TOL[precision]
    print(f"{what}: iters gpu {g['info'].iters} oracle {o['iters']}  errL {eL:.2e}  errS {eS:.2e}")
    assert eL <= tol, (what, eL)
    assert eS <= tol, (what, eS)
    return eL, eS


def case(inst, precision, fixed, **extra):
    M = inst.M.astype(np.float64 if precision == "f64" else np.float32)
    Md = M.astype(np.float64)
    mu0 = workloads.default_mu0(Md)
    o = oracle.fradm(Md, inst.r, inst.lam, mu0, fixed_iters=fixed, **extra)
    g = gpu_solve(M, inst.r, inst.lam, mu0, precision, fixed_iters=fixed, **extra)
    assert g["info"].iters == o["iters"]
    return g, o


# ---------------------------------------------------------------------------


def test_plain_fp64_tolerance_driven_same_stop():
    """400 x 400, r = 5, FP64 workload: the tolerance test stops at the same
    iteration as the oracle and the results agree."""
    inst = workloads.plain_fp64(seed=0)
    mu0 = workloads.default_mu0(inst.M)
    o = oracle.fradm(inst.M, inst.r, inst.lam, mu0, tol=1e-7, max_iter=300)
    g = gpu_solve(inst.M, inst.r, inst.lam, mu0, "f64", tol=1e-7, max_iter=300)
    assert g["info"].status == sfr.SFR_OK
    assert g["info"].iters == o["iters"]
    assert abs(g["info"].rel_residual - o["res"]) <= 1e-6 * o["res"] + 1e-15
    compare(g, o, "f64", "plain_fp64")
    # invariants of the returned factors (FP64)
    r = inst.r
    np.testing.assert_allclose(g["U"].T @ g["U"], np.eye(r), atol=1e-12)
    np.testing.assert_allclose(g["V"].T @ g["V"], np.eye(r), atol=1e-12)
    np.testing.assert_allclose(g["B"], g["B"].T, atol=0)
    assert np.linalg.eigvalsh(g["B"]).min() > 0
    assert abs(g["info"].min_eig_B - np.linalg.eigvalsh(g["B"]).min()) <= 1e-9 * np.abs(g["B"]).max()
    assert np.linalg.matrix_rank(g["U"] @ g["B"] @ g["V"].T) == r
    # planted recovery
    assert rel(g["U"] @ g["B"] @ g["V"].T, inst.L0) <= 1e-5


@pytest.mark.parametrize("precision,shape", [("f64", (400, 400, 5)), ("f32", (1500, 1200, 8))])
def test_default_mu0_from_spectral_norm(precision, shape):
    """A handle created with mu <= 0 takes mu_0 = 1.25 / ||M||_2, with ||M||_2
    from Alg. 4 on M: the reported mu_0 matches the exact spectral norm
    (numpy SVD), and the solve matches the oracle run with that mu_0."""
    m, n, r = shape
    if precision == "f64":
        inst = workloads.plain_fp64(seed=4)
    else:
        inst = workloads.planted(m, n, r, seed=11, frac=0.08, kind="uniform", scale=50.0, dtype=np.float32)
    Md = inst.M.astype(np.float64)
    exact = 1.25 / np.linalg.norm(Md, 2)
    g = gpu_solve(inst.M, r, inst.lam, 0.0, precision, tol=1e-6 if precision == "f32" else 1e-7)
    mu0 = g["info"].mu0
    print(f"{precision}: mu0 gpu {mu0:.12e} exact {exact:.12e} rel {abs(mu0 / exact - 1):.1e}")
    assert abs(mu0 / exact - 1.0) <= 1e-6
    o = oracle.fradm(Md, r, inst.lam, mu0, fixed_iters=g["info"].iters)
    compare(g, o, precision, f"default mu0 {precision}")


@pytest.mark.parametrize("fixed", [1, 2, 3, 8])
def test_fp64_each_sweep_mode(fixed):
    """Iteration 1 (X = M), 2 (Y_1 = 0) and the general sweep."""
    inst = workloads.plain_fp64(seed=3, m=150, n=110, r=4)
    g, o = case(inst, "f64", fixed)
    compare(g, o, "f64", f"fixed{fixed}")
    np.testing.assert_allclose(g["U"], o["U"], atol=1e-8)
    np.testing.assert_allclose(g["V"], o["V"], atol=1e-8)
    np.testing.assert_allclose(g["B"], o["B"], rtol=1e-9, atol=1e-9 * np.abs(o["B"]).max())


@pytest.mark.parametrize("m,n,r,precision", [
    (301, 203, 3, "f32"),     # ragged rows and columns
    (1037, 77, 4, "f32"),     # narrow rows: several rows per wavefront
    (257, 130, 5, "f32"),     # n not a multiple of the vector width (padded copy)
    (211, 77, 3, "f64"),      # odd n in FP64
    (600, 3000, 6, "f32"),    # wide rows: clusters of 3 column slices
    (300, 1500, 4, "f64"),    # wide rows in FP64
    (97, 2500, 12, "f32"),    # few rows, wide
    (3, 50, 2, "f64"),        # fewer rows than one band
    (200, 150, 1, "f64"),     # rank one
    (64, 64, 16, "f32"),
    (500, 64, 20, "f32"),     # r = 20 bucket
    (400, 300, 32, "f64"),    # largest supported rank
    (48, 36000, 20, "f32"),   # clusters wider than one XCD's share of the grid
    (64, 20000, 10, "f32"),   # vector sweep, 20-member clusters: exchange words gathered in batches
    (40, 8000, 10, "f64"),    # the same in FP64 (two words per value)
])
def test_shapes(m, n, r, precision):
    inst = workloads.planted(m, n, r, seed=m + n + r, frac=0.05, kind="uniform", scale=20.0,
                             dtype=np.float64)
    g, o = case(inst, precision, 10)
    compare(g, o, precision, f"{m}x{n} r{r} {precision}")


def test_fp32_large_shape_parity():
    """2000 x 2000, r = 10, 10 % outliers U[-100, 100] in FP32 (the shape of
    the 8000^2 workload at a size the oracle solves in seconds), at the
    oracle's own stopping iteration."""
    inst = workloads.large_fp32(seed=1, m=2000, n=2000, r=10)
    Md = inst.M.astype(np.float64)
    mu0 = workloads.default_mu0(Md)
    o = oracle.fradm(Md, 10, inst.lam, mu0, tol=1e-7)
    g = gpu_solve(inst.M, 10, inst.lam, mu0, "f32", fixed_iters=o["iters"])
    compare(g, o, "f32", "2000^2 r10")
    assert rel(g["U"] @ g["B"] @ g["V"].T, inst.L0.astype(np.float64)) <= 1e-5


def test_rank_equals_min_dim_exact_in_one_iteration():
    rng = np.random.default_rng(5)
    M = rng.standard_normal((40, 12))
    g = gpu_solve(M, 12, 0.1, 0.5, "f64", tol=1e-10)
    assert g["info"].iters == 1
    assert rel(g["U"] @ g["B"] @ g["V"].T, M) <= 1e-12
    assert np.abs(g["S"]).max() <= 1e-10


def test_no_outliers_exact_in_one_iteration_f32():
    rng = np.random.default_rng(6)
    M = (rng.standard_normal((500, 4)) @ rng.standard_normal((4, 300))).astype(np.float32)
    g = gpu_solve(M, 4, 0.05, 0.1, "f32", tol=1e-5)
    assert g["info"].iters == 1
    assert rel(g["U"] @ g["B"] @ g["V"].T, M.astype(np.float64)) <= 1e-6


def test_error_paths():
    rng = np.random.default_rng(7)
    M = rng.standard_normal((50, 40))
    Mn = M.copy(); Mn[3, 7] = np.nan
    g = gpu_solve_status(Mn, 3)
    assert g == sfr.SFR_ERR_NONFINITE
    Mz = M.copy(); Mz[:, :3] = 0.0   # X V_0 = 0 for V_0 = I_{n x r}: P_O undefined
    assert gpu_solve_status(Mz, 3) == sfr.SFR_ERR_RANK
    # max_iter reached
    Mt = torch.from_numpy(M).cuda()
    with sfr.Solver(50, 40, 3, 0.1, 0.05, 0.0, precision="f64", max_iter=2) as s:
        U, B, V, S, info = s.solve(Mt)
        assert info.status == sfr.SFR_WARN_MAXITER and info.iters == 2


def gpu_solve_status(M, r):
    Mt = torch.from_numpy(M).cuda()
    with sfr.Solver(M.shape[0], M.shape[1], r, 0.1, 0.05, 1e-7, precision="f64") as s:
        out = s.solve(Mt, raise_on_error=False)
        return out[4].status


def test_outputs_untouched_on_error():
    M = np.full((30, 20), np.inf)
    Mt = torch.from_numpy(M).cuda()
    with sfr.Solver(30, 20, 2, 0.1, 0.1, 1e-7, precision="f64") as s:
        U = torch.full((30, 2), 7.0, dtype=torch.float64, device="cuda")
        B = torch.full((2, 2), 7.0, dtype=torch.float64, device="cuda")
        V = torch.full((20, 2), 7.0, dtype=torch.float64, device="cuda")
        S = torch.full((30, 20), 7.0, dtype=torch.float64, device="cuda")
        out = s.solve(Mt, out=(U, B, V, S), raise_on_error=False)
        assert out[4].status == sfr.SFR_ERR_NONFINITE
        for t in (U, B, V, S):
            assert bool((t == 7.0).all())


def test_deterministic_and_handle_reuse():
    """Two solves on one handle: bitwise equal on equal input (fixed-order
    reductions, no float atomics), and a different input in between gives
    its own oracle answer (state and exchange slots are reset)."""
    a = workloads.planted(500, 3000, 5, seed=11, frac=0.08, kind="uniform", scale=30.0)
    b = workloads.planted(500, 3000, 5, seed=12, frac=0.08, kind="uniform", scale=30.0)
    mu_a = workloads.default_mu0(a.M); mu_b = workloads.default_mu0(b.M)
    Ma = torch.from_numpy(a.M.astype(np.float32)).cuda()
    Mb = torch.from_numpy(b.M.astype(np.float32)).cuda()
    with sfr.Solver(500, 3000, 5, a.lam, mu_a, 1e-7, precision="f32", fixed_iters=9) as s:
        r1 = [t.clone() for t in s.solve(Ma)[:4]]
        s.solve(Mb)
        r2 = [t.clone() for t in s.solve(Ma)[:4]]
    for x, y in zip(r1, r2):
        assert torch.equal(x, y)
    o = oracle.fradm(b.M.astype(np.float32).astype(np.float64), 5, b.lam, mu_b, fixed_iters=9)
    g = gpu_solve(b.M.astype(np.float32), 5, b.lam, mu_b, "f32", fixed_iters=9)
    compare(g, o, "f32", "reuse")


def test_full_size_8000_fp32_first_iterations():
    """The 8000 x 8000, r = 10 FP32 workload in the launch configuration the
    benchmark times: three iterations (all three sweep modes) against the
    FP64 oracle, L and S compared on every entry of 64 sampled rows."""
    inst = workloads.large_fp32(seed=0)
    Md = inst.M.astype(np.float64)
    mu0 = workloads.default_mu0(inst.M)
    o = oracle.fradm(Md, 10, inst.lam, mu0, fixed_iters=3)
    g = gpu_solve(inst.M, 10, inst.lam, mu0, "f32", fixed_iters=3)
    rows = np.random.default_rng(0).choice(8000, 64, replace=False)
    Lg = g["U"][rows] @ g["B"] @ g["V"].T
    Lo = o["U"][rows] @ o["B"] @ o["V"].T
    assert rel(Lg, Lo) <= 1e-5
    assert rel(g["S"][rows], o["S"][rows]) <= 1e-5
    assert rel(g["S"], o["S"]) <= 1e-5


def test_photometric_full_size_fp32():
    """The photometric-stereo shape of Sec. 5.2 at full size (262144 pixels x
    48 images, r = 3, FP32, Lambertian L0 with specular outliers and
    shadows): the GPU run to the oracle's own stopping iteration (tol 1e-7),
    L and S compared on every entry."""
    inst = workloads.photometric(seed=0)
    Md = inst.M.astype(np.float64)
    mu0 = workloads.default_mu0(Md)
    o = oracle.fradm(Md, 3, inst.lam, mu0, tol=1e-7)
    g = gpu_solve(inst.M, 3, inst.lam, mu0, "f32", fixed_iters=o["iters"])
    assert g["info"].iters == o["iters"]
    compare(g, o, "f32", f"photometric 262144x48 r3, {o['iters']} iterations")


def test_photometric_tolerance_driven_fp32():
    """Same shape at a quarter of the pixels, tolerance-driven on both sides:
    the GPU stops within one iteration of the oracle (the FP32 residual
    decides the stop) and matches the oracle run to the same count."""
    inst = workloads.photometric(seed=3, m=65536)
    Md = inst.M.astype(np.float64)
    mu0 = workloads.default_mu0(Md)
    g = gpu_solve(inst.M, 3, inst.lam, mu0, "f32", tol=1e-6)
    o_ref = oracle.fradm(Md, 3, inst.lam, mu0, tol=1e-6)
    assert abs(g["info"].iters - o_ref["iters"]) <= 1, (g["info"].iters, o_ref["iters"])
    o = oracle.fradm(Md, 3, inst.lam, mu0, fixed_iters=g["info"].iters)
    compare(g, o, "f32", f"photometric 65536x48 r3 tol 1e-6, {g['info'].iters} iterations")


@pytest.mark.parametrize("sweep", ["mfma", "vector"])
@pytest.mark.parametrize("m,n,r", [(300, 1100, 10), (1037, 2048, 4), (64, 5000, 12), (2100, 1024, 1),
                                   (300, 1100, 16), (700, 800, 16), (400, 2100, 13), (200, 2000, 20),
                                   (1037, 700, 24), (150, 1500, 32), (40, 30000, 20)])
def test_both_fp32_sweeps(monkeypatch, sweep, m, n, r):
    """FP32 shapes that both sweeps take: the matrix-core sweep and the vector
    sweep (SFR_SWEEP selects) each against the oracle."""
    monkeypatch.setenv("SFR_SWEEP", sweep)
    inst = workloads.planted(m, n, r, seed=m + n + r, frac=0.08, kind="uniform", scale=30.0, dtype=np.float32)
    g, o = case(inst, "f32", 4)
    compare(g, o, "f32", f"{sweep} {m}x{n} r={r}")


@pytest.mark.parametrize("m,n,r,fixed,bf16", [(300, 6200, 20, 4, False), (130, 9000, 32, 3, False),
                                              (300, 1000, 16, 5, False), (40, 30000, 24, 3, False),
                                              (300, 6200, 20, 4, True)])
def test_both_exchange_forms_bitwise(monkeypatch, m, n, r, fixed, bf16):
    """Matrix-core sweeps of the 4-tile forms with c > 1 members per cluster
    (512-column slices: c = 13, 18, 2 and 59 here, bands with a ragged
    tail): the all-gather and the reduce-then-broadcast exchange (SFR_EXCH
    selects) add the members' partial row products in the same member order,
    so the two solves agree bitwise (FP32 and BF16 operands); the FP32 ones
    match the oracle."""
    monkeypatch.setenv("SFR_SWEEP", "mfma")
    inst = workloads.planted(m, n, r, seed=m + n + r, frac=0.08, kind="uniform", scale=30.0, dtype=np.float32)
    M = inst.M.astype(np.float32)
    Md = M.astype(np.float64)
    mu0 = workloads.default_mu0(Md)
    out = {}
    for form in ("gather", "reduce"):
        monkeypatch.setenv("SFR_EXCH", form)
        out[form] = gpu_solve(M, r, inst.lam, mu0, "f32", fixed_iters=fixed, **({"bf16": True} if bf16 else {}))
        assert out[form]["info"].iters == fixed
    for key in ("U", "B", "V", "S"):
        assert np.array_equal(out["gather"][key], out["reduce"][key]), key
    if not bf16:   # BF16 operands: the two forms are compared with each other only
        o = oracle.fradm(Md, r, inst.lam, mu0, fixed_iters=fixed)
        compare(out["reduce"], o, "f32", f"reduce-then-broadcast {m}x{n} r={r}")


@pytest.mark.parametrize("precision,fixed", [("f32", 9), ("f64", 7), ("f32", 1)])
def test_fixed_count_residual_from_the_S_pass(precision, fixed):
    """A fixed-count solve that returns S ends with the step of its last
    iteration K and takes iteration K's residual ||M - L - S||_F / ||M||_F in
    the pass that writes S; without S it comes from one more sweep.  Both
    match the oracle's residual of iteration K (residual identity of the dual
    update, ||M - L - S|| = ||Y_{K+1} - Y_K|| / mu_K), and the factors of the
    two solves are bitwise the same."""
    m, n, r = (900, 1300, 8) if precision == "f32" else (300, 260, 6)
    dt = np.float32 if precision == "f32" else np.float64
    inst = workloads.planted(m, n, r, seed=5, frac=0.1, kind="uniform", scale=30.0, dtype=dt)
    Md = inst.M.astype(np.float64)
    mu0 = workloads.default_mu0(Md)
    o = oracle.fradm(Md, r, inst.lam, mu0, fixed_iters=fixed)
    Mt = torch.from_numpy(np.ascontiguousarray(inst.M)).cuda()
    with sfr.Solver(m, n, r, inst.lam, mu0, 1e-7, precision=precision, fixed_iters=fixed) as s:
        U1, B1, V1, S1, i1 = s.solve(Mt)
        U2, B2, V2, S2, i2 = s.solve(Mt, want_S=False)
        torch.cuda.synchronize()
    assert S2 is None and i1.iters == i2.iters == fixed
    assert torch.equal(U1, U2) and torch.equal(B1, B2) and torch.equal(V1, V2)
    # a reported figure, not an output: relative 1e-4 in FP32 (its terms are
    # FP32 differences of Y, rounding floor about 3e-8 of ||M||), 1e-9 in FP64
    bar, floor = (1e-4, 3e-8) if precision == "f32" else (1e-9, 1e-15)
    print(f"{precision} K={fixed}: residual from the S pass {i1.rel_residual:.6e}, from sweep K + 1 "
          f"{i2.rel_residual:.6e}, oracle {o['res']:.6e}")
    for info in (i1, i2):
        assert abs(info.rel_residual - o["res"]) <= bar * o["res"] + floor, (info.rel_residual, o["res"])


@pytest.mark.parametrize("spass", ["mfma", "vector", "narrow"])
@pytest.mark.parametrize("m,n,r", [(301, 212, 8), (1037, 700, 10), (77, 3004, 12), (260, 1024, 16),
                                   (500, 68, 20), (130, 904, 24), (150, 1500, 32), (333, 48, 3), (1000, 8, 2)])
def test_both_fp32_S_passes(monkeypatch, spass, m, n, r):
    """The FP32 pass that writes the returned S (and, for a fixed count, the
    last residual) in its forms, selected by SFR_SPASS: the rank-r term on the
    matrix cores (rank buckets from 8), on the vector ALU with one column
    vector per thread, or (n <= 256) the row-packed form that gives every
    thread a column vector of several rows.  Ragged row bands (m not a
    multiple of 16, 64 or 128) and column tiles (n a multiple of 4 only); S and
    the residual against the oracle."""
    monkeypatch.setenv("SFR_SPASS", spass)
    inst = workloads.planted(m, n, r, seed=m + 3 * n + r, frac=0.08, kind="uniform", scale=30.0, dtype=np.float32)
    g, o = case(inst, "f32", 5)
    compare(g, o, "f32", f"S pass {spass} {m}x{n} r={r}")
    assert abs(g["info"].rel_residual - o["res"]) <= 1e-4 * o["res"] + 3e-8, (g["info"].rel_residual, o["res"])


@pytest.mark.parametrize("first", ["kernel", "sweep"])
@pytest.mark.parametrize("m,n,r,precision,fixed", [(300, 1100, 10, "f32", 1), (300, 1100, 10, "f32", 6),
                                                   (257, 2048, 4, "f32", 5), (130, 1500, 32, "f32", 4),
                                                   (97, 4100, 16, "f32", 3), (200, 600, 5, "f64", 1),
                                                   (200, 600, 5, "f64", 7), (1037, 1024, 12, "f64", 3),
                                                   (333, 48, 3, "f32", 1), (1000, 200, 6, "f32", 5),
                                                   (400, 400, 5, "f64", 4), (5000, 80, 20, "f32", 3),
                                                   (3, 50, 2, "f64", 2)])
def test_first_sweep_both_forms(monkeypatch, first, m, n, r, precision, fixed):
    """The first sweep starts from V_0 = I: with P = M[:, :r] it needs only
    Q = M^T P and ||M||_F (SFR_FIRST unset), or the general sweep runs it
    (SFR_FIRST=sweep); both against the oracle, from one iteration on (wide
    rows, and narrow rows packed several to a workgroup; ragged row
    groups)."""
    if first == "sweep":
        monkeypatch.setenv("SFR_FIRST", "sweep")
    dt = np.float32 if precision == "f32" else np.float64
    inst = workloads.planted(m, n, r, seed=m + n + 7 * r, frac=0.08, kind="uniform", scale=30.0, dtype=dt)
    g, o = case(inst, precision, fixed)
    compare(g, o, precision, f"first {first} {m}x{n} r={r} {precision} K={fixed}")
