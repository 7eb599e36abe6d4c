"""sfr_solve_noalloc (the entry point that allocates nothing) against
sfr_solve on a handle: same kernels and arithmetic, so the results must be
bitwise equal; checked on two calls in a row (the second on a smaller
problem, so the shared static scratch keeps the first call's contents), in
FP64 and FP32, tolerance-driven and fixed-count, with M read in place and
through the padded copy, and with the library's default mu_0.  A problem
beyond the static scratch is refused on the host."""
import numpy as np
import pytest
import torch

import workloads
import paper_1503_03004_amd as sfr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    sfr.lib()
    yield


def outputs(m, n, r, dt, fill):
    return (torch.full((m, r), fill, dtype=dt, device="cuda"),
            torch.full((r, r), fill, dtype=torch.float64, device="cuda"),
            torch.full((n, r), fill, dtype=dt, device="cuda"),
            torch.full((m, n), fill, dtype=dt, device="cuda"))


def via_handle(M, r, lam, mu, tol, **opts):
    precision = "f64" if M.dtype == torch.float64 else "f32"
    m, n = M.shape
    with sfr.Solver(m, n, r, lam, mu, tol, precision=precision, **opts) as s:
        out = outputs(m, n, r, M.dtype, 0.0)
        info = s.solve(M, out=out)[4]
    return out, info


def via_noalloc(M, r, lam, mu, tol, **opts):
    m, n = M.shape
    out = outputs(m, n, r, M.dtype, -3.0)
    info = sfr.solve_noalloc(M, r, lam, mu, tol, out, **opts)
    return out, info


def same(a, b):
    (oa, ia), (ob, ib) = a, b
    assert ia.status == ib.status and ia.iters == ib.iters
    assert ia.rel_residual == ib.rel_residual and ia.mu0 == ib.mu0
    for x, y in zip(oa, ob):
        assert torch.equal(x, y)


CASES = [
    # (m, n, r, dtype, opts, second: (m, n))
    (1200, 1500, 8, torch.float32, dict(), (300, 700)),
    (400, 400, 5, torch.float64, dict(), (150, 90)),
    (900, 1030, 10, torch.float32, dict(fixed_iters=9), (257, 130)),
]


@pytest.mark.parametrize("m,n,r,dt,opts,second", CASES)
def test_noalloc_matches_handle_twice(m, n, r, dt, opts, second):
    for k, (mm, nn) in enumerate(((m, n), second)):
        np_dt = np.float64 if dt == torch.float64 else np.float32
        inst = workloads.planted(mm, nn, min(r, mm, nn), seed=mm + nn + k, frac=0.08, kind="uniform", scale=30.0,
                                 dtype=np_dt)
        M = torch.from_numpy(inst.M).cuda()
        mu0 = workloads.default_mu0(inst.M.astype(np.float64))
        tol = 1e-7 if dt == torch.float64 else 1e-6
        rr = min(r, mm, nn)
        a = via_noalloc(M, rr, inst.lam, mu0, tol, **opts)
        b = via_handle(M, rr, inst.lam, mu0, tol, **opts)
        torch.cuda.synchronize()
        print(f"{mm}x{nn} r={rr} {dt}: {a[1].iters} iterations, status {a[1].status}")
        same(a, b)


def test_noalloc_padded_copy_and_default_mu0():
    """n not a multiple of the vector width (M goes through the padded copy
    in the scratch) and mu <= 0 (Alg. 4 estimate in the scratch)."""
    inst = workloads.planted(700, 1001, 6, seed=7, frac=0.08, kind="uniform", scale=30.0, dtype=np.float32)
    M = torch.from_numpy(inst.M).cuda()
    a = via_noalloc(M, 6, inst.lam, 0.0, 1e-6)
    b = via_handle(M, 6, inst.lam, 0.0, 1e-6)
    torch.cuda.synchronize()
    assert a[1].mu0 > 0
    same(a, b)


def test_noalloc_refuses_beyond_the_scratch():
    M = torch.zeros((8000, 8000), dtype=torch.float32, device="cuda")
    out = outputs(8000, 8000, 10, torch.float32, 5.0)
    info = sfr.solve_noalloc(M, 10, 0.01, 1.0, 1e-6, out, raise_on_error=False)
    assert info.status == sfr.SFR_ERR_SCRATCH
    for t in out:
        assert bool((t == 5.0).all())
