"""GPU parity of the batched FR-ADM solver (sfr_create_batch /
sfr_solve_batch): many small independent problems, one workgroup each.

Every item runs Alg. 1 with the Alg. 2 L-step on FP32 data, so each item is
held to the FP32 bar of the single-problem path: relative Frobenius error
<= 1e-5 on L and S against the FP64 oracle at the same iteration count.
Items are independent, so an item's result does not depend on the other
items of its batch: bitwise when the batch's rank bucket is the same
(identical arithmetic), within the FP32 bar across buckets (the padded
rank changes only the order of the r x r rotations).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_1503_03004_amd as sfr

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    sfr.lib()
    yield


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def make(m, n, r, seed, frac=0.08):
    inst = workloads.planted(m, n, r, seed=seed, frac=frac, kind="uniform", scale=50.0, dtype=np.float64)
    M32 = inst.M.astype(np.float32)
    mu0 = workloads.default_mu0(M32.astype(np.float64))
    return dict(M=M32, r=r, lam=inst.lam, mu=mu0, L0=inst.L0)


def run_batch(bs, probs, tol=1e-7, **kw):
    items = [(torch.from_numpy(p["M"]).cuda(), p["r"], p["lam"], p["mu"], p.get("tol", tol)) for p in probs]
    out = bs.solve(items, **kw)
    torch.cuda.synchronize()
    res = []
    for U, B, V, S, info in out:
        res.append(dict(U=U.double().cpu().numpy(), B=B.cpu().numpy(), V=V.double().cpu().numpy(),
                        S=None if S is None else S.double().cpu().numpy(), info=info))
    return res


def check_vs_oracle(p, g, iters, what):
    Md = p["M"].astype(np.float64)
    o = oracle.fradm(Md, p["r"], p["lam"], p["mu"], fixed_iters=iters)
    assert o["rc"] >= 0 and o["iters"] == iters
    Lg = g["U"] @ g["B"] @ g["V"].T
    Lo = o["U"] @ o["B"] @ o["V"].T
    eL, eS = rel(Lg, Lo), rel(g["S"], o["S"])
    print(f"{what}: {p['M'].shape} r={p['r']} iters {iters}  errL {eL:.2e}  errS {eS:.2e}", flush=True)
    assert eL <= TOL, (what, eL)
    assert eS <= TOL, (what, eS)
    r = p["r"]
    assert np.abs(g["U"].T @ g["U"] - np.eye(r)).max() <= 1e-5
    assert np.abs(g["V"].T @ g["V"] - np.eye(r)).max() <= 1e-5
    assert np.array_equal(g["B"], g["B"].T)
    ev = np.linalg.eigvalsh(g["B"]).min()
    assert abs(g["info"].min_eig_B - ev) <= 1e-9 * np.abs(g["B"]).max()
    return o


SHAPES = [
    (64, 32, 2),        # smallest stream shape
    (100, 77, 5),       # ragged rows and columns
    (257, 129, 8),
    (33, 511, 3),       # widest row minus one
    (512, 512, 16),     # largest rank and width
    (2048, 40, 4),      # tallest stream shape
    (3, 50, 2),         # fewer rows than one band
    (700, 300, 12),
    (150, 64, 1),       # rank one
]


@pytest.mark.parametrize("fixed", [1, 2, 3, 9])
def test_mixed_shapes_fixed_iters_match_oracle(fixed):
    """One launch over items of every shape class; each item against the
    oracle after `fixed` iterations (1: X = M; 2: Y_1 = 0; then general)."""
    probs = [make(m, n, r, seed=100 * i + fixed) for i, (m, n, r) in enumerate(SHAPES)]
    with sfr.BatchSolver(len(probs), 2048, 512, 16, fixed_iters=fixed) as bs:
        out = run_batch(bs, probs)
    for p, g in zip(probs, out):
        assert g["info"].status in (sfr.SFR_OK, sfr.SFR_WARN_NOT_SPD)
        assert g["info"].iters == fixed and g["info"].converged
        check_vs_oracle(p, g, fixed, f"fixed{fixed}")


def test_stream_requests_tolerance_driven():
    """Requests drawn from the serving stream (m in [64, 2048], n in
    [32, 512], r in 2..16, 5-15 % outliers U[-50, 50]) solved to a relative
    residual of 1e-6: each stops within one iteration of the oracle's stop
    (the residual is FP32 on the GPU) and matches the oracle run for the
    same number of iterations."""
    reqs = workloads.stream(seed=7, count=10)
    probs = []
    for q in reqs:
        inst = workloads.stream_instance(q, dtype=np.float64)
        M32 = inst.M.astype(np.float32)
        probs.append(dict(M=M32, r=inst.r, lam=inst.lam, mu=workloads.default_mu0(M32.astype(np.float64)),
                          L0=inst.L0, tol=1e-6))
    with sfr.BatchSolver(len(probs), 2048, 512, 16, max_iter=300) as bs:
        out = run_batch(bs, probs)
    for p, g in zip(probs, out):
        info = g["info"]
        assert info.status in (sfr.SFR_OK, sfr.SFR_WARN_NOT_SPD), info
        assert info.converged and info.rel_residual <= 1e-6
        o = oracle.fradm(p["M"].astype(np.float64), p["r"], p["lam"], p["mu"], tol=1e-6, max_iter=300)
        assert abs(o["iters"] - info.iters) <= 1, (o["iters"], info.iters)
        check_vs_oracle(p, g, info.iters, "stream")


def test_alone_vs_mix_same_bucket_bitwise():
    """An item solved alone and inside a mixed batch of the same rank bucket
    gives bit-identical outputs and reports; both for a wide item (n > 128)
    and for a narrow one (n <= 128: the second kernel variant, run beside
    the first on a forked stream)."""
    A = make(300, 200, 7, seed=1)
    C = make(900, 64, 6, seed=3)
    mix = [make(120, 500, 8, seed=2), A, C, make(50, 50, 5, seed=4)]
    with sfr.BatchSolver(4, 1024, 512, 8, max_iter=200) as bs:
        alone = run_batch(bs, [A], tol=1e-6)[0]
        alone_c = run_batch(bs, [C], tol=1e-6)[0]
        out = run_batch(bs, mix, tol=1e-6)
    for a, b in ((alone, out[1]), (alone_c, out[2])):
        for k in ("U", "B", "V", "S"):
            assert np.array_equal(a[k], b[k]), k
        assert a["info"] == b["info"]


def test_alone_vs_mix_across_buckets():
    """r = 3 alone (bucket 3) against r = 3 inside a batch whose largest
    rank is 16: the same iterations, results equal to the FP32 bar."""
    A = make(400, 300, 3, seed=5)
    with sfr.BatchSolver(3, 512, 512, 16, fixed_iters=12) as bs:
        alone = run_batch(bs, [A])[0]
        inmix = run_batch(bs, [make(256, 256, 16, seed=6), A, make(64, 480, 10, seed=7)])[1]
    assert alone["info"].iters == inmix["info"].iters == 12
    La = alone["U"] @ alone["B"] @ alone["V"].T
    Lm = inmix["U"] @ inmix["B"] @ inmix["V"].T
    assert rel(Lm, La) <= TOL and rel(inmix["S"], alone["S"]) <= TOL


def test_batch_matches_single_problem_engine():
    """The batched kernel and the single-problem FP32 engine run the same
    iteration: equal stops and results to the FP32 bar."""
    probs = [make(333, 211, 4, seed=8), make(1500, 480, 10, seed=9)]
    with sfr.BatchSolver(2, 1500, 480, 10, max_iter=300) as bs:
        out = run_batch(bs, probs, tol=1e-6)
    for p, g in zip(probs, out):
        m, n = p["M"].shape
        with sfr.Solver(m, n, p["r"], p["lam"], p["mu"], 1e-6, precision="f32", max_iter=300) as s:
            U, B, V, S, info = s.solve(torch.from_numpy(p["M"]).cuda())
            torch.cuda.synchronize()
        assert abs(info.iters - g["info"].iters) <= 1
        Ls = (U.double() @ B @ V.double().T).cpu().numpy()
        if info.iters == g["info"].iters:
            assert rel(g["U"] @ g["B"] @ g["V"].T, Ls) <= TOL
            assert rel(g["S"], S.double().cpu().numpy()) <= TOL


def test_per_item_errors_are_isolated():
    """A NaN item and a rank-deficient item fail on their own; the other
    items of the launch are solved, and failed items' outputs are left
    untouched."""
    good1, good2 = make(200, 150, 4, seed=10), make(90, 300, 6, seed=11)
    Mnan = good1["M"].copy()
    Mnan[17, 33] = np.nan
    bad_nan = dict(good1, M=Mnan)
    Mr1 = np.outer(np.arange(1.0, 81.0), np.ones(60)).astype(np.float32)    # rank 1, r = 3
    bad_rank = dict(M=Mr1, r=3, lam=0.1, mu=1.0)
    probs = [good1, bad_nan, bad_rank, good2]
    items, outs = [], []
    for p in probs:
        m, n = p["M"].shape
        r = p["r"]
        items.append((torch.from_numpy(p["M"]).cuda(), r, p["lam"], p["mu"], 0.0))
        outs.append((torch.full((m, r), 7.0, device="cuda"), torch.full((r, r), 7.0, dtype=torch.float64,
                                                                         device="cuda"),
                     torch.full((n, r), 7.0, device="cuda"), torch.full((m, n), 7.0, device="cuda")))
    with sfr.BatchSolver(4, 200, 300, 6, fixed_iters=6) as bs:
        res = bs.solve(items, outs=outs, raise_on_error=False)
        torch.cuda.synchronize()
    st = [x[4].status for x in res]
    assert st[1] == sfr.SFR_ERR_NONFINITE and st[2] == sfr.SFR_ERR_RANK
    for k in (1, 2):
        assert all(bool((t == 7.0).all()) for t in outs[k])
    for k in (0, 3):
        assert st[k] in (sfr.SFR_OK, sfr.SFR_WARN_NOT_SPD)
        U, B, V, S, info = res[k]
        g = dict(U=U.double().cpu().numpy(), B=B.cpu().numpy(), V=V.double().cpu().numpy(),
                 S=S.double().cpu().numpy(), info=info)
        check_vs_oracle(probs[k], g, 6, "isolated")
    # the call reports the first error
    with sfr.BatchSolver(4, 200, 300, 6, fixed_iters=6) as bs:
        with pytest.raises(sfr.SFRError) as e:
            bs.solve(items)
        assert e.value.code == sfr.SFR_ERR_NONFINITE


def test_handle_reuse_then_smaller_batch():
    """Two calls in a row on one handle, the second with fewer and smaller
    items, give the outputs of fresh handles (the per-slot workspace keeps
    nothing between calls)."""
    big = [make(800, 400, 9, seed=20), make(640, 512, 12, seed=21), make(100, 100, 2, seed=22)]
    small = [make(64, 40, 9, seed=23)]
    with sfr.BatchSolver(3, 800, 512, 12, fixed_iters=7) as bs:
        run_batch(bs, big)
        second = run_batch(bs, small)[0]
    with sfr.BatchSolver(1, 64, 40, 12, fixed_iters=7) as bs:
        fresh = run_batch(bs, small)[0]
    for k in ("U", "B", "V", "S"):
        assert np.array_equal(second[k], fresh[k]), k
    check_vs_oracle(small[0], second, 7, "reuse")


def test_without_S_and_empty_batch():
    p = make(128, 96, 5, seed=30)
    with sfr.BatchSolver(2, 128, 96, 5, fixed_iters=5) as bs:
        assert bs.solve([]) == []
        g = run_batch(bs, [p], want_S=False)[0]
        assert g["S"] is None
        assert bs.workspace_bytes() >= 2 * (2 * 128 * 96 + 2 * 128 * 16 + 2 * 96 * 16) * 4
    Md = p["M"].astype(np.float64)
    o = oracle.fradm(Md, 5, p["lam"], p["mu"], fixed_iters=5)
    assert rel(g["U"] @ g["B"] @ g["V"].T, o["U"] @ o["B"] @ o["V"].T) <= TOL


def test_items_beyond_the_handle_limits_are_rejected():
    p = make(100, 80, 4, seed=40)
    M = torch.from_numpy(p["M"]).cuda()
    with sfr.BatchSolver(2, 100, 80, 4) as bs:
        for items in ([(M, 4, p["lam"], p["mu"], 1e-6)] * 3,                # count > capacity
                      [(M, 5, p["lam"], p["mu"], 1e-6)],                    # r > max_r
                      [(M, 4, -1.0, p["mu"], 1e-6)],                        # lambda <= 0
                      [(M, 4, p["lam"], p["mu"], float("nan"))]):           # tol NaN
            with pytest.raises(sfr.SFRError) as e:
                bs.solve(items)
            assert e.value.code == sfr.SFR_ERR_ARG
    with sfr.BatchSolver(1, 50, 80, 4) as bs:                                # m > max_m
        with pytest.raises(sfr.SFRError) as e:
            bs.solve([(M, 4, p["lam"], p["mu"], 1e-6)])
        assert e.value.code == sfr.SFR_ERR_ARG


def test_full_capacity_stream_batch():
    """128 stream requests in one launch (a serving-size batch); a sample of
    items against the oracle."""
    reqs = workloads.stream(seed=11, count=128)
    probs = []
    for q in reqs:
        inst = workloads.stream_instance(q, dtype=np.float64)
        M32 = inst.M.astype(np.float32)
        probs.append(dict(M=M32, r=inst.r, lam=inst.lam, mu=workloads.default_mu0(M32.astype(np.float64)),
                          L0=inst.L0))
    with sfr.BatchSolver(128, 2048, 512, 16, fixed_iters=15) as bs:
        out = run_batch(bs, probs)
    assert all(g["info"].iters == 15 for g in out)
    for k in (0, 31, 64, 127):
        check_vs_oracle(probs[k], out[k], 15, f"stream[{k}]")


@pytest.mark.parametrize("form", ["mfma", "vector"])
@pytest.mark.parametrize("fixed", [2, 3, 7])
def test_wide_rank_buckets_in_both_forms(form, fixed, monkeypatch):
    """Wide problems of ranks 8..16 run the matrix-core band loop (16-row
    bands, v_mfma_f32_16x16x4_f32) unless SFR_BATCH_MFMA=0 selects the vector
    one; both against the oracle, every rank bucket from 8 on (r = 9 and 10
    pad to 12 entries in the grouped V layout)."""
    monkeypatch.setenv("SFR_BATCH_MFMA", "1" if form == "mfma" else "0")
    probs = [make(300, 300, r, seed=40 + r) for r in (8, 9, 10, 12, 16)] + [make(1500, 480, 10, seed=9)]
    for p in probs:
        with sfr.BatchSolver(1, p["M"].shape[0], p["M"].shape[1], p["r"], fixed_iters=fixed) as bs:
            g = run_batch(bs, [p])[0]
        check_vs_oracle(p, g, fixed, f"{form} r={p['r']}")


def test_autotune_records_a_form_per_class_and_bucket():
    """sfr_tune_batch times the band-loop forms on the given problems and
    records one per (class, rank bucket) present; solves on the tuned handle
    still match the oracle (every form is exact)."""
    probs = [make(600, 400, 10, seed=50), make(900, 300, 16, seed=51), make(500, 100, 4, seed=52),
             make(700, 64, 12, seed=53), make(300, 200, 3, seed=54)]
    items = [(torch.from_numpy(p["M"]).cuda(), p["r"], p["lam"], p["mu"], 1e-6) for p in probs]
    with sfr.BatchSolver(len(probs), 900, 400, 16, fixed_iters=5) as bs:
        table = bs.autotune(items)
        torch.cuda.synchronize()
        print("tuned:", table)
        assert set(table) == {(False, 10), (False, 16), (True, 4), (True, 12), (False, 3)}
        assert all(v in ("lane groups", "one row per wavefront", "two rows per wavefront", "matrix cores")
                   for v in table.values())
        assert table[(False, 3)] != "matrix cores"        # rank bucket below the matrix-core forms
        assert table[(False, 10)] != "lane groups"        # lane groups only for narrow problems
        out = run_batch(bs, probs)
    for p, g in zip(probs, out):
        check_vs_oracle(p, g, 5, "tuned")


def test_autotune_rejects_items_beyond_the_limits():
    p = make(100, 80, 4, seed=55)
    with sfr.BatchSolver(1, 100, 80, 4) as bs:
        with pytest.raises(sfr.SFRError) as e:
            bs.autotune([(torch.from_numpy(p["M"]).cuda(), 5, p["lam"], p["mu"], 1e-6)])
        assert e.value.code == sfr.SFR_ERR_ARG


BF16_SHAPES = [(600, 300, 8), (900, 512, 16), (400, 200, 12), (1024, 260, 10)]


def test_batched_bf16_every_iteration():
    """Batched BF16 form, every iteration in BF16 (p = X V and Q = X^T P on
    BF16 operands, FP32 accumulation, l in FP32): the unrefined result
    within 1e-3 of the oracle at the same iteration count."""
    probs = [make(m, n, r, seed=300 + i) for i, (m, n, r) in enumerate(BF16_SHAPES)]
    with sfr.BatchSolver(len(probs), 1024, 512, 16, fixed_iters=12, bf16=True) as bs:
        out = run_batch(bs, probs)
    for p, g in zip(probs, out):
        o = oracle.fradm(p["M"].astype(np.float64), p["r"], p["lam"], p["mu"], fixed_iters=12)
        eL = rel(g["U"] @ g["B"] @ g["V"].T, o["U"] @ o["B"] @ o["V"].T)
        eS = rel(g["S"], o["S"])
        print(f"batched all-BF16 {p['M'].shape} r={p['r']}: errL {eL:.2e} errS {eS:.2e}")
        assert eL <= 1e-3 and eS <= 1e-3
        assert eL > 1e-6        # the BF16 operands are really in use


def test_batched_bf16_head_then_fp32():
    """Batched BF16 form with FP32 iterations after (BF16 while the residual
    is above 1e-3), tolerance-driven to 1e-6: within one iteration of the
    oracle's stop and within the FP32 bar of the oracle at the same count."""
    probs = [make(m, n, r, seed=400 + i) for i, (m, n, r) in enumerate(BF16_SHAPES)]
    with sfr.BatchSolver(len(probs), 1024, 512, 16, bf16=True, bf16_tol=1e-3) as bs:
        out = run_batch(bs, probs, tol=1e-6)
    for p, g in zip(probs, out):
        Md = p["M"].astype(np.float64)
        ot = oracle.fradm(Md, p["r"], p["lam"], p["mu"], tol=1e-6)
        assert g["info"].status == sfr.SFR_OK
        assert abs(g["info"].iters - ot["iters"]) <= 1, (g["info"].iters, ot["iters"])
        check_vs_oracle(p, g, g["info"].iters, "batched BF16 head")
