"""GPU tests of continuous batching: the queue form of a batched handle
(persistent kernels fed while they run) and the two servers.

A problem's result must not depend on what else is on the GPU: through the
queue form it is bitwise the same alone and in a mix (each problem's
kernel is chosen by its rank only); through the launch-batching server, whose
launches pick their rank bucket from their largest problem, it is the same
within the FP32 bar of 1e-5.  Every result is also checked against the FP64
oracle on a sample.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_1503_03004_amd as sfr
from paper_1503_03004_amd import serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    sfr.lib()
    yield


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def requests(count, seed=3, max_m=700):
    out = []
    for q in workloads.stream(seed=seed, count=count, rate=2000.0):
        q = dict(q, m=min(q["m"], max_m))
        q["r"] = min(q["r"], q["m"], q["n"])
        inst = workloads.stream_instance(q)
        out.append(dict(q, inst=inst, Mt=torch.from_numpy(inst.M).cuda(), lam=inst.lam,
                        mu=workloads.default_mu0(inst.M.astype(np.float64))))
    return out


def wait(bs, ticket, timeout=60.0):
    t0 = time.time()
    while True:
        res = bs.queue_poll(ticket)
        if res is not None:
            return res
        assert time.time() - t0 < timeout, "queue result not collected in time"
        time.sleep(1e-4)


def host(res):
    U, B, V, S, info = res
    return [t.double().cpu().numpy() for t in (U, B, V, S)], info


def test_queue_alone_and_in_a_mix():
    reqs = requests(40)
    with sfr.BatchSolver(64, 700, 512, 16) as bs:
        bs.queue_start()
        tickets = [bs.queue_submit(q["Mt"], q["r"], q["lam"], q["mu"], 1e-6) for q in reqs]
        assert all(t is not None for t in tickets)
        mix = [host(wait(bs, t)) for t in tickets]
        alone = [host(wait(bs, bs.queue_submit(q["Mt"], q["r"], q["lam"], q["mu"], 1e-6))) for q in reqs]
        bs.queue_stop()
    for (a, ia), (b, ib) in zip(mix, alone):
        assert ia.status == ib.status == sfr.SFR_OK and ia.iters == ib.iters
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    # parity against the oracle at the GPU's iteration count, on a sample
    for q, ((U, B, V, S), info) in list(zip(reqs, mix))[:: 7]:
        Md = q["inst"].M.astype(np.float64)
        o = oracle.fradm(Md, q["r"], q["lam"], q["mu"], fixed_iters=info.iters)
        eL = rel(U @ B @ V.T, o["U"] @ o["B"] @ o["V"].T)
        eS = rel(S, o["S"])
        print(f"{q['m']}x{q['n']} r={q['r']}: {info.iters} it, L {eL:.1e} S {eS:.1e}, orth {info.orth_err:.1e}")
        assert eL <= 1e-5 and eS <= 1e-5
        assert info.orth_err <= 1e-5


def test_queue_busy_and_relaunch_after_idle():
    """Two slots: a third submission is refused while both are in flight;
    after the kernels have ended from idleness, a submission relaunches them
    and gives the same result as before."""
    reqs = requests(3, seed=5)
    with sfr.BatchSolver(2, 700, 512, 16) as bs:
        bs.queue_start()
        t0 = bs.queue_submit(reqs[0]["Mt"], reqs[0]["r"], reqs[0]["lam"], reqs[0]["mu"], 1e-6)
        t1 = bs.queue_submit(reqs[1]["Mt"], reqs[1]["r"], reqs[1]["lam"], reqs[1]["mu"], 1e-6)
        assert t0 is not None and t1 is not None
        assert bs.queue_submit(reqs[2]["Mt"], reqs[2]["r"], reqs[2]["lam"], reqs[2]["mu"], 1e-6) is None
        first = host(wait(bs, t0))
        wait(bs, t1)
        time.sleep(3.0)      # about a second of idleness ends the persistent kernels
        again = host(wait(bs, bs.queue_submit(reqs[0]["Mt"], reqs[0]["r"], reqs[0]["lam"], reqs[0]["mu"], 1e-6)))
        bs.queue_stop()
        # the handle runs batches again once the queue has stopped
        out = bs.solve([(reqs[2]["Mt"], reqs[2]["r"], reqs[2]["lam"], reqs[2]["mu"], 1e-6)])
        assert out[0][4].status == sfr.SFR_OK
    for x, y in zip(first[0], again[0]):
        assert np.array_equal(x, y)


def test_queue_server_stream():
    """The queue server on a Poisson stream: every request is solved, and
    each result is bitwise the one the same request gets alone."""
    reqs = requests(48, seed=7)
    arrivals = workloads.stream(seed=7, count=48, rate=2000.0)
    rq = [serve.Request(M=q["Mt"], r=q["r"], lam=q["lam"], mu=q["mu"], tol=1e-6, arrival=a["t"])
          for q, a in zip(reqs, arrivals)]
    with serve.QueueServer(max_m=700, max_n=512, max_r=16, capacity=32) as qs:
        wall = qs.run(rq)
        lat = [q.latency * 1e3 for q in rq]
        print(f"queue server: {len(rq)} requests in {wall:.3f} s, p50 {serve.percentile(lat, 50):.2f} ms, "
              f"p99 {serve.percentile(lat, 99):.2f} ms, max in flight {qs.max_in_flight}")
        bs = qs.solver
        bs.queue_start()
        for q in rq:
            alone = host(wait(bs, bs.queue_submit(q.M, q.r, q.lam, q.mu, q.tol)))
            mix = host(q.result)
            assert mix[1].status == sfr.SFR_OK and mix[1].iters == alone[1].iters
            for x, y in zip(mix[0], alone[0]):
                assert np.array_equal(x, y)
        bs.queue_stop()


def test_batch_server_alone_and_in_a_mix():
    """The launch-batching server: each request's result is the result of
    the same request solved alone, within 1e-5 (a launch takes the rank
    bucket of its largest problem)."""
    reqs = requests(32, seed=9)
    arrivals = workloads.stream(seed=9, count=32, rate=4000.0)
    rq = [serve.Request(M=q["Mt"], r=q["r"], lam=q["lam"], mu=q["mu"], tol=1e-6, arrival=a["t"])
          for q, a in zip(reqs, arrivals)]
    with serve.BatchServer(max_m=700, max_n=512, max_r=16, workers=2, capacity=32) as srv:
        srv.run(rq)
        solver = srv.solvers[0]
        for q in rq:
            (U, B, V, S), info = host(q.result)
            (Ua, Ba, Va, Sa), ia = host(solver.solve([(q.M, q.r, q.lam, q.mu, q.tol)])[0])
            assert info.status == ia.status == sfr.SFR_OK
            assert abs(info.iters - ia.iters) <= 1
            if info.iters == ia.iters:
                assert rel(U @ B @ V.T, Ua @ Ba @ Va.T) <= 1e-5
                assert rel(S, Sa) <= 1e-5
