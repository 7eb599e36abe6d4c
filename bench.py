#!/usr/bin/env python3
"""Benchmark of the S-FR hot path on one MI355X.

A step is one FR-ADM iteration (Alg. 1 with the Alg. 2 L-step): the fused
sweep over M and Y, the column-partial/Gram reduction and the FP64 r x r
step.  The timed region runs exactly --steps iterations through the C ABI
(sfr_solve with fixed_iters = steps, which also writes U, B, V and S once
at the end), with the input already resident in HBM.

Default workload: m = n = 8000, r = 10, FP32 storage, L0 = A B^T with
N(0,1) factors, 10 % Bernoulli outliers U[-100, 100] (seeded synthetic).

Printed: one JSON line with the iteration rate, the fused sweep's HBM
roofline fraction (HIP start/stop events bound to every sweep dispatch,
taken in a second run of the same K iterations), a full
tolerance-driven solve rate with p50/p99 latency, the
relative error against the FP64 oracle on the same input, and the oracle's
own rate on the host (cpu_baseline).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("sweep.hip", "sweep_mfma.hip", "exchange.hpp", "sfr_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1503_03004_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def host_info() -> dict:
    """CPU model, logical CPUs and memory of the host that times the oracle."""
    model, mem_kib = None, None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    mem_kib = int(line.split()[1])
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(),
            "mem_gib": round(mem_kib / 2 ** 20, 1) if mem_kib else None}


def copy_bandwidth_gbs(dev) -> float:
    """Read + write bandwidth of a plain device copy (torch copy_ of 512 MiB),
    mean of 10 copies timed with HIP events: the achievable streaming rate
    on this device, reported beside the published peak."""
    import torch
    src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 10 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def measured_traffic(workload: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary, if it was taken on the current sweep source."""
    path = os.path.join(ROOT, "profiles", f"sweep_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("sweep_source_sha") != sweep_source_hash():
        return None
    return d.get("bytes_per_launch")


def _oracle_worker(seed, iters, barrier, queue):
    """One oracle process of the all-cores leg: draws the 8000^2 input itself,
    waits for the others, then times `iters` FR-ADM iterations (one thread)."""
    import oracle
    import workloads
    inst = workloads.large_fp32(seed=seed)
    Md = inst.M.astype(np.float64)
    mu0 = workloads.default_mu0(inst.M)
    barrier.wait()
    t = time.perf_counter()
    oracle.fradm(Md, inst.r, inst.lam, mu0, fixed_iters=iters)
    queue.put(time.perf_counter() - t)


def oracle_all_cores(seed: int, iters: int, procs: int) -> dict:
    """The oracle as it stands, on every core of the host share at once: one
    single-threaded process per core, each running `iters` iterations of the
    same 8000^2 r = 10 workload, started together.  Aggregate throughput =
    procs * iters / (slowest process's time)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        barrier = ctx.Barrier(procs)
        queue = ctx.Queue()
        ps = [ctx.Process(target=_oracle_worker, args=(seed, iters, barrier, queue)) for _ in range(procs)]
        for p in ps:
            p.start()
        import queue as queue_mod
        times = []
        while len(times) < procs:
            try:
                times.append(queue.get(timeout=2))
            except queue_mod.Empty:
                if any(p.exitcode not in (None, 0) for p in ps):
                    for p in ps:
                        p.kill()
                    raise RuntimeError("an oracle process of the all-cores leg failed")
        for p in ps:
            p.join()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    slowest = max(times)
    return {"value": procs * iters / slowest, "unit": "iters/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs} concurrent single-threaded oracle processes, {iters} FR-ADM iterations each of the "
                      f"same 8000x8000 r=10 input, FP64; aggregate over the slowest ({slowest:.1f} s)"}


def rel(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", default="large_fp32",
                    choices=["large_fp32", "plain_fp64", "photometric", "tsvd_fp32", "serving", "nystrom", "large_rank"])
    ap.add_argument("--requests", type=int, default=4000, help="serving: requests in the Poisson stream")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: mean arrival rate (requests/s)")
    ap.add_argument("--workers", type=int, default=4, help="serving: concurrent batched launches")
    ap.add_argument("--max-batch", type=int, default=0, help="serving: requests per launch (0: capacity)")
    ap.add_argument("--no-autotune", action="store_true", help="serving: keep the built-in band-loop forms")
    ap.add_argument("--queue-capacity", type=int, default=512, help="serving: slots of the queue server")
    ap.add_argument("--nys-l", type=int, default=80, help="nystrom: sampled rows and columns l (default 4r = 80)")
    ap.add_argument("--solves", type=int, default=5, help="tolerance-driven solves timed for solves/s")
    ap.add_argument("--m", type=int, default=2000, help="large_rank: rows")
    ap.add_argument("--n", type=int, default=2000, help="large_rank: columns")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-config4", action="store_true",
                    help="large_fp32: skip the 40000^2 FR-Nys / full FR-ADM figures in the default line")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="large_fp32: skip the 400^2 FP64, photometric and serving figures in the default line")
    ap.add_argument("--all-cores-iters", type=int, default=2,
                    help="large_fp32: oracle iterations per process in the all-cores CPU leg (0: skip)")
    ap.add_argument("--oracle-iters", type=int, default=12, help="oracle iterations timed on the host (about 1 s each)")
    ap.add_argument("--rank", type=int, default=0, help="large_fp32 / tsvd_fp32: rank r (default 10)")
    ap.add_argument("--bf16-iters", type=int, default=0,
                    help="BF16-operand contractions for the first K iterations of every solve, FP32 after")
    ap.add_argument("--bf16-tol", type=float, default=1e-3,
                    help="with --bf16-iters: tolerance-driven solves leave BF16 at this residual")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration under rocprofv3)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the row-sharded multi-GPU form is a design note only).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_1503_03004_amd as sfr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "serving":
        return serving(args)
    if args.workload == "nystrom":
        return nystrom(args)
    if args.workload == "large_rank":
        return large_rank(args)

    def single(args):
        """One FR-ADM / Alg. 4 workload: the timed fixed-count solve, the
        tolerance-driven solves and (unless --no-cpu-baseline) the oracle leg."""
        t0 = time.time()
        tsvd = args.workload == "tsvd_fp32"
        if args.workload in ("large_fp32", "tsvd_fp32"):
            rk = args.rank or 10
            inst = workloads.large_fp32(seed=args.seed, r=rk)
            precision, esz, tol = "f32", 4, 1e-6
            desc = f"FR-ADM, m=n=8000, r={rk}, FP32, 10% outliers U[-100,100]"
            if tsvd:
                tol = 1e-6
                desc = f"FixedRankOptFull (Alg. 4) rank-{rk} TSVD of the same 8000x8000 FP32 matrix"
        elif args.workload == "plain_fp64":
            inst = workloads.plain_fp64(seed=args.seed)
            precision, esz, tol = "f64", 8, 1e-7
            desc = "FR-ADM, m=n=400, r=5, FP64, 5% outliers U[-50,50]"
        else:
            inst = workloads.photometric(seed=args.seed)
            precision, esz, tol = "f32", 4, 1e-6
            desc = "FR-ADM, photometric stereo shape m=262144 x n=48, r=3, FP32"
        m, n = inst.M.shape
        r = inst.r
        mu0 = workloads.default_mu0(inst.M)
        # BF16 head (FP32 FR-ADM only): fixed-count solves take BF16 for their
        # first --bf16-iters iterations, tolerance-driven ones until --bf16-tol
        bf_fixed, bf_tol = {}, {}
        if args.bf16_iters > 0:
            if precision != "f32" or tsvd:
                print("bench.py: --bf16-iters applies to FP32 FR-ADM workloads", file=sys.stderr)
                sys.exit(2)
            bf_fixed = dict(bf16=True, bf16_iters=args.bf16_iters)
            bf_tol = dict(bf16=True, bf16_tol=args.bf16_tol)
        tdt = torch.float64 if precision == "f64" else torch.float32
        M = torch.from_numpy(np.ascontiguousarray(inst.M)).to(device=dev, dtype=tdt)
        torch.cuda.synchronize()
        print(f"[bench] workload {args.workload} {m}x{n} r={r} ready in {time.time() - t0:.1f}s", file=sys.stderr,
              flush=True)

        stream = torch.cuda.current_stream()
        if args.calibrate_copy:
            # a plain copy kernel of known size: reads and writes 256 MiB each
            src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
        def run(solver, out=None, stream=None):
            """One solve: FR-ADM (U, B, V, S, info) or Alg. 4 (U, B, V, None, info)."""
            if tsvd:
                U_, B_, V_, inf_ = solver.tsvd(M, out=None if out is None else out[:3], stream=stream)
                return U_, B_, V_, None, inf_
            return solver.solve(M, out=out, stream=stream)

        # ---- the timed handle and its outputs are set up first, so that the
        # warm-up runs right before the timed solve
        K = args.steps
        solver = sfr.Solver(m, n, r, inst.lam, mu0, tol, precision=precision, fixed_iters=K, **bf_fixed)
        U = torch.empty((m, r), dtype=tdt, device=dev)
        Bm = torch.empty((r, r), dtype=torch.float64, device=dev)
        V = torch.empty((n, r), dtype=tdt, device=dev)
        S = torch.empty((m, n), dtype=tdt, device=dev)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)

        # ---- warmup: W untimed iterations (a handle of their own)
        if args.warmup > 0:
            with sfr.Solver(m, n, r, inst.lam, mu0, tol, precision=precision, fixed_iters=args.warmup, **bf_fixed) as w:
                run(w)
        torch.cuda.synchronize()

        # ---- timed: exactly K iterations (plus the output pass writing U, B, V, S)
        ev0.record(stream)
        _, _, _, _, info = run(solver, out=(U, Bm, V, S), stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        assert info.iters == K, info
        value = K / (ms / 1e3)
        solver.close()
        # ---- the same K iterations again with HIP events bound to every sweep
        # dispatch (kept out of the run above: the events cost a few us a launch)
        with sfr.Solver(m, n, r, inst.lam, mu0, tol, precision=precision, fixed_iters=K, profile=True,
                        **bf_fixed) as sp:
            _, _, _, _, pinfo = run(sp, out=(U, Bm, V, S), stream=stream)
        torch.cuda.synchronize()
        sweep_ms = pinfo.sweep_ms
        print(f"[bench] {K} iterations in {ms:.3f} ms; sweep {sweep_ms * 1e3:.1f} us avg over {pinfo.sweeps_timed}",
              file=sys.stderr, flush=True)

        bytes_per_el = (1 if tsvd else 3) * esz  # read M (, read Y_{k-1}, write Y_k)
        alg_bytes = bytes_per_el * m * n
        achieved = alg_bytes / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else 0.0
        copy_gbs = copy_bandwidth_gbs(dev)
        print(f"[bench] plain device copy: {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
        # the committed counters were taken on the default configuration only
        default_cfg = (not args.rank or args.rank == 10) and not bf_fixed
        traffic = measured_traffic(args.workload) if default_cfg else None
        sweep_name = "sweep_mfma_kernel" if (bf_fixed or r > 10 or tsvd) else "sweep_kernel"

        # ---- full tolerance-driven solves: solves/s and latency percentiles
        lat = []
        solve_iters = None
        Ls = None
        with sfr.Solver(m, n, r, inst.lam, mu0, tol, precision=precision, max_iter=300, **bf_tol) as s2:
            for i in range(max(1, args.solves)):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                U2, B2, V2, S2, inf2 = run(s2, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                lat.append(e0.elapsed_time(e1))
                solve_iters = inf2.iters
            rec_err = None
            if inst.L0 is not None and not tsvd:
                rows = np.random.default_rng(1).choice(m, min(m, 256), replace=False)
                Lr = (U2.double()[rows] @ B2 @ V2.double().T).cpu().numpy()
                rec_err = rel(Lr, inst.L0[rows].astype(np.float64))
        lat = np.array(lat)
        print(f"[bench] tolerance-driven solve: {solve_iters} iterations, p50 {np.percentile(lat, 50):.2f} ms",
              file=sys.stderr, flush=True)

        # ---- FP64 oracle on the same input: host rate and parity of the first iterations
        cpu = None
        parity = None
        if not args.no_cpu_baseline:
            import oracle
            Md = inst.M.astype(np.float64)
            oi = args.oracle_iters
            t1 = time.perf_counter()
            if tsvd:
                Uo, Bo, Vo, _ = oracle.fr_full(Md, np.eye(m, r), np.eye(r), np.eye(n, r), oi)
                o = {"U": Uo, "B": Bo, "V": Vo, "S": None}
            else:
                o = oracle.fradm(Md, r, inst.lam, mu0, fixed_iters=oi)
            tc = time.perf_counter() - t1
            cpu = {"value": oi / tc, "unit": "iters/s", "cores": 1, "kind": "oracle", "host": host_info(),
                   "sample": f"{oi} {'Alg. 4 steps' if tsvd else 'FR-ADM iterations'} of the same {m}x{n} r={r} "
                             f"input, FP64, one thread ({tc:.1f} s)"}
            # a BF16 head of the same share of the iterations as in the timed run
            bf_par = dict(bf_fixed, bf16_iters=max(1, (args.bf16_iters * oi) // K)) if bf_fixed else {}
            with sfr.Solver(m, n, r, inst.lam, mu0, tol, precision=precision, fixed_iters=oi, **bf_par) as s3:
                U3, B3, V3, S3, _ = run(s3)
            torch.cuda.synchronize()
            rows = np.random.default_rng(2).choice(m, min(m, 128), replace=False)
            Lg = (U3.double()[rows] @ B3 @ V3.double().T).cpu().numpy()
            Lo = o["U"][rows] @ o["B"] @ o["V"].T
            parity = {"iterations": oi, **({"bf16_iters": bf_par["bf16_iters"]} if bf_par else {}),
                      "rel_err_L": rel(Lg, Lo),
                      "rel_err_S": None if tsvd else rel(S3.double()[rows].cpu().numpy(), o["S"][rows]),
                      "rows_sampled": int(rows.size)}
            print(f"[bench] oracle {oi} iterations in {tc:.1f} s; parity {parity}", file=sys.stderr, flush=True)

        out = {
            "metric": "iters/s & solves/s at rel-err<=1e-5 vs FP64 oracle; %HBM roofline; p50/p99",
            "value": value,
            "unit": "iters/s",
            "n_gpus": 1,
            "steps": K,
            "warmup": args.warmup,
            "ms_per_step": ms / K,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "bf16-operands+f32" if bf_fixed else precision,
            "data": "synthetic",
            "config": {"workload": desc, "m": m, "n": n, "r": r, "lambda": inst.lam, "mu0": mu0,
                       "rho": 1.5, "mu_bar": 1e9, "seed": args.seed,
                       **({"bf16_iters": args.bf16_iters, "bf16_tol": args.bf16_tol} if bf_fixed else {})},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                         "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                         "kernel": sweep_name, "sweep_us": sweep_ms * 1e3,
                         "alg_bytes_per_launch": alg_bytes},
            "cpu_baseline": cpu,
            "solves_per_s": 1e3 / float(np.mean(lat)),
            "solve_iters": solve_iters,
            "solve_tol": tol,
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "parity_vs_oracle": parity,
            "recovery_rel_err_L": rec_err,
            "paper_context": ("Appendix, Alg. 4 (FixedRankOptFull): Q-linear convergence to the TSVD; the paper "
                              "prints no timing for this shape") if tsvd else
                             ("Table 1, FR-ADM 8000^2 r=10 (outliers in [-1,1]): 28 iterations in 27.42 s "
                              "(~1.0 it/s) on a 3.2 GHz desktop CPU; not the same workload"),
        }
        return out, default_cfg

    out, default_cfg = single(args)
    default_line = args.workload == "large_fp32" and default_cfg
    if default_line and not args.no_cpu_baseline and args.all_cores_iters > 0:
        procs = max(1, min(16, os.cpu_count() or 1))
        out["cpu_baseline_all_cores"] = oracle_all_cores(args.seed, args.all_cores_iters, procs)
        print(f"[bench] oracle on {procs} cores: {out['cpu_baseline_all_cores']['value']:.2f} iters/s",
              file=sys.stderr, flush=True)
    if default_line and not args.no_config4:
        torch.cuda.empty_cache()
        c4 = nystrom_measure(args, l=80)
        out["config4_nystrom"] = {k: c4[k] for k in ("config", "value", "unit", "ms_per_step", "nys_iters",
                                                     "nys_rel_err_vs_L0", "full_fradm", "parity_vs_oracle",
                                                     "cpu_baseline", "roofline")}
    if default_line and not args.no_other_configs:
        # the other workloads of the metric, each measured here as its own
        # --workload run measures it (compact keys; the full lines come from
        # bench.py --workload plain_fp64 | photometric | serving)
        keep = ("config", "value", "unit", "ms_per_step", "dtype", "solves_per_s", "solve_iters", "p50_ms",
                "p99_ms", "parity_vs_oracle", "recovery_rel_err_L", "cpu_baseline")
        for wl, key in (("plain_fp64", "config1_fp64_400"), ("photometric", "config3_photometric")):
            torch.cuda.empty_cache()
            sub = argparse.Namespace(**vars(args))
            sub.workload, sub.rank, sub.bf16_iters = wl, 0, 0
            o, _ = single(sub)
            out[key] = {k: o.get(k) for k in keep}
            out[key]["roofline"] = {k: o["roofline"].get(k) for k in ("bound", "achieved", "peak", "unit", "frac",
                                                                        "kernel", "sweep_us")}
        torch.cuda.empty_cache()
        sub = argparse.Namespace(**vars(args))
        sub.workload, sub.requests = "serving", min(args.requests, 2000)
        o = serving_measure(sub)
        out["config5_serving"] = {k: o.get(k) for k in ("config", "value", "unit", "p50_ms", "p99_ms",
                                                         "saturated_solves_per_s", "slowest_request_alone_ms",
                                                         "failed", "failed_queue", "parity_vs_oracle",
                                                         "cpu_baseline", "roofline")}
    print(json.dumps(out), flush=True)


FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X, published (packed FP32)


def nystrom(args):
    print(json.dumps(nystrom_measure(args, l=args.nys_l)), flush=True)


def nystrom_measure(args, l):
    """FR-Nys workload (Alg. 3): m = n = 40000, r = 20, l = 4r = 80 sampled
    rows and columns, FP32, L0 = A B^T with N(0,1) factors and 7 % Laplace(0,
    20) outliers, drawn on the device.  value = FR-Nys solves/s (tol 1e-6 on
    both sub-solves); beside it the full FR-ADM solve of the same matrix (mu_0
    = 1.25/||M||_2 from the library's device default) and both results'
    relative error against the planted L0 on 20000 sampled entries: the two
    compared at their final error.  Parity: a 25-iteration FR-Nys solve
    against the oracle's Alg. 3 on the same two gathered blocks (20000 sampled
    entries of L), whose host time is the CPU baseline."""
    import torch
    import workloads
    import paper_1503_03004_amd as sfr

    m = n = 40000
    r, tol, fixed = 20, 1e-6, 25
    t0 = time.time()
    M, A, B, lam = workloads.nystrom_large_device(seed=args.seed)
    assert bool(torch.isfinite(M).all()), "non-finite input"
    perm = workloads.row_permutation(m, seed=args.seed + 11)
    pt = torch.from_numpy(perm).cuda()
    C = M[pt, :l].double().cpu().numpy()
    Rb = M[pt[:l]].double().cpu().numpy()
    mu_l, mu_t = workloads.default_mu0(C), workloads.default_mu0(Rb)
    rng = np.random.default_rng(5)
    ti = rng.integers(0, m, 20000)          # shuffled-order row index
    tj = rng.integers(0, n, 20000)
    rows_t = torch.from_numpy(perm[ti]).cuda()
    cols_t = torch.from_numpy(tj).cuda()
    L0 = (A[rows_t].double() * B[cols_t].double()).sum(1)
    torch.cuda.synchronize()
    print(f"[bench] nystrom 40000^2 r={r} l={l} ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    def sampled_L(U, Bc, V):
        return ((U[rows_t].double() @ Bc) * V[cols_t].double()).sum(1)

    def err_L0(U, Bc, V):
        return float(torch.linalg.norm(sampled_L(U, Bc, V) - L0) / torch.linalg.norm(L0))

    U = torch.empty(m, r, device="cuda", dtype=torch.float32)
    V = torch.empty(n, r, device="cuda", dtype=torch.float32)
    Bm = torch.empty(r, r, device="cuda", dtype=torch.float64)
    S = torch.empty_like(M)
    out = (U, Bm, V, S)
    K = max(1, args.solves)

    # ---- FR-Nys, tolerance-driven
    with sfr.Solver(m, n, r, lam, 1.0, tol, precision="f32", nystrom_l=l, mu_left=mu_l, mu_top=mu_t) as s:
        s.solve_nys(M, perm, out=out)                       # warm
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(K):
            _, _, _, _, ninfo = s.solve_nys(M, perm, out=out)
        torch.cuda.synchronize()
        nys_ms = 1e3 * (time.perf_counter() - t1) / K
    nys_err = err_L0(U, Bm, V)
    print(f"[bench] FR-Nys: {nys_ms:.2f} ms per solve ({ninfo.iters}/{ninfo.iters_top} iterations), "
          f"error vs L0 {nys_err:.2e}", file=sys.stderr, flush=True)

    # ---- full FR-ADM on the same matrix: mu_0 from the device default, then
    # timed with that mu_0 (and once more with the sweep events bound)
    with sfr.Solver(m, n, r, lam, 0.0, tol, precision="f32") as s:
        _, _, _, _, finfo = s.solve(M, out=out)
    mu0 = finfo.mu0
    with sfr.Solver(m, n, r, lam, mu0, tol, precision="f32") as s:
        s.solve(M, out=out)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(2):
            _, _, _, _, finfo = s.solve(M, out=out)
        torch.cuda.synchronize()
        full_ms = 1e3 * (time.perf_counter() - t1) / 2
    full_err = err_L0(U, Bm, V)
    with sfr.Solver(m, n, r, lam, mu0, tol, precision="f32", profile=True) as s:
        _, _, _, _, pinfo = s.solve(M, out=out)
    torch.cuda.synchronize()
    sweep_gbs = 12.0 * m * n / (pinfo.sweep_ms * 1e-3) / 1e9 if pinfo.sweep_ms > 0 else 0.0
    print(f"[bench] full FR-ADM: {full_ms:.1f} ms per solve ({finfo.iters} iterations), error vs L0 {full_err:.2e}; "
          f"sweep {pinfo.sweep_ms * 1e3:.0f} us ({sweep_gbs:.0f} GB/s)", file=sys.stderr, flush=True)

    # ---- parity and the oracle's host time: 25 iterations on both blocks
    with sfr.Solver(m, n, r, lam, 1.0, tol, precision="f32", nystrom_l=l, mu_left=mu_l, mu_top=mu_t,
                    fixed_iters=fixed) as s:
        s.solve_nys(M, perm, out=out)
    torch.cuda.synchronize()
    Lg = sampled_L(U, Bm, V).cpu().numpy()
    cpu, parity = None, None
    if not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        o = oracle.frnys_blocks(C, Rb, r, lam, mu_l, mu_t, fixed_iters=fixed)
        tc = time.perf_counter() - t1
        Lo = oracle.nys_entries(o["LL"], o["Wp"], o["LT"], ti, tj)
        parity = {"iterations": fixed, "rel_err_L_sampled": rel(Lg, Lo), "entries_sampled": len(ti)}
        cpu = {"value": 1.0 / tc, "unit": "solves/s", "cores": 1, "kind": "oracle", "host": host_info(),
               "sample": f"Alg. 3 on the two gathered blocks ({m}x{l} and {l}x{n}), {fixed} iterations each, FP64, "
                         f"one thread ({tc:.1f} s); the dense m x n S pass is not included"}
        print(f"[bench] oracle {tc:.1f} s; parity {parity}", file=sys.stderr, flush=True)

    # whole-solve algorithmic bytes of FR-Nys: the dense S pass (read M,
    # write S) and the sub-solves (read, read Y, write Y per element and
    # iteration of the two l-wide blocks)
    nys_bytes = 8.0 * m * n + 12.0 * l * (m + n) * (ninfo.iters + ninfo.iters_top) / 2.0
    nys_gbs = nys_bytes / (nys_ms * 1e-3) / 1e9
    out_line = {
        "metric": "iters/s & solves/s at rel-err<=1e-5 vs FP64 oracle; %HBM roofline; p50/p99",
        "value": 1e3 / nys_ms,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": 1,
        "ms_per_step": nys_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"FR-Nys, m=n=40000, r=20, l={l}, FP32, 7% Laplace(0,20) outliers, tol {tol}",
                   "m": m, "n": n, "r": r, "l": l, "lambda": lam, "mu_left": mu_l, "mu_top": mu_t,
                   "seed": args.seed},
        "roofline": {"bound": "hbm", "achieved": nys_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": nys_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "FR-Nys solve (dense S pass + sub-solves, whole-solve bytes / solve time)",
                     "alg_bytes_per_solve": nys_bytes},
        "cpu_baseline": cpu,
        "nys_iters": [ninfo.iters, ninfo.iters_top],
        "nys_rel_err_vs_L0": nys_err,
        "full_fradm": {"ms_per_solve": full_ms, "iters": finfo.iters, "mu0": mu0, "rel_err_vs_L0": full_err,
                       "sweep_us": pinfo.sweep_ms * 1e3, "sweep_gbs": sweep_gbs,
                       "sweep_frac": sweep_gbs / HBM_PEAK_GBS, "speedup_of_nys": full_ms / nys_ms},
        "parity_vs_oracle": parity,
        "paper_context": "Sec. 5.1: FR-Nys is faster than FR-ADM at low rank on large matrices",
    }
    return out_line


FP32_MFMA_PEAK_TFLOPS = 157.3    # MI355X, published dense FP32 matrix


def large_rank(args):
    """Large-rank workload (Sec. 5.1, Table 2: r = 0.1 m; Sec. 5.3 clustering
    shapes): m x n (default 2000 x 2000), r = --rank (default 200), FP32,
    L0 = A B^T with N(0,1) factors and 10 % outliers uniform in [-1, 1] (the
    synthetic set-up of Sec. 5.1), mu_0 = 1.25/||M||_2.  value = FR-ADM
    iterations/s over --steps fixed iterations; beside it a tolerance-driven
    solve (1e-6) and parity of --oracle-iters iterations against the FP64
    oracle, whose host time is the CPU baseline.  roofline: the three m x n
    contractions' 6 m n r flops per iteration over the whole iteration's
    time (every kernel of the iteration, the r x r algebra included) against
    the dense FP32 matrix peak."""
    import torch
    import workloads
    import paper_1503_03004_amd as sfr

    m, n = args.m, args.n
    r = args.rank or 200
    t0 = time.time()
    inst = workloads.planted(m, n, r, seed=args.seed, frac=0.10, kind="uniform", scale=1.0, dtype=np.float32)
    Md = inst.M.astype(np.float64)
    mu0 = workloads.default_mu0(Md)
    M = torch.from_numpy(inst.M).cuda()
    torch.cuda.synchronize()
    print(f"[bench] large_rank {m}x{n} r={r} ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    K = args.steps
    if args.warmup > 0:
        with sfr.Solver(m, n, r, inst.lam, mu0, 1e-6, precision="f32", fixed_iters=args.warmup) as w:
            w.solve(M)
    torch.cuda.synchronize()
    U = torch.empty((m, r), device="cuda")
    Bm = torch.empty((r, r), dtype=torch.float64, device="cuda")
    V = torch.empty((n, r), device="cuda")
    S = torch.empty((m, n), device="cuda")
    with sfr.Solver(m, n, r, inst.lam, mu0, 1e-6, precision="f32", fixed_iters=K) as s:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, _, _, info = s.solve(M, out=(U, Bm, V, S))
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t1)
    assert info.iters == K
    with sfr.Solver(m, n, r, inst.lam, mu0, 1e-6, precision="f32") as s:
        s.solve(M, out=(U, Bm, V, S))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, _, _, tinfo = s.solve(M, out=(U, Bm, V, S))
        torch.cuda.synchronize()
        solve_ms = 1e3 * (time.perf_counter() - t1)
        rows = np.random.default_rng(1).choice(m, min(m, 256), replace=False)
        rec = rel((U.double()[rows] @ Bm @ V.double().T).cpu().numpy(), inst.L0[rows])
    print(f"[bench] {K} iterations in {ms:.1f} ms; tolerance-driven solve {tinfo.iters} iterations {solve_ms:.1f} ms",
          file=sys.stderr, flush=True)
    flops = 6.0 * m * n * r
    achieved = flops * K / (ms * 1e-3) / 1e12
    cpu, parity = None, None
    if not args.no_cpu_baseline:
        import oracle
        oi = max(1, min(args.oracle_iters, 3))
        t1 = time.perf_counter()
        o = oracle.fradm(Md, r, inst.lam, mu0, fixed_iters=oi)
        tc = time.perf_counter() - t1
        with sfr.Solver(m, n, r, inst.lam, mu0, 1e-6, precision="f32", fixed_iters=oi) as s3:
            U3, B3, V3, S3, _ = s3.solve(M)
        torch.cuda.synchronize()
        rows = np.random.default_rng(2).choice(m, min(m, 128), replace=False)
        Lg = (U3.double()[rows] @ B3 @ V3.double().T).cpu().numpy()
        Lo = o["U"][rows] @ o["B"] @ o["V"].T
        parity = {"iterations": oi, "rel_err_L": rel(Lg, Lo),
                  "rel_err_S": rel(S3.double()[rows].cpu().numpy(), o["S"][rows]), "rows_sampled": int(rows.size)}
        cpu = {"value": oi / tc, "unit": "iters/s", "cores": 1, "kind": "oracle", "host": host_info(),
               "sample": f"{oi} FR-ADM iterations of the same {m}x{n} r={r} input, FP64, one thread ({tc:.1f} s)"}
        print(f"[bench] oracle {oi} iterations in {tc:.1f} s; parity {parity}", file=sys.stderr, flush=True)
    out = {
        "metric": "iters/s & solves/s at rel-err<=1e-5 vs FP64 oracle; %HBM roofline; p50/p99",
        "value": K / (ms * 1e-3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"FR-ADM large rank, m={m}, n={n}, r={r}, FP32, 10% outliers U[-1,1]",
                   "m": m, "n": n, "r": r, "lambda": inst.lam, "mu0": mu0, "seed": args.seed},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_MFMA_PEAK_TFLOPS, "traffic": None,
                     "kernel": "whole iteration (GEMM tiles, Grams, FP64 r x r algebra)",
                     "alg_flops_per_iteration": flops},
        "cpu_baseline": cpu,
        "solves_per_s": 1e3 / solve_ms,
        "solve_iters": tinfo.iters,
        "solve_ms": solve_ms,
        "recovery_rel_err_L": rec,
        "parity_vs_oracle": parity,
        "paper_context": "Table 2 (r = 0.1 m): FR-ADM 2000^2 r=200, 35 iterations in 7.53 s; 8000^2 r=800, 21 "
                         "iterations in 166 s (3.2 GHz desktop CPU; outliers in [-1,1])",
    }
    print(json.dumps(out), flush=True)


def serving(args):
    print(json.dumps(serving_measure(args)), flush=True)


def serving_measure(args):
    """Serving workload: a Poisson stream of independent decompositions
    (m U[64, 2048], n U[32, 512], r U{2..16}, 5-15 % outliers U[-50, 50],
    FP32, tol 1e-6 on the relative residual) through the continuous-batching
    server over sfr_solve_batch.  value = solves/s over the stream at the
    offered rate; also p50/p99 arrival-to-completion latency, the saturated
    capacity (every request present at t = 0), and the batched kernel's
    FP32 arithmetic rate in one full launch."""
    import torch
    import workloads
    import paper_1503_03004_amd as sfr
    from paper_1503_03004_amd import serve

    tol = 1e-6
    t0 = time.time()
    reqs = workloads.stream_device(seed=args.seed, count=args.requests, rate=args.rate)
    torch.cuda.synchronize()
    print(f"[serving] {len(reqs)} requests drawn on the device in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)

    def requests(arrivals=True, subset=None):
        src = reqs if subset is None else [reqs[i] for i in subset]
        return [serve.Request(M=q["M"], r=q["r"], lam=q["lam"], mu=q["mu"], tol=tol,
                              arrival=q["t"] if arrivals else 0.0) for q in src]

    server = serve.BatchServer(max_m=2048, max_n=512, max_r=16, workers=args.workers, capacity=256,
                               max_batch=args.max_batch or None)
    server.run(requests(False, range(min(64, len(reqs)))))          # warm-up, untimed
    # autotune the band-loop form per problem class and rank bucket on a sample of the stream
    tuned = server.tune(requests(False, range(min(256, len(reqs))))) if not args.no_autotune else {}
    torch.cuda.synchronize()
    print(f"[serving] autotuned forms: {tuned}", file=sys.stderr, flush=True)

    # ---- the stream at its offered rate
    server.launches, server.batch_sizes = 0, []
    run_reqs = requests(True)
    wall = server.run(run_reqs)
    lat_ms = [1e3 * q.latency for q in run_reqs]
    bad = [q.result[4].status for q in run_reqs if q.result[4].status < 0]
    iters = [q.result[4].iters for q in run_reqs]
    value = len(run_reqs) / wall
    mean_batch = float(np.mean(server.batch_sizes))
    stream_launches = server.launches
    print(f"[serving] offered {args.rate:.0f}/s: {value:.0f} solves/s, p50 {serve.percentile(lat_ms, 50):.2f} ms, "
          f"p99 {serve.percentile(lat_ms, 99):.2f} ms, {server.launches} launches (mean batch {mean_batch:.1f})",
          file=sys.stderr, flush=True)

    # ---- saturation: every request present at t = 0
    server.launches, server.batch_sizes = 0, []
    sat = requests(False)
    wall_sat = server.run(sat)
    capacity = len(sat) / wall_sat
    print(f"[serving] saturated: {capacity:.0f} solves/s", file=sys.stderr, flush=True)
    server.close()
    launch_server = {"solves_per_s": value, "p50_ms": serve.percentile(lat_ms, 50),
                     "p99_ms": serve.percentile(lat_ms, 99), "saturated_solves_per_s": capacity,
                     "launches": stream_launches, "mean_batch": mean_batch, "workers": args.workers,
                     "note": "launch batching (sfr_solve_batch): a worker launches what has arrived and "
                             "retires the batch when the launch returns"}

    # ---- continuous batching: the queue server (persistent kernels fed while they run)
    qserver = serve.QueueServer(max_m=2048, max_n=512, max_r=16, capacity=args.queue_capacity)
    qserver.run(requests(False, range(min(64, len(reqs)))))         # warm-up, untimed
    torch.cuda.synchronize()
    q_reqs = requests(True)
    q_wall = qserver.run(q_reqs)
    q_lat = [1e3 * q.latency for q in q_reqs]
    q_value = len(q_reqs) / q_wall
    q_bad = [q.result[4].status for q in q_reqs if q.result[4].status < 0]
    q_inflight = qserver.max_in_flight
    print(f"[serving] queue server, offered {args.rate:.0f}/s: {q_value:.0f} solves/s, "
          f"p50 {serve.percentile(q_lat, 50):.2f} ms, p99 {serve.percentile(q_lat, 99):.2f} ms, "
          f"max in flight {q_inflight}", file=sys.stderr, flush=True)
    q_sat = requests(False)
    q_wall_sat = qserver.run(q_sat)
    q_capacity = len(q_sat) / q_wall_sat
    print(f"[serving] queue server saturated: {q_capacity:.0f} solves/s", file=sys.stderr, flush=True)
    # the slowest single request alone (the floor of any tail latency)
    slow = max(range(len(reqs)), key=lambda i: reqs[i]["m"] * reqs[i]["n"] * reqs[i]["r"])
    alone = requests(False, [slow])
    qserver.run(alone)
    slowest_alone_ms = 1e3 * alone[0].latency
    qserver.close()
    print(f"[serving] slowest request alone (m n r largest): {slowest_alone_ms:.2f} ms", file=sys.stderr, flush=True)

    # ---- one full launch timed with HIP events: the kernel's arithmetic rate
    cap = 256
    idx = list(range(min(cap, len(reqs))))
    one = requests(False, idx)
    bs = sfr.BatchSolver(len(one), 2048, 512, 16)
    stream = torch.cuda.current_stream()
    bs.solve([(q.M, q.r, q.lam, q.mu, q.tol) for q in one], stream=stream)     # warm
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    res = bs.solve([(q.M, q.r, q.lam, q.mu, q.tol) for q in one], stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    launch_ms = e0.elapsed_time(e1)
    bs.close()
    flops = 0.0
    hbm = 0.0
    for q, rr in zip(one, res):
        m, n = q.M.shape
        k = rr[4].iters + 1               # sweeps run: the stopping test of k follows sweep k + 1
        flops += k * m * n * 6.0 * q.r    # l, p and q products: 3 r FMAs per element and sweep
        hbm += k * m * n * 12.0           # read M, read Y_{k-1}, write Y_k
    tflops = flops / (launch_ms * 1e-3) / 1e12
    gbs = hbm / (launch_ms * 1e-3) / 1e9

    # ---- the same requests through the single-problem engine (sfr_solve),
    # one solve after another on the same stream, handles created beforehand;
    # results compared with the batched ones at the same tolerance
    handles = [sfr.Solver(q.M.shape[0], q.M.shape[1], q.r, q.lam, q.mu, tol, precision="f32") for q in one]
    for h, q in zip(handles, one):
        h.solve(q.M, stream=stream)                                     # warm
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    singles = [h.solve(q.M, stream=stream) for h, q in zip(handles, one)]
    torch.cuda.synchronize()
    single_rate = len(one) / (time.perf_counter() - t1)
    for h in handles:
        h.close()
    same, dL, dS = 0, [], []
    for rb, ro in zip(res, singles):
        if rb[4].iters != ro[4].iters:
            continue
        same += 1
        Lb = (rb[0].double() @ rb[1] @ rb[2].double().T).cpu().numpy()
        Lo = (ro[0].double() @ ro[1] @ ro[2].double().T).cpu().numpy()
        dL.append(rel(Lb, Lo))
        dS.append(rel(rb[3].double().cpu().numpy(), ro[3].double().cpu().numpy()))
    # ---- the batched BF16 form (BF16 p and Q products while the residual is
    # above 1e-3, FP32 after) on the same requests, one launch
    bs16 = sfr.BatchSolver(len(one), 2048, 512, 16, bf16=True, bf16_tol=1e-3)
    bs16.solve([(q.M, q.r, q.lam, q.mu, q.tol) for q in one], stream=stream)     # warm
    torch.cuda.synchronize()
    e0.record(stream)
    res16 = bs16.solve([(q.M, q.r, q.lam, q.mu, q.tol) for q in one], stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    bf16_ms = e0.elapsed_time(e1)
    bs16.close()
    dL16 = []
    for rb, r16 in zip(res, res16):
        if rb[4].iters != r16[4].iters:
            continue
        Lb = (rb[0].double() @ rb[1] @ rb[2].double().T).cpu().numpy()
        L16 = (r16[0].double() @ r16[1] @ r16[2].double().T).cpu().numpy()
        dL16.append(max(rel(L16, Lb), rel(r16[3].double().cpu().numpy(), rb[3].double().cpu().numpy())))
    d16 = np.array(dL16) if dL16 else np.zeros(0)
    bf16_batched = {"solves_per_s": len(one) / (bf16_ms * 1e-3), "launch_ms": bf16_ms, "requests": len(one),
                    "same_iters_as_fp32_batched": len(dL16),
                    "max_rel_diff_vs_fp32_batched": max(dL16) if dL16 else None,
                    "median_rel_diff_vs_fp32_batched": float(np.median(d16)) if d16.size else None,
                    "within_1e-5_of_fp32_batched": int((d16 <= 1e-5).sum()),
                    "within_1e-3_of_fp32_batched": int((d16 <= 1e-3).sum()),
                    "note": "BF16 p and Q products while the residual > 1e-3 (matrix-core form, rank bucket >= 8), "
                            "FP32 iterations after; same tol as the FP32 per-instance solves"}
    print(f"[serving] batched BF16 form: {bf16_batched}", file=sys.stderr, flush=True)
    per_instance = {"solves_per_s": single_rate, "requests": len(one), "same_iters": same,
                    "max_rel_diff_L": max(dL) if dL else None, "max_rel_diff_S": max(dS) if dS else None,
                    "batched_one_launch_solves_per_s": len(one) / (launch_ms * 1e-3),
                    "note": "sfr_solve per request, sequential on one stream, FP32, same tol; diffs against "
                            "the batched results of the same requests"}
    print(f"[serving] per-problem engine: {single_rate:.0f} solves/s on the same {len(one)} requests "
          f"(batched, one launch: {len(one) / (launch_ms * 1e-3):.0f}/s); {per_instance}", file=sys.stderr, flush=True)

    # ---- FP64 oracle on a bounded sample of the stream: host rate and parity
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        errs = []
        t1 = time.perf_counter()
        done = 0
        for i, q in enumerate(run_reqs):
            Md = q.M.double().cpu().numpy()
            o = oracle.fradm(Md, q.r, q.lam, q.mu, tol=tol, max_iter=300)
            done += 1
            g = q.result
            if o["iters"] == g[4].iters:
                Lg = (g[0].double() @ g[1] @ g[2].double().T).cpu().numpy()
                errs.append(max(rel(Lg, o["U"] @ o["B"] @ o["V"].T), rel(g[3].double().cpu().numpy(), o["S"])))
            if time.perf_counter() - t1 > 12.0:
                break
        tc = time.perf_counter() - t1
        cpu = {"value": done / tc, "unit": "solves/s", "cores": 1, "kind": "oracle", "host": host_info(),
               "sample": f"the first {done} requests of the stream solved to tol {tol} in FP64 on one thread "
                         f"({tc:.1f} s)"}
        parity = {"requests_compared": len(errs), "max_rel_err": max(errs) if errs else None,
                  "note": "requests whose oracle solve stopped at the GPU's iteration count"}
        print(f"[serving] oracle: {done} solves in {tc:.1f} s; parity {parity}", file=sys.stderr, flush=True)

    out = {
        "metric": "solves/s of a Poisson stream of independent decompositions; p50/p99 latency",
        "value": q_value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(run_reqs),
        "warmup": 64,
        "ms_per_step": 1e3 * q_wall / len(q_reqs),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson {args.rate:.0f} req/s, m U[64,2048], n U[32,512], r U{{2..16}}, "
                               f"5-15% outliers U[-50,50], FP32, tol {tol}",
                   "requests": len(run_reqs), "rate": args.rate, "server": "queue (persistent kernels)",
                   "queue_capacity": qserver.capacity, "seed": args.seed},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": None, "kernel": "batch_kernel",
                     "launch_ms": launch_ms, "problems_per_launch": len(one), "hbm_alg_gbs": gbs},
        "cpu_baseline": cpu,
        "p50_ms": serve.percentile(q_lat, 50),
        "p99_ms": serve.percentile(q_lat, 99),
        "saturated_solves_per_s": q_capacity,
        "max_in_flight": q_inflight,
        "failed_queue": len(q_bad),
        "slowest_request_alone_ms": slowest_alone_ms,
        "launch_server": launch_server,
        "per_instance_fp32": per_instance,
        "bf16_batched": bf16_batched,
        "autotuned": {f"{'narrow' if k[0] else 'wide'} r<={k[1]}": v for k, v in tuned.items()},
        "median_iters": float(np.median(iters)),
        "failed": len(bad),
        "parity_vs_oracle": parity,
    }
    return out


if __name__ == "__main__":
    main()
