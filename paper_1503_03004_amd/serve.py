"""Continuous-batching front end for many independent decompositions.

Requests (M, r, lambda, mu_0, tol) arrive over time; every problem is solved
by the batched FR-ADM kernel (one workgroup per problem, the whole iteration
on one CU; sfr_solve_batch).  The server keeps `workers` batched handles,
each with its own HIP stream and host thread, so up to `workers` launches
are on the GPU at once: a worker takes every request that has arrived (up to
its capacity), launches, and when the launch returns retires the batch and
takes the next one.  A request's latency is the time from its arrival to the
return of the launch that solved it.

Admission is by device memory: each handle holds `capacity` workspace slots
sized for the largest admitted problem, and the capacity is cut so that all
handles fit in a fraction of the free HBM reported by the runtime.  Requests
beyond the handles' limits (n > 512, r > 16, m > max_m) are rejected at
submission.

QueueServer is the continuous form: persistent kernels take requests one by
one while they run (no launch boundary), admission is by free slot and by
free HBM at admission time.

This module only schedules: all arithmetic runs in the HIP library.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

from ._binding import BatchSolver, SFRError

# limits of the batched kernel (sfr_create_batch)
MAX_N = 512
MAX_R = 16


def slot_bytes(max_m: int, max_n: int) -> int:
    """Device workspace of one batched slot: two Y buffers (max_m x ldy),
    two P (max_m x 16) and two Q (max_n x 16) buffers, FP32, and its
    descriptor."""
    ldy = (max_n + 3) // 4 * 4
    return 4 * (2 * max_m * ldy + 2 * max_m * 16 + 2 * max_n * 16) + 256


@dataclass
class Request:
    M: object                 # float32 CUDA tensor, row-major
    r: int
    lam: float
    mu: float
    tol: float
    arrival: float = 0.0      # seconds after the start of the run
    # filled by the server
    start: float = field(default=float("nan"))
    done: float = field(default=float("nan"))
    result: tuple | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class BatchServer:
    def __init__(self, max_m: int, max_n: int = MAX_N, max_r: int = MAX_R, *, workers: int = 4,
                 capacity: int = 256, max_batch: int | None = None, hbm_fraction: float = 0.5,
                 want_S: bool = True, rho: float = 1.5, mu_bar: float = 1e9, max_iter: int = 300):
        import torch
        if not (1 <= max_n <= MAX_N and 1 <= max_r <= MAX_R and max_m >= 1):
            raise ValueError("batched limits: n <= 512, r <= 16")
        free, _ = torch.cuda.mem_get_info()
        per_slot = slot_bytes(max_m, max_n)
        fit = int(free * hbm_fraction) // (workers * per_slot)
        if fit < 1:
            raise MemoryError("not enough free device memory for one batched slot per worker")
        self.capacity = min(int(capacity), fit)
        # requests per launch: smaller launches leave room for the next ones
        # (a launch lasts as long as its slowest problem)
        self.max_batch = self.capacity if max_batch is None else max(1, min(int(max_batch), self.capacity))
        self.max_m, self.max_n, self.max_r = int(max_m), int(max_n), int(max_r)
        self.want_S = want_S
        self.workers = int(workers)
        self.solvers = [BatchSolver(self.capacity, max_m, max_n, max_r, rho=rho, mu_bar=mu_bar, max_iter=max_iter)
                        for _ in range(self.workers)]
        self.streams = [torch.cuda.Stream() for _ in range(self.workers)]
        self.classes = worker_classes(self.workers)
        self.launches = 0
        self.batch_sizes: list[int] = []

    def tune(self, sample: list[Request]) -> dict:
        """Autotune every worker's handle on a sample of requests (the
        band-loop form per problem class and rank bucket, sfr_tune_batch).
        Returns the table chosen by the first handle."""
        items = [(q.M, q.r, q.lam, q.mu, q.tol) for q in sample[: self.capacity] if self.admissible(q)]
        table = {}
        for w, bs in enumerate(self.solvers):
            t = bs.autotune(items, stream=self.streams[w])
            if w == 0:
                table = t
        return table

    def admissible(self, req: Request) -> bool:
        m, n = req.M.shape
        return m <= self.max_m and n <= self.max_n and 1 <= req.r <= min(self.max_r, m, n)

    def run(self, requests: list[Request]) -> float:
        """Release the requests at their arrival times (seconds from now),
        solve them all, and return the wall time of the run.  Each request
        gets .start, .done (seconds from the start) and .result =
        (U, B, V, S, Info)."""
        import torch
        for q in requests:
            if not self.admissible(q):
                raise ValueError("request beyond the server's limits")
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
        # one queue per class: narrow problems (n <= 128) run in the library's
        # second kernel variant; keeping the classes apart means a launch
        # never needs the handle's side stream, so the streams in use stay
        # at one per worker (HIP maps streams onto a few hardware queues, and
        # launches that share one run one after the other)
        queues = {False: collections.deque(), True: collections.deque()}
        cv = threading.Condition()
        state = {"released": 0, "error": None}
        total = len(requests)
        t0 = time.perf_counter()

        def worker(w: int):
            bs, st = self.solvers[w], self.streams[w]
            pending = queues[self.classes[w]]
            if st is not None:
                torch.cuda.set_stream(st)
            while True:
                with cv:
                    while not pending and state["released"] < total and state["error"] is None:
                        cv.wait()
                    if state["error"] is not None or (not pending and state["released"] >= total):
                        return
                    batch = [pending.popleft() for _ in range(min(len(pending), self.max_batch))]
                now = time.perf_counter() - t0
                for q in batch:
                    q.start = now
                try:
                    out = bs.solve([(q.M, q.r, q.lam, q.mu, q.tol) for q in batch], want_S=self.want_S,
                                   stream=st, raise_on_error=False)
                except SFRError as e:          # argument or device failure: stop the run
                    with cv:
                        state["error"] = e
                        cv.notify_all()
                    return
                done = time.perf_counter() - t0
                for q, res in zip(batch, out):
                    q.done = done
                    q.result = res
                with cv:
                    self.launches += 1
                    self.batch_sizes.append(len(batch))

        threads = [threading.Thread(target=worker, args=(w,), daemon=True) for w in range(self.workers)]
        for t in threads:
            t.start()
        for i in order:
            q = requests[i]
            delay = q.arrival - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            with cv:
                queues[is_narrow(q)].append(q)
                state["released"] += 1
                cv.notify_all()
        with cv:
            cv.notify_all()
        for t in threads:
            t.join()
        if state["error"] is not None:
            raise state["error"]
        return time.perf_counter() - t0

    def close(self):
        for s in self.solvers:
            s.close()
        self.solvers = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class QueueServer:
    """Continuous batching on the queue form of a batched handle
    (sfr_queue_*): persistent kernels take problems one by one while they
    run, so a request is submitted the moment it arrives (if a workspace
    slot and device memory are free), starts as soon as a workgroup is free,
    and is collected as soon as it is solved -- no launch boundary, and no
    wait for the slowest problem of a batch.

    Admission: a request needs one of the handle's `capacity` workspace
    slots (sized for the largest admissible problem, all of them cut to fit
    `hbm_fraction` of the free HBM at construction) and, at admission time,
    room in device memory for its outputs: the free HBM the runtime reports
    is read before each round of admissions, and requests wait while it is
    below `reserve_bytes`.  A request's latency is the time from its arrival
    to the poll that collects its result.

    This class only schedules: all arithmetic runs in the HIP library."""

    def __init__(self, max_m: int, max_n: int = MAX_N, max_r: int = MAX_R, *, capacity: int = 1024,
                 hbm_fraction: float = 0.5, reserve_bytes: int = 1 << 30, want_S: bool = True,
                 grid_large: int = 0, grid_small: int = 0, rho: float = 1.5, mu_bar: float = 1e9,
                 max_iter: int = 300):
        import torch
        if not (1 <= max_n <= MAX_N and 1 <= max_r <= MAX_R and max_m >= 1):
            raise ValueError("batched limits: n <= 512, r <= 16")
        free, _ = torch.cuda.mem_get_info()
        fit = int(free * hbm_fraction) // slot_bytes(max_m, max_n)
        if fit < 1:
            raise MemoryError("not enough free device memory for one batched slot")
        self.capacity = min(int(capacity), fit)
        self.max_m, self.max_n, self.max_r = int(max_m), int(max_n), int(max_r)
        self.want_S = want_S
        self.reserve_bytes = int(reserve_bytes)
        self.grid = (int(grid_large), int(grid_small))
        self.solver = BatchSolver(self.capacity, max_m, max_n, max_r, rho=rho, mu_bar=mu_bar, max_iter=max_iter)
        self.max_in_flight = 0
        self.held_for_memory = 0

    def admissible(self, req: Request) -> bool:
        m, n = req.M.shape
        return m <= self.max_m and n <= self.max_n and 1 <= req.r <= min(self.max_r, m, n)

    def run(self, requests: list[Request]) -> float:
        """Release the requests at their arrival times (seconds from now),
        solve them all, and return the wall time of the run.  Each request
        gets .start (submission), .done (collection, seconds from the start)
        and .result = (U, B, V, S, Info)."""
        import torch
        for q in requests:
            if not self.admissible(q):
                raise ValueError("request beyond the server's limits")
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
        bs = self.solver
        bs.queue_start(*self.grid)
        waiting = collections.deque()
        in_flight = {}
        nxt = 0
        remaining = len(requests)
        t0 = time.perf_counter()
        try:
            while remaining:
                now = time.perf_counter() - t0
                while nxt < len(order) and requests[order[nxt]].arrival <= now:
                    waiting.append(requests[order[nxt]])
                    nxt += 1
                progressed = False
                if waiting:
                    free, _ = torch.cuda.mem_get_info()
                    if free < self.reserve_bytes:
                        self.held_for_memory += 1
                    else:
                        while waiting:
                            q = waiting[0]
                            t = bs.queue_submit(q.M, q.r, q.lam, q.mu, q.tol, want_S=self.want_S)
                            if t is None:
                                break          # every slot in flight: wait for a retirement
                            waiting.popleft()
                            q.start = time.perf_counter() - t0
                            in_flight[t] = q
                            progressed = True
                        self.max_in_flight = max(self.max_in_flight, len(in_flight))
                for t in list(in_flight):
                    res = bs.queue_poll(t)
                    if res is not None:
                        q = in_flight.pop(t)
                        q.done = time.perf_counter() - t0
                        q.result = res
                        remaining -= 1
                        progressed = True
                if not progressed:
                    nxt_t = requests[order[nxt]].arrival if nxt < len(order) else None
                    wait = 5e-5 if nxt_t is None else min(5e-5, max(0.0, nxt_t - (time.perf_counter() - t0)))
                    if wait > 0:
                        time.sleep(wait)
        finally:
            bs.queue_stop()
        return time.perf_counter() - t0

    def close(self):
        if self.solver is not None:
            self.solver.close()
        self.solver = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


NARROW_N = 128   # problems with at most this many columns use the narrow kernel variant


def is_narrow(req: Request) -> bool:
    return req.M.shape[1] <= NARROW_N


def worker_classes(workers: int) -> list[bool]:
    """Class served by each worker (True: narrow).  About a fifth of the
    stream is narrow (n uniform in [32, 512]), and narrow problems are the
    cheaper ones, so one worker in four serves them (at least one)."""
    if workers == 1:
        raise ValueError("the server needs two workers or more (one per problem class)")
    nn = max(1, workers // 4)
    return [False] * (workers - nn) + [True] * nn


def percentile(values, p: float) -> float:
    """p-th percentile (0..100) by linear interpolation between order
    statistics."""
    v = sorted(values)
    if not v:
        return float("nan")
    x = (len(v) - 1) * p / 100.0
    lo = int(x)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (x - lo)
