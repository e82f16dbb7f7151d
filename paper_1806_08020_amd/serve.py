"""Continuous-batching server for eigen-solves (the served production form).

Requests of uneven size arrive over time (seeded Poisson arrivals).  The
request loop admits them as device memory and slots free up:

* admission is by HBM footprint: the CSR arrays, start vectors and the
  solve's workspace must fit the remaining budget;
* small solves (n <= small_n) go to the batched engine (`ppa.Batch`): every
  engine step is one launch that advances all admitted small solves, one
  workgroup each, and new solves join free slots between steps;
* larger solves run whole on worker threads, each with its own HIP stream,
  through the single-solve path (`ppa.Poly.build` + `ppa.eigs`), so their
  kernels overlap on the device with the batch launches and with each other;
* each request's latency runs from its arrival to its result.

All numerical work happens in libppa; this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

from . import ppa
from . import workloads as W


@dataclass
class Request:
    rid: int
    csr: W.CSR
    d: int
    m: int
    k: int
    nev: int
    b: np.ndarray
    v0: np.ndarray
    rtol: float = 1e-8
    max_cycles: int = 30
    arrival: float = 0.0          # seconds after the start of the run
    precision: str = "f64"        # "f64" or "mixed" (FP32 pi(A)v on either path)
    graph: bool = False           # stream path: replay restart cycles from HIP graphs
    lowsync: bool = False         # stream path: delayed-reorthogonalisation Gram-Schmidt


@dataclass
class Completion:
    rid: int
    result: ppa.EigsOut | None
    error: str | None
    path: str                     # "batch" or "stream"
    arrival: float
    admitted: float
    finished: float
    footprint: int
    n: int

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def csr_bytes(csr: W.CSR) -> int:
    return int(csr.nnz) * 12 + 4 * (csr.n + 1)


def stream_footprint(rq: Request) -> int:
    """Upper bound of the device bytes of a single-solve request: CSR (+FP32
    copy), b, v0, the two Krylov bases and temporaries, the GMRES basis."""
    n = rq.csr.n
    ld = (n + 31) // 32 * 32
    f = csr_bytes(rq.csr) + 16 * n
    if rq.precision == "mixed":
        f += 4 * rq.csr.nnz + 4 * 6 * n
    f += 8 * ld * (2 * (rq.m + 1) + 4 * rq.nev + 12)
    f += 8 * ld * (rq.d + 5) + 8 * ld
    return int(f)


def batch_footprint(rq: Request) -> int:
    return csr_bytes(rq.csr) + 16 * rq.csr.n + ppa.batch_workspace_bytes(
        rq.csr.n, rq.d, rq.m, rq.nev, int(rq.csr.nnz), rq.precision)


def _solve_stream(rq: Request, stream: torch.cuda.Stream, window: str = "auto",
                  tune: bool = True) -> ppa.EigsOut:
    with torch.cuda.stream(stream):
        A = ppa.Matrix(rq.csr, want_f32=(rq.precision == "mixed"), window=window, tune=tune)
        b = torch.as_tensor(rq.b, device="cuda")
        v0 = torch.as_tensor(rq.v0, device="cuda")
        P = ppa.Poly.build(A, rq.d, b, lowsync=rq.lowsync)
        r = ppa.eigs(A, P, v0, rq.m, rq.k, rq.nev, rtol=rq.rtol, max_cycles=rq.max_cycles,
                     precision=rq.precision, graph=rq.graph, lowsync=rq.lowsync)
        stream.synchronize()
    return r


class Server:
    def __init__(self, hbm_budget: int, max_slots: int = 256, small_n: int = 16384,
                 stream_workers: int = 3, matrix_window: str = "auto", matrix_tune: bool = False):
        """matrix_window, matrix_tune: SpMV kernel choice for the matrices of
        whole solves (ppa.Matrix's ``window`` and ``tune``).  A served matrix
        is used for one solve, so by default it skips the timing of kernel
        variants at creation, which would cost more than it saves."""
        self.budget = int(hbm_budget)
        self.matrix_window = matrix_window
        self.matrix_tune = matrix_tune
        self.small_n = small_n
        self.batch_stream = torch.cuda.Stream()
        self.batch = ppa.Batch(max_slots, stream=self.batch_stream)
        self.max_slots = max_slots
        self.workers = stream_workers
        self.streams = [torch.cuda.Stream() for _ in range(stream_workers)]
        self.pool = ThreadPoolExecutor(max_workers=stream_workers)
        self.stats = {"batch_steps": 0, "max_in_flight": 0, "max_used_bytes": 0}

    def is_small(self, rq: Request) -> bool:
        return rq.csr.n <= self.small_n and rq.m <= 64 and rq.nev <= 32 and rq.d <= 126

    def run(self, requests: list[Request], clock=time.perf_counter) -> list[Completion]:
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting: deque[Request] = deque()
        in_batch: dict[int, tuple] = {}      # slot -> (req, admitted, footprint)
        in_stream: dict = {}                 # future -> (req, admitted, footprint, stream)
        free_streams = list(self.streams)
        used = 0
        done: list[Completion] = []
        t0 = clock()
        total = len(requests)
        for rq in requests:
            fp = batch_footprint(rq) if self.is_small(rq) else stream_footprint(rq)
            if fp > self.budget:
                raise ValueError(f"request {rq.rid} needs {fp} bytes, above the whole budget")
        while len(done) < total:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission: in arrival order, every request that fits now
            for rq in list(waiting):
                small = self.is_small(rq)
                fp = batch_footprint(rq) if small else stream_footprint(rq)
                if used + fp > self.budget:
                    continue
                if small:
                    if len(in_batch) >= self.max_slots:
                        continue
                    with torch.cuda.stream(self.batch_stream):
                        rp = torch.as_tensor(rq.csr.rowptr).to("cuda", non_blocking=False)
                        ci = torch.as_tensor(rq.csr.colind).to("cuda", non_blocking=False)
                        va = torch.as_tensor(rq.csr.vals).to("cuda", non_blocking=False)
                        b = torch.as_tensor(rq.b).to("cuda")
                        v0 = torch.as_tensor(rq.v0).to("cuda")
                    slot = self.batch.submit(rp, ci, va, rq.d, rq.m, rq.k, rq.nev, b, v0,
                                             rtol=rq.rtol, max_cycles=rq.max_cycles,
                                             precision=rq.precision)
                    if slot is None:
                        continue
                    in_batch[slot] = (rq, clock() - t0, fp)
                else:
                    if not free_streams:
                        continue
                    st = free_streams.pop()
                    fut = self.pool.submit(_solve_stream, rq, st, self.matrix_window, self.matrix_tune)
                    in_stream[fut] = (rq, clock() - t0, fp, st)
                used += fp
                waiting.remove(rq)
            self.stats["max_in_flight"] = max(self.stats["max_in_flight"], len(in_batch) + len(in_stream))
            self.stats["max_used_bytes"] = max(self.stats["max_used_bytes"], used)
            progressed = False
            if in_batch:
                fin, _ = self.batch.step()
                self.stats["batch_steps"] += 1
                progressed = True
                t = clock() - t0
                for slot in fin:
                    rq, ta, fp = in_batch.pop(slot)
                    try:
                        res, err = self.batch.result(slot), None
                    except ppa.PPAError as e:
                        res, err = None, str(e)
                    done.append(Completion(rq.rid, res, err, "batch", rq.arrival, ta, t, fp, rq.csr.n))
                    used -= fp
            for fut in [f for f in in_stream if f.done()]:
                rq, ta, fp, st = in_stream.pop(fut)
                try:
                    res, err = fut.result(), None
                except ppa.PPAError as e:
                    res, err = None, str(e)
                done.append(Completion(rq.rid, res, err, "stream", rq.arrival, ta, clock() - t0, fp, rq.csr.n))
                used -= fp
                free_streams.append(st)
                progressed = True
            if not progressed:
                if in_stream:
                    time.sleep(0.0005)
                elif pending and not waiting:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - (clock() - t0))))
        return sorted(done, key=lambda c: c.rid)

    def close(self):
        self.pool.shutdown(wait=True)


# ---------------------------------------------------------------- served mix
def served_mix(count: int = 512, seed: int = 5, rate: float = 50.0, side_max: int = 1000,
               max_cycles: int = 30, precision: str = "f64", graph: bool = False) -> list[Request]:
    """The served workload: 2-D convection-diffusion operators with grid side
    log-uniform in [32, side_max], beta*h uniform in [0, 0.8], nev uniform in
    {5..20}, d uniform in {10..60}, Arnoldi(max(30, 2(nev+5)), nev+5),
    rtol 1e-8, Poisson arrivals at `rate` per second."""
    rng = np.random.default_rng([seed, 2])
    t = 0.0
    out = []
    for i in range(count):
        side = int(round(np.exp(rng.uniform(np.log(32), np.log(side_max)))))
        bh = float(rng.uniform(0.0, 0.8))
        nev = int(rng.integers(5, 21))
        d = int(rng.integers(10, 61))
        t += float(rng.exponential(1.0 / rate))
        csr = W.convdiff_2d(side, bh)
        b, v0 = W.start_vectors(csr.n, 1000 * seed + i)
        k = nev + 5
        m = max(30, 2 * k)
        out.append(Request(i, csr, d, m, k, nev, b, v0, 1e-8, max_cycles, t, precision, graph))
    return out


def summarize(done: list[Completion], wall: float) -> dict:
    lat = np.array([c.latency for c in done])
    ok = [c for c in done if c.result is not None]
    pairs = sum(c.result.nconv for c in ok)
    conv = sum(1 for c in ok if c.result.converged)
    return {
        "requests": len(done),
        "converged": conv,
        "errors": sum(1 for c in done if c.error),
        "eigenpairs": int(pairs),
        "eigenpairs_per_s": pairs / wall if wall > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "wall_s": wall,
        "batch_requests": sum(1 for c in done if c.path == "batch"),
        "stream_requests": sum(1 for c in done if c.path == "stream"),
        "by_path": {path: _path_summary([c for c in done if c.path == path])
                    for path in ("batch", "stream")},
    }


def _path_summary(done: list[Completion]) -> dict:
    """Latency and work of the requests one path served (batched engine or
    whole solves on worker streams)."""
    if not done:
        return {"requests": 0}
    lat = np.array([c.latency for c in done])
    ok = [c for c in done if c.result is not None]
    return {"requests": len(done), "converged": sum(1 for c in ok if c.result.converged),
            "eigenpairs": int(sum(c.result.nconv for c in ok)),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_n": float(np.mean([c.n for c in done])),
            "fp32_cycles": int(sum(c.result.fp32_cycles for c in ok)),
            "cycles": int(sum(c.result.cycles for c in ok))}
