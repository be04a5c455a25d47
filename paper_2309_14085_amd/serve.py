"""Serving loop: build + solve requests admitted by an HBM budget, overlapping on one GPU.

Requests arrive over time (Poisson arrivals).  A request is admitted, in
arrival order, as soon as a worker slot is free and its estimated device
memory fits the remaining HBM budget.  Each worker builds the request's
representation (host, through h2s_build) and solves its right-hand sides
(h2s_solve) on a stream of its own, so the device work of admitted requests
overlaps.  The C calls release the Python interpreter lock, so the host
builds of different requests also run side by side.

The system solved is the second-kind form of the paper's kernel systems:
with quadrature weight w = |domain| / N on the kernel, (w K + I) x = b, i.e.
(K + I / w) x = b / w; `shift = N / |domain|` is passed to h2s_build and b is
scaled by 1 / w.  Latency is completion time minus arrival time.

Every numeric step runs in libh2s.so; this module only schedules.
"""
import math
import os
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import h2s, inputs


@dataclass
class Request:
    rid: int
    arrival: float        # seconds after the start of the run
    d: int
    n: int
    nrhs: int
    seed: int
    eps: float = 0.0      # 0: 1e-8 in 2D, 1e-6 in 3D

    @property
    def kind(self):
        return h2s.LOG_R if self.d == 2 else h2s.INV_R

    @property
    def tol(self):
        return self.eps or (1e-8 if self.d == 2 else 1e-6)

    @property
    def shift(self):
        return self.n / float(2 ** self.d)  # 1 / w, the domain [-1, 1]^d has measure 2^d


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = 0.0
    done: float = 0.0
    build_s: float = 0.0
    solve_s: float = 0.0
    est_bytes: int = 0
    device_bytes: int = 0
    iterations: list = field(default_factory=list)
    residuals: list = field(default_factory=list)
    converged: bool = False
    x: np.ndarray = None
    error: str = ""

    @property
    def latency(self):
        return self.done - self.arrival


def make_requests(count, rate, seed, n_range=(16384, 131072), n_range_3d=None, nrhs_max=4):
    """count requests with exponential inter-arrival times (rate per second), d in {2, 3}
    uniform, N log-uniform in n_range (n_range_3d for d = 3), 1..nrhs_max right-hand sides."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        d = int(rng.integers(2, 4))
        lo, hi = n_range if d == 2 or n_range_3d is None else n_range_3d
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        out.append(Request(i, t, d, n, int(rng.integers(1, nrhs_max + 1)), 10_000 + 7 * i))
    return out


def estimate_bytes(req):
    """Device memory of one request: representation in FP64 and FP32, solve workspace
    (restart 50), right-hand sides and solutions; per point, from measured builds."""
    per_point = 3600 if req.d == 2 else 16000
    return req.n * (per_point + 51 * 8 + 16 * req.nrhs)


class Server:
    def __init__(self, hbm_budget_bytes=16 << 30, workers=4, host_threads=None, keep_x=False):
        self.budget = int(hbm_budget_bytes)
        self.workers = int(workers)
        cores = min(os.cpu_count() or 1, 16)
        self.host_threads = host_threads or max(1, cores // self.workers)
        self.keep_x = keep_x

    def run(self, requests):
        import torch
        h2s.load()
        dev = torch.device("cuda:0")
        pending = queue.Queue()      # arrived, not yet admitted (arrival order)
        admitted = queue.Queue()     # admitted, waiting for a worker
        results = {r.rid: Result(r.rid, r.arrival) for r in requests}
        lock = threading.Condition()
        state = {"used": 0, "inflight": 0, "peak_inflight": 0, "peak_used": 0, "remaining": len(requests)}
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        def arrivals():
            for r in sorted(requests, key=lambda r: r.arrival):
                delay = r.arrival - now()
                if delay > 0:
                    time.sleep(delay)
                with lock:
                    pending.put(r)
                    lock.notify_all()

        def admitter():
            served = 0
            while served < len(requests):
                r = pending.get()
                est = min(estimate_bytes(r), self.budget)
                with lock:
                    while state["inflight"] >= self.workers or state["used"] + est > self.budget:
                        lock.wait()
                    state["used"] += est
                    state["inflight"] += 1
                    state["peak_inflight"] = max(state["peak_inflight"], state["inflight"])
                    state["peak_used"] = max(state["peak_used"], state["used"])
                res = results[r.rid]
                res.admitted, res.est_bytes = now(), est
                admitted.put(r)
                served += 1
            for _ in range(self.workers):
                admitted.put(None)

        def worker():
            stream = torch.cuda.Stream()
            while True:
                r = admitted.get()
                if r is None:
                    return
                res = results[r.rid]
                try:
                    self._serve_one(r, res, stream, dev, torch)
                except Exception as e:  # the request fails, the server goes on
                    res.error = f"{type(e).__name__}: {e}"
                res.done = now()
                with lock:
                    state["used"] -= res.est_bytes
                    state["inflight"] -= 1
                    state["remaining"] -= 1
                    lock.notify_all()

        threads = [threading.Thread(target=arrivals), threading.Thread(target=admitter)]
        threads += [threading.Thread(target=worker) for _ in range(self.workers)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        wall = now()
        out = [results[r.rid] for r in requests]
        return out, self.summary(out, requests, wall, state)

    def _serve_one(self, r, res, stream, dev, torch):
        pts = inputs.uniform_points(r.n, r.d, r.seed)
        B = inputs.normal_rhs(r.n, r.nrhs, r.seed + 1) * r.shift  # b / w
        t = time.perf_counter()
        T = h2s.build(pts, kind=r.kind, leaf_size=64, eps=r.tol, shift=r.shift, host_threads=self.host_threads,
                      stream=stream)
        res.build_s = time.perf_counter() - t
        try:
            with torch.cuda.stream(stream):
                b = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev, non_blocking=False).t()
                t = time.perf_counter()
                x, info = T.solve(b if r.nrhs > 1 else b[:, 0].contiguous(), rtol=1e-8, stream=stream,
                                  raise_on_fail=False)
                stream.synchronize()
                res.solve_s = time.perf_counter() - t
                res.iterations = [i["iterations"] for i in info]
                res.residuals = [i["residual"] for i in info]
                res.converged = all(i["converged"] for i in info)
                res.device_bytes = T.stats()["device_bytes"]
                if self.keep_x:
                    res.x = x.cpu().numpy()
        finally:
            T.free()

    @staticmethod
    def summary(out, requests, wall, state):
        ok = [o for o in out if not o.error]
        lat = np.array([o.latency for o in ok]) if ok else np.array([np.nan])
        by_id = {o.rid: o for o in out}
        pts_rhs = sum(r.n * r.nrhs for r in requests if not by_id[r.rid].error)
        return {"requests": len(out), "failed": len(out) - len(ok), "converged": sum(o.converged for o in ok),
                "wall_s": wall, "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean()), "throughput_req_per_s": len(ok) / wall,
                "points_x_rhs_per_s": pts_rhs / wall, "peak_inflight": state["peak_inflight"],
                "peak_budget_used_bytes": state["peak_used"],
                "mean_build_s": float(np.mean([o.build_s for o in ok])) if ok else float("nan"),
                "mean_solve_s": float(np.mean([o.solve_s for o in ok])) if ok else float("nan"),
                "max_iterations": max((max(o.iterations) for o in ok if o.iterations), default=0),
                "max_residual": max((max(o.residuals) for o in ok if o.residuals), default=float("nan"))}
