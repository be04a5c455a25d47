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
import sys
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


# Device bytes per point of a request's representation in FP64 and FP32 at the largest sizes
# served (from measured builds; the floor of the admission estimate); and of the multi-RHS product buffers of one
# precision (32 columns of charges, near-field potentials and coefficients), which a solve of
# several right-hand sides allocates for its inner and its FP64 products.
REP_BYTES_PER_POINT = {2: 4500, 3: 16000}
BATCH_BYTES_PER_POINT = {2: 1300, 3: 2600}


def batch_bytes(req):
    return 2 * BATCH_BYTES_PER_POINT[req.d] * req.n if req.nrhs > 1 else 0


def solve_bytes(req, restart=50):
    """The library's solve workspace of a request: Krylov basis, work vectors and state of every
    column solved in lockstep ((restart + 1) + 3 vectors each) and one column's workspace."""
    cols = min(req.nrhs, 32)
    return req.n * 8 * ((restart + 1 + 3) * cols + (restart + 1 + 3))


def estimate_bytes(req, rep_per_point=None):
    """Device memory of one request: its representation (rep_per_point[d] bytes per point, by
    default REP_BYTES_PER_POINT), the multi-RHS product buffers when it has several right-hand
    sides, its solve workspace, and b and x."""
    per_point = (rep_per_point or REP_BYTES_PER_POINT)[req.d]
    return int(req.n * per_point) + batch_bytes(req) + solve_bytes(req) + 16 * req.n * req.nrhs


class CachingAllocator:
    """The library's device memory from PyTorch's caching allocator (installed with
    h2s_set_allocator): a finished request's blocks stay cached in the process and serve the next
    request's representation and Krylov workspace without hipMalloc / hipFree.  Blocks are freed
    only after the request's stream has finished with them (the solve synchronises before
    h2s_free), so a reused block is never still in use."""

    def __init__(self, torch):
        self.torch = torch
        self.lock = threading.Lock()
        self.live, self.bytes, self.peak, self.calls = {}, 0, 0, 0

    def alloc(self, nbytes):
        p = self.torch.cuda.caching_allocator_alloc(nbytes, device=0)
        with self.lock:
            self.live[p] = nbytes
            self.bytes += nbytes
            self.peak = max(self.peak, self.bytes)
            self.calls += 1
        return p

    def free(self, p):
        with self.lock:
            self.bytes -= self.live.pop(p, 0)
        self.torch.cuda.caching_allocator_delete(p)

    def install(self):
        h2s.set_allocator(self.alloc, self.free)

    @staticmethod
    def uninstall():
        h2s.set_allocator()


class Server:
    """Admission: a request waits until a worker is free and its estimated device bytes fit the
    remaining budget.  The estimate of the representation is REP_BYTES_PER_POINT, raised by what
    h2s_get_stats reports for finished requests (the largest bytes per point seen for each d,
    times 1.25).  Bytes per point grow with N (boxes on the boundary have fewer neighbours, and
    small trees have more of them), so a floor measured at the largest sizes keeps what was
    learned from small requests from under-reserving large ones."""

    def __init__(self, hbm_budget_bytes=16 << 30, workers=4, host_threads=None, keep_x=False, allocator=None,
                 progress=None):
        self.progress = progress  # a label: one line per finished request goes to stderr
        self.budget = int(hbm_budget_bytes)
        self.workers = int(workers)
        cores = min(os.cpu_count() or 1, 16)
        self.host_threads = host_threads or max(1, cores // self.workers)
        self.keep_x = keep_x
        self.allocator = allocator
        self.learned = {}  # d -> representation bytes per point measured so far

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
                with lock:
                    per = {d: max(REP_BYTES_PER_POINT[d], 1.25 * self.learned.get(d, 0.0)) for d in (2, 3)}
                est = min(estimate_bytes(r, per), self.budget)
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
                if self.progress:
                    print(f"{self.progress}: request {r.rid} d={r.d} n={r.n} nrhs={r.nrhs} latency {res.latency:.2f} s "
                          f"(build {res.build_s:.2f} s){' ' + res.error if res.error else ''}", file=sys.stderr, flush=True)
                with lock:
                    if res.device_bytes:
                        rep = max(res.device_bytes - solve_bytes(r) - batch_bytes(r), 0) / r.n
                        self.learned[r.d] = max(self.learned.get(r.d, 0.0), rep)
                    state["used"] -= res.est_bytes
                    state["inflight"] -= 1
                    state["remaining"] -= 1
                    lock.notify_all()

        if self.allocator is not None:
            self.allocator.install()
        threads = [threading.Thread(target=arrivals), threading.Thread(target=admitter)]
        threads += [threading.Thread(target=worker) for _ in range(self.workers)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        if self.allocator is not None:
            self.allocator.uninstall()
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
                "max_residual": max((max(o.residuals) for o in ok if o.residuals), default=float("nan")),
                "max_device_bytes": max((o.device_bytes for o in ok), default=0),
                "est_over_device_bytes_min": min((o.est_bytes / o.device_bytes for o in ok if o.device_bytes),
                                                 default=float("nan")),
                "est_worst_request": min(([r.d, r.n, r.nrhs, by_id[r.rid].est_bytes, by_id[r.rid].device_bytes]
                                          for r in requests if by_id[r.rid].device_bytes and not by_id[r.rid].error),
                                         key=lambda v: v[3] / v[4], default=None)}


def run_loads(count, loads=(0.5, 0.9), calib=16, seed=5, n_range=(16384, 131072), n_range_3d=(16384, 32768),
              nrhs_max=16, workers=4, budget=64 << 30, caching=True, progress=False):
    """The serving stream at offered loads relative to the server's solo throughput: first a
    saturated calibration run (calib requests of the same distribution, all arriving at once)
    measures the throughput mu; then, for each load L, count requests arrive as a Poisson stream
    at rate L mu.  Each request builds its own representation (uniform points in [-1,1]^d, log r
    in 2D or 1/r in 3D, in the weighted second-kind form) and solves 1..nrhs_max right-hand
    sides to 1e-8.  Returns {"solo_throughput_req_per_s": mu, "loads": {L: summary}}."""
    import torch
    alloc = CachingAllocator(torch) if caching else None
    cal = make_requests(calib, rate=1e9, seed=seed + 1000, n_range=n_range, n_range_3d=n_range_3d, nrhs_max=nrhs_max)
    _, s0 = Server(hbm_budget_bytes=budget, workers=workers, allocator=alloc,
                   progress="calibration" if progress else None).run(cal)
    mu = s0["throughput_req_per_s"]
    out = {"solo_throughput_req_per_s": mu, "calibration": s0, "loads": {}}
    for L in loads:
        reqs = make_requests(count, rate=L * mu, seed=seed, n_range=n_range, n_range_3d=n_range_3d, nrhs_max=nrhs_max)
        _, sm = Server(hbm_budget_bytes=budget, workers=workers, allocator=alloc,
                       progress=f"load {L}" if progress else None).run(reqs)
        sm["offered_load"] = L
        sm["arrival_rate_per_s"] = L * mu
        out["loads"][str(L)] = sm
    if alloc is not None:
        out["caching_allocator"] = {"calls": alloc.calls, "peak_bytes": alloc.peak, "live_bytes_at_end": alloc.bytes}
    return out


def main(argv=None):
    import argparse
    import json
    p = argparse.ArgumentParser(description="build + solve serving stream at offered loads (defaults: 512 "
                                            "requests, N up to 2^20 in 2D and 3D, 1-16 right-hand sides)")
    p.add_argument("--requests", type=int, default=512)
    p.add_argument("--loads", default="0.5,0.9")
    p.add_argument("--calib", type=int, default=16)
    p.add_argument("--workers", type=int, default=4)
    p.add_argument("--budget-gib", type=float, default=200.0)
    p.add_argument("--n-min", type=int, default=16384)
    p.add_argument("--n-max-2d", type=int, default=1048576)
    p.add_argument("--n-max-3d", type=int, default=1048576)
    p.add_argument("--nrhs-max", type=int, default=16)
    p.add_argument("--seed", type=int, default=5)
    p.add_argument("--no-caching", action="store_true")
    a = p.parse_args(argv)
    res = run_loads(a.requests, loads=tuple(float(x) for x in a.loads.split(",")), calib=a.calib, seed=a.seed,
                    n_range=(a.n_min, a.n_max_2d), n_range_3d=(a.n_min, a.n_max_3d), nrhs_max=a.nrhs_max,
                    workers=a.workers, budget=int(a.budget_gib * (1 << 30)), caching=not a.no_caching, progress=True)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
