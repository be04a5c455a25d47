"""Serving loop (paper_2309_14085_amd/serve.py): requests admitted by an HBM
budget and solved concurrently must each give the same solution as when
solved alone (the kernels use no atomics and every reduction has a fixed
order, so the solutions are equal bit for bit), reach the 1e-8 residual,
and respect the budget and the worker count.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_14085_amd import h2s, serve as _serve
    h2s.load()
    return _serve


def test_each_result_same_alone_and_in_the_mix(serve, orc, inputs):
    reqs = serve.make_requests(6, rate=50.0, seed=5, n_range=(4096, 16384), n_range_3d=(4096, 8192), nrhs_max=3)
    budget = 2 * max(serve.estimate_bytes(r) for r in reqs)  # at most two of the largest at a time
    print("serving mix", [(r.d, r.n, r.nrhs) for r in reqs], flush=True)
    mix, summary = serve.Server(hbm_budget_bytes=budget, workers=3, keep_x=True).run(reqs)
    print(summary, flush=True)
    assert summary["failed"] == 0 and summary["converged"] == len(reqs)
    assert summary["peak_inflight"] <= 3 and summary["peak_budget_used_bytes"] <= budget
    for r, res in zip(reqs, mix):
        assert max(res.residuals) <= 1e-8
        alone_req = serve.Request(r.rid, 0.0, r.d, r.n, r.nrhs, r.seed)
        alone, _ = serve.Server(workers=1, keep_x=True).run([alone_req])
        assert np.array_equal(res.x, alone[0].x), r.rid
    # the residual of one request measured with the oracle product
    r = reqs[0]
    pts = inputs.uniform_points(r.n, r.d, r.seed)
    B = inputs.normal_rhs(r.n, r.nrhs, r.seed + 1) * r.shift
    O = orc.Tree(pts, orc.LOG_R if r.d == 2 else orc.INV_R, 64, r.tol, shift=r.shift)
    X = mix[0].x.reshape(r.n, -1) if r.nrhs > 1 else mix[0].x[:, None]
    for c in range(r.nrhs):
        res = np.linalg.norm(B[:, c] - O.apply(X[:, c])) / np.linalg.norm(B[:, c])
        assert res <= 1.01e-8, (c, res)


def test_failing_allocator_reports_out_of_memory_and_leaks_nothing(serve, inputs):
    """h2s_set_allocator with an allocator that fails after k successful allocations: the build
    returns OUT_OF_MEMORY and frees every block it took (the handle owns them until then), and
    the default allocator works again afterwards."""
    from paper_2309_14085_amd import h2s
    pts = inputs.uniform_points(20000, 2, 71)
    live, count = {}, [0]

    def make(k):
        def alloc(nbytes):
            if count[0] >= k:
                return 0
            count[0] += 1
            p = torch.cuda.caching_allocator_alloc(nbytes, device=0)
            live[p] = nbytes
            return p

        def free(p):
            live.pop(p)
            torch.cuda.caching_allocator_delete(p)
        return alloc, free

    try:
        for k in (0, 5, 20):
            count[0] = 0
            h2s.set_allocator(*make(k))
            print(f"failing allocator after {k}", flush=True)
            with pytest.raises(h2s.H2SError) as e:
                h2s.build(pts, kind=h2s.LOG_R, leaf_size=64, eps=1e-8)
            assert e.value.status == h2s.ERR_OUT_OF_MEMORY
            assert count[0] == k and not live, (k, len(live))
        # enough allocations: the build and a product go through the callbacks, and h2s_free
        # returns every block
        count[0] = 0
        h2s.set_allocator(*make(10 ** 6))
        T = h2s.build(pts, kind=h2s.LOG_R, leaf_size=64, eps=1e-8)
        y = T.apply(torch.ones(20000, dtype=torch.float64, device="cuda:0"))
        torch.cuda.synchronize()
        assert live and torch.isfinite(y).all()
        T.free()
        assert not live
    finally:
        h2s.set_allocator()
    T = h2s.build(pts, kind=h2s.LOG_R, leaf_size=64, eps=1e-8)
    T.free()


def test_hbm_budget_caps_the_handle(inputs):
    """h2s_build_opts.hbm_budget_bytes: a budget below the representation makes the build return
    OUT_OF_MEMORY with every block returned; a budget that fits the representation only lets
    single-column products run and makes the first multi-RHS product (whose buffers are allocated
    on first use) return OUT_OF_MEMORY, after which the handle still works; a larger budget
    serves both, with results equal to an unbudgeted handle's."""
    from paper_2309_14085_amd import h2s
    n = 20000
    pts = inputs.uniform_points(n, 2, 72)
    dev = torch.device("cuda:0")
    q = torch.from_numpy(inputs.normal_rhs(n, 4, 73)).to(dev)  # column-major (n, 4)
    live = {}

    def alloc(nbytes):
        p = torch.cuda.caching_allocator_alloc(nbytes, device=0)
        live[p] = nbytes
        return p

    def free(p):
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    ref = h2s.build(pts, kind=h2s.LOG_R, leaf_size=64, eps=1e-8)
    y1 = ref.apply(q[:, 0].contiguous()).clone()
    rep_bytes = ref.stats()["device_bytes"]  # the representation and what a single-column product uses
    Y4 = ref.apply(q).clone()
    full_bytes = ref.stats()["device_bytes"]
    assert full_bytes > rep_bytes
    try:
        h2s.set_allocator(alloc, free)
        print(f"budget: representation {rep_bytes} B, with the multi-RHS buffers {full_bytes} B", flush=True)
        with pytest.raises(h2s.H2SError) as e:
            h2s.build(pts, kind=h2s.LOG_R, leaf_size=64, eps=1e-8, hbm_budget_bytes=rep_bytes // 2)
        assert e.value.status == h2s.ERR_OUT_OF_MEMORY and not live
        T = h2s.build(pts, kind=h2s.LOG_R, leaf_size=64, eps=1e-8, hbm_budget_bytes=rep_bytes)
        assert T.stats()["device_bytes"] <= rep_bytes
        assert torch.equal(T.apply(q[:, 0].contiguous()), y1)
        with pytest.raises(h2s.H2SError) as e:
            T.apply(q)
        assert e.value.status == h2s.ERR_OUT_OF_MEMORY
        assert T.stats()["device_bytes"] <= rep_bytes
        assert torch.equal(T.apply(q[:, 0].contiguous()), y1)
        T.free()
        assert not live
        T = h2s.build(pts, kind=h2s.LOG_R, leaf_size=64, eps=1e-8, hbm_budget_bytes=full_bytes)
        assert torch.equal(T.apply(q), Y4) and torch.equal(T.apply(q[:, 0].contiguous()), y1)
        T.free()
        assert not live
    finally:
        h2s.set_allocator()
    ref.free()


def test_caching_allocator_serves_the_same_results(serve):
    """The serving loop with its caching allocator (PyTorch's, behind h2s_set_allocator) gives
    every request the same solution bit for bit as with hipMalloc, and returns every block."""
    reqs = serve.make_requests(5, rate=50.0, seed=9, n_range=(4096, 16384), n_range_3d=(4096, 8192), nrhs_max=4)
    plain, _ = serve.Server(workers=2, keep_x=True).run(reqs)
    alloc = serve.CachingAllocator(torch)
    cached, summary = serve.Server(workers=2, keep_x=True, allocator=alloc).run(reqs)
    print(summary, alloc.calls, alloc.peak, flush=True)
    print([(r.d, r.n, r.nrhs, o.est_bytes, o.device_bytes) for r, o in zip(reqs, cached)], flush=True)
    assert summary["failed"] == 0 and summary["converged"] == len(reqs)
    assert alloc.calls > 0 and alloc.bytes == 0 and not alloc.live
    for a, b in zip(plain, cached):
        assert np.array_equal(a.x, b.x), a.rid
    # the admission estimate covers what the library allocated
    assert summary["est_over_device_bytes_min"] >= 1.0


def test_offered_loads_report_latency_percentiles(serve):
    """The load-driven stream (calibration, then Poisson arrivals at 0.5 and 0.9 of the measured
    throughput) at a small size: every request converges, p50 <= p99, and the higher load does
    not finish its stream faster than its arrivals."""
    res = serve.run_loads(6, loads=(0.5, 0.9), calib=3, n_range=(4096, 16384), n_range_3d=(4096, 8192), nrhs_max=6,
                          workers=2, budget=8 << 30)
    print(res, flush=True)
    assert res["solo_throughput_req_per_s"] > 0
    for L in ("0.5", "0.9"):
        sm = res["loads"][L]
        assert sm["failed"] == 0 and sm["converged"] == 6 and sm["max_residual"] <= 1e-8
        assert 0 < sm["p50_s"] <= sm["p99_s"]
    assert res["caching_allocator"]["live_bytes_at_end"] == 0
