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
