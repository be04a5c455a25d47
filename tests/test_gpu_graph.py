"""The product captured in a HIP graph (torch.cuda.graph on the caller's stream).

h2s_apply forks its near field onto the handle's second stream and joins it
back with events, and enqueues no memset, so a capture on the caller's stream
takes the whole product.  Each replay, with eager work of the program between
replays, must equal the eager product bit for bit (the kernels use no atomics),
also after the captured input buffer is refilled.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def lib():
    from paper_2309_14085_amd import h2s
    h2s.load()
    return h2s


@pytest.mark.parametrize("m", [1, 8])
def test_graph_replays_equal_eager(lib, orc, inputs, m):
    n = 20000
    print(f"graph capture m={m}", flush=True)
    dev = _dev()
    pts = inputs.uniform_points(n, 2, 81)
    T = lib.build(pts, kind=0, leaf_size=64, eps=1e-8)
    Q0 = inputs.normal_rhs(n, m, 82)
    Q1 = inputs.normal_rhs(n, m, 83)

    def as_dev(Q):
        X = torch.from_numpy(np.ascontiguousarray(Q.T)).to(dev).t()  # (n, m) column-major
        return X[:, 0].contiguous() if m == 1 else X

    x_static = as_dev(Q0)
    y_static = torch.zeros_like(x_static)
    # eager first: creates the handle's second stream and any block buffers outside the capture
    ref0 = T.apply(x_static).clone()
    ref1 = T.apply(as_dev(Q1)).clone()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        T.apply(x_static, y_static, stream=s)
    torch.cuda.synchronize()
    other = T.apply(as_dev(Q1))  # eager work of the program between replays
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y_static, ref0), rep
        other = T.apply(as_dev(Q1), other)
        torch.cuda.synchronize()
    # refill the captured input: the replay computes the new product
    x_static.copy_(as_dev(Q1))
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(y_static, ref1)
    # and the replayed product matches the oracle
    O = orc.Tree(pts, 0, 64, 1e-8)
    y = y_static.cpu().numpy().reshape(n, -1, order="F") if m > 1 else y_static.cpu().numpy()[:, None]
    for c in range(m):
        want = O.apply(Q1[:, c])
        assert np.linalg.norm(y[:, c] - want) / np.linalg.norm(want) <= 1e-12
