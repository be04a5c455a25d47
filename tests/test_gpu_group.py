"""Tree groups (h2s_group_apply): the products of many trees of uneven size, each captured as a
graph of its own and launched on a stream of the group's own (forked from and joined back into
the caller's stream), must equal each tree's own h2s_apply bit for bit on every replay (with
other work of the program between replays), after the inputs are refilled (same pointers), and
after other vectors force new captures."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_14085_amd import h2s
    h2s.load()
    return h2s


# d, n, kind, param, shift, variant, prec, leaf size, eps
SPECS = [(2, 2000, 0, 0.0, 0.0, 0, 0, 64, 1e-8), (2, 9000, 0, 0.0, 0.0, 1, 0, 64, 1e-8),
         (3, 5000, 1, 0.0, 0.0, 0, 0, 64, 1e-6), (2, 30000, 0, 0.0, 0.0, 0, 1, 64, 1e-8),
         (3, 12000, 1, 0.0, 0.0, 0, 1, 64, 1e-6), (2, 4096, 2, 0.2, 1e-2, 0, 0, 32, 1e-10),
         (3, 3000, 6, 0.0, 50.0, 0, 0, 32, 1e-8), (2, 700, 4, 0.05, 0.0, 0, 0, 64, 1e-10),
         (2, 20000, 0, 0.0, 0.0, 0, 2, 64, 1e-8), (3, 2500, 5, 0.1, 0.0, 1, 0, 32, 1e-8), (2, 50, 0, 0.0, 0.0, 0, 0, 64, 1e-8)]


def test_group_equals_each_tree(lib, inputs):
    dev = torch.device("cuda:0")
    trees, xs = [], []
    for i, (d, n, kind, param, shift, variant, prec, nmax, eps) in enumerate(SPECS):
        trees.append(lib.build(inputs.uniform_points(n, d, 300 + i), kind=kind, leaf_size=nmax, eps=eps,
                               variant=variant, prec=prec, param=param, shift=shift))
        xs.append(torch.from_numpy(inputs.normal_rhs(n, 1, 400 + i)[:, 0]).to(dev))
    refs = [T.apply(x).clone() for T, x in zip(trees, xs)]
    torch.cuda.synchronize()
    G = lib.Group(trees)
    ys = [torch.zeros_like(x) for x in xs]
    for rep in range(3):
        print(f"group replay {rep}", flush=True)
        G.apply(xs, ys)
        torch.cuda.synchronize()
        for i in range(len(trees)):
            assert torch.equal(ys[i], refs[i]), (rep, i)
        trees[3].apply(xs[3])  # eager work of the program between replays
        torch.cuda.synchronize()
    # new contents, same pointers: the captured graphs read them
    for i, x in enumerate(xs):
        x.copy_(torch.from_numpy(inputs.normal_rhs(len(x), 1, 500 + i)[:, 0]).to(dev))
    refs2 = [T.apply(x).clone() for T, x in zip(trees, xs)]
    G.apply(xs, ys)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(ys, refs2))
    # other vectors: new captures
    xs2 = [x.clone() for x in xs]
    ys2 = [torch.full_like(x, 7.0) for x in xs]
    G.apply(xs2, ys2)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(ys2, refs2))
    G.free()



def test_fused_classes_equal_each_tree(lib, inputs):
    """Trees of one precision, kernel function and dimension run fused (one launch per step for
    the whole class): classes of uneven sizes and depths, including kernel parameters that differ
    between members, beside a lone tree that keeps its own graph."""
    dev = torch.device("cuda:0")
    specs = []
    for i, n in enumerate((500, 1200, 4096, 9000, 20000, 41000, 3000, 64, 15000, 700, 30000, 2500)):
        specs.append((2, n, 0, 0.0, 0.0, 0, 64, 1e-8))              # FP64 log r, 2D
    for i, n in enumerate((3000, 12000, 800, 26000, 5000, 9000)):
        specs.append((3, n, 1, 0.0, 0.0, 1, 64, 1e-6))              # FP32 1/r, 3D
    for i, (n, h) in enumerate(((2000, 0.2), (6000, 0.1), (4000, 0.3), (9000, 0.15))):
        specs.append((2, n, 2, h, 1e-2, 0, 32, 1e-10))              # FP64 Gaussian, different h
    for i, n in enumerate((3000, 8000, 1500)):
        specs.append((3, n, 6, 0.0, 60.0, 0, 32, 1e-8))             # FP64 NTI multiquadric
    specs.append((3, 7000, 3, 0.0, 0.0, 0, 48, 1e-10))              # a lone exp(-r) tree
    trees, xs = [], []
    for i, (d, n, kind, param, shift, prec, nmax, eps) in enumerate(specs):
        trees.append(lib.build(inputs.uniform_points(n, d, 700 + i), kind=kind, leaf_size=nmax, eps=eps, prec=prec,
                               param=param, shift=shift))
        xs.append(torch.from_numpy(inputs.normal_rhs(n, 1, 800 + i)[:, 0]).to(dev))
    refs = [T.apply(x).clone() for T, x in zip(trees, xs)]
    torch.cuda.synchronize()
    print(f"fused group of {len(trees)} trees", flush=True)
    G = lib.Group(trees)
    ys = [torch.zeros_like(x) for x in xs]
    for rep in range(2):
        G.apply(xs, ys)
        torch.cuda.synchronize()
        for i in range(len(trees)):
            assert torch.equal(ys[i], refs[i]), (rep, i, specs[i])
    ys2 = [torch.full_like(x, -1.0) for x in xs]  # other output vectors: the tables are refreshed
    G.apply(xs, ys2)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(ys2, refs))
    G.free()

@pytest.mark.skip(reason="capturing the products of many trees as parallel branches of ONE HIP graph (a capture "
                         "origin stream forking one stream per tree, each forking its tree's near-field and M2L "
                         "streams) ended the host process with a segmentation fault inside the group apply, whose "
                         "cause is not identified; groups capture one graph per tree instead")
def test_group_captured_as_one_graph():
    pass
