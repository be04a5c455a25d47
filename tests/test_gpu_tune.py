"""Autotuner and launch schedule (h2s_tune, h2s_set_schedule): a schedule only spreads the
same per-thread ordered sums over other blocks and streams, so every product must equal the
product under the default schedule bit for bit, and the tuner installs a valid schedule no
slower than the one it started from."""
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


@pytest.mark.parametrize("d,kind,eps,prec", [(2, 0, 1e-8, 0), (3, 1, 1e-6, 0), (2, 0, 1e-8, 1)])
def test_schedules_do_not_change_the_product(lib, orc, inputs, d, kind, eps, prec):
    n = 40000 if d == 2 else 30000
    print(f"schedule d={d} kind={kind} prec={prec}", flush=True)
    pts = inputs.uniform_points(n, d, 90 + d)
    q = inputs.normal_rhs(n, 1, 95 + d)[:, 0]
    T = lib.build(pts, kind=kind, leaf_size=64, eps=eps, prec=prec)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(q).to(dev)
    ref = T.apply(x).clone()
    k = T.stats()["kappa"]
    for share in (0.0, 1.0, 0.33):
        for m2l_stream in (0, 1, 2):
            T.set_schedule(near_first=share, up_threads=[64] * 33, dn_threads=[512] * 33, m2l_stream=m2l_stream)
            assert torch.equal(T.apply(x), ref), (share, m2l_stream)
    T.set_schedule(near_first=0.6, up_threads=[512] * 33, dn_threads=[64] * 33)
    assert torch.equal(T.apply(x), ref)
    y = torch.zeros_like(x)
    info = T.tune(x, y, reps=3)
    torch.cuda.synchronize()
    print(f"  tune: {info}, schedule {T.schedule()['near_first']}, "
          f"up {T.schedule()['up_threads'][1:k + 1]}, dn {T.schedule()['dn_threads'][1:k]}", flush=True)
    assert torch.equal(y, ref)
    assert info["candidates"] > 8 * k and 0 < info["ms_tuned"] <= info["ms_entry"]
    sc = T.schedule()
    assert 0.0 <= sc["near_first"] <= 1.0
    assert all(w % 64 == 0 and 64 <= w <= 512 for w in sc["up_threads"][1:k + 1] + sc["dn_threads"][1:k])
    assert torch.equal(T.apply(x), ref)
    if prec == 0:
        want = orc.Tree(pts, kind, 64, eps).apply(q)
        assert np.linalg.norm(ref.cpu().numpy() - want) / np.linalg.norm(want) <= 1e-12
