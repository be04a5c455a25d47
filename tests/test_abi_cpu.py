"""The C ABI on the CPU: library loads, exports every declared symbol, validates
arguments before allocating, and its host build equals the oracle's bit for bit.

No compute call reaches the GPU here (host_only handles only).
"""
import ctypes

import numpy as np
import pytest


@pytest.fixture(scope="module")
def lib():
    from paper_2309_14085_amd import h2s
    h2s.load()
    return h2s


def test_exports_every_declared_symbol(lib):
    names = lib.header_functions()
    assert {"h2s_build", "h2s_apply", "h2s_apply_phases", "h2s_free", "h2s_get_stats", "h2s_export",
            "h2s_set_allocator", "h2s_status_string", "h2s_last_error"} <= set(names)
    so = lib.load()
    for n in names:
        assert hasattr(so, n), n


def _raw_build(lib, pts, n, d, k, o):
    h = ctypes.c_void_p(12345)
    p = pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if pts is not None else None
    st = lib.load().h2s_build(p, n, d, ctypes.byref(k) if k else None, ctypes.byref(o) if o else None, None,
                              ctypes.byref(h))
    return st, h.value


def test_validation_before_allocation(lib):
    pts = np.random.default_rng(0).uniform(-1, 1, (100, 2))
    k = lib.Kernel(lib.LOG_R, 0.0, 0.0, 0.0)
    o = lib.BuildOpts(64, 1e-8, 1e-8, 0, 0, 0, 1)
    assert _raw_build(lib, pts, 100, 2, k, o)[0] == lib.OK
    bad = [
        (None, 100, 2, k, o),
        (pts, 0, 2, k, o),
        (pts, 100, 4, k, o),
        (pts, 100, 2, None, o),
        (pts, 100, 2, lib.Kernel(9, 0, 0, 0), o),
        (pts, 100, 2, lib.Kernel(lib.GAUSSIAN, 0.0, 1.0, 0.0), o),
        (pts, 100, 2, lib.Kernel(lib.RBF_AR, 0.0, 0.0, 0.0), o),
        (pts, 100, 2, lib.Kernel(lib.RBF_AR, float("nan"), 0.0, 0.0), o),
        (pts, 100, 2, lib.Kernel(lib.RBF_LOG, -0.1, 0.0, 0.0), o),
        (pts, 100, 2, lib.Kernel(lib.RBF_LOG, 1.0, 0.0, 0.0), o),
        (pts, 100, 2, lib.Kernel(lib.NTI_MQ, 0.0, 1.0, 0.0), o),  # 3D only
        (pts, 100, 2, lib.Kernel(7, 0.0, 1.0, 0.0), o),
        (pts, 100, 2, k, lib.BuildOpts(0, 1e-8, 1e-8, 0, 0, 0, 1)),
        (pts, 100, 2, k, lib.BuildOpts(64, -1.0, 1e-8, 0, 0, 0, 1)),
        (pts, 100, 2, k, lib.BuildOpts(64, float("nan"), 1e-8, 0, 0, 0, 1)),
        (pts, 100, 2, k, lib.BuildOpts(64, 1e-8, 1e-8, 5, 0, 0, 1)),
        (pts, 100, 2, k, lib.BuildOpts(64, 1e-8, 1e-8, 0, 7, 0, 1)),
    ]
    for args in bad:
        st, h = _raw_build(lib, *args)
        assert st == lib.ERR_INVALID_ARG and h is None, args
    nanpts = pts.copy()
    nanpts[5, 1] = np.inf
    st, h = _raw_build(lib, nanpts, 100, 2, k, o)
    assert st == lib.ERR_INVALID_ARG and h is None
    assert "finite" in lib.last_error()


def test_host_only_handle(lib, inputs):
    pts = inputs.uniform_points(4096, 2, 1)
    T = lib.build(pts, host_only=True)
    s = T.stats()
    assert s["kappa"] == 3 and s["n"] == 4096 and s["near_pairs"] == 288 and s["device_bytes"] == 0
    assert s["far_pairs"] == 96 + 576 and s["ver_pairs"] == 4 + 32 + 160
    st = T.apply_ptr(1 << 20, 2 << 20)
    assert st == lib.ERR_UNSUPPORTED
    assert lib.load().h2s_free(None) == lib.OK
    assert lib.status_string(lib.ERR_DEVICE) == "device error"
    assert T.solve_ptr(1 << 20, 2 << 20) == lib.ERR_UNSUPPORTED


def test_solve_defaults_and_validation(lib, inputs):
    import ctypes
    o = lib.SolveOpts()
    assert lib.load().h2s_solve_opts_default(ctypes.byref(o)) == lib.OK
    assert (o.restart, o.max_iter, o.max_refine, o.inner_prec, o.use_x0) == (50, 10000, 1000, lib.FP32, 0)
    assert (o.rtol, o.inner_rtol) == (1e-8, 1e-6)
    assert lib.load().h2s_solve_opts_default(None) == lib.ERR_INVALID_ARG
    T = lib.build(inputs.uniform_points(300, 2, 5), host_only=True)
    assert lib.load().h2s_solve(None, ctypes.c_void_p(8), ctypes.c_void_p(16), 1, 1, 1, None, None, None) == \
        lib.ERR_INVALID_ARG
    # the host-only handle is rejected before any argument reaches the device
    bad = lib.SolveOpts()
    lib.load().h2s_solve_opts_default(ctypes.byref(bad))
    bad.restart = 0
    assert T.solve_ptr(1 << 20, 2 << 20, opts=bad) == lib.ERR_UNSUPPORTED


CASES = [
    (2, 4096, 0, 64, 1e-8, 0, 0.0, 1000),
    (2, 4096, 0, 64, 1e-8, 1, 0.0, 1000),
    (3, 5000, 1, 64, 1e-6, 0, 0.0, 7),
    (2, 3000, 2, 32, 1e-10, 0, 0.3, 8),
    (3, 3000, 3, 20, 1e-12, 1, 0.0, 9),
    (2, 4000, 4, 64, 1e-10, 0, 0.05, 10),
    (3, 3000, 5, 32, 1e-8, 1, 0.1, 11),
    (3, 3000, 6, 32, 1e-8, 0, 0.0, 12),
    (3, 3000, 6, 64, 1e-6, 1, 0.0, 13),
]


@pytest.mark.parametrize("case", CASES + [(2, 3000, 0, 32, 1e-10, 0, 0.0, -14), (3, 3000, 1, 32, 1e-6, 1, 0.0, -15)])
def test_host_build_equals_oracle_bitwise(lib, orc, inputs, case, tmp_path):
    """(a negative seed: the point set with 40 exact duplicates, which both builds take once into
    their cross approximations)"""
    d, n, kind, nmax, eps, variant, param, seed = case
    pts = inputs.uniform_points(n, d, abs(seed))
    if seed < 0:
        pts = inputs.with_coincident_points(pts, 40, -seed)
        n = len(pts)
    O = orc.Tree(pts, kind, nmax, eps, variant=variant, param=param)
    L = lib.build(pts, kind=kind, leaf_size=nmax, eps=eps, variant=variant, param=param, host_only=True)
    ex = L.export(tmp_path / "rep.bin")
    assert np.array_equal(ex["perm"], O.perm())
    lev = ex["lev_off"]
    K = O.kappa
    assert len(lev) == K + 2
    for l in range(K + 1):
        b = O.boxes(l)
        g0, g1 = lev[l], lev[l + 1]
        assert np.array_equal(ex["box_begin"][g0:g1], b["begin"])
        for which, nm in ((0, "near"), (1, "far"), (2, "ver")):
            if (which == 0 and l != K) or (which and l == 0):
                continue
            off, idx = O.lists(which, l)
            eo, ei = ex[nm + "_off"], ex[nm + "_idx"]
            for x in range(g1 - g0):
                assert np.array_equal(ei[eo[g0 + x]:eo[g0 + x + 1]] - g0, idx[off[x]:off[x + 1]])
        for f, fn in ((0, "far"), (1, "ver")):
            if variant == 1 and f == 1:
                continue
            rk, co = ex[f"fam_{fn}_rank"], ex[f"fam_{fn}_coef_off"]
            oo, orow = ex[f"fam_{fn}_op_off"], ex[f"fam_{fn}_op_rows"]
            for x in range(g1 - g0):
                g = g0 + x
                r = max(O.rank(f, l, x), 0)
                assert rk[g] == r
                if r == 0:
                    continue
                pr, pc = O.pivots(f, l, x)
                assert np.array_equal(ex[f"fam_{fn}_piv_row"][co[g]:co[g + 1]], pr)
                assert np.array_equal(ex[f"fam_{fn}_piv_col"][co[g]:co[g + 1]], pc)
                mine = ex[f"fam_{fn}_op"][oo[g]:oo[g + 1]]
                mine = mine.reshape(r, orow[g]).T if l == K else mine.reshape(orow[g], r)
                assert np.array_equal(mine, O.operator(f, l, x))
    if variant == 1:
        pairs = ex["pairs"].reshape(-1, 6)
        data = ex["pair_data"]
        for l in range(1, K + 1):
            op = O.hph_pairs(l)
            mine = pairs[pairs[:, 0] == l]
            assert len(mine) == len(op)
            for (lv, gx, gy, r, ou, ov), (x, y, ub, vb) in zip(mine, op):
                assert (gx - lev[l], gy - lev[l], r) == (x, y, ub.shape[1])
                nx, ny = ub.shape[0], vb.shape[0]
                assert np.array_equal(data[ou:ou + r * nx].reshape(r, nx).T, ub)
                assert np.array_equal(data[ov:ov + r * ny].reshape(r, ny).T, vb)


def test_schedule_defaults_and_validation(lib, inputs):
    """The launch schedule of a host-only handle: defaults cover the widest box of each level in
    whole wavefronts, invalid schedules are rejected without change, valid ones round-trip."""
    T = lib.build(inputs.uniform_points(4096, 2, 1), host_only=True)
    k = T.stats()["kappa"]
    sc = T.schedule()
    assert sc["near_first"] == 0.8 and sc["m2l_stream"] == 2
    for l in range(1, k + 1):
        assert sc["up_threads"][l] % 64 == 0 and 64 <= sc["up_threads"][l] <= 512
        if l < k:
            assert sc["dn_threads"][l] % 64 == 0 and 64 <= sc["dn_threads"][l] <= 512
    for bad in ({"near_first": 1.5}, {"near_first": float("nan")}, {"m2l_stream": 3}, {"m2l_stream": -1},
                {"up_threads": {k: 96}},
                {"up_threads": {1: 1024}}, {"dn_threads": {1: 0}}):
        with pytest.raises(lib.H2SError) as e:
            T.set_schedule(**bad)
        assert e.value.status == lib.ERR_INVALID_ARG
        assert T.schedule() == sc
    T.set_schedule(near_first=0.25, up_threads={k: 128, 1: 512}, dn_threads={1: 256}, m2l_stream=0)
    sc2 = T.schedule()
    assert sc2["near_first"] == 0.25 and sc2["up_threads"][k] == 128 and sc2["up_threads"][1] == 512
    assert sc2["m2l_stream"] == 0
    assert sc2["dn_threads"][1] == 256
    # tuning needs a device handle
    st = lib.load().h2s_tune(T.handle, ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), 1, None, None)
    assert st == lib.ERR_UNSUPPORTED


def test_nti_multiquadric_rejects_fp32_m2l(lib, inputs):
    """The float far field of H2S_FP32_M2L is not built for the NTI multiquadric."""
    pts = inputs.uniform_points(500, 3, 2)
    k = lib.Kernel(lib.NTI_MQ, 0.0, 1.0, 0.0)
    assert _raw_build(lib, pts, 500, 3, k, lib.BuildOpts(64, 1e-6, 1e-6, 0, lib.FP32_M2L, 0, 1))[0] == lib.ERR_UNSUPPORTED
    assert _raw_build(lib, pts, 500, 3, k, lib.BuildOpts(64, 1e-6, 1e-6, 0, lib.FP32, 0, 1))[0] == lib.OK


def test_group_validation(lib, inputs):
    """Tree groups reject NULL / empty arrays, duplicates and host-only trees before touching a device."""
    T = lib.build(inputs.uniform_points(300, 2, 5), host_only=True)
    so = lib.load()
    h = ctypes.c_void_p(77)
    assert so.h2s_group_create(None, 1, ctypes.byref(h)) == lib.ERR_INVALID_ARG and h.value is None
    arr = (ctypes.c_void_p * 2)(T.handle, T.handle)
    assert so.h2s_group_create(arr, 0, ctypes.byref(h)) == lib.ERR_INVALID_ARG
    assert so.h2s_group_create(arr, 2, ctypes.byref(h)) == lib.ERR_INVALID_ARG  # duplicate
    assert so.h2s_group_create(arr, 1, ctypes.byref(h)) == lib.ERR_UNSUPPORTED  # host_only
    assert so.h2s_group_free(None) == lib.OK


def test_binding_rejects_vectors_of_the_wrong_shape_before_any_launch(lib):
    """The binding checks every vector's rows, type and layout before it passes a pointer on:
    a short x or y would otherwise be read or written past its end by the kernels."""
    import torch
    pts = np.random.default_rng(3).uniform(-1, 1, (300, 2))
    T = lib.build(pts, leaf_size=32, eps=1e-6, host_only=True)
    good = torch.zeros(300, dtype=torch.float64)
    for bad in (torch.zeros(299, dtype=torch.float64), torch.zeros(301, dtype=torch.float64),
                torch.zeros((299, 2), dtype=torch.float64), torch.zeros((300, 2, 1), dtype=torch.float64)):
        with pytest.raises(ValueError):
            T.apply(bad)
        with pytest.raises(ValueError):
            T.apply(good, y=bad)
        with pytest.raises(ValueError):
            T.solve(bad)
    with pytest.raises(ValueError):
        T.apply(torch.zeros((300, 2), dtype=torch.float64), y=torch.zeros((300, 3), dtype=torch.float64))
    with pytest.raises(TypeError):  # right shape, but a host tensor
        T.apply(good)
    with pytest.raises(TypeError):
        T.apply(good.float())
    T.free()


@pytest.mark.parametrize("d,kind,variant", [(2, 0, 0), (2, 0, 1), (3, 1, 0), (3, 1, 1)])
def test_oracle_import_of_the_library_export(lib, orc, inputs, tmp_path, d, kind, variant):
    """The oracle's import mode reads the library's export and runs its own MVP on it.  The host
    build takes the same integer decisions as the oracle's build, so the imported product equals
    the oracle's own product bit for bit, part by part; this pins the reader (layouts, offsets,
    the row-major to column-major turn of the stacked transfers, the (H2+H)* factors)."""
    n = 3000
    pts = inputs.uniform_points(n, d, 321 + d)
    q = inputs.normal_rhs(n, 1, 654)[:, 0]
    T = lib.build(pts, kind=kind, leaf_size=32, eps=1e-8, variant=variant, shift=0.5, host_only=True)
    path = tmp_path / "rep.h2sx"
    T.export(path)
    T.free()
    imp = orc.Tree.from_export(path, kind, shift=0.5)
    own = orc.Tree(pts, kind, 32, 1e-8, variant=variant, shift=0.5)
    assert (imp.kappa, imp.variant, imp.n) == (own.kappa, variant, n)
    for a, b in zip(imp.apply_parts(q), own.apply_parts(q)):
        assert np.array_equal(a, b)


def test_oracle_import_rejects_a_damaged_file(orc, tmp_path):
    p = tmp_path / "bad.h2sx"
    p.write_bytes(b"H2SX" + b"\x01\x00\x00\x00" + b"\x05\x00\x00\x00" + b"\x00" * 20)
    with pytest.raises(ValueError):
        orc.Tree.from_export(p, 0)
    with pytest.raises(ValueError):
        orc.Tree.from_export(tmp_path / "missing.h2sx", 0)

def test_build_opts_layout_matches_the_header(lib):
    """BuildOpts mirrors h2s_build_opts field by field (x86-64 alignment): the budget field sits
    last, after the two int32 flags, at offset 40 of 48 bytes."""
    import ctypes as ct
    assert ct.sizeof(lib.BuildOpts) == 48
    assert lib.BuildOpts.host_only.offset == 36 and lib.BuildOpts.hbm_budget_bytes.offset == 40
    T = lib.build(np.random.default_rng(3).uniform(-1, 1, (2000, 2)), host_only=True, hbm_budget_bytes=1)
    assert T.stats()["device_bytes"] == 0  # a host-only handle holds no device memory: the budget never binds
