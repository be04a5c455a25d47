"""Benchmark: H2* fast MVP throughput on one MI355X.

Workload: 2D, N = 2^20 points i.i.d. uniform in [-1,1]^2 (seed 1001), kernel
log|x-y| with K_ii = 0, leaf size 64, NCA tolerance 1e-8, one N(0,1)
right-hand side (seed 2001).  A step is one complete product y = K~ x through
h2s_apply (charges to tree order, P2M, M2M, M2L, L2L, L2P, near field,
scatter) with x and y resident in HBM.  `value` is the FP64 H2* rate in
points/s; the FP32 form and the (H2+H)* variant are timed beside it.

Prints one JSON line (see the fields below).  --gpus N > 1 is not supported:
the library and this benchmark run on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks used for the roofline fraction.
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=25)  # the clocks settle over the first ~20 products
    p.add_argument("--profile-steps", type=int, default=3)
    p.add_argument("--workload", default="2d_log_n1048576")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--only", default="", help="comma list of h2star_fp64,h2star_fp32,h2star_fp32m2l,h2plush_fp64")
    p.add_argument("--calib-copy", action="store_true",
                   help="also run one plain 256 MiB device copy (reference for the HBM byte counters)")
    p.add_argument("--no-solve", action="store_true", help="skip the RBF interpolation solve beside the MVP")
    p.add_argument("--no-multi-rhs", action="store_true", help="skip the 3D 32-RHS batched product beside the MVP")
    p.add_argument("--no-serve", action="store_true", help="skip the serving run (build + solve requests)")
    p.add_argument("--no-tune", action="store_true", help="skip the autotuned-schedule leg of the FP64 product")
    p.add_argument("--no-group", action="store_true", help="skip the tree-group leg (many small trees, one launch)")
    p.add_argument("--profile-only", action="store_true",
                   help="skip the timed steps and the solve, multi-RHS and serving legs: warm-up and the per-class "
                        "profiled steps only (for rocprofv3 runs)")
    return p.parse_args()


def time_variant(h2s, torch, pts, q, w, variant, prec, steps, warmup, prof_steps):
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    T = h2s.build(pts, kind=w.kind, leaf_size=w.nmax, eps=w.eps, variant=variant, prec=prec,
                  param=w.param, shift=w.shift)
    t_init = time.perf_counter() - t0
    x = torch.from_numpy(q).to(dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    if steps == 0:
        T.set_profiling(True)  # profile-only runs: every launch in the profiled schedule
    for _ in range(warmup):
        T.apply(x, y)
    torch.cuda.synchronize()
    if steps == 0:
        T.profile()  # discard the warm-up record
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        T.apply(x, y)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / steps if steps else float("nan")
    T.set_profiling(True)
    for _ in range(prof_steps):
        T.apply(x, y)
    prof = T.profile()
    T.set_profiling(False)
    torch.cuda.synchronize()
    stats = T.stats()
    out = y.cpu().numpy()
    T.free()
    return dict(ms=ms, wall_ms=1e3 * wall / steps if steps else float("nan"), t_init=t_init, stats=stats,
                kernels={k: {"avg_ms": v[0] / max(v[1], 1), "launches_per_step": v[1] / max(prof_steps, 1)}
                         for k, v in prof.items() if v[1]}), out


def time_tuned(h2s, torch, pts, q, w, steps, warmup):
    """The FP64 H2* product under the default schedule and under the one h2s_tune installs
    (same tree, same vectors; the two products must be equal bit for bit)."""
    dev = torch.device("cuda:0")
    T = h2s.build(pts, kind=w.kind, leaf_size=w.nmax, eps=w.eps, param=w.param, shift=w.shift)
    x = torch.from_numpy(q).to(dev)
    y = torch.empty_like(x)

    def timed():
        for _ in range(warmup):
            T.apply(x, y)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):
            T.apply(x, y)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    ms_default = timed()
    ref = y.clone()
    t0 = time.perf_counter()
    info = T.tune(x, y, reps=5)
    tune_s = time.perf_counter() - t0
    ms_tuned = timed()
    equal = bool(torch.equal(y, ref))
    sc, k = T.schedule(), T.stats()["kappa"]
    T.free()
    return {"ms_default": ms_default, "ms_tuned": ms_tuned, "speedup": ms_default / ms_tuned,
            "points_per_s_tuned": w.n / (ms_tuned * 1e-3), "tune_s": tune_s, "candidates": info["candidates"],
            "bitwise_equal": equal,
            "schedule": {"near_first": sc["near_first"], "m2l_stream": sc["m2l_stream"],
                         "up_threads_by_level": sc["up_threads"][1:k + 1], "dn_threads_by_level": sc["dn_threads"][1:k]}}


def time_group(h2s, torch, count=32, seed=7, reps=10):
    """count 2D log r trees (n_max 64, eps 1e-8) of N log-uniform in [2^12, 2^15]: one
    h2s_group_apply (one fused class: one launch per step for all trees) against count h2s_apply
    calls on one stream."""
    import numpy as np
    from paper_2309_14085_amd import inputs
    rng = np.random.default_rng(seed)
    sizes = [int(round(np.exp(rng.uniform(np.log(4096), np.log(32768))))) for _ in range(count)]
    dev = torch.device("cuda:0")
    trees = [h2s.build(inputs.uniform_points(n, 2, 3000 + i), kind=0, leaf_size=64, eps=1e-8)
             for i, n in enumerate(sizes)]
    xs = [torch.from_numpy(inputs.normal_rhs(n, 1, 4000 + i)[:, 0]).to(dev) for i, n in enumerate(sizes)]
    ys = [torch.empty_like(x) for x in xs]
    G = h2s.Group(trees)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    ms_seq = timed(lambda: [T.apply(x, y) for T, x, y in zip(trees, xs, ys)])
    ref = [y.clone() for y in ys]
    ms_group = timed(lambda: G.apply(xs, ys))
    equal = all(bool(torch.equal(a, b)) for a, b in zip(ys, ref))
    G.free()
    for T in trees:
        T.free()
    total = int(sum(sizes))
    return {"trees": count, "n_min": min(sizes), "n_max": max(sizes), "points": total,
            "ms_one_by_one": ms_seq, "ms_group": ms_group, "speedup": ms_seq / ms_group,
            "points_per_s_group": total / (ms_group * 1e-3), "bitwise_equal": equal}


def time_solve(h2s, torch, w):
    """GMRES(50) + iterative refinement to 1e-8 (FP32 Krylov products, FP64 residuals) on the
    RBF interpolation system.  Build and a one-step warm-up solve (uploads, workspace) untimed;
    then one timed solve from x = 0."""
    dev = torch.device("cuda:0")
    T = h2s.build(w.points(), kind=w.kind, leaf_size=w.nmax, eps=w.eps, param=w.param, shift=w.shift)
    b = torch.from_numpy(w.rhs()[:, 0].copy()).to(dev)
    x, _ = T.solve(b, rtol=1e-8, max_iter=1, raise_on_fail=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = T.solve(b, x=x, rtol=1e-8, max_iter=100000, raise_on_fail=False)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    T.free()
    i = info[0]
    return {"workload": w.name, "n": w.n, "kernel": "exp(-r^2/0.1^2), K_ii = 1, shift 1e-2", "restart": 50,
            "inner": "fp32", "rtol": 1e-8, "seconds": sec, "iterations": i["iterations"],
            "refinements": i["refinements"], "ms_per_iteration": 1e3 * sec / max(i["iterations"], 1),
            "residual_fp64": i["residual"], "converged": i["converged"]}


def time_multi_rhs(h2s, torch, w, reps=3):
    """H2* product of 32 right-hand sides: one h2s_apply with nrhs = 32 (blocks of 8 columns
    through the batched kernels) against 32 single-column applies, in FP64; then the same
    32-column product with the far-field M2L on the matrix cores in float (FP32_M2L) and with
    bfloat16 inputs (FP32_BF16M2L), each with its error against the FP64 product (which the
    GPU tests hold within 1e-12 of the oracle).  Builds untimed."""
    import numpy as np
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    T = h2s.build(w.points(), kind=w.kind, leaf_size=w.nmax, eps=w.eps)
    t_init = time.perf_counter() - t0
    Q = np.asfortranarray(w.rhs())
    X = torch.from_numpy(Q).to(dev)                      # (n, m), column-major
    X = X.t().contiguous().t() if X.stride(0) != 1 else X
    Yb = torch.empty((w.nrhs, w.n), dtype=torch.float64, device=dev).t()
    Ys = torch.empty_like(Yb)
    T.apply(X, Yb)
    for c in range(w.nrhs):
        T.apply(X[:, c].contiguous(), Ys[:, c])
    torch.cuda.synchronize()
    cols = [X[:, c].contiguous() for c in range(w.nrhs)]
    outs = [torch.empty(w.n, dtype=torch.float64, device=dev) for _ in range(w.nrhs)]

    def timed(fn):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    ms_b = timed(lambda: T.apply(X, Yb))
    ms_s = timed(lambda: [T.apply(cols[c], outs[c]) for c in range(w.nrhs)])
    for c in range(w.nrhs):
        Ys[:, c] = outs[c]
    diff = float(((Yb - Ys).norm(dim=0) / Ys.norm(dim=0)).max())
    st = T.stats()
    T.free()
    # M2L flops of the far field per 32-column product (2 per multiply-add), for the matrix-core rate
    far_flops = 2.0 * st["m2l_evals_family"][0] * w.nrhs
    lowp = {}
    for name, prec in (("fp32_m2l", h2s.FP32_M2L), ("bf16_m2l", h2s.FP32_BF16M2L)):
        Tl = h2s.build(w.points(), kind=w.kind, leaf_size=w.nmax, eps=w.eps, prec=prec)
        Yl = torch.empty_like(Yb)
        Tl.apply(X, Yl)
        torch.cuda.synchronize()
        ms_l = timed(lambda: Tl.apply(X, Yl))
        err = (Yl - Yb).norm(dim=0) / Yb.norm(dim=0)
        errmax = (Yl - Yb).abs().amax(dim=0) / Yb.abs().amax(dim=0)
        lowp[name] = {"batched_ms": ms_l, "speedup_vs_fp64_batched": ms_b / ms_l,
                      "points_x_rhs_per_s": w.n * w.nrhs / (ms_l * 1e-3),
                      "rel_err_vs_fp64_max_column": float(err.max()), "rel_err_vs_fp64_median_column": float(err.median()),
                      "max_elem_err_vs_fp64": float(errmax.max()),
                      "far_m2l_mfma": "f32 16x16x4" if prec == h2s.FP32_M2L else "bf16 16x16x32, f32 accumulation"}
        Tl.free()
    return {"workload": w.name, "n": w.n, "d": w.d, "kernel": "1/r (K_ii = 0)", "nca_tol": w.eps, "nrhs": w.nrhs,
            "dtype": "f64", "batched_ms": ms_b, "per_vector_ms": ms_s, "speedup": ms_s / ms_b,
            "points_x_rhs_per_s_batched": w.n * w.nrhs / (ms_b * 1e-3),
            "points_x_rhs_per_s_per_vector": w.n * w.nrhs / (ms_s * 1e-3),
            "max_rel_diff_batched_vs_per_vector": diff, "t_init_s": t_init,
            "m2l_evals_per_rhs": st["m2l_evals"], "p2p_evals_per_rhs": st["p2p_evals"],
            "far_m2l_flops_per_product": far_flops, "low_precision": lowp}


def time_serving(count=32, workers=4, budget=64 << 30):
    """The build + solve serving stream at 0.5x and 0.9x of the server's measured throughput
    (the stream of 512 requests with N up to 2^20 and 1-16 right-hand sides, at smaller sizes and
    counts: d in {2, 3}, N log-uniform in [2^14, 2^17] (2D) / [2^14, 2^15] (3D), 1-16 right-hand sides, log r (2D) or 1/r (3D) in second-kind form,
    GMRES to 1e-8), admitted by learned device bytes within a 64 GiB budget, 4 workers, the
    library's memory from the caching allocator."""
    from paper_2309_14085_amd import serve
    res = serve.run_loads(count, loads=(0.5, 0.9), calib=8, seed=5, n_range=(16384, 131072),
                          n_range_3d=(16384, 32768), nrhs_max=16, workers=workers, budget=budget)
    res.update({"workers": workers, "hbm_budget_bytes": budget, "requests_per_load": count,
                "requests_spec": "d in {2,3}; N log-uniform 2^14..2^17 (2D), 2^14..2^15 (3D); 1-16 RHS; "
                                 "(w K + I) x = b, w = 2^d / N; GMRES(50) FP32 Krylov to 1e-8; "
                                 "the full stream has N up to 2^20 (its host builds take up to ~25 s each)"})
    return res


def algorithmic_work(stats, kernel, prec):
    """Algorithmic HBM bytes and kernel evaluations of one launch of a kernel class.

    Bytes count each stored operator entry, coordinate, charge and output once:
    P2M and L2P each read one copy of the stored leaf bases (the rows that are
    not exact unit rows), M2M and L2L one copy of the stored transfers; points
    d FP64 (FP32 in the FP32 policies) per point, charges, near-field
    potentials, y, perm and the int16 row maps.  Evaluations are the near-field
    pairs (ordered leaf pairs of N*, as Sec. 5.1.2 sums them) and the M2L
    entries sum_X sum_{Y in IL(X)} r_X r_Y."""
    n, d = stats["n"], stats["d"]
    basis_b = 8 if prec == 0 else 4
    pt_b = 8 if prec == 0 else 4
    leaf = stats["leaf_basis_stored"] or stats["leaf_basis_entries"]
    tr = stats["transfer_stored"] or stats["transfer_entries"]
    if kernel == "near":
        return n * (d * pt_b + 8 + 8), stats["p2p_evals"]
    if kernel == "leaf_down":
        return n * (8 + 8 + 4 + 4 + 8) + leaf * basis_b, 0
    if kernel == "leaf_up":
        return n * (8 + 4 + 8 + 4) + leaf * basis_b, 0
    if kernel == "m2l_far":
        return 0, stats["m2l_evals_family"][0]
    if kernel == "m2l_ver":
        return 0, stats["m2l_evals_family"][1]
    if kernel in ("m2m", "l2l"):
        return tr * 8, 0
    if kernel == "pair_part":
        return stats["pair_entries"] * basis_b, 0
    return 0, 0


CLASSES = ("leaf_up", "m2m", "m2l_far", "m2l_ver", "l2l", "pair_part", "leaf_down", "near")


def product_roofline(stats, kernels, ms, r_eval, prec):
    """Whole-product roofline: T* = max(B / BW_peak, E / R_eval), B the algorithmic bytes and E the
    kernel evaluations of every phase (algorithmic_work summed over the classes the product runs),
    BW_peak the published 8 TB/s and R_eval the measured register-resident evaluation rate of the
    same kernel function.  frac = T* / t_MVP; `binding` names the larger term.  Per-class
    fractions use each class's isolated time from the profiling hooks."""
    B = E = 0
    per = {}
    for c in CLASSES:
        if c not in kernels:
            continue
        b, e = algorithmic_work(stats, c, prec)
        B, E = B + b, E + e
        t = kernels[c]["avg_ms"] * kernels[c]["launches_per_step"] * 1e-3
        if e:
            per[c] = {"bound": "alu", "evals": e, "ms": t * 1e3, "geval_s": e / t / 1e9, "frac": e / t / r_eval}
        elif b:
            per[c] = {"bound": "hbm", "bytes": b, "ms": t * 1e3, "gb_s": b / t / 1e9, "frac": b / t / 1e9 / HBM_PEAK_GBS}
    t_hbm = B / (HBM_PEAK_GBS * 1e9)
    t_eval = E / r_eval
    t_star = max(t_hbm, t_eval)
    return {"t_star_ms": t_star * 1e3, "t_mvp_ms": ms, "frac": t_star / (ms * 1e-3),
            "binding": "alu (kernel evaluations)" if t_eval >= t_hbm else "hbm",
            "bytes": B, "evals": E, "t_hbm_ms": t_hbm * 1e3, "t_eval_ms": t_eval * 1e3,
            "r_eval_measured": r_eval, "bw_peak_gb_s": HBM_PEAK_GBS,
            "frac_if_no_overlap": (t_hbm + t_eval) / (ms * 1e-3), "per_kernel": per}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    if a.profile_only:  # rocprofv3 runs trace the product alone
        a.no_solve = a.no_multi_rhs = a.no_serve = a.no_tune = a.no_group = True
    import numpy as np
    import torch

    from paper_2309_14085_amd import h2s, inputs

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    h2s.load()
    if a.calib_copy:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = inputs.workload(a.workload)
    pts, q = w.points(), np.ascontiguousarray(w.rhs()[:, 0])
    todo = [("h2star_fp64", h2s.H2STAR, h2s.FP64), ("h2star_fp32", h2s.H2STAR, h2s.FP32),
            ("h2star_fp32m2l", h2s.H2STAR, h2s.FP32_M2L), ("h2plush_fp64", h2s.H2_PLUS_H, h2s.FP64)]
    if a.only:
        todo = [t for t in todo if t[0] in a.only.split(",")]
    res, outs = {}, {}
    for name, variant, prec in todo:
        print(f"# building and timing {name}", file=sys.stderr, flush=True)
        r, y = time_variant(h2s, torch, pts, q, w, variant, prec, 0 if a.profile_only else a.steps, a.warmup,
                            a.profile_steps)
        r["points_per_s"] = w.n / (r["ms"] * 1e-3)
        res[name], outs[name] = r, y
        print(f"# {name}: {r['ms']:.3f} ms/step, {r['points_per_s']:.3e} points/s, init {r['t_init']:.1f}s",
              file=sys.stderr, flush=True)
    ref = outs.get("h2star_fp64")
    for name in outs:
        if ref is not None and name != "h2star_fp64":
            res[name]["rel_err_vs_fp64_h2star"] = float(np.linalg.norm(outs[name] - ref) / np.linalg.norm(ref))

    main_name = "h2star_fp64" if "h2star_fp64" in res else next(iter(res))
    m = res[main_name]
    kernels = m["kernels"]
    prec_main = 0 if main_name.endswith("fp64") else 1
    r_eval = h2s.eval_rate(w.kind, w.d, h2s.FP64 if prec_main == 0 else h2s.FP32, param=w.param)
    print(f"# measured R_eval: {r_eval:.4e} evaluations/s", file=sys.stderr, flush=True)
    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches_per_step"])
        roofline = roofline_entry(dom, kernels[dom], m["stats"], prec_main, r_eval)
        if not a.profile_only:
            roofline["whole_product"] = product_roofline(m["stats"], kernels, m["ms"], r_eval, prec_main)
        for name in res:
            if name != main_name and res[name]["kernels"] and not a.profile_only:
                pv = 0 if name.endswith("fp64") else 1
                res[name]["whole_product"] = product_roofline(res[name]["stats"], res[name]["kernels"],
                                                              res[name]["ms"], r_eval, pv)

    tuned = None
    if not a.no_tune and main_name == "h2star_fp64":
        print("# autotuning the launch schedule of the FP64 product", file=sys.stderr, flush=True)
        tuned = time_tuned(h2s, torch, pts, q, w, a.steps, a.warmup)
        print(f"# tuned: {tuned}", file=sys.stderr, flush=True)

    group = None
    if not a.no_group:
        print("# 32 small trees: one group apply against one apply each", file=sys.stderr, flush=True)
        group = time_group(h2s, torch)
        print(f"# group: {group}", file=sys.stderr, flush=True)

    solve = None
    if not a.no_solve:
        print("# building and timing the RBF interpolation solve", file=sys.stderr, flush=True)
        solve = time_solve(h2s, torch, inputs.workload("2d_gauss_rbf_n262144"))
        print(f"# solve: {solve}", file=sys.stderr, flush=True)

    multi = None
    if not a.no_multi_rhs:
        print("# building and timing the 32-RHS batched product", file=sys.stderr, flush=True)
        multi = time_multi_rhs(h2s, torch, inputs.workload("3d_invr_n262144_m32"))
        print(f"# multi-rhs: {multi}", file=sys.stderr, flush=True)

    served = None
    if not a.no_serve:
        print("# serving build + solve requests", file=sys.stderr, flush=True)
        served = time_serving()
        print(f"# serving: {served}", file=sys.stderr, flush=True)

    cpu = None
    if not a.no_cpu_baseline:
        print("# oracle on the host cores: build, MVPs at all and at 8 threads, sampled direct sum",
              file=sys.stderr, flush=True)
        cpu, oracle_out = cpu_baseline(pts, q, w, want_hph="h2plush_fp64" in outs)
        for name, y in outs.items():
            ref_o = oracle_out["h2plush" if name.startswith("h2plush") else "h2star"]
            if ref_o is not None:
                res[name]["rel_err_vs_oracle"] = float(np.linalg.norm(y - ref_o) / np.linalg.norm(ref_o))
                res[name]["max_rel_err_vs_oracle"] = float(np.abs(y - ref_o).max() / np.abs(ref_o).max())
            rows, exact = oracle_out["rows"], oracle_out["direct_rows"]
            res[name]["rel_err_vs_direct_sampled"] = float(np.linalg.norm(y[rows] - exact) / np.linalg.norm(exact))
        cpu["oracle_rel_err_vs_direct_sampled"] = oracle_out["oracle_vs_direct"]

    line = {
        "metric": "H2* MVP points/s and % roofline at stated rel err vs FP64; solve p50/p99",
        "value": m["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": m["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: uniform points in [-1,1]^2 (seed 1001), N(0,1) rhs (seed 2001)",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "kernel": "log r (K_ii = 0)", "leaf_size": w.nmax,
                   "nca_tol": w.eps, "nrhs": 1, "variant": "H2*(b+t)"},
        "rel_err_vs_oracle": m.get("rel_err_vs_oracle"),
        "rel_err_vs_direct_sampled": m.get("rel_err_vs_direct_sampled"),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "tuned_schedule": tuned,
        "tree_group": group,
        "solve": solve,
        "multi_rhs": multi,
        "serving": served,
        "variants": {k: {kk: vv for kk, vv in v.items() if kk != "stats"} for k, v in res.items()},
        "ranks": {"far_max_by_level": m["stats"]["rank_max_level"][0],
                  "ver_max_by_level": m["stats"]["rank_max_level"][1],
                  "far_avg_by_level": [round(x, 1) for x in m["stats"]["rank_avg_level"][0]],
                  "ver_avg_by_level": [round(x, 1) for x in m["stats"]["rank_avg_level"][1]]},
        "work": {k: m["stats"][k] for k in ("p2p_evals", "m2l_evals", "operator_bytes", "device_bytes",
                                            "near_pairs", "far_pairs", "ver_pairs")},
    }
    print(json.dumps(line))


def roofline_entry(name, k, stats, prec, r_eval=None):
    """Roofline of the dominant kernel class (one launch per step for the leaf and M2L classes).

    Kernel-evaluation classes are bound by FP64 VALU issue: the chip issues
    256 CUs x 4 SIMDs x 16 FP64 lanes per clock at 2.4 GHz, and one
    evaluation of log r (distance, table-driven logarithm, multiply-add)
    takes VALU_PER_EVAL vector instructions in the compiled inner loop, so
    the peak is the issue rate divided by that count.  Operator-streaming
    classes are bound by HBM bandwidth."""
    avg_s = k["avg_ms"] * 1e-3
    byts, evals = algorithmic_work(stats, name, prec)
    traffic = measured_traffic(name)
    if evals:
        per_eval = VALU_PER_EVAL.get(name, VALU_PER_EVAL["near"])
        peak = VALU_LANE_ISSUE_PER_S / per_eval / 1e9
        ach = evals / avg_s / 1e9
        out = {"kernel": name, "bound": "alu", "achieved": ach, "peak": peak, "unit": "Geval/s",
               "frac": ach / peak, "traffic": traffic, "evals_per_launch": evals,
               "valu_instr_per_eval": per_eval, "avg_launch_ms": k["avg_ms"],
               "fp64_tflops": ach * FP64_FLOPS_PER_EVAL / 1e3, "fp64_flops_per_eval": FP64_FLOPS_PER_EVAL,
               "frac_of_fp64_peak": ach * FP64_FLOPS_PER_EVAL / 1e3 / FP64_PEAK_TFLOPS}
        if r_eval:
            out["r_eval_measured_geval_s"] = r_eval / 1e9
            out["frac_of_measured_r_eval"] = ach / (r_eval / 1e9)
        return out
    ach = byts / avg_s / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "bytes_per_launch": byts, "avg_launch_ms": k["avg_ms"]}


# FP64 VALU lane-instructions per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (the 78.6 TFLOP/s FP64 vector peak counts one FMA per lane-instruction as 2 flops).
VALU_LANE_ISSUE_PER_S = 256 * 4 * 16 * 2.4e9
# Vector instructions per log-r kernel evaluation in the compiled FP64 2D inner
# loops (4 evaluations per iteration, loop control included): the near field
# 73 / 4, M2L 77 / 4.
VALU_PER_EVAL = {"near": 18.25, "m2l_far": 19.25, "m2l_ver": 19.25}
# FP64 flops of one evaluation (FMA = 2): squared distance 5, reduction
# r = m c - 1 and the degree-5 series 12, the exponent term 2, multiply-add 2.
FP64_FLOPS_PER_EVAL = 21

COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters_2d_log_n1048576.json")


KERNEL_SOURCES = ("h2s_kernels.hip", "h2s_kfun.hpp", "h2s_device.hpp")


def kernel_sources_sha256():
    """SHA-256 over the sources the single-column product kernels are compiled from, in order."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2309_14085_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary,
    or None if that summary was taken on other kernel sources."""
    try:
        c = json.load(open(COUNTERS))
    except (OSError, ValueError):
        return None
    if kernel_sources_sha256() != c.get("kernels_sha256"):
        return None
    k = c.get("per_launch_bytes", {}).get(kernel)
    return None if k is None else k["fetch"] + k["write"]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pts, q, w, want_hph=False, direct_rows=1024):
    """The oracle's H2* MVP on the host cores (build untimed), same inputs: the median of 2 MVPs
    with every host thread and again with 8 threads (the paper's thread count), and the oracle's
    compensated direct sum on `direct_rows` seeded rows (scaled to the full product).  Returns the
    record and the oracle's products (H2*, and (H2+H)* if asked) with the sampled direct rows, for
    the GPU results' errors."""
    import numpy as np

    import oracle
    oracle.set_threads(0)
    all_threads = oracle.num_threads()
    t0 = time.perf_counter()
    T = oracle.Tree(pts, w.kind, w.nmax, w.eps)
    t_build = time.perf_counter() - t0

    def mvps(threads):
        oracle.set_threads(threads)
        times, y = [], None
        for _ in range(2):
            t0 = time.perf_counter()
            y = T.apply(q)
            times.append(time.perf_counter() - t0)
        return float(np.median(times)), y

    t_all, y_h2 = mvps(0)
    t_8, _ = mvps(8)
    oracle.set_threads(0)
    del T
    y_hph = None
    if want_hph:
        y_hph = oracle.Tree(pts, w.kind, w.nmax, w.eps, variant=1).apply(q)
    rows = np.sort(np.random.default_rng(7).choice(w.n, direct_rows, replace=False))
    t0 = time.perf_counter()
    exact = oracle.direct(pts, q, w.kind, param=w.param, shift=w.shift, rows=rows)
    t_dir = time.perf_counter() - t0
    rec = {"value": w.n / t_all, "unit": "points/s", "cores": all_threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"full workload {w.name}: oracle FP64 H2* build ({t_build:.1f} s, untimed) then 2 MVPs, "
                     f"median {t_all:.2f} s with {all_threads} threads",
           "threads_8": {"value": w.n / t_8, "mvp_s": t_8, "cores": 8},
           "direct_sum": {"rows": direct_rows, "seconds": t_dir, "cores": all_threads,
                          "full_product_s_est": t_dir * w.n / direct_rows,
                          "points_per_s_est": direct_rows / t_dir},
           "build_s": t_build}
    out = {"h2star": y_h2, "h2plush": y_hph, "rows": rows, "direct_rows": exact,
           "oracle_vs_direct": float(np.linalg.norm(y_h2[rows] - exact) / np.linalg.norm(exact))}
    return rec, out


if __name__ == "__main__":
    main()
