"""Python binding of the C ABI in include/h2s.h (argument marshalling only).

Every step of the product runs in libh2s.so (host build in C++, MVP in HIP
kernels).  PyTorch provides device memory and streams.  There is no fallback:
if the library is missing, loading raises.
"""
import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libh2s.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "h2s.h")

OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NOT_CONVERGED, ERR_UNSUPPORTED, ERR_INTERNAL = range(7)
LOG_R, INV_R, GAUSSIAN, EXP_R, RBF_AR, RBF_LOG, NTI_MQ = 0, 1, 2, 3, 4, 5, 6
H2STAR, H2_PLUS_H = 0, 1
FP64, FP32, FP32_M2L, FP32_BF16M2L = 0, 1, 2, 3
PHASE_NEAR, PHASE_FAR, PHASE_VER, PHASE_ALL = 1, 2, 4, 7
PROF_NAMES = ("leaf_up", "m2m", "m2l_far", "l2l", "pair_part", "pair_sum", "leaf_down", "m2l_ver", "near")


class Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("param", ctypes.c_double), ("diag", ctypes.c_double),
                ("shift", ctypes.c_double)]


class BuildOpts(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("eps_far", ctypes.c_double), ("eps_ver", ctypes.c_double),
                ("variant", ctypes.c_int), ("prec", ctypes.c_int), ("host_threads", ctypes.c_int32),
                ("host_only", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("kappa", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("n", ctypes.c_int64), ("boxes", ctypes.c_int64),
                ("near_pairs", ctypes.c_int64), ("far_pairs", ctypes.c_int64), ("ver_pairs", ctypes.c_int64),
                ("rank_sum", ctypes.c_int64 * 2), ("rank_max", ctypes.c_int32 * 2),
                ("p2p_evals", ctypes.c_int64), ("m2l_evals", ctypes.c_int64), ("m2l_evals_family", ctypes.c_int64 * 2),
                ("leaf_basis_entries", ctypes.c_int64), ("transfer_entries", ctypes.c_int64),
                ("pair_entries", ctypes.c_int64),
                ("operator_bytes", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("build_seconds", ctypes.c_double),
                ("rank_max_level", (ctypes.c_int32 * 32) * 2), ("rank_avg_level", (ctypes.c_double * 32) * 2),
                ("leaf_basis_stored", ctypes.c_int64), ("transfer_stored", ctypes.c_int64)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if name in ("rank_max_level", "rank_avg_level"):
                v = [list(row)[: self.kappa + 1] for row in v]
            elif hasattr(v, "__len__"):
                v = list(v)
            out[name] = v
        return out


_lib = None


class H2SError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_string(status)}: {msg}")
        self.status = status


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("inner_prec", ctypes.c_int), ("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
                ("use_x0", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("near_first", ctypes.c_double), ("up_threads", ctypes.c_int32 * 33),
                ("dn_threads", ctypes.c_int32 * 33), ("m2l_stream", ctypes.c_int32)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("ms_entry", ctypes.c_double), ("ms_tuned", ctypes.c_double), ("candidates", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("refinements", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("residual", ctypes.c_double)]


def load():
    """Load libh2s.so (built by paper_2309_14085_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.h2s_build.argtypes = [f64p, i64, i32, ctypes.POINTER(Kernel), ctypes.POINTER(BuildOpts), vp,
                              ctypes.POINTER(vp)]
    lib.h2s_apply.argtypes = [vp, vp, vp, i32, i64, i64, vp]
    lib.h2s_apply_phases.argtypes = [vp, u32, vp, vp, i32, i64, i64, vp]
    lib.h2s_free.argtypes = [vp]
    lib.h2s_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.h2s_export.argtypes = [vp, ctypes.c_char_p]
    lib.h2s_set_allocator.argtypes = [vp, vp, vp]
    lib.h2s_set_profiling.argtypes = [vp, i32]
    lib.h2s_get_profile.argtypes = [vp, f64p, ctypes.POINTER(i64)]
    lib.h2s_status_string.restype = ctypes.c_char_p
    lib.h2s_status_string.argtypes = [ctypes.c_int]
    lib.h2s_last_error.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    lib.h2s_solve_opts_default.argtypes = [ctypes.POINTER(SolveOpts)]
    lib.h2s_solve.argtypes = [vp, vp, vp, i32, i64, i64, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), vp]
    lib.h2s_group_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
    lib.h2s_group_apply.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.h2s_group_free.argtypes = [vp]
    lib.h2s_get_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
    lib.h2s_set_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
    lib.h2s_tune.argtypes = [vp, vp, vp, i32, ctypes.POINTER(TuneInfo), vp]
    lib.h2s_eval_rate.argtypes = [ctypes.POINTER(Kernel), i32, i32, f64p, vp]
    lib.h2s_apply_noalloc.argtypes = [vp, vp, vp, i32, i64, i64, vp]
    for name in ("h2s_build", "h2s_apply", "h2s_apply_phases", "h2s_free", "h2s_get_stats", "h2s_export",
                 "h2s_set_allocator", "h2s_last_error", "h2s_set_profiling", "h2s_get_profile",
                 "h2s_solve_opts_default", "h2s_solve", "h2s_get_schedule", "h2s_set_schedule", "h2s_tune",
                 "h2s_group_create", "h2s_group_apply", "h2s_group_free", "h2s_eval_rate", "h2s_apply_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def header_functions():
    """Names of the functions include/h2s.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(h2s_\w+)\s*\(", text, re.M)))


def status_string(s):
    return load().h2s_status_string(int(s)).decode()


def last_error():
    buf = ctypes.create_string_buffer(512)
    load().h2s_last_error(buf, 512)
    return buf.value.decode()


def check(status):
    if status != OK:
        raise H2SError(status, last_error())


def _stream_ptr(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return ctypes.c_void_p(0)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


class Tree:
    """Handle returned by h2s_build."""

    def __init__(self, handle, n, d):
        self._h = handle
        self.n, self.d = n, d

    def __del__(self):
        self.free()

    def free(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.h2s_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def _check_shape(self, v, name, ncols=None):
        """Reject a vector the kernels would read or write out of bounds: it must be a vector or
        an (n, m) matrix with n rows (and ncols columns when given)."""
        import torch
        if not isinstance(v, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if v.dim() not in (1, 2) or v.shape[0] != self.n:
            raise ValueError(f"{name} must have {self.n} rows (got shape {tuple(v.shape)})")
        if v.dim() == 2 and v.shape[1] == 0:
            raise ValueError(f"{name} has no columns")
        if ncols is not None and (1 if v.dim() == 1 else v.shape[1]) != ncols:
            raise ValueError(f"{name} must have {ncols} columns (got shape {tuple(v.shape)})")

    @staticmethod
    def _check_type(v, name):
        import torch
        if v.dtype != torch.float64 or not v.is_cuda:
            raise TypeError(f"{name} must be a CUDA float64 tensor")

    def _check_vec(self, v, name, ncols=None):
        self._check_shape(v, name, ncols)
        self._check_type(v, name)

    def _out_ld(self, y, name, m):
        """Leading dimension of an output y (checked like an input), which must be contiguous in
        its rows (column-major)."""
        self._check_vec(y, name, m)
        if y.stride(0) != 1:
            raise ValueError(f"{name} must be column-major (stride(0) == 1)")
        return self.n if y.dim() == 1 or y.shape[1] == 1 else y.stride(1)

    def apply(self, x, y=None, mask=PHASE_ALL, stream=None):
        """y = K~ x for a CUDA float64 tensor x of shape (n,) or column-major (n, m)."""
        import torch
        self._check_shape(x, "x")
        if y is not None:
            self._check_shape(y, "y", 1 if x.dim() == 1 else x.shape[1])
        self._check_type(x, "x")
        if x.dim() == 1:
            xx = x.contiguous()
            m, ldx = 1, self.n
        else:
            if x.stride(0) != 1:
                x = x.t().contiguous().t()
            xx, m, ldx = x, x.shape[1], x.stride(1) if x.shape[1] > 1 else self.n
        if y is None:
            y = torch.empty_strided(tuple(x.shape), (1,) if x.dim() == 1 else (1, self.n), dtype=torch.float64,
                                    device=x.device)
        ldy = self._out_ld(y, "y", m)
        check(load().h2s_apply_phases(self._h, mask, ctypes.c_void_p(xx.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                      m, ldx, ldy, _stream_ptr(stream)))
        return y

    def apply_noalloc_ptr(self, x_ptr, y_ptr, nrhs, ldx=None, ldy=None, stream=None):
        """Raw-pointer form of h2s_apply_noalloc (pointers as ints); returns the status."""
        return load().h2s_apply_noalloc(self._h, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr), nrhs,
                                        ldx or self.n, ldy or self.n, _stream_ptr(stream))

    def apply_ptr(self, x_ptr, y_ptr, nrhs=1, ldx=None, ldy=None, mask=PHASE_ALL, stream=None):
        """Raw-pointer form of h2s_apply_phases (pointers as ints)."""
        return load().h2s_apply_phases(self._h, mask, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr), nrhs,
                                       ldx or self.n, ldy or self.n, _stream_ptr(stream))

    def solve(self, b, x=None, restart=50, rtol=1e-8, inner_prec=FP32, inner_rtol=1e-6, max_iter=10000,
              max_refine=1000, use_x0=False, stream=None, raise_on_fail=True):
        """Solve K~ x = b (h2s_solve) for a CUDA float64 b of shape (n,) or column-major (n, m).

        Returns (x, [info dict per right-hand side]).  NOT_CONVERGED raises unless raise_on_fail is False."""
        import torch
        self._check_shape(b, "b")
        if x is not None:
            self._check_shape(x, "x", 1 if b.dim() == 1 else b.shape[1])
        self._check_type(b, "b")
        if b.dim() == 1:
            bb, m, ldb = b.contiguous(), 1, self.n
        else:
            if b.stride(0) != 1:
                b = b.t().contiguous().t()
            bb, m, ldb = b, b.shape[1], b.stride(1) if b.shape[1] > 1 else self.n
        if x is None:
            x = torch.zeros_like(bb) if bb.dim() == 1 else torch.zeros(
                (m, self.n), dtype=torch.float64, device=b.device).t()
        ldx = self._out_ld(x, "x", m)
        o = SolveOpts()
        check(load().h2s_solve_opts_default(ctypes.byref(o)))
        o.restart, o.rtol, o.inner_prec, o.inner_rtol = restart, rtol, inner_prec, inner_rtol
        o.max_iter, o.max_refine, o.use_x0 = max_iter, max_refine, int(bool(use_x0))
        infos = (SolveInfo * m)()
        rc = load().h2s_solve(self._h, ctypes.c_void_p(bb.data_ptr()), ctypes.c_void_p(x.data_ptr()), m, ldb, ldx,
                              ctypes.byref(o), infos, _stream_ptr(stream))
        if rc != OK and (rc != ERR_NOT_CONVERGED or raise_on_fail):
            check(rc)
        return x, [{"iterations": i.iterations, "refinements": i.refinements, "converged": bool(i.converged),
                    "residual": i.residual, "status": rc} for i in infos]

    def solve_ptr(self, b_ptr, x_ptr, nrhs=1, ldb=None, ldx=None, opts=None, infos=None, stream=None):
        """Raw-pointer form of h2s_solve (pointers as ints); returns the status."""
        return load().h2s_solve(self._h, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr), nrhs, ldb or self.n,
                                ldx or self.n, None if opts is None else ctypes.byref(opts), infos,
                                _stream_ptr(stream))

    def set_profiling(self, on=True):
        check(load().h2s_set_profiling(self._h, int(bool(on))))

    def schedule(self):
        """The launch schedule: {"near_first", "up_threads", "dn_threads", "m2l_stream"}
        (widths per level 0..32)."""
        sc = Schedule()
        check(load().h2s_get_schedule(self._h, ctypes.byref(sc)))
        return {"near_first": sc.near_first, "up_threads": list(sc.up_threads), "dn_threads": list(sc.dn_threads),
                "m2l_stream": sc.m2l_stream}

    def set_schedule(self, near_first=None, up_threads=None, dn_threads=None, m2l_stream=None):
        """Replace fields of the launch schedule (others kept); see h2s_set_schedule."""
        cur = self.schedule()
        sc = Schedule()
        sc.near_first = cur["near_first"] if near_first is None else float(near_first)
        sc.m2l_stream = cur["m2l_stream"] if m2l_stream is None else int(m2l_stream)
        for name, new in (("up_threads", up_threads), ("dn_threads", dn_threads)):
            vals = list(cur[name])
            if new is not None:
                for l, w in (new.items() if isinstance(new, dict) else enumerate(new)):
                    vals[l] = int(w)
            getattr(sc, name)[:] = vals
        check(load().h2s_set_schedule(self._h, ctypes.byref(sc)))

    def tune(self, x, y, reps=5, stream=None):
        """Autotune the launch schedule on device vectors x, y (CUDA float64, length n); y = K~ x on return.
        Returns {"ms_entry", "ms_tuned", "candidates"}."""
        self._check_vec(x, "x", 1)
        self._out_ld(y, "y", 1)
        if x.dim() == 1 and x.stride(0) != 1:
            raise ValueError("x must be contiguous")
        info = TuneInfo()
        check(load().h2s_tune(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), int(reps),
                              ctypes.byref(info), _stream_ptr(stream)))
        return {"ms_entry": info.ms_entry, "ms_tuned": info.ms_tuned, "candidates": info.candidates}

    def profile(self):
        """{kernel class: (total ms, launches)} since the last call; waits for the recorded events."""
        ms = (ctypes.c_double * len(PROF_NAMES))()
        cnt = (ctypes.c_int64 * len(PROF_NAMES))()
        check(load().h2s_get_profile(self._h, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(PROF_NAMES)}

    def stats(self):
        s = Stats()
        check(load().h2s_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def export(self, path):
        check(load().h2s_export(self._h, str(path).encode()))
        return read_export(path)



class Group:
    """Trees applied together: one captured graph per tree, each launched on a stream of the
    group's own (h2s_group_apply)."""

    def __init__(self, trees):
        self.trees = list(trees)  # the trees must outlive the group
        arr = (ctypes.c_void_p * len(self.trees))(*[T.handle for T in self.trees])
        h = ctypes.c_void_p()
        check(load().h2s_group_create(arr, len(self.trees), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        self.free()

    def free(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.h2s_group_free(self._h)
            self._h = None

    def apply(self, xs, ys, stream=None):
        """ys[i] = K~_i xs[i] for CUDA float64 vectors (one per tree), ordered on stream."""
        n = len(self.trees)
        if len(xs) != n or len(ys) != n:
            raise ValueError("one x and one y per tree")
        for T, x, y in zip(self.trees, xs, ys):
            T._check_vec(x, "x", 1)
            T._out_ld(y, "y", 1)
            if x.stride(0) != 1:
                raise ValueError("x must be contiguous")
        xa = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        ya = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
        check(load().h2s_group_apply(self._h, xa, ya, _stream_ptr(stream)))
        return ys

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p))
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = None


def set_allocator(alloc=None, free=None):
    """h2s_set_allocator with Python callables: alloc(nbytes) -> device pointer (int) or 0 on
    failure, free(ptr).  None, None restores hipMalloc / hipFree.  Affects later builds only."""
    global _allocator_refs
    lib = load()
    if alloc is None and free is None:
        check(lib.h2s_set_allocator(None, None, None))
        _allocator_refs = None
        return

    def _a(ctx, nbytes, out):
        try:
            p = int(alloc(int(nbytes)) or 0)
        except Exception:  # a failing allocator reports failure, it does not raise into C
            p = 0
        out[0] = p or None
        return 0 if p else 1

    def _f(ctx, ptr):
        try:
            free(int(ptr))
        except Exception:
            pass

    refs = (_ALLOC_FN(_a), _FREE_FN(_f))
    check(lib.h2s_set_allocator(ctypes.cast(refs[0], ctypes.c_void_p), ctypes.cast(refs[1], ctypes.c_void_p), None))
    _allocator_refs = refs  # the C library holds these pointers


def build(points, kind=LOG_R, leaf_size=64, eps=1e-8, eps_ver=None, variant=H2STAR, prec=FP64, param=0.0,
          diag=None, shift=0.0, host_threads=0, host_only=False, stream=None, hbm_budget_bytes=0):
    """h2s_build on host points (n, d) float64.  hbm_budget_bytes > 0 caps the device memory the
    handle may ever hold (an allocation beyond it fails as OUT_OF_MEMORY)."""
    lib = load()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, d = pts.shape
    if diag is None:
        diag = 0.0 if kind in (LOG_R, INV_R, RBF_AR, RBF_LOG) else 1.0
    k = Kernel(kind, param, diag, shift)
    o = BuildOpts(leaf_size, eps, eps if eps_ver is None else eps_ver, variant, prec, host_threads, int(host_only),
                  int(hbm_budget_bytes))
    h = ctypes.c_void_p()
    check(lib.h2s_build(pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n, d, ctypes.byref(k), ctypes.byref(o),
                        _stream_ptr(stream) if not host_only else ctypes.c_void_p(0), ctypes.byref(h)))
    return Tree(h, n, d)


def eval_rate(kind=LOG_R, d=2, prec=FP64, param=0.0, stream=None):
    """h2s_eval_rate: peak kernel evaluations per second of the device kernel function
    (register-resident loop, fastest of five launches)."""
    out = ctypes.c_double()
    k = Kernel(kind, param, 0.0, 0.0)
    check(load().h2s_eval_rate(ctypes.byref(k), d, prec, ctypes.byref(out), _stream_ptr(stream)))
    return out.value


_DT = {1: np.int32, 2: np.int64, 3: np.float64}


def read_export(path):
    """Parse the named-array container written by h2s_export."""
    with open(path, "rb") as f:
        buf = f.read()
    if buf[:4] != b"H2SX":
        raise ValueError("not an h2s export file")
    count = int(np.frombuffer(buf, np.uint32, 1, 8)[0])
    pos, out = 12, {}
    for _ in range(count):
        name = buf[pos:pos + 32].split(b"\0", 1)[0].decode()
        dtype, ndim = np.frombuffer(buf, np.uint32, 2, pos + 32)
        dims = np.frombuffer(buf, np.int64, int(ndim), pos + 40)
        pos += 40 + 8 * int(ndim)
        cnt = int(np.prod(dims)) if ndim else 1
        dt = np.dtype(_DT[int(dtype)])
        out[name] = np.frombuffer(buf, dt, cnt, pos).reshape(tuple(int(x) for x in dims)).copy()
        pos += cnt * dt.itemsize
    return out
