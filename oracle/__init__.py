"""Python view of the plain-C FP64 oracle (oracle/h2s_oracle.c).

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this package.  It shares no code with the
library in paper_2309_14085_amd/.

Kernel kinds: 0 = log r, 1 = 1/r, 2 = exp(-r^2/h^2), 3 = exp(-r),
4 = a/r (r >= a) | r/a (r < a), 5 = log r/log a (r >= a) | (r log r - 1)/(a log a - 1) (r < a),
6 = (|x-y|^2 + (c(x) - c(y))^2 + 1)^(3/2) with c(x) = exp(-(x_1 + x_3)) (3D only).
Variants: 0 = H2*(b+t), 1 = (H2+H)*.
Families: 0 = far field (B2T NCA), 1 = vertex sharing (T2B NCA).
Lists: 0 = near field N* (leaf level), 1 = IL_far, 2 = IL_ver.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

LOG_R, INV_R, GAUSS, EXP_R, RBF_AR, RBF_LOG, NTI_MQ = 0, 1, 2, 3, 4, 5, 6
H2STAR, H2_PLUS_H = 0, 1
FAR, VER = 0, 1
NEAR_LIST, FAR_LIST, VER_LIST = 0, 1, 2

_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    lib.orc_build.restype = ctypes.c_void_p
    lib.orc_build.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_double,
                              ctypes.c_double, ctypes.c_int]
    lib.orc_free.argtypes = [ctypes.c_void_p]
    lib.orc_apply.argtypes = [ctypes.c_void_p, _f64p, _f64p, _f64p, _f64p]
    lib.orc_direct.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, _f64p, _i64p, ctypes.c_int64, _f64p]
    lib.orc_aca_dense.restype = ctypes.c_int64
    lib.orc_aca_dense.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, _i64p, _i64p,
                                  _f64p, _f64p]
    lib.orc_info.restype = ctypes.c_int64
    lib.orc_info.argtypes = [ctypes.c_void_p, _i64p]
    lib.orc_cube.argtypes = [ctypes.c_void_p, _f64p]
    lib.orc_perm.argtypes = [ctypes.c_void_p, _i64p]
    lib.orc_nbox.restype = ctypes.c_int64
    lib.orc_nbox.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc_boxes.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64p, _i32p, _i64p, _i64p, _i64p]
    lib.orc_list_len.restype = ctypes.c_int64
    lib.orc_list_len.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.orc_list.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _i64p, _i64p]
    lib.orc_rank.restype = ctypes.c_int64
    lib.orc_rank.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64]
    lib.orc_pivots.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _i64p, _i64p]
    lib.orc_operator.restype = ctypes.c_int64
    lib.orc_operator.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _f64p]
    lib.orc_hph_npairs.restype = ctypes.c_int64
    lib.orc_hph_npairs.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc_hph_pair.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, _i64p, _f64p, _f64p]
    lib.orc_tree_points.argtypes = [ctypes.c_void_p, _f64p]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_import.restype = ctypes.c_void_p
    lib.orc_import.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.orc_depth.restype = ctypes.c_int
    lib.orc_depth.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int64]
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def default_diag(kind):
    """K(x, x): 0 for log r, 1/r and the two piecewise RBFs, whose systems leave out
    j = i (the paper's convention), 1 for the Gaussian, exp(-r) and the NTI multiquadric
    (its value at x = y)."""
    return 0.0 if kind in (LOG_R, INV_R, RBF_AR, RBF_LOG) else 1.0


def _check_dim(kind, d):
    if kind == NTI_MQ and d != 3:
        raise ValueError("the NTI multiquadric is defined in 3D only")


def direct(points, q, kind, param=0.0, diag=None, shift=0.0, rows=None):
    """Direct product phi = (K + shift I) q, compensated FP64 (rows: optional subset)."""
    lib = _load()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, d = pts.shape
    _check_dim(kind, d)
    q = np.ascontiguousarray(q, dtype=np.float64)
    if diag is None:
        diag = default_diag(kind)
    if rows is None:
        out = np.empty(n)
        lib.orc_direct(_p(pts, _f64p), n, d, kind, param, diag, shift, _p(q, _f64p), None, n, _p(out, _f64p))
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.empty(len(rows))
        lib.orc_direct(_p(pts, _f64p), n, d, kind, param, diag, shift, _p(q, _f64p), _p(rows, _i64p),
                       len(rows), _p(out, _f64p))
    return out


def aca_dense(M, eps):
    """ACA of an explicit matrix: returns (row pivots, col pivots, U, V) with M ~ U V^T."""
    lib = _load()
    M = np.ascontiguousarray(M, dtype=np.float64)
    nI, nJ = M.shape
    mr = max(1, min(nI, nJ))
    prow = np.zeros(mr, np.int64)
    pcol = np.zeros(mr, np.int64)
    U = np.zeros((mr, nI))
    V = np.zeros((mr, nJ))
    r = lib.orc_aca_dense(_p(M, _f64p), nI, nJ, eps, _p(prow, _i64p), _p(pcol, _i64p), _p(U, _f64p), _p(V, _f64p))
    return prow[:r].copy(), pcol[:r].copy(), U[:r].T.copy(), V[:r].T.copy()


def depth(n, d, nmax):
    """Leaf level kappa of the uniform 2^d tree for n points and leaf size nmax."""
    return int(_load().orc_depth(n, d, nmax))


def num_threads():
    return _load().orc_num_threads()


def set_threads(n):
    """Threads of the oracle's parallel loops from now on (n <= 0: every host core)."""
    _load().orc_set_threads(int(n))


class Tree:
    """An oracle H2* / (H2+H)* representation built from user-order points."""

    def __init__(self, points, kind, nmax, eps_far, eps_ver=None, variant=H2STAR, param=0.0,
                 diag=None, shift=0.0):
        lib = _load()
        pts = np.ascontiguousarray(points, dtype=np.float64)
        n, d = pts.shape
        _check_dim(kind, d)
        if eps_ver is None:
            eps_ver = eps_far
        if diag is None:
            diag = default_diag(kind)
        self.kind, self.param, self.diag, self.shift = kind, param, diag, shift
        self._h = lib.orc_build(_p(pts, _f64p), n, d, kind, param, diag, shift, nmax, eps_far, eps_ver, variant)
        if not self._h:
            raise ValueError("oracle build rejected its arguments")
        info = np.zeros(6, np.int64)
        lib.orc_info(self._h, _p(info, _i64p))
        self.d, self.n, self.kappa, self.variant, self.nmax, self.total_boxes = (int(v) for v in info)

    @classmethod
    def from_export(cls, path, kind, param=0.0, diag=None, shift=0.0):
        """Import mode: the representation another builder wrote to `path` (the library's
        export container: tree, permutation, lists, pivots, FP64 operators, (H2+H)* factors),
        for the kernel it was built with.  apply() then runs the MVP of Sec. 5.1.2 / 5.2.2 on
        exactly those operators."""
        lib = _load()
        if diag is None:
            diag = default_diag(kind)
        h = lib.orc_import(str(path).encode(), kind, param, diag, shift)
        if not h:
            raise ValueError(f"oracle import rejected {path}")
        self = cls.__new__(cls)
        self.kind, self.param, self.diag, self.shift = kind, param, diag, shift
        self._h = h
        info = np.zeros(6, np.int64)
        lib.orc_info(self._h, _p(info, _i64p))
        self.d, self.n, self.kappa, self.variant, self.nmax, self.total_boxes = (int(v) for v in info)
        return self

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    def apply_parts(self, q):
        """(near, far, vertex) potentials in user order; near includes shift*q."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        near, far, ver = np.empty(self.n), np.empty(self.n), np.empty(self.n)
        _lib.orc_apply(self._h, _p(q, _f64p), _p(near, _f64p), _p(far, _f64p), _p(ver, _f64p))
        return near, far, ver

    def apply(self, q):
        near, far, ver = self.apply_parts(q)
        return near + far + ver

    def cube(self):
        out = np.zeros(4)
        _lib.orc_cube(self._h, _p(out, _f64p))
        return out[: self.d].copy(), float(out[3])

    def perm(self):
        out = np.zeros(self.n, np.int64)
        _lib.orc_perm(self._h, _p(out, _i64p))
        return out

    def tree_points(self):
        out = np.zeros((self.n, self.d))
        _lib.orc_tree_points(self._h, _p(out, _f64p))
        return out

    def boxes(self, level):
        nb = _lib.orc_nbox(self._h, level)
        morton = np.zeros(nb, np.int64)
        coord = np.zeros((nb, self.d), np.int32)
        begin = np.zeros(nb, np.int64)
        end = np.zeros(nb, np.int64)
        parent = np.zeros(nb, np.int64)
        _lib.orc_boxes(self._h, level, _p(morton, _i64p), _p(coord, _i32p), _p(begin, _i64p), _p(end, _i64p),
                       _p(parent, _i64p))
        return dict(morton=morton, coord=coord, begin=begin, end=end, parent=parent)

    def lists(self, which, level):
        nb = _lib.orc_nbox(self._h, level)
        ln = _lib.orc_list_len(self._h, which, level)
        off = np.zeros(nb + 1, np.int64)
        idx = np.zeros(max(ln, 1), np.int64)
        _lib.orc_list(self._h, which, level, _p(off, _i64p), _p(idx, _i64p))
        return off, idx[:ln].copy()

    def rank(self, fam, level, box):
        return int(_lib.orc_rank(self._h, fam, level, box))

    def pivots(self, fam, level, box):
        r = self.rank(fam, level, box)
        if r <= 0:
            return np.zeros(0, np.int64), np.zeros(0, np.int64)
        row = np.zeros(r, np.int64)
        col = np.zeros(r, np.int64)
        _lib.orc_pivots(self._h, fam, level, box, _p(row, _i64p), _p(col, _i64p))
        return row, col

    def operator(self, fam, level, box):
        """Leaf: U_X (n_X x r).  Non-leaf: stacked L2L operators (sum r_c x r)."""
        r = self.rank(fam, level, box)
        if r <= 0:
            return np.zeros((0, 0))
        nrow = _lib.orc_operator(self._h, fam, level, box, None)
        out = np.zeros((r, nrow))
        _lib.orc_operator(self._h, fam, level, box, _p(out, _f64p))
        return out.T.copy()

    def hph_pairs(self, level):
        np_ = _lib.orc_hph_npairs(self._h, level)
        b = self.boxes(level)
        out = []
        for p in range(np_):
            info = np.zeros(3, np.int64)
            _lib.orc_hph_pair(self._h, level, p, _p(info, _i64p), None, None)
            x, y, r = (int(v) for v in info)
            nx = int(b["end"][x] - b["begin"][x])
            ny = int(b["end"][y] - b["begin"][y])
            ub = np.zeros((max(r, 0), nx))
            vb = np.zeros((max(r, 0), ny))
            _lib.orc_hph_pair(self._h, level, p, _p(info, _i64p), _p(ub, _f64p), _p(vb, _f64p))
            out.append((x, y, ub.T.copy(), vb.T.copy()))
        return out
