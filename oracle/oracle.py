"""ctypes front-end of the FP64 CPU oracle (``smash_oracle.c``).

TEST INFRASTRUCTURE ONLY: only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It never touches the
HIP library and the HIP library never touches it.

The oracle follows the paper step by step (Sec. 3.1 partition, eqs. (3.3)-(3.5)
pair lists, eq. (2.2) interpolation basis, Thm. 2.4 / eq. (2.14) compr,
eqs. (3.6)-(3.20) level-wise construction, Sec. 3.4 product); the C source
names the passage each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smash_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KERNELS = {"inv_r": 0, "log_r": 1, "exp_r": 2, "cauchy": 3, "double_layer": 4}

# export codes (mirrored from smash_oracle.c)
EX_PERM_X, EX_PERM_Y, EX_NODES, EX_BOXES, EX_L, EX_LM = 1, 2, 3, 4, 5, 6
EX_NEAR_PTR, EX_NEAR_IDX, EX_RANKS = 7, 8, 9
EX_ROW_SEL, EX_ROW_G, EX_COL_SEL, EX_COL_G, EX_ROW_GRID, EX_COL_GRID = 10, 11, 12, 13, 14, 15
EX_SIZES, EX_LEVELS, EX_SWAPS, EX_MARGINS, EX_DECISION_MARGINS = 16, 17, 18, 19, 20
_DOUBLE_EXPORTS = {EX_BOXES, EX_ROW_G, EX_COL_G, EX_MARGINS, EX_DECISION_MARGINS}
# columns of EX_DECISION_MARGINS per side (row side first, then column side)
DECISIONS = ("pivot", "rank cutoff", "swap", "SVD cutoff")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.oracle_build.argtypes = [dp, C.c_int64, dp, C.c_int64, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                   C.c_double, C.c_double, C.c_double, C.c_int, dp,
                                   C.c_double, C.c_int, dp, C.POINTER(C.c_void_p)]
        L.oracle_build.restype = C.c_int
        L.oracle_build_basis.argtypes = list(L.oracle_build.argtypes[:-1]) + [
            C.c_int, C.POINTER(C.c_void_p)]
        L.oracle_build_basis.restype = C.c_int
        L.oracle_taylor_basis.argtypes = [dp, C.c_int, C.c_double, C.c_double, C.c_int, dp]
        L.oracle_taylor_basis.restype = None
        L.oracle_build_tree.argtypes = [dp, C.c_int64, dp, C.c_int64, C.c_int, C.c_int, C.c_int,
                                        C.c_int, C.c_int, C.c_double, C.c_int, dp, C.c_double,
                                        C.c_int, dp, C.POINTER(C.c_void_p)]
        L.oracle_build_tree.restype = C.c_int
        L.oracle_matvec.argtypes = [C.c_void_p, dp, C.c_int64, dp]
        L.oracle_matvec.restype = C.c_int
        L.oracle_export.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(C.c_int64)]
        L.oracle_export.restype = C.c_int
        L.oracle_destroy.argtypes = [C.c_void_p]
        L.oracle_destroy.restype = None
        L.oracle_dense_matvec.argtypes = [dp, C.c_int64, dp, C.c_int64, C.c_int, C.c_int,
                                          C.c_double, dp, dp, dp, C.c_int64, dp]
        L.oracle_dense_matvec.restype = None
        L.oracle_cauchy_like_dense.argtypes = [dp, C.c_int64, dp, C.c_int64, dp, dp, C.c_int,
                                               dp, C.c_int64, dp]
        L.oracle_cauchy_like_dense.restype = None
        L.oracle_cauchy_like_matvec.argtypes = [C.c_void_p, dp, dp, C.c_int, dp, C.c_int64, dp]
        L.oracle_cauchy_like_matvec.restype = C.c_int
        L.oracle_dense_rows.argtypes = [dp, C.c_int64, dp, C.c_int64, C.c_int, C.c_int,
                                        C.c_double, dp, dp, C.POINTER(C.c_int64), C.c_int64,
                                        dp, C.c_int64, dp]
        L.oracle_dense_rows.restype = None
        L.oracle_kernel_block.argtypes = [dp, dp, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                          C.c_double, dp, dp, dp]
        L.oracle_kernel_block.restype = None
        L.oracle_compr.argtypes = [dp, C.c_int, C.c_int, C.c_double, C.c_double, ip, ip, dp, ip]
        L.oracle_compr.restype = C.c_int
        L.oracle_interp_basis.argtypes = [dp, C.c_int, C.c_int, dp, dp, C.c_int, dp]
        L.oracle_interp_basis.restype = None
        L.oracle_left_svd.argtypes = [dp, C.c_int, C.c_int, C.c_double, dp, dp]
        L.oracle_left_svd.restype = C.c_int
        L.oracle_well_separated_boxes.argtypes = [dp, dp, dp, dp, C.c_int, C.c_double]
        L.oracle_well_separated_boxes.restype = C.c_int
        L.oracle_point_key.argtypes = [dp, C.c_int, C.c_int, dp, dp, C.c_int]
        L.oracle_point_key.restype = C.c_uint64
        L.oracle_order_rule.argtypes = [C.c_double, C.c_double]
        L.oracle_order_rule.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _data(a, n):
    """per-point data (n x 3: m_1, m_2, diagonal) of the double-layer kernel"""
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (n, 3):
        raise ValueError("point data must be (n, 3)")
    return a


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


class Oracle:
    """An oracle construction: tree, pair lists, IDs; ``matvec`` applies it."""

    def __init__(self, x, y=None, *, kernel="inv_r", leaf=32, order=10, adm=1, tol=1e-10,
                 tau=None, eps_svd=None, f=2.0, diag=None, root=None, max_depth=0,
                 point_data=None, tree_only=False, basis="chebyshev"):
        x = _f64(x)
        if x.ndim == 1:
            x = x[:, None]
        same = y is None
        y = x if same else _f64(y)
        if y.ndim == 1:
            y = y[:, None]
        d = x.shape[1]
        kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        if tau is None:
            tau = 0.6 if d == 1 else 0.7
        if eps_svd is None:
            eps_svd = tol
        if diag is None:
            diag = 1.0 if kid == 2 else 0.0
        has_root = root is not None
        rlo = np.zeros(3)
        side = 0.0
        if has_root:
            rlo[:d] = np.asarray(root[0], dtype=np.float64).reshape(-1)[:d]
            side = float(root[1])
        self.d, self.kid, self.adm, self.diag = d, kid, adm, diag
        self.x, self.y, self.same = x, y, same
        self.point_data = _data(point_data, x.shape[0])
        h = C.c_void_p()
        if tree_only:  # partition and pair lists only (no generators, no product)
            rc = lib().oracle_build_tree(_dp(x), x.shape[0], _dp(y), y.shape[0], int(same), d,
                                         kid, int(leaf), int(adm), float(tau), int(has_root),
                                         _dp(rlo), side, int(max_depth), _dp(self.point_data),
                                         C.byref(h))
        else:
            if basis not in ("chebyshev", "taylor"):
                raise ValueError("basis must be 'chebyshev' or 'taylor'")
            rc = lib().oracle_build_basis(_dp(x), x.shape[0], _dp(y), y.shape[0], int(same), d,
                                          kid, int(leaf), int(order), int(adm), float(tol),
                                          float(tau), float(eps_svd), float(f), float(diag),
                                          int(has_root), _dp(rlo), side, int(max_depth),
                                          _dp(self.point_data), int(basis == "taylor"),
                                          C.byref(h))
        if rc != 0:
            raise OracleError("oracle_build failed with code %d" % rc)
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and h.value:
            lib().oracle_destroy(h)
            self._h = None

    def export(self, what):
        n = C.c_int64(0)
        rc = lib().oracle_export(self._h, what, None, C.byref(n))
        if rc != 0:
            raise OracleError("export %d failed" % what)
        dt = np.float64 if what in _DOUBLE_EXPORTS else np.int32
        out = np.zeros(max(n.value, 1), dtype=dt)
        if n.value:
            lib().oracle_export(self._h, what, out.ctypes.data_as(C.c_void_p), C.byref(n))
        return out[: n.value]

    # convenient views ---------------------------------------------------
    def sizes(self):
        s = self.export(EX_SIZES)
        return dict(nx=int(s[0]), ny=int(s[1]), nnodes=int(s[2]), nlevels=int(s[3]),
                    nL=int(s[4]), nLm=int(s[5]), d=int(s[6]), adm=int(s[7]))

    def nodes(self):
        return self.export(EX_NODES).reshape(-1, 8)

    def boxes(self):
        return self.export(EX_BOXES).reshape(-1, 6)

    def L(self):
        return self.export(EX_L).reshape(-1, 2)

    def Lm(self):
        return self.export(EX_LM).reshape(-1, 2)

    def ranks(self):
        return self.export(EX_RANKS).reshape(-1, 6)

    def matvec(self, Q):
        Q = _f64(Q)
        vec = Q.ndim == 1
        if vec:
            Q = Q[:, None]
        Q = np.ascontiguousarray(Q)
        Z = np.zeros((self.x.shape[0], Q.shape[1]))
        rc = lib().oracle_matvec(self._h, _dp(Q), Q.shape[1], _dp(Z))
        if rc != 0:
            raise OracleError("oracle_matvec failed with code %d" % rc)
        return Z[:, 0] if vec else Z

    def cauchy_like_matvec(self, w, v, Q):
        """sum_l w_l o (C-hat (v_l o Q)) over the generator columns l (eq. (6.2)),
        C-hat this handle's approximation; w: (nx, p), v: (ny, p)."""
        w, v = np.ascontiguousarray(_f64(w)), np.ascontiguousarray(_f64(v))
        Q = _f64(Q)
        vec = Q.ndim == 1
        Q = np.ascontiguousarray(Q[:, None] if vec else Q)
        p = w.shape[1]
        Z = np.zeros((self.x.shape[0], Q.shape[1]))
        rc = lib().oracle_cauchy_like_matvec(self._h, _dp(w), _dp(v), p, _dp(Q), Q.shape[1],
                                             _dp(Z))
        if rc != 0:
            raise OracleError("oracle_cauchy_like_matvec failed with code %d" % rc)
        return Z[:, 0] if vec else Z

    def per_node(self, side="row"):
        """List of (grid, sel, G) per node (root entry is empty)."""
        rk = self.ranks()
        if side == "row":
            grid, sel, G = self.export(EX_ROW_GRID), self.export(EX_ROW_SEL), self.export(EX_ROW_G)
            mcol, kcol = 0, 1
        else:
            grid, sel, G = self.export(EX_COL_GRID), self.export(EX_COL_SEL), self.export(EX_COL_G)
            mcol, kcol = 2, 3
        out = [(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, 0)))]
        og = og2 = 0
        for i in range(1, rk.shape[0]):
            m, k = int(rk[i, mcol]), int(rk[i, kcol])
            out.append((grid[og:og + m], sel[og:og + m], G[og2:og2 + (m - k) * k].reshape(m - k, k)))
            og += m
            og2 += (m - k) * k
        return out


def _pts(a):
    a = _f64(a)
    return a[:, None] if a.ndim == 1 else a


def dense_matvec(x, y, Q, kernel="inv_r", diag=None, data_x=None, data_y=None):
    """Exact A Q with A = [kappa(x, y)] (definition of A in Sec. 3); data_x,
    data_y: the points' data for the double-layer kernel."""
    x, y = _pts(x), _pts(y)
    data_x, data_y = _data(data_x, x.shape[0]), _data(data_y, y.shape[0])
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    if diag is None:
        diag = 1.0 if kid == 2 else 0.0
    Q = _f64(Q)
    vec = Q.ndim == 1
    Q = np.ascontiguousarray(Q[:, None] if vec else Q)
    Z = np.zeros((x.shape[0], Q.shape[1]))
    lib().oracle_dense_matvec(_dp(x), x.shape[0], _dp(y), y.shape[0], x.shape[1], kid,
                              float(diag), _dp(data_x), _dp(data_y), _dp(Q), Q.shape[1], _dp(Z))
    return Z[:, 0] if vec else Z


def cauchy_like_dense(x, y, w, v, Q):
    """Exact A Q for the Cauchy-like matrix of eq. (6.1): a_ij = sum_l w_il v_jl /
    (x_i - y_j), points on the real line; w: (nx, p), v: (ny, p)."""
    x, y = np.ascontiguousarray(_f64(x).ravel()), np.ascontiguousarray(_f64(y).ravel())
    w, v = np.ascontiguousarray(_f64(w)), np.ascontiguousarray(_f64(v))
    Q = _f64(Q)
    vec = Q.ndim == 1
    Q = np.ascontiguousarray(Q[:, None] if vec else Q)
    Z = np.zeros((x.shape[0], Q.shape[1]))
    lib().oracle_cauchy_like_dense(_dp(x), x.shape[0], _dp(y), y.shape[0], _dp(w), _dp(v),
                                   w.shape[1], _dp(Q), Q.shape[1], _dp(Z))
    return Z[:, 0] if vec else Z


def dense_rows(x, y, rows, Q, kernel="inv_r", diag=None, data_x=None, data_y=None):
    """Exact rows of A Q for the given original row indices."""
    x, y = _pts(x), _pts(y)
    data_x, data_y = _data(data_x, x.shape[0]), _data(data_y, y.shape[0])
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    if diag is None:
        diag = 1.0 if kid == 2 else 0.0
    Q = _f64(Q)
    vec = Q.ndim == 1
    Q = np.ascontiguousarray(Q[:, None] if vec else Q)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    Z = np.zeros((rows.shape[0], Q.shape[1]))
    lib().oracle_dense_rows(_dp(x), x.shape[0], _dp(y), y.shape[0], x.shape[1], kid,
                            float(diag), _dp(data_x), _dp(data_y),
                            rows.ctypes.data_as(C.POINTER(C.c_int64)),
                            rows.shape[0], _dp(Q), Q.shape[1], _dp(Z))
    return Z[:, 0] if vec else Z


def kernel_block(P, Qp, kernel="inv_r", diag=None, data_P=None, data_Q=None):
    P, Qp = _pts(P), _pts(Qp)
    data_P, data_Q = _data(data_P, P.shape[0]), _data(data_Q, Qp.shape[0])
    kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    if diag is None:
        diag = 1.0 if kid == 2 else 0.0
    B = np.zeros((P.shape[0], Qp.shape[0]))
    lib().oracle_kernel_block(_dp(P), _dp(Qp), P.shape[0], Qp.shape[0], P.shape[1], kid,
                              float(diag), _dp(data_P), _dp(data_Q), _dp(B))
    return B


def compr(Cm, tol, f=2.0):
    """compr of eq. (2.14) on an m x c matrix: returns (k, skel, rest, G, nswaps)."""
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    m, c = Cm.shape
    k = C.c_int(0)
    ns = C.c_int(0)
    sel = np.zeros(max(m, 1), dtype=np.int32)
    G = np.zeros(max(m * c, 1))
    rc = lib().oracle_compr(_dp(Cm), m, c, float(tol), float(f), C.byref(k),
                            sel.ctypes.data_as(C.POINTER(C.c_int)), _dp(G), C.byref(ns))
    if rc != 0:
        raise OracleError("compr failed with code %d" % rc)
    kk = k.value
    return kk, sel[:kk].copy(), sel[kk:m].copy(), G[: (m - kk) * kk].reshape(m - kk, kk).copy(), ns.value


def interp_basis(pts, lo, hi, p):
    pts = _pts(pts)
    m, d = pts.shape
    lo3 = np.zeros(3)
    hi3 = np.zeros(3)
    lo3[:d] = lo
    hi3[:d] = hi
    out = np.zeros((m, p ** d))
    lib().oracle_interp_basis(_dp(pts), m, d, _dp(lo3), _dp(hi3), p, _dp(out))
    return out


def taylor_basis(pts, lo, hi, p):
    """The Taylor basis (2.4)-(2.5) with r = p terms of the interval [lo, hi] at
    the given points (m x p)."""
    pts = np.ascontiguousarray(_f64(pts).ravel())
    Cm = np.zeros((pts.shape[0], p))
    lib().oracle_taylor_basis(_dp(pts), pts.shape[0], float(lo), float(hi), int(p), _dp(Cm))
    return Cm


def left_svd(A, eps):
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    S = np.zeros((m, m))
    sig = np.zeros(m)
    ks = lib().oracle_left_svd(_dp(A), m, n, float(eps), _dp(S), _dp(sig))
    return S[:, :ks].copy(), sig


def well_separated(lo_i, hi_i, lo_j, hi_j, tau):
    a = [np.zeros(3) for _ in range(4)]
    for t, v in enumerate((lo_i, hi_i, lo_j, hi_j)):
        v = np.atleast_1d(np.asarray(v, dtype=np.float64))
        a[t][: v.shape[0]] = v
    d = np.atleast_1d(lo_i).shape[0]
    return bool(lib().oracle_well_separated_boxes(_dp(a[0]), _dp(a[1]), _dp(a[2]), _dp(a[3]), d,
                                                  float(tau)))


def point_key_of(xv, adm, lo, hi, max_split):
    xv = np.atleast_1d(np.asarray(xv, dtype=np.float64))
    d = xv.shape[0]
    x3, lo3, hi3 = np.zeros(3), np.zeros(3), np.zeros(3)
    x3[:d], lo3[:d], hi3[:d] = xv, lo, hi
    return int(lib().oracle_point_key(_dp(x3), d, int(adm), _dp(lo3), _dp(hi3), int(max_split)))


def order_rule(eps, tau):
    """Sec. 6.1 heuristic expansion order for tolerance eps and ratio tau."""
    return int(lib().oracle_order_rule(float(eps), float(tau)))
