"""Thin ctypes binding of libsmash (include/smash.h).

Argument marshalling only: torch device tensors become raw pointers and the
current torch stream becomes the hipStream_t; every step of the construction
and of the product runs in the HIP library.  If the library is not built,
``lib()`` raises -- there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmash.so")

KERNELS = {"inv_r": 0, "log_r": 1, "exp_r": 2, "cauchy": 3, "double_layer": 4}
ADM = {"weak": 0, "hss": 0, "strong": 1, "h2": 1}
PREC = {"f64": 0, "f32": 1, "bf16": 2}

EX = dict(perm_x=1, perm_y=2, nodes=3, boxes=4, L=5, Lm=6, near_ptr=7, near_idx=8, ranks=9,
          row_sel=10, row_G=11, col_sel=12, col_G=13, row_grid=14, col_grid=15, sizes=16,
          levels=17, coupling=18, near=19)
_F64_EXPORTS = {"boxes", "row_G", "col_G"}


class SmashError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("smash error %d: %s" % (code, msg))
        self.code = code


COUPLING = {"auto": 0, "stored": 1, "evaluated": 2}
# size of the library's per-device array used by smash_matvec_noalloc
NOALLOC_SCRATCH_BYTES = 64 << 20


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("tau", C.c_double), ("eps_svd", C.c_double),
                ("srrqr_f", C.c_double), ("diag_value", C.c_double), ("eval_prec", C.c_int32),
                ("apply_prec", C.c_int32), ("has_root_box", C.c_int32),
                ("root_lo", C.c_double * 3), ("root_side", C.c_double), ("max_depth", C.c_int32),
                ("batched", C.c_int32), ("timing", C.c_int32),
                ("mv_split_nodes", C.c_int32), ("graphs", C.c_int32),
                ("mv_xcd_run", C.c_int32), ("coupling_mode", C.c_int32),
                ("coupling_chunk", C.c_int64), ("alloc", C.c_void_p), ("free", C.c_void_p),
                ("alloc_ctx", C.c_void_p), ("point_data", C.c_void_p), ("basis", C.c_int32)]

# smash_alloc_fn / smash_free_fn
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)


def torch_allocator_hooks(device=None):
    """(alloc, free) hooks that take a handle's device memory from torch's
    caching allocator on the stream the library names, so torch accounts for
    it (torch.cuda.memory_allocated) and one memory budget covers both."""
    import torch
    dev = torch.cuda.current_device() if device is None else device

    def _alloc(ctx, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
        except Exception:
            return None

    def _free(ctx, ptr, nbytes, stream):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    return ALLOC_FN(_alloc), FREE_FN(_free)


class Info(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("dim", C.c_int32), ("nlevels", C.c_int32),
                ("nnodes", C.c_int64), ("nleaves", C.c_int64), ("n_admissible", C.c_int64),
                ("n_inadmissible", C.c_int64), ("sum_rank_row", C.c_int64),
                ("sum_rank_col", C.c_int64), ("max_rank_row", C.c_int32),
                ("max_rank_col", C.c_int32), ("coupling_entries", C.c_int64),
                ("near_entries", C.c_int64), ("g_entries_row", C.c_int64),
                ("g_entries_col", C.c_int64), ("index_entries", C.c_int64),
                ("device_bytes", C.c_int64), ("total_swaps", C.c_int64),
                ("apply_prec", C.c_int32), ("eval_prec", C.c_int32),
                ("symmetric_reuse", C.c_int32), ("build_ms", C.c_double),
                ("phase_ms", C.c_double * 16), ("phase_calls", C.c_int64 * 16),
                ("graph_captures", C.c_int64), ("graph_replays", C.c_int64),
                ("coupling_evaluated", C.c_int32), ("coupling_chunks", C.c_int32),
                ("coupling_ws_entries", C.c_int64), ("bytes_dense", C.c_int64),
                ("bytes_hss0", C.c_int64), ("bytes_smash", C.c_int64),
                ("build_peak_bytes", C.c_int64)]

BASES = {"chebyshev": 0, "taylor": 1}  # SMASH_BASIS_*

PHASES = ["tree", "pairs", "near_svd", "compr", "slots", "blocks", "mv_gather", "mv_up",
          "mv_coupling", "mv_down", "mv_near_out"]


_lib = None
EXPORTED = ["smash_default_options", "smash_build", "smash_build_xy", "smash_matvec",
            "smash_matvec_noalloc", "smash_matvec_cauchy_like", "smash_matvec_batched", "smash_set_product_shape", "smash_info", "smash_export", "smash_destroy",
            "smash_estimate_footprint", "smash_estimate_footprint_mode", "smash_trim",
            "smash_last_error"]


def lib():
    """Load libsmash.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsmash.so is not built (run python -m "
                               "paper_1705_05443_amd.build_lib); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.smash_default_options.argtypes = [C.POINTER(Options)]
        L.smash_build.argtypes = [vp, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_int32, C.c_double, C.POINTER(Options), vp, C.POINTER(vp)]
        L.smash_build_xy.argtypes = [vp, C.c_int64, vp, C.c_int64, C.c_int32, C.c_int32,
                                     C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                     C.POINTER(Options), vp, C.POINTER(vp)]
        L.smash_matvec.argtypes = [vp, vp, C.c_int64, C.c_int32, C.c_int32, vp, C.c_int64, vp]
        L.smash_matvec_noalloc.argtypes = L.smash_matvec.argtypes
        L.smash_matvec_cauchy_like.argtypes = [vp, vp, C.c_int64, C.c_int32, C.c_int32, vp, vp,
                                               C.c_int32, vp, C.c_int64, vp]
        L.smash_matvec_batched.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(vp),
                                           C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                           C.POINTER(vp), C.POINTER(C.c_int64), C.c_int32, vp]
        L.smash_set_product_shape.argtypes = [vp, C.c_int32, C.c_int32]
        L.smash_estimate_footprint.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                               C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                               C.POINTER(C.c_int64)]
        L.smash_estimate_footprint_mode.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                                    C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                                    C.c_int32, C.POINTER(C.c_int64)]
        L.smash_info.argtypes = [vp, C.POINTER(Info)]
        L.smash_export.argtypes = [vp, C.c_int32, vp, C.POINTER(C.c_int64)]
        L.smash_destroy.argtypes = [vp]
        L.smash_trim.argtypes = [C.c_int32]
        L.smash_last_error.restype = C.c_char_p
        for f in ("smash_default_options", "smash_build", "smash_build_xy", "smash_matvec",
                  "smash_matvec_noalloc", "smash_matvec_batched",
                  "smash_set_product_shape", "smash_info", "smash_export", "smash_destroy",
                  "smash_estimate_footprint", "smash_estimate_footprint_mode", "smash_trim"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise SmashError(rc, lib().smash_last_error().decode())


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def trim(device=-1):
    """Return the library's cached device memory (idle build chunks and the
    free part of the default memory pool) to the device (smash_trim)."""
    _check(lib().smash_trim(int(device)))


def estimate_footprint(n, dim, kernel="inv_r", leaf=64, order=8, adm="strong", tol=1e-8,
                       apply_prec="f64", coupling="stored"):
    """Upper estimate of a handle's device bytes (smash_estimate_footprint_mode)
    for the stored or the evaluated coupling form."""
    b = C.c_int64(0)
    _check(lib().smash_estimate_footprint_mode(int(n), int(dim), KERNELS[kernel], int(leaf),
                                               int(order), ADM[adm], float(tol),
                                               PREC[apply_prec], COUPLING[coupling],
                                               C.byref(b)))
    return b.value


def matvec_batched(handles, Xs, outs=None, stream=None):
    """Products of several handles in one library call (smash_matvec_batched):
    returns [h.matvec(X) for h, X in zip(handles, Xs)], 2-D (n, nrhs) tensors
    of one vector precision; `outs` may give the result tensors."""
    import torch
    if len(handles) != len(Xs) or (outs is not None and len(outs) != len(Xs)):
        raise ValueError("handles, Xs (and outs) must have the same length")
    if not handles:
        return []
    precs = {h.apply_prec == "f64" for h in handles}
    if len(precs) != 1:
        raise TypeError("all handles must share the vector precision")
    dt = torch.float64 if precs.pop() else torch.float32
    Xc, Yc = [], []
    for c, (h, X) in enumerate(zip(handles, Xs)):
        if X.dim() != 2 or X.dtype != dt or not X.is_cuda:
            raise TypeError("X must be a 2-D CUDA tensor of the vector precision")
        X = X if X.stride(1) == 1 else X.contiguous()
        Y = (torch.empty((h.nx, X.shape[1]), dtype=dt, device=X.device) if outs is None
             else outs[c])
        if (not Y.is_cuda or Y.dtype != dt or tuple(Y.shape) != (h.nx, X.shape[1])
                or Y.stride(1) != 1):
            raise TypeError("out must be a CUDA (nx, nrhs) tensor with unit column stride")
        Xc.append(X)
        Yc.append(Y)
    n = len(handles)
    vp = C.c_void_p
    hs = (vp * n)(*[h._h.value for h in handles])
    xs = (vp * n)(*[X.data_ptr() for X in Xc])
    ys = (vp * n)(*[Y.data_ptr() for Y in Yc])
    ldx = (C.c_int64 * n)(*[X.stride(0) for X in Xc])
    ldy = (C.c_int64 * n)(*[Y.stride(0) for Y in Yc])
    nr = (C.c_int32 * n)(*[X.shape[1] for X in Xc])
    _check(lib().smash_matvec_batched(n, hs, xs, ldx, nr, ys, ldy,
                                      PREC["f64" if dt == torch.float64 else "f32"],
                                      _stream_ptr(stream)))
    return Yc


class Smash:
    """A device-resident SMASH construction (the C handle).

    x, y: CUDA float64 point arrays (n x dim); y None means Y = X.  The
    remaining keywords map onto smash_build's arguments and smash_options
    (include/smash.h).  tuned: take the product's launch shape from the
    autotuner table (autotune.lookup) for this size bin, with nrhs_hint as
    the expected right-hand-side count; explicit mv_split_nodes / mv_xcd_run
    win.  graphs: replay repeated products from captured HIP graphs.
    coupling: "auto", "stored" or "evaluated" (SMASH_COUPLING_*): keep the
    coupling blocks, or evaluate them inside every product in chunks of
    coupling_chunk entries (0: 256 MiB worth).  allocator: None (the
    library's own pool), "torch" (torch's caching allocator, see
    torch_allocator_hooks) or an (alloc, free) pair of ALLOC_FN / FREE_FN.
    basis: "chebyshev" (interpolation, eq. (2.2)) or "taylor" (eqs. (2.4)-(2.5),
    order = the number of terms r; points on the line only).
    """

    def __init__(self, x, y=None, *, kernel="inv_r", leaf=64, order=8, adm="strong", tol=1e-8,
                 tau=None, eps_svd=None, f=2.0, diag=0.0, eval_prec="f64", apply_prec="f64",
                 root=None, max_depth=0, batched=True, timing=False, mv_split_nodes=None,
                 mv_xcd_run=None, graphs=True, tuned=True, nrhs_hint=16, coupling="auto",
                 coupling_chunk=0, allocator=None, stream=None, point_data=None,
                 basis="chebyshev"):
        import torch
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64):
            raise TypeError("x must be a CUDA float64 tensor")
        x = x.contiguous()
        if x.dim() == 1:
            x = x[:, None]
        if y is not None:
            y = y.contiguous()
            if y.dim() == 1:
                y = y[:, None]
        opt = Options()
        lib().smash_default_options(C.byref(opt))
        if tau is not None:
            opt.tau = tau
        if eps_svd is not None:
            opt.eps_svd = eps_svd
        opt.srrqr_f = f
        opt.diag_value = diag
        if eval_prec not in ("f64", "f32"):
            raise ValueError("eval_prec must be 'f64' or 'f32'")
        opt.eval_prec = PREC[eval_prec]
        opt.apply_prec = PREC[apply_prec]
        if root is not None:
            opt.has_root_box = 1
            lo = list(np.atleast_1d(np.asarray(root[0], dtype=np.float64)))
            for t, v in enumerate(lo[:3]):
                opt.root_lo[t] = v
            opt.root_side = float(root[1])
        opt.max_depth = max_depth
        opt.batched = 1 if batched else 0
        opt.timing = 1 if timing else 0
        if tuned and (mv_split_nodes is None or mv_xcd_run is None):
            from . import autotune
            ny_ = x.shape[0] if y is None else y.shape[0]
            shp = autotune.lookup(max(x.shape[0], ny_), x.shape[1], adm, apply_prec, nrhs_hint)
            if shp:
                if mv_split_nodes is None:
                    mv_split_nodes = shp["mv_split_nodes"]
                if mv_xcd_run is None:
                    mv_xcd_run = shp["mv_xcd_run"]
        if mv_split_nodes is not None:
            opt.mv_split_nodes = int(mv_split_nodes)
        if mv_xcd_run is not None:
            opt.mv_xcd_run = int(mv_xcd_run)
        opt.graphs = 1 if graphs else 0
        if coupling not in COUPLING:
            raise ValueError("coupling must be 'auto', 'stored' or 'evaluated'")
        opt.coupling_mode = COUPLING[coupling]
        opt.coupling_chunk = int(coupling_chunk)
        if basis not in BASES:
            raise ValueError("basis must be 'chebyshev' or 'taylor'")
        opt.basis = BASES[basis]
        self._hooks = None
        if allocator is not None:
            self._hooks = torch_allocator_hooks() if allocator == "torch" else tuple(allocator)
            opt.alloc = C.cast(self._hooks[0], C.c_void_p)
            opt.free = C.cast(self._hooks[1], C.c_void_p)
        if point_data is not None:  # the double-layer kernel's per-point data, n x 3
            if not (isinstance(point_data, torch.Tensor) and point_data.is_cuda
                    and point_data.dtype == torch.float64):
                raise TypeError("point_data must be a CUDA float64 tensor")
            point_data = point_data.contiguous()
            opt.point_data = point_data.data_ptr()
        self.apply_prec = apply_prec
        self.nx = x.shape[0]
        self.ny = x.shape[0] if y is None else y.shape[0]
        self._keep = (x, y, point_data)
        h = C.c_void_p()
        kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        a = ADM[adm] if isinstance(adm, str) else int(adm)
        sp = _stream_ptr(stream)
        if y is None:
            rc = lib().smash_build(C.c_void_p(x.data_ptr()), x.shape[0], x.shape[1], kid,
                                   leaf, order, a, tol, C.byref(opt), sp, C.byref(h))
        else:
            rc = lib().smash_build_xy(C.c_void_p(x.data_ptr()), x.shape[0],
                                      C.c_void_p(y.data_ptr()), y.shape[0], x.shape[1], kid,
                                      leaf, order, a, tol, C.byref(opt), sp, C.byref(h))
        _check(rc)
        self._h = h

    def matvec(self, X, out=None, stream=None):
        """Y = A-hat X, original point order; X: (ny, nrhs) or (ny,), float64 for an
        FP64-apply handle, float32 for FP32 and BF16 apply."""
        return self._product(lib().smash_matvec, X, out, stream)

    def matvec_noalloc(self, X, out=None, stream=None):
        """The same product through smash_matvec_noalloc: no device allocation by
        the library (its vectors live in the library's per-device array of
        NOALLOC_SCRATCH_BYTES); `out` must be given by callers that cannot
        allocate."""
        return self._product(lib().smash_matvec_noalloc, X, out, stream)

    def _product(self, fn, X, out, stream):
        import torch
        dt = torch.float64 if self.apply_prec == "f64" else torch.float32
        vec = X.dim() == 1
        if vec:
            X = X[:, None]
        if X.dtype != dt or not X.is_cuda:
            raise TypeError("X must be a CUDA tensor of the apply precision")
        if X.stride(1) != 1:
            X = X.contiguous()
        R = X.shape[1]
        if out is None:
            out = torch.empty((self.nx, R), dtype=dt, device=X.device)
        elif (not out.is_cuda or out.dtype != dt or out.dim() != 2
              or tuple(out.shape) != (self.nx, R) or out.stride(1) != 1):
            raise TypeError("out must be a CUDA (nx, nrhs) tensor of the vector precision "
                            "with unit column stride")
        _check(fn(self._h, C.c_void_p(X.data_ptr()), X.stride(0), R,
                  PREC["f64" if self.apply_prec == "f64" else "f32"], C.c_void_p(out.data_ptr()),
                  out.stride(0), _stream_ptr(stream)))
        return out[:, 0] if vec else out

    def matvec_cauchy_like(self, X, w, v, out=None, stream=None):
        """Y = sum_l w_l o (A-hat (v_l o X)) through smash_matvec_cauchy_like: the
        Cauchy-like matrix with generators w (nx, p) and v (ny, p), CUDA float64
        tensors (eqs. (6.1)-(6.2)); X and out as for matvec."""
        import torch
        for g, n in ((w, self.nx), (v, self.ny)):
            if not (isinstance(g, torch.Tensor) and g.is_cuda and g.dtype == torch.float64
                    and g.dim() == 2 and g.shape[0] == n):
                raise TypeError("w and v must be CUDA float64 tensors of shape (nx, p), (ny, p)")
        if w.shape[1] != v.shape[1]:
            raise ValueError("w and v must have the same number of columns")
        w, v = w.contiguous(), v.contiguous()
        p = w.shape[1]

        def fn(h, X, ldx, R, dt, Y, ldy, s):
            return lib().smash_matvec_cauchy_like(h, X, ldx, R, dt, C.c_void_p(w.data_ptr()),
                                                  C.c_void_p(v.data_ptr()), p, Y, ldy, s)
        return self._product(fn, X, out, stream)

    def set_product_shape(self, mv_split_nodes, mv_xcd_run):
        """Launch shape of the products (see smash_set_product_shape)."""
        _check(lib().smash_set_product_shape(self._h, int(mv_split_nodes), int(mv_xcd_run)))

    def info(self):
        inf = Info()
        _check(lib().smash_info(self._h, C.byref(inf)))
        out = {k: getattr(inf, k) for k, _ in Info._fields_ if k not in ("phase_ms", "phase_calls")}
        out["phase_ms"] = {n: inf.phase_ms[i] for i, n in enumerate(PHASES)}
        out["phase_calls"] = {n: inf.phase_calls[i] for i, n in enumerate(PHASES)}
        return out

    def export(self, what):
        n = C.c_int64(0)
        code = EX[what]
        _check(lib().smash_export(self._h, code, None, C.byref(n)))
        if what in ("coupling", "near"):
            dt = np.float64 if self.apply_prec == "f64" else np.float32
        else:
            dt = np.float64 if what in _F64_EXPORTS else np.int32
        out = np.zeros(max(n.value, 1), dtype=dt)
        _check(lib().smash_export(self._h, code, out.ctypes.data_as(C.c_void_p), C.byref(n)))
        return out[: n.value]

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().smash_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
