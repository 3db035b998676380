"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad arguments before touching any device."""
import ctypes as C
import os
import re

import pytest

from paper_1705_05443_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "smash.h")).read()
    return sorted(set(re.findall(r"\b(smash_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(api.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = api.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_invalid_arguments_are_rejected_without_a_device():
    L = api.lib()
    opt = api.Options()
    assert L.smash_default_options(C.byref(opt)) == 0
    assert opt.struct_size == C.sizeof(api.Options)
    assert opt.coupling_mode == 0 and opt.coupling_chunk == 0  # auto, default chunk
    h = C.c_void_p()
    dummy = C.c_void_p(16)  # never dereferenced: validation fails first
    # dim out of range
    assert L.smash_build(dummy, 10, 4, 0, 8, 4, 1, 1e-6, C.byref(opt), None, C.byref(h)) == -1
    # 1/(x-y) needs dim 1
    assert L.smash_build(dummy, 10, 2, 3, 8, 4, 1, 1e-6, C.byref(opt), None, C.byref(h)) == -2
    # order out of range, leaf < 1, bad admissibility, bad tol
    assert L.smash_build(dummy, 10, 2, 0, 8, 0, 1, 1e-6, C.byref(opt), None, C.byref(h)) == -1
    assert L.smash_build(dummy, 10, 2, 0, 0, 4, 1, 1e-6, C.byref(opt), None, C.byref(h)) == -1
    assert L.smash_build(dummy, 10, 2, 0, 8, 4, 7, 1e-6, C.byref(opt), None, C.byref(h)) == -1
    assert L.smash_build(dummy, 10, 2, 0, 8, 4, 1, -1.0, C.byref(opt), None, C.byref(h)) == -1
    # NULL points, n < 1
    assert L.smash_build(None, 10, 2, 0, 8, 4, 1, 1e-6, C.byref(opt), None, C.byref(h)) == -1
    assert L.smash_build(dummy, 0, 2, 0, 8, 4, 1, 1e-6, C.byref(opt), None, C.byref(h)) == -1
    # options: wrong struct size, tau outside (0,1), f <= 1, unknown precision
    bad = api.Options()
    L.smash_default_options(C.byref(bad))
    bad.struct_size = 3
    assert L.smash_build(dummy, 10, 2, 0, 8, 4, 1, 1e-6, C.byref(bad), None, C.byref(h)) == -1
    for field, val in (("tau", 1.5), ("srrqr_f", 1.0), ("apply_prec", 9), ("eval_prec", 9),
                       ("eval_prec", 2), ("mv_split_nodes", -1), ("mv_xcd_run", 0),
                       ("mv_xcd_run", 5000), ("coupling_mode", 3), ("coupling_mode", -1),
                       ("coupling_chunk", -5)):
        L.smash_default_options(C.byref(bad))
        setattr(bad, field, val)
        assert L.smash_build(dummy, 10, 2, 0, 8, 4, 1, 1e-6, C.byref(bad), None, C.byref(h)) == -1
    assert h.value is None
    assert b"tau" in L.smash_last_error() or len(L.smash_last_error()) > 0
    # NULL handle everywhere
    assert L.smash_matvec(None, dummy, 1, 1, 0, dummy, 1, None) == -1
    assert L.smash_matvec_noalloc(None, dummy, 1, 1, 0, dummy, 1, None) == -1
    info = api.Info()
    assert L.smash_info(None, C.byref(info)) == -1
    n = C.c_int64(0)
    assert L.smash_export(None, 1, None, C.byref(n)) == -1
    assert L.smash_set_product_shape(None, 16, 16) == -1
    assert L.smash_destroy(None) == 0


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        api.Smash(torch.zeros(4, 2, dtype=torch.float64))


def test_footprint_estimate_by_coupling_form():
    """The evaluated form never estimates above the stored one, the AUTO form
    estimates as the stored one, and an unknown form is rejected."""
    L = api.lib()
    b = C.c_int64(0)
    for n, d, k in ((1000, 1, 0), (65536, 2, 1), (30000, 3, 0), (200000, 3, 2)):
        s = api.estimate_footprint(n, d, list(api.KERNELS)[k], coupling="stored")
        e = api.estimate_footprint(n, d, list(api.KERNELS)[k], coupling="evaluated")
        a = api.estimate_footprint(n, d, list(api.KERNELS)[k], coupling="auto")
        assert 0 < e <= s and a == s
        assert L.smash_estimate_footprint(n, d, k, 64, 8, 1, 1e-6, 0, C.byref(b)) == 0
        assert b.value == s
    assert L.smash_estimate_footprint_mode(1000, 2, 0, 64, 8, 1, 1e-6, 0, 7, C.byref(b)) == -1
    assert L.smash_estimate_footprint_mode(1000, 2, 0, 64, 8, 1, 1e-6, 0, 2, None) == -1


def test_batched_products_reject_bad_arguments_before_running():
    L = api.lib()
    vp = C.c_void_p
    one = lambda t, v: (t * 1)(v)  # noqa: E731
    args = dict(hs=one(vp, None), xs=one(vp, 16), ldx=one(C.c_int64, 4), nr=one(C.c_int32, 4),
                ys=one(vp, 16), ldy=one(C.c_int64, 4))
    call = lambda n, a: L.smash_matvec_batched(n, a["hs"], a["xs"], a["ldx"], a["nr"], a["ys"],  # noqa: E731
                                               a["ldy"], 0, None)
    assert call(-1, args) == -1
    assert call(0, args) == 0  # nothing to do
    assert call(1, args) == -1  # NULL handle
    assert b"entry 0" in L.smash_last_error()
    assert L.smash_matvec_batched(1, None, args["xs"], args["ldx"], args["nr"], args["ys"],
                                  args["ldy"], 0, None) == -1


def test_allocator_hooks_must_come_in_pairs():
    L = api.lib()
    opt = api.Options()
    L.smash_default_options(C.byref(opt))
    assert opt.alloc is None and opt.free is None and opt.alloc_ctx is None
    hook = api.ALLOC_FN(lambda ctx, n, s: None)
    opt.alloc = C.cast(hook, C.c_void_p)
    h = C.c_void_p()
    dummy = C.c_void_p(16)
    assert L.smash_build(dummy, 10, 2, 0, 8, 4, 1, 1e-6, C.byref(opt), None, C.byref(h)) == -1
    assert b"allocator hooks" in L.smash_last_error()
    assert not h.value
