"""Host-only checks of the C ABI library: it loads without a GPU, exports every
function include/gs2.h declares, and rejects bad arguments before touching
the device."""
import ctypes as C

import pytest

from paper_2104_01196_amd import native


def test_library_exports_every_declared_symbol():
    L = native.lib()
    names = native.declared_functions()
    assert {"gs2_setup", "gs2_apply", "jr_apply", "gs_trisolve_apply", "gmres_solve", "gs2_destroy",
            "gs2_status_string", "gs2_setup_batched", "gmres_solve_batched"} <= set(names)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_defaults():
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, 1, 2, 3):
        assert native.status_string(code) not in ("", "unknown status")
    assert native.status_string(12345) == "unknown status"
    o = native.Options()
    native.lib().gs2_default_options(C.byref(o))
    assert (o.precision, o.inner_damping, o.compact, o.build_levels, o.autotune, o.lanes_per_row,
            o.rhs_per_item, o.spmv_format, o.basis_loads) == (0, 1.0, 0, 0, 1, 0, 0, 0, 0)


def test_argument_errors_without_device():
    L = native.lib()
    out = C.c_void_p()
    assert L.gs2_setup(None, 1, 1, 1.0, 0, None, None, C.byref(out)) == native.ERR_ARG
    d = native.CsrDesc(4, 4, 8, 8, 8)  # bogus but non-null pointers: rejected on the arguments alone
    for args in [(0, 1, 1.0, 0), (1, -1, 1.0, 0), (1, 1, 0.0, 0), (1, 1, 2.0, 0), (1, 1, 1.0, 3)]:
        assert L.gs2_setup(C.byref(d), *args, None, None, C.byref(out)) == native.ERR_ARG
    bad = native.Options(7, 1.0, 0, 0, 1, 0)
    assert L.gs2_setup(C.byref(d), 1, 1, 1.0, 0, C.byref(bad), None, C.byref(out)) == native.ERR_ARG
    for field, val in (("basis_loads", 3), ("spmv_format", 4), ("format", 4)):
        o = native.Options()
        L.gs2_default_options(C.byref(o))
        setattr(o, field, val)
        assert L.gs2_setup(C.byref(d), 1, 1, 1.0, 0, C.byref(o), None, C.byref(out)) == native.ERR_ARG, field
    info = native.SolveInfo()
    assert L.gmres_solve(C.byref(d), 8, 8, 0, 1e-8, 10, 0, None, C.byref(info), None) == native.ERR_ARG
    assert info.status == native.ERR_ARG
    assert L.gmres_solve(C.byref(d), 8, 8, 10, 1e-8, 10, native.PREC_GS2, None, C.byref(info), None) == native.ERR_ARG
    assert L.gs2_apply(None, 8, 16, None) == native.ERR_ARG
