"""ctypes binding of libgs2.so (include/gs2.h), same names as the C ABI.

Argument marshalling only: tensors must already live on the GPU; their data
pointers and torch's current HIP stream are handed to the library, which does
all of the work.  There is no fallback path: if the library is missing or a
call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs2.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gs2.h")

OK, ERR_ARG, ERR_BAD_CSR, ERR_ZERO_DIAG, ERR_NONFINITE, ERR_NOMEM, ERR_HIP, ERR_FP16_RANGE, ERR_NO_LEVELS = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
ERR_SCRATCH = -9
NOALLOC_SCRATCH_DOUBLES = 524288  # fixed scratch of the allocation-free entry point (doubles per device)
NOT_CONVERGED, BREAKDOWN_EXACT, STAGNATED = 1, 2, 3
BREAKDOWN = BREAKDOWN_EXACT  # earlier name of the same code
FORWARD, BACKWARD, SYMMETRIC = 0, 1, 2
FP64, FP32, FP16_SCALED = 0, 1, 2
FORMAT_AUTO, FORMAT_SELL, FORMAT_DIA, FORMAT_BLOCK3 = 0, 1, 2, 3
LDS_AUTO, LDS_OFF, LDS_ON = 0, 1, 2
XCD_AUTO, XCD_DISPATCH_ORDER, XCD_RANGES = 0, 1, 2
PREC_NONE, PREC_GS2, PREC_JR, PREC_GS_TRISOLVE, PREC_MTGS = 0, 1, 2, 3, 4


class Gs2Error(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


class CsrDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("colind", C.c_void_p),
                ("val", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("inner_damping", C.c_double), ("compact", C.c_int),
                ("build_levels", C.c_int), ("autotune", C.c_int), ("lanes_per_row", C.c_int),
                ("rhs_per_item", C.c_int), ("orthogonalization", C.c_int), ("blocks", C.c_int),
                ("local_sweeps", C.c_int), ("team_rows", C.c_int), ("team_wait_ms", C.c_int),
                ("format", C.c_int), ("rows_per_lane", C.c_int), ("lds_staging", C.c_int),
                ("xcd_ranges", C.c_int), ("stagnation_cycles", C.c_int), ("spmv_format", C.c_int),
                ("basis_loads", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("relres", C.c_double), ("converged", C.c_int),
                ("status", C.c_int), ("seconds", C.c_double)]


_lib = None


def lib():
    """Load libgs2.so (built by paper_2104_01196_amd.build)."""
    global _lib
    if _lib is None:
        # torch bundles its own HIP runtime; load it first so that libgs2
        # binds to that same runtime instead of bringing a second one.
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2104_01196_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        L.gs2_default_options.argtypes = [C.POINTER(Options)]
        L.gs2_setup.argtypes = [C.POINTER(CsrDesc), i, i, d, i, C.POINTER(Options), vp, C.POINTER(vp)]
        L.gs2_apply.argtypes = [vp, vp, vp, vp]
        L.jr_apply.argtypes = [vp, i, d, vp, vp, vp]
        L.gs_trisolve_apply.argtypes = [vp, i, d, vp, vp, vp]
        L.mtgs_apply.argtypes = [vp, i, d, vp, vp, vp]
        L.gmres_solve.argtypes = [C.POINTER(CsrDesc), vp, vp, i, d, i, i, vp, C.POINTER(SolveInfo), vp]
        L.cg_solve.argtypes = [C.POINTER(CsrDesc), vp, vp, d, i, i, vp, C.POINTER(SolveInfo), vp]
        L.gs2_destroy.argtypes = [vp]
        L.gs2_destroy.restype = None
        L.gs2_status_string.argtypes = [i]
        L.gs2_status_string.restype = C.c_char_p
        i64p = C.POINTER(C.c_int64)
        ip = C.POINTER(C.c_int)
        L.gs2_handle_query.argtypes = [vp, i64p, i64p, i64p, i64p, ip, ip, ip]
        L.gs2_handle_schedule.argtypes = [vp, ip, ip, ip, ip, ip, ip, ip, ip, ip]
        L.gs2_gmres_schedule.argtypes = [vp, ip, ip, ip, ip, ip]
        L.gs2_gmres_basis_schedule.argtypes = [vp, ip, ip, ip]
        L.gs2_inner_residuals.argtypes = [vp, vp, i, C.POINTER(C.c_double), vp]
        L.gs2_inner_residuals_noalloc.argtypes = [vp, vp, i, vp, vp]
        L.gs2_profile.argtypes = [i]
        L.gs2_graphs.argtypes = [i]
        L.gs2_profile_kernel_count.argtypes = []
        L.gs2_profile_read.argtypes = [i, C.POINTER(C.c_char_p), i64p, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        if hasattr(L, "gs2_setup_batched"):
            L.gs2_setup_batched.argtypes = [C.POINTER(CsrDesc), i, i, i, d, i, C.POINTER(Options), i, i, vp,
                                            C.POINTER(vp)]
            L.gmres_solve_batched.argtypes = [vp, i, vp, vp, d, i, C.POINTER(SolveInfo), vp]
            L.gs2_destroy_batched.argtypes = [vp]
            L.gs2_batched_schedule.argtypes = [vp, ip, ip, ip]
            L.gs2_destroy_batched.restype = None
        _lib = L
    return _lib


def declared_functions() -> list[str]:
    """Function names declared in include/gs2.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*([a-z_0-9]+)\s*\(", txt, flags=re.M)))


def status_string(code: int) -> str:
    try:
        return lib().gs2_status_string(int(code)).decode()
    except RuntimeError:
        return "library not loaded"


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t, dtype, n=None, what="tensor"):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{what} must have {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class DeviceCSR:
    """CSR matrix resident on the GPU: int32 rowptr/colind, float64 val."""

    def __init__(self, n, rowptr, colind, val):
        import torch

        self.n = int(n)
        self.rowptr, self.colind, self.val = rowptr, colind, val
        self.nnz = int(colind.numel())
        _ptr(rowptr, torch.int32, self.n + 1, "rowptr")
        _ptr(colind, torch.int32, None, "colind")
        _ptr(val, torch.float64, self.nnz, "val")

    @classmethod
    def from_host(cls, A, device="cuda"):
        """From any object with n, rowptr, colind, val (numpy arrays)."""
        import torch

        return cls(A.n, torch.as_tensor(A.rowptr, dtype=torch.int32, device=device),
                   torch.as_tensor(A.colind, dtype=torch.int32, device=device),
                   torch.as_tensor(A.val, dtype=torch.float64, device=device))

    def desc(self) -> CsrDesc:
        return CsrDesc(self.n, self.nnz, self.rowptr.data_ptr(), self.colind.data_ptr(), self.val.data_ptr())


class Handle:
    """Owns a gs2_handle*; freed by gs2_destroy (or on garbage collection)."""

    def __init__(self, ptr, n, keep=None):
        self.ptr = ptr
        self.n = n
        self._keep = keep

    def __del__(self):
        try:
            gs2_destroy(self)
        except Exception:
            pass


def gs2_setup(A: DeviceCSR, sweeps=1, inner=1, damping=1.0, variant=FORWARD, precision=FP64, inner_damping=1.0,
              compact=False, build_levels=False, autotune=True, lanes_per_row=0, orthogonalization=0, blocks=1,
              local_sweeps=1, format=FORMAT_AUTO, rows_per_lane=0, lds_staging=0, stagnation_cycles=0,
              spmv_format=FORMAT_AUTO, xcd_ranges=0, basis_loads=0, stream=None) -> Handle:
    opt = Options(precision=precision, inner_damping=inner_damping, compact=int(compact),
                  build_levels=int(build_levels), autotune=int(autotune), lanes_per_row=lanes_per_row,
                  orthogonalization=orthogonalization, blocks=blocks, local_sweeps=local_sweeps, format=format,
                  rows_per_lane=rows_per_lane, lds_staging=lds_staging, xcd_ranges=xcd_ranges,
                  stagnation_cycles=stagnation_cycles, spmv_format=spmv_format, basis_loads=basis_loads)
    out = C.c_void_p()
    d = A.desc()
    st = lib().gs2_setup(C.byref(d), sweeps, inner, damping, variant, C.byref(opt), _stream(stream), C.byref(out))
    if st != OK:
        raise Gs2Error(st, "gs2_setup")
    return Handle(out, A.n)


def gs2_apply(h: Handle, v, z, stream=None):
    import torch

    st = lib().gs2_apply(h.ptr, _ptr(v, torch.float64, h.n, "v"), _ptr(z, torch.float64, h.n, "z"), _stream(stream))
    if st != OK:
        raise Gs2Error(st, "gs2_apply")


def jr_apply(h: Handle, sweeps, damping, v, z, stream=None):
    import torch

    st = lib().jr_apply(h.ptr, sweeps, damping, _ptr(v, torch.float64, h.n, "v"), _ptr(z, torch.float64, h.n, "z"),
                        _stream(stream))
    if st != OK:
        raise Gs2Error(st, "jr_apply")


def gs_trisolve_apply(h: Handle, variant, damping, v, z, stream=None):
    import torch

    st = lib().gs_trisolve_apply(h.ptr, variant, damping, _ptr(v, torch.float64, h.n, "v"),
                                 _ptr(z, torch.float64, h.n, "z"), _stream(stream))
    if st != OK:
        raise Gs2Error(st, "gs_trisolve_apply")


def mtgs_apply(h: Handle, variant, damping, v, z, stream=None):
    import torch

    st = lib().mtgs_apply(h.ptr, variant, damping, _ptr(v, torch.float64, h.n, "v"),
                          _ptr(z, torch.float64, h.n, "z"), _stream(stream))
    if st != OK:
        raise Gs2Error(st, "mtgs_apply")


def gmres_solve(A: DeviceCSR, b, x, restart=30, rtol=1e-8, maxit=10000, prec_kind=PREC_GS2, prec: Handle = None,
                stream=None, raise_on_error=True) -> dict:
    """Returns the gs2_solve_info fields as a dict.  Hard errors raise;
    GS2_NOT_CONVERGED / GS2_BREAKDOWN_EXACT / GS2_STAGNATED are reported in the dict."""
    import torch

    info = SolveInfo()
    d = A.desc()
    st = lib().gmres_solve(C.byref(d), _ptr(b, torch.float64, A.n, "b"), _ptr(x, torch.float64, A.n, "x"), restart,
                           rtol, maxit, prec_kind, prec.ptr if prec is not None else None, C.byref(info),
                           _stream(stream))
    if st < 0 and raise_on_error:
        raise Gs2Error(st, "gmres_solve")
    return {"iterations": info.iterations, "restarts": info.restarts, "relres": info.relres,
            "converged": bool(info.converged), "status": info.status, "seconds": info.seconds}


def cg_solve(A: DeviceCSR, b, x, rtol=1e-8, maxit=10000, prec_kind=PREC_GS2, prec: Handle = None, stream=None,
             raise_on_error=True) -> dict:
    """Preconditioned CG; returns the gs2_solve_info fields as a dict."""
    import torch

    info = SolveInfo()
    d = A.desc()
    st = lib().cg_solve(C.byref(d), _ptr(b, torch.float64, A.n, "b"), _ptr(x, torch.float64, A.n, "x"), rtol, maxit,
                        prec_kind, prec.ptr if prec is not None else None, C.byref(info), _stream(stream))
    if st < 0 and raise_on_error:
        raise Gs2Error(st, "cg_solve")
    return {"iterations": info.iterations, "restarts": info.restarts, "relres": info.relres,
            "converged": bool(info.converged), "status": info.status, "seconds": info.seconds}


def gs2_destroy(h: Handle):
    if h is not None and h.ptr:
        lib().gs2_destroy(h.ptr)
        h.ptr = None


def gs2_handle_query(h: Handle) -> dict:
    v = [C.c_int64() for _ in range(4)] + [C.c_int() for _ in range(3)]
    st = lib().gs2_handle_query(h.ptr, *[C.byref(x) for x in v])
    if st != OK:
        raise Gs2Error(st, "gs2_handle_query")
    keys = ["n", "nnz_l", "nnz_u", "bytes_stored", "lanes_per_row", "levels_l", "levels_u"]
    return {k: x.value for k, x in zip(keys, v)}


def gs2_handle_schedule(h: Handle) -> dict:
    v = [C.c_int() for _ in range(9)]
    st = lib().gs2_handle_schedule(h.ptr, *[C.byref(x) for x in v])
    if st != OK:
        raise Gs2Error(st, "gs2_handle_schedule")
    keys = ["format", "lanes_per_row", "rows_per_lane", "vector_bytes", "lds_staging", "xcd_ranges", "ndiag_l",
            "ndiag_u", "tuned"]
    return {k: x.value for k, x in zip(keys, v)}


def gs2_gmres_schedule(h: Handle) -> dict:
    """The layout of gmres_solve's copy of A with this handle (zeros before its first solve)."""
    v = [C.c_int() for _ in range(5)]
    st = lib().gs2_gmres_schedule(h.ptr, *[C.byref(x) for x in v])
    if st != OK:
        raise Gs2Error(st, "gs2_gmres_schedule")
    return {k: x.value for k, x in zip(["format", "lanes_per_row", "rows_per_lane", "ndiag", "tuned"], v)}


def gs2_gmres_basis_schedule(h: Handle) -> dict:
    """Arnoldi steps from which the basis passes keep fewer loads in flight (-1 never; zeros before the first solve)."""
    v = [C.c_int() for _ in range(3)]
    st = lib().gs2_gmres_basis_schedule(h.ptr, *[C.byref(x) for x in v])
    if st != OK:
        raise Gs2Error(st, "gs2_gmres_basis_schedule")
    return {k: x.value for k, x in zip(["dot_narrow_from", "update_narrow_from", "tuned"], v)}


def gs2_inner_residuals(h: Handle, r, inner: int, stream=None):
    """||r - (wL + D) g_j|| / ||r|| for j = 0..inner (numpy array)."""
    import numpy as np
    import torch

    out = (C.c_double * (inner + 1))()
    st = lib().gs2_inner_residuals(h.ptr, _ptr(r, torch.float64, h.n, "r"), inner, out, _stream(stream))
    if st != OK:
        raise Gs2Error(st, "gs2_inner_residuals")
    return np.array(out[:], dtype=np.float64)


def gs2_inner_residuals_noalloc(h: Handle, r, inner: int, out, stream=None):
    """The allocation-free variant: writes the inner + 1 ratios into the
    float64 GPU tensor `out` on the stream, without allocating or
    synchronising (partial sums in the library's fixed per-device scratch)."""
    import torch

    st = lib().gs2_inner_residuals_noalloc(h.ptr, _ptr(r, torch.float64, h.n, "r"), inner,
                                           _ptr(out, torch.float64, inner + 1, "out"), _stream(stream))
    if st != OK:
        raise Gs2Error(st, "gs2_inner_residuals_noalloc")


def gs2_profile(enable: bool):
    lib().gs2_profile(1 if enable else 0)


def gs2_graphs(enable: bool) -> bool:
    """Switch the HIP-graph replay of GMRES restart cycles; returns the previous setting."""
    return bool(lib().gs2_graphs(1 if enable else 0))


def gs2_profile_read() -> dict:
    """{kernel name: {"launches", "ms", "bytes"}} for kinds with launches."""
    L = lib()
    out = {}
    for kid in range(L.gs2_profile_kernel_count()):
        name, cnt, ms, by = C.c_char_p(), C.c_int64(), C.c_double(), C.c_double()
        st = L.gs2_profile_read(kid, C.byref(name), C.byref(cnt), C.byref(ms), C.byref(by))
        if st != OK:
            raise Gs2Error(st, "gs2_profile_read")
        if cnt.value:
            out[name.value.decode()] = {"launches": cnt.value, "ms": ms.value, "bytes": by.value}
    return out


class BatchHandle:
    def __init__(self, ptr, sizes, nrhs, keep=None):
        self.ptr = ptr
        self.sizes = list(sizes)
        self.nrhs = nrhs
        self._keep = keep

    def __del__(self):
        try:
            gs2_destroy_batched(self)
        except Exception:
            pass


def gs2_setup_batched(mats, sweeps=2, inner=2, damping=1.0, variant=FORWARD, precision=FP32, restart=20, nrhs=4,
                      inner_damping=1.0, autotune=True, lanes_per_row=0, rhs_per_item=0, compact=False, team_rows=0,
                      team_wait_ms=0, stream=None) -> BatchHandle:
    """mats: list of DeviceCSR.  team_rows: rows x right-hand sides per
    workgroup of an item's team (0 = library default, < 0 = one workgroup
    per item); team_wait_ms: longest team barrier wait (0 = default, < 0 =
    none, which abandons every team item: the error path, for tests)."""
    descs = (CsrDesc * len(mats))(*[m.desc() for m in mats])
    opt = Options(precision, inner_damping, int(compact), 0, int(autotune), lanes_per_row, rhs_per_item, 0, 1, 1,
                  team_rows, team_wait_ms)
    out = C.c_void_p()
    st = lib().gs2_setup_batched(descs, len(mats), sweeps, inner, damping, variant, C.byref(opt), restart, nrhs,
                                 _stream(stream), C.byref(out))
    if st != OK:
        raise Gs2Error(st, "gs2_setup_batched")
    return BatchHandle(out, [m.n for m in mats], nrhs, keep=mats)


def gs2_batched_schedule(bh: BatchHandle) -> dict:
    """Lanes per row, right-hand sides per work item and whether they were timed."""
    v = [C.c_int() for _ in range(3)]
    st = lib().gs2_batched_schedule(bh.ptr, *[C.byref(x) for x in v])
    if st != OK:
        raise Gs2Error(st, "gs2_batched_schedule")
    return {k: x.value for k, x in zip(["lanes_per_row", "rhs_per_item", "tuned"], v)}


def gmres_solve_batched(bh: BatchHandle, nrhs, B, X, rtol=1e-8, maxit=10000, stream=None, raise_on_error=True):
    import torch

    tot = sum(bh.sizes) * nrhs
    infos = (SolveInfo * (len(bh.sizes) * nrhs))()
    st = lib().gmres_solve_batched(bh.ptr, nrhs, _ptr(B, torch.float64, tot, "B"), _ptr(X, torch.float64, tot, "X"),
                                   rtol, maxit, infos, _stream(stream))
    if st < 0 and raise_on_error:
        raise Gs2Error(st, "gmres_solve_batched")
    return st, [{"iterations": f.iterations, "restarts": f.restarts, "relres": f.relres,
                 "converged": bool(f.converged), "status": f.status} for f in infos]


def gs2_destroy_batched(bh: BatchHandle):
    if bh is not None and bh.ptr:
        lib().gs2_destroy_batched(bh.ptr)
        bh.ptr = None
