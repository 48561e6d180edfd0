"""CPU oracle: plain single-threaded float64 GS2 / JR / Gauss-Seidel / GMRES.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the library under
paper_2104_01196_amd never does, and the two share no code.  The arithmetic
lives in gs2_oracle.c (built with gcc -O2 -ffp-contract=off, no OpenMP); this
module only marshals numpy arrays through ctypes.

Parity status per function (what pins it lives in tests/test_oracle_*.py):
  spmv, gs2_apply / gs2_sweep, jr_sweep, sor_sweep, levels, gmres,
  round_f16, gs2_apply_lp (FP32 / FP16-scaled, including the binary32 rounding
  of its row sums), gs2c_sweep (compact form), pcg, inner_residuals (dense
  Neumann partial sums at damping != 1, and the n_j -> depth limit): all
  pinned.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs2_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-shared", "-fPIC"]

FORWARD, BACKWARD, SYMMETRIC = 0, 1, 2
PREC_NONE, PREC_GS2, PREC_JR, PREC_SOR, PREC_MTGS = 0, 1, 2, 3, 4
_PREC = {"none": PREC_NONE, "gs2": PREC_GS2, "jr": PREC_JR, "sor": PREC_SOR, "mtgs": PREC_MTGS}
FP64, FP32, FP16S = 0, 1, 2
OK, ERR_ARG, ERR_ZERO_DIAG, ERR_NONFINITE, ERR_NOMEM, ERR_FP16_RANGE = 0, -1, -3, -4, -5, -7
NOT_CONVERGED, BREAKDOWN = 1, 2


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, no GPU code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


class _Prec(C.Structure):
    _fields_ = [("kind", C.c_int), ("variant", C.c_int), ("sweeps", C.c_int), ("inner", C.c_int),
                ("omega", C.c_double), ("gamma", C.c_double), ("precision", C.c_int), ("compact", C.c_int),
                ("blocks", C.c_int), ("local_sweeps", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("relres", C.c_double),
                ("converged", C.c_int), ("status", C.c_int)]


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        csr = [C.c_int, _i32p, _i32p, _f64p]
        L.or_spmv.argtypes = csr + [_f64p, _f64p]
        L.or_diag.argtypes = csr + [_f64p]
        L.or_gs2_sweep.argtypes = csr + [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, _f64p, _f64p]
        L.or_gs2_apply.argtypes = L.or_gs2_sweep.argtypes
        L.or_gs2c_sweep.argtypes = L.or_gs2_sweep.argtypes
        L.or_jr_sweep.argtypes = csr + [C.c_int, C.c_double, _f64p, _f64p]
        L.or_sor_sweep.argtypes = csr + [C.c_int, C.c_int, C.c_double, _f64p, _f64p]
        L.or_levels.argtypes = [C.c_int, _i32p, _i32p, C.c_int, _i32p]
        L.or_inner_residuals.argtypes = csr + [C.c_int, C.c_double, _f64p, _f64p]
        L.or_round_f16.argtypes = [C.c_double]
        L.or_round_f16.restype = C.c_double
        L.or_gs2_apply_lp.argtypes = csr + [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, _f64p, _f64p]
        L.or_gmres.argtypes = csr + [_f64p, _f64p, C.c_int, C.c_double, C.c_int, C.POINTER(_Prec), C.c_int,
                                     C.POINTER(_Info), C.c_void_p]
        L.or_pcg.argtypes = csr + [_f64p, _f64p, C.c_double, C.c_int, C.POINTER(_Prec), C.POINTER(_Info)]
        L.or_colors.argtypes = [C.c_int, _i32p, _i32p, _i32p]
        L.or_gs2_block_sweep.argtypes = csr + [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                               _f64p, _f64p]
        L.or_mtgs_sweep.argtypes = csr + [C.c_int, C.c_int, C.c_double, _f64p, _f64p]
        _lib = L
    return _lib


def _csr(A):
    return (int(A.n), np.ascontiguousarray(A.rowptr, np.int32), np.ascontiguousarray(A.colind, np.int32),
            np.ascontiguousarray(A.val, np.float64))


def _vec(v):
    return np.ascontiguousarray(v, np.float64)


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


def _chk(st):
    if st < 0:
        raise OracleError(st)
    return st


def spmv(A, x):
    y = np.empty(A.n)
    lib().or_spmv(*_csr(A), _vec(x), y)
    return y


def diag(A):
    d = np.empty(A.n)
    _chk(lib().or_diag(*_csr(A), d))
    return d


def gs2_sweep(A, b, x0, variant=FORWARD, sweeps=1, inner=1, omega=1.0, gamma=1.0):
    """Stand-alone GS2 iteration from x0 (returns a new array)."""
    x = _vec(x0).copy()
    _chk(lib().or_gs2_sweep(*_csr(A), variant, sweeps, inner, omega, gamma, _vec(b), x))
    return x


def gs2_apply(A, v, variant=FORWARD, sweeps=1, inner=1, omega=1.0, gamma=1.0):
    """Preconditioner form: GS2 on A z = v from z = 0."""
    z = np.empty(A.n)
    _chk(lib().or_gs2_apply(*_csr(A), variant, sweeps, inner, omega, gamma, _vec(v), z))
    return z


def gs2c_sweep(A, b, x0, variant=FORWARD, sweeps=1, inner=1, omega=1.0, gamma=1.0):
    """Compact two-stage form from x0."""
    x = _vec(x0).copy()
    _chk(lib().or_gs2c_sweep(*_csr(A), variant, sweeps, inner, omega, gamma, _vec(b), x))
    return x


def jr_sweep(A, b, x0, sweeps=1, omega=1.0):
    x = _vec(x0).copy()
    _chk(lib().or_jr_sweep(*_csr(A), sweeps, omega, _vec(b), x))
    return x


def sor_sweep(A, b, x0, variant=FORWARD, sweeps=1, omega=1.0):
    x = _vec(x0).copy()
    _chk(lib().or_sor_sweep(*_csr(A), variant, sweeps, omega, _vec(b), x))
    return x


def levels(A, lower=True):
    lv = np.empty(A.n, np.int32)
    nlev = lib().or_levels(int(A.n), np.ascontiguousarray(A.rowptr, np.int32),
                           np.ascontiguousarray(A.colind, np.int32), 1 if lower else 0, lv)
    return lv, nlev


def gs2_block_sweep(A, b, x0, blocks=1, variant=FORWARD, sweeps=1, local_sweeps=1, inner=1, omega=1.0, gamma=1.0):
    """Hybrid block-Jacobi GS2: `sweeps` global sweeps, each freezing the
    off-block values and running `local_sweeps` local GS2 sweeps per block."""
    x = _vec(x0).copy()
    _chk(lib().or_gs2_block_sweep(*_csr(A), blocks, variant, sweeps, local_sweeps, inner, omega, gamma, _vec(b), x))
    return x


def colors(A):
    """Greedy first-fit coloring in natural order on the symmetrised pattern."""
    c = np.empty(A.n, np.int32)
    ncol = lib().or_colors(int(A.n), np.ascontiguousarray(A.rowptr, np.int32),
                           np.ascontiguousarray(A.colind, np.int32), c)
    _chk(ncol)
    return c, ncol


def mtgs_sweep(A, b, x0, variant=FORWARD, sweeps=1, omega=1.0):
    """Multicolor Gauss-Seidel / SOR sweeps from x0."""
    x = _vec(x0).copy()
    _chk(lib().or_mtgs_sweep(*_csr(A), variant, sweeps, omega, _vec(b), x))
    return x


def inner_residuals(A, r, inner, omega=1.0):
    out = np.empty(inner + 1)
    _chk(lib().or_inner_residuals(*_csr(A), inner, omega, _vec(r), out))
    return out


def round_f16(x: float) -> float:
    return lib().or_round_f16(float(x))


def gs2_apply_lp(A, v, precision=FP32, variant=FORWARD, sweeps=1, inner=1, omega=1.0, gamma=1.0):
    """Reduced-precision (FP32 or FP16-scaled) GS2 apply from zero, inner damping gamma."""
    z = np.empty(A.n)
    _chk(lib().or_gs2_apply_lp(*_csr(A), precision, variant, sweeps, inner, omega, gamma, _vec(v), z))
    return z


def gmres(A, b, x0=None, restart=30, rtol=1e-8, maxit=10000, prec="none", variant=FORWARD, sweeps=1, inner=1,
          omega=1.0, gamma=1.0, precision=FP64, compact=False, cgs2=False, history=False, blocks=1, local_sweeps=1):
    """Restarted flexible GMRES(m).  prec in {"none", "gs2", "jr", "sor"}.

    Returns (x, info dict).  info: iterations, restarts, relres, converged,
    status, seconds (wall time of the solve, setup included), and history
    (relative residual estimates) when requested.
    """
    kind = _PREC[prec]
    P = _Prec(kind, variant, sweeps, inner, omega, gamma, precision, 1 if compact else 0, blocks, local_sweeps)
    info = _Info()
    x = np.zeros(A.n) if x0 is None else _vec(x0).copy()
    hist = np.full(maxit + 2, np.nan) if history else None
    t0 = time.perf_counter()
    lib().or_gmres(*_csr(A), _vec(b), x, restart, rtol, maxit, C.byref(P), 1 if cgs2 else 0, C.byref(info),
                   hist.ctypes.data_as(C.c_void_p) if hist is not None else None)
    dt = time.perf_counter() - t0
    out = {"iterations": info.iterations, "restarts": info.restarts, "relres": info.relres,
           "converged": bool(info.converged), "status": info.status, "seconds": dt}
    if history:
        out["history"] = hist[: info.iterations + 1]
    return x, out


def pcg(A, b, x0=None, rtol=1e-8, maxit=10000, prec="none", variant=SYMMETRIC, sweeps=1, inner=1, omega=1.0,
        gamma=1.0, precision=FP64, compact=False, blocks=1, local_sweeps=1):
    """Preconditioned conjugate gradients.  Returns (x, info dict)."""
    kind = _PREC[prec]
    P = _Prec(kind, variant, sweeps, inner, omega, gamma, precision, 1 if compact else 0, blocks, local_sweeps)
    info = _Info()
    x = np.zeros(A.n) if x0 is None else _vec(x0).copy()
    t0 = time.perf_counter()
    lib().or_pcg(*_csr(A), _vec(b), x, rtol, maxit, C.byref(P), C.byref(info))
    dt = time.perf_counter() - t0
    return x, {"iterations": info.iterations, "restarts": info.restarts, "relres": info.relres,
               "converged": bool(info.converged), "status": info.status, "seconds": dt}
