"""Pins of the oracle's reduced-precision preconditioner forms (FP32 and
diagonally scaled FP16 storage with FP32 arithmetic).

The paper fixes only that the preconditioner runs in single precision while
the Krylov solver stays in double (Section 10).  The forms are defined in
symmetrically scaled variables (exact-arithmetic invariant); these tests pin
(1) the binary16 rounding against numpy's IEEE conversion, (2) exactness on
dyadic data where no rounding can occur, so the reduced forms must equal the
float64 textbook form bit for bit, and (3) error bounds against float64.
"""
import numpy as np
import pytest

import oracle
from gen import poisson2d, laplace3d, random_sparse, vardiff3d, CSR

F, B, S = oracle.FORWARD, oracle.BACKWARD, oracle.SYMMETRIC


def test_round_f16_all_bit_patterns():
    h = np.arange(65536, dtype=np.uint32).astype(np.uint16).view(np.float16)
    d = h.astype(np.float64)
    out = np.array([oracle.round_f16(x) for x in d])
    fin = np.isfinite(d)
    assert np.array_equal(out[fin], d[fin])
    assert np.all(np.isinf(out[np.isinf(d)]) & (np.sign(out[np.isinf(d)]) == np.sign(d[np.isinf(d)])))
    assert np.all(np.isnan(out[np.isnan(d)]))


def test_round_f16_random_and_ties():
    rng = np.random.default_rng(0)
    xs = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-9, 5, 20000),
        rng.uniform(65000, 66000, 2000) * rng.choice([-1, 1], 2000),
    ])
    # exact midpoints between consecutive finite halfs (ties -> even)
    h = np.arange(0, 0x7BFF, dtype=np.uint16).view(np.float16).astype(np.float64)
    mids = (h[:-1] + h[1:]) / 2
    xs = np.concatenate([xs, mids, -mids, [65519.99, 65520.0, 65504.0, 2.0 ** -25, 2.0 ** -26, 3 * 2.0 ** -26]])
    with np.errstate(over="ignore"):
        ref = xs.astype(np.float16).astype(np.float64)
    out = np.array([oracle.round_f16(x) for x in xs])
    assert np.array_equal(out, ref)


def dyadic_problem(N):
    A = poisson2d(N)  # d = 4: scale 1/2, scaled off-diagonals -1/4, all exact
    v = np.random.default_rng(1).integers(-8, 9, A.n).astype(np.float64)
    return A, v


@pytest.mark.parametrize("prec", [oracle.FP32, oracle.FP16S])
@pytest.mark.parametrize("variant,sweeps,inner", [(F, 1, 1), (F, 2, 3), (B, 1, 2), (S, 2, 1), (F, 3, 0)])
def test_reduced_forms_exact_on_dyadic_data(prec, variant, sweeps, inner):
    """Every scaled value, product and partial sum is a short dyadic rational,
    exactly representable in binary32, so the reduced form must reproduce the
    float64 textbook (unscaled) result exactly."""
    A, v = dyadic_problem(6)
    z64 = oracle.gs2_apply(A, v, variant, sweeps, inner, 1.0)
    zlp = oracle.gs2_apply_lp(A, v, prec, variant, sweeps, inner, 1.0)
    assert np.array_equal(z64, zlp)


@pytest.mark.parametrize("prec", [oracle.FP32, oracle.FP16S])
@pytest.mark.parametrize("variant,sweeps,inner,w,gamma", [(F, 1, 2, 1.0, 0.5), (S, 1, 2, 0.5, 0.5),
                                                          (F, 2, 2, 0.5, 0.5), (B, 1, 3, 1.0, 0.75),
                                                          (F, 1, 3, 0.5, 0.25)])
def test_reduced_forms_inner_damping_exact_on_dyadic_data(prec, variant, sweeps, inner, w, gamma):
    """Inner damping (Section 9) in the reduced forms: with dyadic damping
    factors and few enough sweeps every value stays a dyadic rational short
    enough for binary32, so the reduced form with gamma must equal the
    float64 textbook form with the same gamma bit for bit; a gamma dropped,
    applied to the wrong term or to the wrong iterate changes the result."""
    A, v = dyadic_problem(6)
    z64 = oracle.gs2_apply(A, v, variant, sweeps, inner, w, gamma)
    zlp = oracle.gs2_apply_lp(A, v, prec, variant, sweeps, inner, w, gamma)
    assert np.array_equal(z64, zlp)
    assert not np.array_equal(z64, oracle.gs2_apply(A, v, variant, sweeps, inner, w, 1.0))


def test_reduced_forms_refuse_compact_and_blocks():
    """The reduced-precision forms are defined for the non-compact sweep over
    the whole matrix: the oracle's GMRES refuses the others in them."""
    A, v = dyadic_problem(6)
    for kw in (dict(compact=True), dict(blocks=2)):
        _, info = oracle.gmres(A, v, restart=10, rtol=1e-8, prec="gs2", precision=oracle.FP32, **kw)
        assert info["status"] == -1 and info["iterations"] == 0, (kw, info)  # argument error


@pytest.mark.parametrize("mk", [lambda: random_sparse(200, seed=7, avg_offdiag=6, neg_diag_rows=10),
                                lambda: vardiff3d(6, seed=3), lambda: laplace3d(6)])
@pytest.mark.parametrize("variant,sweeps,inner", [(F, 2, 1), (S, 1, 2)])
def test_reduced_forms_error_bounds(mk, variant, sweeps, inner):
    """Relative 2-norm error against float64: a few hundred unit roundoffs of
    the storage format (each stored value and each partial sum carries one)."""
    A = mk()
    v = np.random.default_rng(2).standard_normal(A.n)
    z64 = oracle.gs2_apply(A, v, variant, sweeps, inner, 0.9)
    e32 = np.linalg.norm(oracle.gs2_apply_lp(A, v, oracle.FP32, variant, sweeps, inner, 0.9) - z64) / np.linalg.norm(z64)
    e16 = np.linalg.norm(oracle.gs2_apply_lp(A, v, oracle.FP16S, variant, sweeps, inner, 0.9) - z64) / np.linalg.norm(z64)
    assert e32 < 300 * 2.0 ** -24
    assert 2.0 ** -24 * 0.01 < e16 < 300 * 2.0 ** -11
    assert e32 < e16


def test_fp16_range_error():
    """Scaled entries beyond binary16 range are rejected (not silently inf)."""
    A = CSR(2, np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32), np.array([1e-6, 1.0, 1.0, 1e-6]))
    with pytest.raises(oracle.OracleError) as e:
        oracle.gs2_apply_lp(A, np.ones(2), oracle.FP16S)
    assert e.value.status == oracle.ERR_FP16_RANGE


def test_gmres_reduced_precision_reaches_tolerance():
    """The FP64 outer Krylov loop recovers full accuracy with an FP32 / FP16
    preconditioner, with about the same iteration count (Section 10)."""
    A = vardiff3d(10, seed=9)
    b = np.random.default_rng(3).standard_normal(A.n)
    its = {}
    for p in (oracle.FP64, oracle.FP32, oracle.FP16S):
        x, info = oracle.gmres(A, b, restart=50, rtol=1e-8, prec="gs2", variant=S, sweeps=1, inner=1, precision=p)
        assert info["converged"] and info["relres"] <= 1e-8
        its[p] = info["iterations"]
    assert abs(its[oracle.FP32] - its[oracle.FP64]) <= 1
    assert abs(its[oracle.FP16S] - its[oracle.FP64]) <= max(2, its[oracle.FP64] // 10)


# ------------------------------------------------ binary32 accumulation pin
#
# The reduced forms accumulate every row sum in binary32 (Section 10: the
# preconditioner runs in single precision).  On a unit-diagonal matrix the
# scaling is exact (s = 1) and every entry below is representable in binary32
# and binary16 (2^-24 is the smallest binary16 subnormal), so only the
# rounding of the partial sums can change the result.  Row 3 sums, in CSR
# order, 1 * 1 + 2^-24 * 1 + 2^-24 * 1:
#   binary32: 1 + 2^-24 lies halfway between 1 and 1 + 2^-23; round to
#             nearest even keeps 1 (even significand); the second 2^-24 is
#             again a tie and again gives 1.  The sum is 1.
#   binary64: 1 + 2^-24 + 2^-24 = 1 + 2^-23 exactly.
# With v_3 = 2 the inner step gives g_3 = 2 - 1 = 1 in binary32, while an
# accumulation in binary64 would give 2 - (1 + 2^-23) = 1 - 2^-23, which is
# representable in binary32 (spacing 2^-24 below 1) and so survives the
# final rounding.

def _tie_matrix(lower=True):
    """4x4 unit-diagonal matrix whose only coupled row sums 1, 2^-24, 2^-24
    (in CSR order) against the identity rows."""
    e = 2.0 ** -24
    if lower:  # row 3: columns 0, 1, 2 off the diagonal
        rp = np.array([0, 1, 2, 3, 7], np.int32)
        ci = np.array([0, 1, 2, 0, 1, 2, 3], np.int32)
        va = np.array([1.0, 1.0, 1.0, 1.0, e, e, 1.0])
        row = 3
    else:  # row 0: columns 1, 2, 3 off the diagonal
        rp = np.array([0, 4, 5, 6, 7], np.int32)
        ci = np.array([0, 1, 2, 3, 1, 2, 3], np.int32)
        va = np.array([1.0, 1.0, e, e, 1.0, 1.0, 1.0])
        row = 0
    return CSR(4, rp, ci, va), row


@pytest.mark.parametrize("prec", [oracle.FP32, oracle.FP16S])
@pytest.mark.parametrize("lower", [True, False])
def test_binary32_accumulation_inner_sum(prec, lower):
    """One GS2 half with one inner sweep from zero: the coupled row's inner
    sum must round in binary32 (result exactly 1.0), while the float64
    textbook form gives 1 - 2^-23."""
    A, row = _tie_matrix(lower)
    v = np.ones(4)
    v[row] = 2.0
    variant = F if lower else B
    z = oracle.gs2_apply_lp(A, v, prec, variant, 1, 1, 1.0)
    expect = np.ones(4)  # identity rows: z = v = 1; coupled row: 2 - 1 = 1
    assert np.array_equal(z, expect), z
    z64 = oracle.gs2_apply(A, v, variant, 1, 1, 1.0)
    assert z64[row] == 1.0 - 2.0 ** -23


@pytest.mark.parametrize("prec", [oracle.FP32, oracle.FP16S])
@pytest.mark.parametrize("lower", [True, False])
def test_binary32_accumulation_residual_sum(prec, lower):
    """Two Jacobi-Richardson sweeps (n_j = 0): the second sweep's outer
    residual of the coupled row is, in binary32 and CSR order,
    ((2 - 2) - 1*1) - 2^-24 - 2^-24 = -1 (both subtractions are ties that
    round to the even -1), so x = 2 + (-1) = 1 exactly; in binary64 the
    residual is -(1 + 2^-23) and x = 1 - 2^-23."""
    A, row = _tie_matrix(lower)
    v = np.ones(4)
    v[row] = 2.0
    variant = F if lower else B
    z = oracle.gs2_apply_lp(A, v, prec, variant, 2, 0, 1.0)
    assert np.array_equal(z, np.ones(4)), z
    z64 = oracle.gs2_apply(A, v, variant, 2, 0, 1.0)
    assert z64[row] == 1.0 - 2.0 ** -23
