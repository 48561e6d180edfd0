"""Pins of the oracle's preconditioned conjugate gradients and of the
symmetry of the SGS2 preconditioner it relies on."""
import numpy as np
import pytest

import oracle
from gen import poisson2d, vardiff3d, laplace3d


def dense_op(fn, n):
    return np.column_stack([fn(e) for e in np.eye(n)])


@pytest.mark.parametrize("mk", [lambda: poisson2d(5), lambda: vardiff3d(3, seed=2)])
@pytest.mark.parametrize("sweeps,inner,w", [(1, 1, 1.0), (2, 2, 0.9), (1, 0, 0.8)])
def test_sgs2_operator_symmetric_positive(mk, sweeps, inner, w):
    """For symmetric A the symmetric two-stage operator is symmetric: the
    Neumann sum with U is the transpose of the one with L (L^T = U), and the
    forward/backward composition mirrors itself.  It is also positive
    definite on these M-matrices, so it is a valid CG preconditioner."""
    A = mk()
    P = dense_op(lambda v: oracle.gs2_apply(A, v, oracle.SYMMETRIC, sweeps, inner, w), A.n)
    assert np.abs(P - P.T).max() <= 1e-13 * np.abs(P).max()
    assert np.linalg.eigvalsh((P + P.T) / 2).min() > 0


@pytest.mark.parametrize("prec,kw", [("none", {}), ("gs2", dict(variant=oracle.SYMMETRIC, sweeps=1, inner=1)),
                                     ("jr", dict(sweeps=1, omega=0.8)), ("sor", dict(variant=oracle.SYMMETRIC))])
def test_pcg_a_norm_optimality(prec, kw):
    """x_k minimises the A-norm error over x0 + span{M^-1 r0, (M^-1 A) M^-1 r0, ...}:
    compare with the Galerkin solution on the explicitly built basis."""
    A = vardiff3d(4, seed=3)
    M = A.dense()
    rng = np.random.default_rng(1)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)

    def Pinv(v):
        if prec == "none":
            return v.copy()
        if prec == "gs2":
            return oracle.gs2_apply(A, v, kw["variant"], kw["sweeps"], kw["inner"], 1.0)
        if prec == "jr":
            return oracle.jr_sweep(A, v, np.zeros(A.n), kw["sweeps"], kw["omega"])
        return oracle.sor_sweep(A, v, np.zeros(A.n), kw["variant"], 1, 1.0)

    r0 = b - M @ x0
    for k in (1, 3, 6):
        x, info = oracle.pcg(A, b, x0, rtol=1e-30, maxit=k, prec=prec, **kw)
        assert info["iterations"] == k
        K, v = [], Pinv(r0)
        for _ in range(k):
            K.append(v / np.linalg.norm(v))
            v = Pinv(M @ K[-1])
        K = np.linalg.qr(np.column_stack(K))[0]
        y = np.linalg.solve(K.T @ M @ K, K.T @ r0)
        xs = np.linalg.solve(M, b)
        err = lambda z: np.sqrt((z - xs) @ M @ (z - xs))  # noqa: E731
        # the minimum A-norm error is well conditioned even when the basis is not
        assert err(x) == pytest.approx(err(x0 + K @ y), rel=1e-7, abs=1e-12)
        np.testing.assert_allclose(x, x0 + K @ y, rtol=1e-5, atol=1e-6)


def test_pcg_finite_termination_and_status():
    A = poisson2d(6)
    b = np.random.default_rng(2).standard_normal(A.n)
    x, info = oracle.pcg(A, b, rtol=1e-12, maxit=200)
    assert info["converged"] and info["iterations"] <= A.n + 5
    np.testing.assert_allclose(A.dense() @ x, b, atol=1e-10 * np.linalg.norm(b))
    _, info = oracle.pcg(A, b, rtol=1e-14, maxit=3)
    assert info["status"] == oracle.NOT_CONVERGED and info["iterations"] == 3
    x, info = oracle.pcg(A, np.zeros(A.n))
    assert info["converged"] and info["iterations"] == 0 and not x.any()


def test_pcg_reduced_precision_keeps_iterations():
    """Single-precision SGS2 keeps the CG iteration count (Section 10)."""
    A = laplace3d(10)
    b = np.random.default_rng(4).standard_normal(A.n)
    its = [oracle.pcg(A, b, prec="gs2", variant=oracle.SYMMETRIC, sweeps=1, inner=1, precision=p)[1]["iterations"]
           for p in (oracle.FP64, oracle.FP32, oracle.FP16S)]
    assert abs(its[1] - its[0]) <= 1 and abs(its[2] - its[0]) <= 2
