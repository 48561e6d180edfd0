"""Pins of the oracle's restarted, flexible, right-preconditioned GMRES."""
import numpy as np
import pytest

import oracle
from gen import poisson2d, random_sparse, CSR, config_problem


def test_finite_termination_unpreconditioned():
    A = random_sparse(24, seed=21, avg_offdiag=6, dominance=0.6)  # not diagonally dominant
    b = np.random.default_rng(0).standard_normal(A.n)
    x, info = oracle.gmres(A, b, restart=A.n, rtol=1e-12, maxit=A.n, prec="none")
    assert info["converged"] and info["iterations"] <= A.n
    np.testing.assert_allclose(A.dense() @ x, b, rtol=0, atol=1e-10 * np.linalg.norm(b))


@pytest.mark.parametrize("prec,kw", [("none", {}), ("gs2", dict(sweeps=1, inner=1)),
                                     ("gs2", dict(variant=oracle.SYMMETRIC, sweeps=2, inner=2, omega=0.9)),
                                     ("jr", dict(sweeps=2, omega=0.8)), ("sor", dict(sweeps=1, omega=1.1))])
def test_minimal_residual_property(prec, kw):
    """After k Arnoldi steps without restart, x_k minimises ||b - A x|| over
    x0 + span{M^-1 r0, M^-1 A M^-1 r0, ...} (M^-1 linear here).  Compare with
    numpy.linalg.lstsq over that explicitly built basis."""
    A = random_sparse(30, seed=22, avg_offdiag=5, dominance=1.1)
    M = A.dense()
    rng = np.random.default_rng(1)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)

    def P(v):
        if prec == "none":
            return v.copy()
        if prec == "gs2":
            return oracle.gs2_apply(A, v, kw.get("variant", 0), kw["sweeps"], kw["inner"], kw.get("omega", 1.0))
        if prec == "jr":
            return oracle.jr_sweep(A, v, np.zeros(A.n), kw["sweeps"], kw["omega"])
        return oracle.sor_sweep(A, v, np.zeros(A.n), 0, kw["sweeps"], kw["omega"])

    r0 = b - M @ x0
    for k in (1, 3, 6):
        x, info = oracle.gmres(A, b, x0, restart=50, rtol=1e-30, maxit=k, prec=prec, **kw)
        assert info["iterations"] == k
        W, v = [], r0 / np.linalg.norm(r0)
        for _ in range(k):
            z = P(v)
            W.append(z)
            v = M @ z
            v /= np.linalg.norm(v)
        W = np.column_stack(W)
        y = np.linalg.lstsq(M @ W, r0, rcond=None)[0]
        best = np.linalg.norm(r0 - M @ W @ y)
        assert np.linalg.norm(b - M @ x) == pytest.approx(best, rel=1e-7, abs=1e-12)


def test_jr1_iteration_count_independent_of_damping():
    """w D^{-1} is a scalar multiple of D^{-1}; GMRES iterates do not change
    (the paper's JR(1) column is the same for every damping factor)."""
    p = config_problem(1, size=24)
    its = []
    for w in (1.0, 0.9, 0.8, 0.7):
        _, info = oracle.gmres(p["A"], p["b"], restart=30, rtol=1e-8, prec="jr", sweeps=1, omega=w)
        assert info["converged"]
        its.append(info["iterations"])
    assert len(set(its)) == 1


def test_exact_preconditioner_one_step():
    """Lower-triangular A: forward GS, and GS2 with inner >= DAG depth, are
    exact inverses, so GMRES converges in one step."""
    A0 = poisson2d(5)
    M = np.tril(A0.dense())
    import scipy.sparse as sp

    T = sp.csr_matrix(M)
    A = CSR(T.shape[0], T.indptr.astype(np.int32), T.indices.astype(np.int32), T.data.astype(np.float64))
    b = np.random.default_rng(3).standard_normal(A.n)
    for prec, kw in [("sor", dict(sweeps=1)), ("gs2", dict(sweeps=1, inner=8))]:
        x, info = oracle.gmres(A, b, restart=10, rtol=1e-10, prec=prec, **kw)
        assert info["converged"] and info["iterations"] == 1


def test_identity_breakdown_and_zero_rhs():
    n = 12
    A = CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    b = np.random.default_rng(4).standard_normal(n)
    x, info = oracle.gmres(A, b, restart=5, rtol=1e-12, prec="none")
    assert info["converged"] and info["iterations"] == 1
    np.testing.assert_allclose(x, b, rtol=1e-14)
    x, info = oracle.gmres(A, np.zeros(n), restart=5, rtol=1e-12, prec="none")
    assert info["converged"] and info["iterations"] == 0 and not x.any()


def test_not_converged_and_nonfinite_status():
    p = config_problem(1, size=16)
    _, info = oracle.gmres(p["A"], p["b"], restart=5, rtol=1e-12, maxit=7, prec="none")
    assert info["status"] == oracle.NOT_CONVERGED and info["iterations"] == 7 and not info["converged"]
    b = p["b"].copy()
    b[3] = np.nan
    _, info = oracle.gmres(p["A"], b, restart=5, prec="none")
    assert info["status"] == oracle.ERR_NONFINITE


def test_zero_diagonal_rejected():
    A = poisson2d(3)
    A.val[A.colind == np.repeat(np.arange(A.n), np.diff(A.rowptr))] *= np.r_[1, 1, 0, [1] * 6]
    with pytest.raises(oracle.OracleError) as e:
        oracle.gs2_apply(A, np.ones(A.n))
    assert e.value.status == oracle.ERR_ZERO_DIAG


def test_mgs_and_cgs2_agree():
    p = config_problem(1, size=32)
    a = oracle.gmres(p["A"], p["b"], restart=30, prec="gs2", sweeps=1, inner=1)
    c = oracle.gmres(p["A"], p["b"], restart=30, prec="gs2", sweeps=1, inner=1, cgs2=True)
    assert abs(a[1]["iterations"] - c[1]["iterations"]) <= 1
    np.testing.assert_allclose(a[0], c[0], rtol=1e-6, atol=1e-7)


def test_solution_accuracy_config1():
    """GS2(1,1)-GMRES(30) on the 64^2 Poisson problem reaches 1e-8."""
    p = config_problem(1)
    x, info = oracle.gmres(p["A"], p["b"], restart=30, rtol=1e-8, prec="gs2", sweeps=1, inner=1)
    assert info["converged"] and info["relres"] <= 1e-8
    assert np.linalg.norm(x - p["x_true"]) / np.linalg.norm(p["x_true"]) < 1e-4


@pytest.mark.parametrize("cgs2", [False, True])
def test_happy_breakdown_ends_the_cycle(cgs2):
    """Happy breakdown (reading of the stopping rule: the Krylov space has
    become invariant).  A = diag(1..6) and b in the span of its first two
    eigenvectors: the Krylov space of b has dimension 2, so the second
    Arnoldi step leaves only rounding noise (h_{3,2} ~ 1e-17).  rtol = 0 keeps
    the residual-estimate test from ending the cycle (the recorded estimate
    after step 2 is nonzero), so only the breakdown branch can: the first cycle
    must end after exactly 2 steps with the exact solution, and the third step
    then belongs to a second cycle."""
    n = 6
    d = np.arange(1, n + 1, dtype=np.float64)
    A = CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d.copy())
    b = np.array([0.3, 0.7, 0, 0, 0, 0])
    # one cycle only: the breakdown leaves the cycle after step 2 with the exact solution
    x, info = oracle.gmres(A, b, restart=10, rtol=0.0, maxit=2, prec="none", cgs2=cgs2, history=True)
    assert info["iterations"] == 2 and info["restarts"] == 0
    assert info["history"][2] > 0.0  # the estimate did not reach rtol = 0
    np.testing.assert_allclose(x, b / d, rtol=0, atol=1e-15)
    # a third step: it must start a second cycle (restart count 1)
    x, info = oracle.gmres(A, b, restart=10, rtol=0.0, maxit=3, prec="none", cgs2=cgs2, history=True)
    assert info["iterations"] == 3 and info["restarts"] == 1, info
    assert info["history"][2] > 0.0
    np.testing.assert_allclose(x, b / d, rtol=0, atol=1e-15)
