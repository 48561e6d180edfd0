"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test compares the oracle's sparse, step-by-step arithmetic with something
independent of it: a dense closed form from a different equation of the
paper, a library routine (numpy / scipy), a closed-form spectrum, a structural
invariant, or brute force on a tiny input.  A dropped term, a wrong sign, a
wrong triangle or a transposed operand in the oracle fails at least one of
them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from gen import laplace1d, laplace3d, poisson2d, random_sparse, vardiff3d, elasticity_q1

F, B, S = oracle.FORWARD, oracle.BACKWARD, oracle.SYMMETRIC


def parts(A):
    M = A.dense()
    return np.tril(M, -1), np.diag(np.diag(M)), np.triu(M, 1), M


def operator(fn, n):
    """Dense matrix of a linear map given as a function of a vector."""
    return np.column_stack([fn(e) for e in np.eye(n)])


def rho(G):
    return np.max(np.abs(np.linalg.eigvals(G)))


MATS = {
    "rand_nonsym": lambda: random_sparse(40, seed=1, avg_offdiag=5, long_rows=2, long_len=30, diag_only_rows=3),
    "rand_negdiag": lambda: random_sparse(30, seed=2, avg_offdiag=4, neg_diag_rows=5),
    "poisson2d_5": lambda: poisson2d(5),
    "vardiff3d_3": lambda: vardiff3d(3, seed=5),
}


# ------------------------------------------------------------------ SpMV

@pytest.mark.parametrize("name", list(MATS))
def test_spmv_matches_dense(name):
    A = MATS[name]()
    x = np.random.default_rng(0).standard_normal(A.n)
    np.testing.assert_allclose(oracle.spmv(A, x), A.dense() @ x, rtol=1e-14, atol=1e-14)


# ---------------------------------------------------- exact GS / SOR (Section 3)

@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("w", [1.0, 0.8, 1.3])
def test_sor_is_triangular_solve(name, w):
    """One SOR sweep x1 = x0 + w (D + wL)^{-1}(b - A x0) (forward) or with U
    (backward), computed by scipy's triangular solver on the dense factors."""
    A = MATS[name]()
    L, D, U, M = parts(A)
    rng = np.random.default_rng(3)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    fwd = x0 + w * sla.solve_triangular(D + w * L, b - M @ x0, lower=True)
    np.testing.assert_allclose(oracle.sor_sweep(A, b, x0, F, 1, w), fwd, rtol=1e-12, atol=1e-12)
    bwd = x0 + w * sla.solve_triangular(D + w * U, b - M @ x0, lower=False)
    np.testing.assert_allclose(oracle.sor_sweep(A, b, x0, B, 1, w), bwd, rtol=1e-12, atol=1e-12)
    sym = fwd + w * sla.solve_triangular(D + w * U, b - M @ fwd, lower=False)
    np.testing.assert_allclose(oracle.sor_sweep(A, b, x0, S, 1, w), sym, rtol=1e-12, atol=1e-12)
    two = fwd + w * sla.solve_triangular(D + w * L, b - M @ fwd, lower=True)
    np.testing.assert_allclose(oracle.sor_sweep(A, b, x0, F, 2, w), two, rtol=1e-12, atol=1e-12)


# --------------------------------------------- GS2 against the Neumann form (Section 4)

def neumann_half(L, D, T, M, b, x, s, w, gamma=1.0):
    """x + w g_s, with g_s = sum_{k<=s} (-w D^{-1} T)^k D^{-1} r for gamma = 1
    (the degree-s Neumann expansion of Section 4); for gamma != 1 the affine
    inner map g -> G g + c with G = (1-gamma) I - gamma w D^{-1} T,
    c = gamma D^{-1} r, started at D^{-1} r, summed in closed form."""
    Dinv = np.diag(1.0 / np.diag(D))
    r = b - M @ x
    if gamma == 1.0:
        K = -w * Dinv @ T
        g = sum(np.linalg.matrix_power(K, k) @ (Dinv @ r) for k in range(s + 1))
    else:
        n = len(b)
        G = (1 - gamma) * np.eye(n) - gamma * w * Dinv @ T
        c = gamma * Dinv @ r
        g = np.linalg.matrix_power(G, s) @ (Dinv @ r) + sum(np.linalg.matrix_power(G, k) @ c for k in range(s))
    return x + w * g


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("s", [0, 1, 2, 4])
@pytest.mark.parametrize("w", [1.0, 0.7])
def test_gs2_matches_neumann_sum(name, s, w):
    A = MATS[name]()
    L, D, U, M = parts(A)
    rng = np.random.default_rng(11)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    f = neumann_half(L, D, L, M, b, x0, s, w)
    np.testing.assert_allclose(oracle.gs2_sweep(A, b, x0, F, 1, s, w), f, rtol=1e-11, atol=1e-11)
    bk = neumann_half(L, D, U, M, b, x0, s, w)
    np.testing.assert_allclose(oracle.gs2_sweep(A, b, x0, B, 1, s, w), bk, rtol=1e-11, atol=1e-11)
    sy = neumann_half(L, D, U, M, b, f, s, w)
    np.testing.assert_allclose(oracle.gs2_sweep(A, b, x0, S, 1, s, w), sy, rtol=1e-11, atol=1e-11)
    f2 = neumann_half(L, D, L, M, b, f, s, w)
    np.testing.assert_allclose(oracle.gs2_sweep(A, b, x0, F, 2, s, w), f2, rtol=1e-11, atol=1e-11)
    # preconditioner form: zero initial guess
    z = neumann_half(L, D, L, M, b, np.zeros(A.n), s, w)
    np.testing.assert_allclose(oracle.gs2_apply(A, b, F, 1, s, w), z, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("gamma", [0.5, 0.8])
def test_gs2_inner_damping_closed_form(gamma):
    A = MATS["rand_nonsym"]()
    L, D, U, M = parts(A)
    rng = np.random.default_rng(5)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    for s in (1, 3):
        ref = neumann_half(L, D, L, M, b, x0, s, 0.9, gamma)
        np.testing.assert_allclose(oracle.gs2_sweep(A, b, x0, F, 1, s, 0.9, gamma), ref, rtol=1e-11, atol=1e-11)


def test_jr_is_gs2_with_zero_inner_bitwise():
    A = MATS["rand_nonsym"]()
    rng = np.random.default_rng(9)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    for sw, w in [(1, 1.0), (3, 0.7)]:
        a = oracle.jr_sweep(A, b, x0, sw, w)
        g = oracle.gs2_sweep(A, b, x0, F, sw, 0, w)
        assert np.array_equal(a, g)
    # JR from zero is w D^{-1} b
    d = np.diag(A.dense())
    np.testing.assert_allclose(oracle.jr_sweep(A, b, np.zeros(A.n), 1, 0.6), 0.6 * b / d, rtol=1e-15)


# ----------------------------------------------- nilpotency of D^{-1}L (Section 4)

@pytest.mark.parametrize("mk,depth", [(lambda: laplace1d(8), 7), (lambda: poisson2d(4), 6),
                                       (lambda: laplace3d(3), 6), (lambda: poisson2d(6), 10)])
def test_levels_and_nilpotency(mk, depth):
    """In natural order the longest path of L's DAG is n-1 (1D), 2(N-1) (2D)
    and 3(N-1) (3D).  With s >= that depth the Neumann series is exact and GS2
    equals exact GS; with s = depth - 1 it does not."""
    A = mk()
    lv, nlev = oracle.levels(A, lower=True)
    assert nlev - 1 == depth
    lvu, nlevu = oracle.levels(A, lower=False)
    assert nlevu - 1 == depth
    L, D, U, M = parts(A)
    exact = np.linalg.inv(D + L)
    P_exact = operator(lambda v: oracle.gs2_apply(A, v, F, 1, depth), A.n)
    np.testing.assert_allclose(P_exact, exact, rtol=0, atol=1e-14 * np.abs(exact).max())
    P_short = operator(lambda v: oracle.gs2_apply(A, v, F, 1, depth - 1), A.n)
    assert np.abs(P_short - exact).max() > 1e-6
    # the whole GS2 sweep from any x0 equals the exact GS sweep
    rng = np.random.default_rng(1)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    np.testing.assert_allclose(oracle.gs2_sweep(A, b, x0, S, 2, depth), oracle.sor_sweep(A, b, x0, S, 2, 1.0),
                               rtol=1e-12, atol=1e-12)


def test_nilpotency_lattice_path_count():
    """2D N=4: the only term GS2(5) lacks is (-D^{-1}L)^6 D^{-1}, whose largest
    entry counts the 20 monotone lattice paths from corner to corner, times
    4^-7 (every step and the final D^{-1} divide by 4)."""
    A = poisson2d(4)
    L, D, U, M = parts(A)
    diff = np.abs(operator(lambda v: oracle.gs2_apply(A, v, F, 1, 5), A.n) - np.linalg.inv(D + L)).max()
    assert diff == pytest.approx(20 * 4.0 ** -7, rel=1e-12)


def test_levels_brute_force():
    A = random_sparse(25, seed=4, avg_offdiag=3)
    M = A.dense() != 0
    n = A.n

    def longest(i, lower):
        nb = [j for j in range(n) if M[i, j] and ((j < i) if lower else (j > i))]
        return 0 if not nb else 1 + max(longest(j, lower) for j in nb)

    for lower in (True, False):
        lv, nlev = oracle.levels(A, lower)
        ref = [longest(i, lower) for i in range(n)]
        assert list(lv) == ref and nlev == max(ref) + 1


# ----------------------------------------- residual recurrences (Section 5)

def stand_alone_residuals(A, b, x0, k, fn):
    x = x0.copy()
    out = []
    for _ in range(k):
        x = fn(x)
        out.append(b - A.dense() @ x)
    return out


def test_residual_recurrence_gs2_and_sgs2_and_jr():
    """r_{k+1} = (I - A D^-1 [I - L D^-1]) r_k for GS2 with one inner sweep,
    the product of the forward and backward factors for SGS2(1), and
    (I - A D^-1)^2 = I - A D^-1 [I - (L+U) D^-1] for two JR sweeps."""
    A = poisson2d(5)
    L, D, U, M = parts(A)
    n = A.n
    I = np.eye(n)
    Di = np.diag(1.0 / np.diag(D))
    rng = np.random.default_rng(2)
    b, x0 = rng.standard_normal(n), rng.standard_normal(n)
    r0 = b - M @ x0
    Rg = I - M @ Di @ (I - L @ Di)
    Ru = I - M @ Di @ (I - U @ Di)
    for k, r in enumerate(stand_alone_residuals(A, b, x0, 3, lambda x: oracle.gs2_sweep(A, b, x, F, 1, 1)), 1):
        np.testing.assert_allclose(r, np.linalg.matrix_power(Rg, k) @ r0, rtol=1e-10, atol=1e-10)
    for k, r in enumerate(stand_alone_residuals(A, b, x0, 2, lambda x: oracle.gs2_sweep(A, b, x, S, 1, 1)), 1):
        np.testing.assert_allclose(r, np.linalg.matrix_power(Ru @ Rg, k) @ r0, rtol=1e-10, atol=1e-10)
    J2 = I - M @ Di @ (I - (L + U) @ Di)
    np.testing.assert_allclose(J2, np.linalg.matrix_power(I - M @ Di, 2), atol=1e-13)
    for k, r in enumerate(stand_alone_residuals(A, b, x0, 2, lambda x: oracle.jr_sweep(A, b, x, 2, 1.0)), 1):
        np.testing.assert_allclose(r, np.linalg.matrix_power(J2, k) @ r0, rtol=1e-10, atol=1e-10)
    r3 = stand_alone_residuals(A, b, x0, 1, lambda x: oracle.jr_sweep(A, b, x, 3, 1.0))[0]
    np.testing.assert_allclose(r3, np.linalg.matrix_power(I - M @ Di, 3) @ r0, rtol=1e-10, atol=1e-10)


# ------------------------------------------------------ closed-form spectra

def iteration_matrix(A, fn):
    """Error propagation of a stationary iteration: apply it with b = 0."""
    z = np.zeros(A.n)
    return operator(lambda e: fn(z, e), A.n)


@pytest.mark.parametrize("N", [4, 8])
def test_jacobi_and_gs_spectral_radius_2d(N):
    A = poisson2d(N)
    c = np.cos(np.pi / (N + 1))
    GJ = iteration_matrix(A, lambda b, e: oracle.jr_sweep(A, b, e, 1, 1.0))
    assert rho(GJ) == pytest.approx(c, abs=1e-10)
    GGS = iteration_matrix(A, lambda b, e: oracle.sor_sweep(A, b, e, F, 1, 1.0))
    assert rho(GGS) == pytest.approx(c * c, abs=1e-7)  # consistently ordered: rho_GS = rho_J^2


@pytest.mark.parametrize("w", [0.5, 0.8, 1.0])
def test_damped_jacobi_spectrum_1d_3d(w):
    for A, mus in [(laplace1d(9), [np.cos(k * np.pi / 10) for k in range(1, 10)]),
                   (laplace3d(3), [(np.cos(i * np.pi / 4) + np.cos(j * np.pi / 4) + np.cos(k * np.pi / 4)) / 3
                                   for i in range(1, 4) for j in range(1, 4) for k in range(1, 4)])]:
        G = iteration_matrix(A, lambda b, e: oracle.jr_sweep(A, b, e, 1, w))
        ref = max(abs(1 - w * (1 - m)) for m in mus)
        assert rho(G) == pytest.approx(ref, abs=1e-10)


def test_gs2_spectra_szyld_bound_and_limit():
    """Two-stage theory for regular splittings (Section 5): the s-inner-sweep
    method satisfies rho(T_{s+1}) >= rho(T_1)^{s+1} with T_1 = Jacobi; the radius
    decreases with s and reaches rho_GS once s >= the DAG depth (6 for 2D N=4).
    N = 4 values: 0.809 (s=0) > 0.7248 (s=1) > ... > 0.6545 = cos^2(pi/5)."""
    A = poisson2d(4)
    rj = np.cos(np.pi / 5)
    radii = []
    for s in range(0, 8):
        G = iteration_matrix(A, lambda b, e, s=s: oracle.gs2_sweep(A, b, e, F, 1, s, 1.0))
        radii.append(rho(G))
        assert radii[-1] >= rj ** (s + 1) - 1e-12
    assert radii[0] == pytest.approx(rj, abs=1e-12)
    assert radii[1] == pytest.approx(0.7248, abs=5e-5)
    assert all(a >= b - 1e-9 for a, b in zip(radii, radii[1:]))
    assert radii[6] == pytest.approx(rj ** 2, abs=1e-6) and radii[7] == pytest.approx(rj ** 2, abs=1e-6)


# ----------------------------------------------------------- compact form

def test_compact_equals_noncompact_only_for_exact_inner():
    """Eq. (one-stage) and eq. (one-stage-2) agree for the exact M; with an
    approximate inverse (few inner sweeps) eq. (two-stage-3) differs from
    eq. (two-stage) (Section 4, compact form)."""
    A = poisson2d(4)
    rng = np.random.default_rng(8)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    for w in (1.0, 0.8):
        exact_c = oracle.gs2c_sweep(A, b, x0, S, 2, 6, w)
        exact_n = oracle.gs2_sweep(A, b, x0, S, 2, 6, w)
        np.testing.assert_allclose(exact_c, exact_n, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(exact_c, oracle.sor_sweep(A, b, x0, S, 2, w), rtol=1e-12, atol=1e-12)
        assert np.abs(oracle.gs2c_sweep(A, b, x0, F, 1, 1, w) - oracle.gs2_sweep(A, b, x0, F, 1, 1, w)).max() > 1e-4


def test_compact_closed_form():
    """x1 = w Mhat (b - [U + (1 - 1/w) D] x0), Mhat the Neumann sum of degree s."""
    A = MATS["rand_nonsym"]()
    L, D, U, M = parts(A)
    rng = np.random.default_rng(12)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    w, s = 0.8, 2
    Di = np.diag(1 / np.diag(D))
    K = -w * Di @ L
    Mhat = sum(np.linalg.matrix_power(K, k) for k in range(s + 1)) @ Di
    ref = w * Mhat @ (b - (U + (1 - 1 / w) * D) @ x0)
    np.testing.assert_allclose(oracle.gs2c_sweep(A, b, x0, F, 1, s, w), ref, rtol=1e-11, atol=1e-11)


# ------------------------------------------------------- inner diagnostic

def test_inner_residual_diagnostic():
    A = poisson2d(4)
    L, D, U, M = parts(A)
    r = np.random.default_rng(4).standard_normal(A.n)
    out = oracle.inner_residuals(A, r, 7)
    # j = 0: r - D D^{-1} r - L D^{-1} r = -L D^{-1} r
    assert out[0] == pytest.approx(np.linalg.norm(L @ (r / np.diag(D))) / np.linalg.norm(r), rel=1e-12)
    assert out[6] < 1e-14 and out[7] < 1e-14
    assert all(out[j] > 1e-8 for j in range(6))


@pytest.mark.parametrize("name", ["rand_nonsym", "rand_negdiag", "vardiff3d_3"])
@pytest.mark.parametrize("w", [0.8, 1.3])
def test_inner_residual_diagnostic_damped(name, w):
    """The diagnostic for a damping w != 1 (Section 8, inner convergence):
    g_j is the dense Neumann partial sum sum_{k<=j} (-w D^{-1} L)^k D^{-1} r
    (Section 4), and the reported value is ||r - (wL + D) g_j|| / ||r||."""
    A = MATS[name]()
    L, D, U, M = parts(A)
    r = np.random.default_rng(11).standard_normal(A.n)
    J = 6
    out = oracle.inner_residuals(A, r, J, omega=w)
    Di = np.diag(1 / np.diag(D))
    K = -w * Di @ L
    g = np.zeros(A.n)
    term = Di @ r
    for j in range(J + 1):
        g = g + term
        ref = np.linalg.norm(r - (w * L + D) @ g) / np.linalg.norm(r)
        assert out[j] == pytest.approx(ref, rel=1e-10, abs=1e-15), (j, out[j], ref)
        term = K @ term
