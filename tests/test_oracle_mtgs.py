"""Pins of the oracle's multicolor Gauss-Seidel (Section 6, multi-threaded
Gauss-Seidel): a valid coloring, equivalence with sequential GS on the
color-permuted matrix, and the red-black spectrum of the 2D Laplacian."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from gen import CSR, poisson2d, laplace3d, random_sparse, vardiff3d, elasticity_q1


def permuted(A, perm):
    S = A.to_scipy()[perm][:, perm].tocsr()
    S.sort_indices()
    return CSR(A.n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))


MATS = [lambda: poisson2d(6), lambda: laplace3d(4), lambda: vardiff3d(4, seed=1), lambda: elasticity_q1(3, 3, 3),
        lambda: random_sparse(60, seed=9, avg_offdiag=4)]


@pytest.mark.parametrize("mk", MATS)
def test_coloring_valid_and_greedy(mk):
    A = mk()
    c, ncol = oracle.colors(A)
    S = A.to_scipy()
    P = ((S + S.T) != 0).tocoo()
    off = P.row != P.col
    assert not np.any(c[P.row[off]] == c[P.col[off]])
    deg = np.diff(((S + S.T) != 0).tocsr().indptr) - 1
    assert ncol == c.max() + 1 and ncol <= deg.max() + 1
    # first fit: every row's color is the smallest absent among earlier neighbours
    Pc = ((S + S.T) != 0).tocsr()
    for i in range(A.n):
        nb = Pc.indices[Pc.indptr[i]:Pc.indptr[i + 1]]
        used = set(c[nb[nb < i]])
        assert c[i] == min(set(range(ncol + 1)) - used)


def test_natural_order_stencils_two_colors():
    assert oracle.colors(poisson2d(8))[1] == 2 and oracle.colors(laplace3d(5))[1] == 2


@pytest.mark.parametrize("mk", MATS)
@pytest.mark.parametrize("variant,sweeps,w", [(oracle.FORWARD, 1, 1.0), (oracle.BACKWARD, 2, 0.8),
                                              (oracle.SYMMETRIC, 1, 1.1)])
def test_mtgs_is_gs_on_color_ordering(mk, variant, sweeps, w):
    """Sweeping colors in turn is sequential GS/SOR on the matrix whose rows
    and columns are sorted by color (stable within a color)."""
    A = mk()
    c, _ = oracle.colors(A)
    perm = np.argsort(c, kind="stable")
    rng = np.random.default_rng(3)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    x = oracle.mtgs_sweep(A, b, x0, variant, sweeps, w)
    Ap = permuted(A, perm)
    xp = oracle.sor_sweep(Ap, b[perm], x0[perm], variant, sweeps, w)
    np.testing.assert_allclose(x[perm], xp, rtol=1e-13, atol=1e-13)


def test_red_black_spectral_radius():
    """Red-black ordering of the 5-point Laplacian is consistently ordered, so
    rho(GS) = rho_J^2 = cos^2(pi/(N+1)) as in natural order."""
    N = 7
    A = poisson2d(N)
    z = np.zeros(A.n)
    G = np.column_stack([oracle.mtgs_sweep(A, z, e, oracle.FORWARD, 1, 1.0) for e in np.eye(A.n)])
    assert np.max(np.abs(np.linalg.eigvals(G))) == pytest.approx(np.cos(np.pi / (N + 1)) ** 2, abs=1e-8)


def test_mtgs_preconditioned_solvers():
    A = vardiff3d(8, seed=6)
    b = np.random.default_rng(1).standard_normal(A.n)
    _, ig = oracle.gmres(A, b, restart=30, prec="mtgs", variant=oracle.SYMMETRIC)
    _, ic = oracle.pcg(A, b, prec="mtgs", variant=oracle.SYMMETRIC)
    _, i0 = oracle.pcg(A, b, prec="none")
    assert ig["converged"] and ic["converged"] and ic["iterations"] < i0["iterations"]
