"""Generator checks: exact sizes, structure and the physics each stand-in
must carry (symmetry, definiteness, M-matrix signs, rigid-body modes)."""
import numpy as np
import pytest

from gen import (poisson2d, laplace3d, vardiff3d, elasticity_q1, convdiff2d, convdiff_batch, random_sparse,
                 config_problem)
from gen.problems import _q1_reference


def test_sizes():
    assert (poisson2d(64).n, poisson2d(64).nnz) == (4096, 20224)
    A = laplace3d(16)
    assert (A.n, A.nnz) == (16 ** 3, 7 * 16 ** 3 - 6 * 16 ** 2)
    A = vardiff3d(8, seed=1)
    assert (A.n, A.nnz) == (512, 7 * 512 - 6 * 64)
    A = elasticity_q1(5, 5, 5)
    assert (A.n, A.nnz) == (375, (3 * 5 - 2) ** 3 * 9)
    A = convdiff2d(20, 10.0, 1.0)
    assert (A.n, A.nnz) == (400, 5 * 400 - 4 * 20)
    for A in (poisson2d(7), laplace3d(5), vardiff3d(5), elasticity_q1(3, 4, 3), convdiff2d(9, 3.0, 4.0),
              random_sparse(50, seed=3, long_rows=2, long_len=70, diag_only_rows=2)):
        A.check()


def test_full_size_counts_formula():
    """Full-size configurations (counts from closed forms, no assembly)."""
    N = 128
    assert 7 * N ** 3 - 6 * N ** 2 == 14581760
    N = 192
    assert (N ** 3, 7 * N ** 3 - 6 * N ** 2) == (7077888, 49324032)
    assert 190 ** 3 * 9 == 61731000  # 64^3 free Q1 nodes x 3 dof


def test_laplacians_symmetric_zero_interior_rowsum():
    for A in (poisson2d(6), laplace3d(5)):
        M = A.dense()
        assert np.array_equal(M, M.T)
        rs = M.sum(1)
        assert np.all(rs >= 0) and np.sum(rs == 0) > 0
        assert np.linalg.eigvalsh(M).min() > 0


def test_vardiff_spd_m_matrix():
    M = vardiff3d(5, seed=4).dense()
    assert np.allclose(M, M.T, rtol=0, atol=0)
    off = M - np.diag(np.diag(M))
    assert np.all(off <= 0)
    rs = np.diag(M) + off.sum(1)
    assert np.all(rs >= -1e-12 * np.diag(M)) and np.any(rs > 1e-3)  # weakly dominant, strictly at the boundary
    np.linalg.cholesky(M)


def test_convdiff_m_matrix_and_upwinding():
    A = convdiff2d(8, 30.0, 2.5)
    M = A.dense()
    off = M - np.diag(np.diag(M))
    assert np.all(off <= 0)
    assert np.all(np.diag(M) + off.sum(1) >= -1e-12)
    h = 1 / 9
    wx, wy = 30 * np.cos(2.5), 30 * np.sin(2.5)  # wx < 0: x+ neighbour is upwind
    i = 4 * 8 + 4
    assert M[i, i + 1] == pytest.approx(-1 - h * abs(wx)) and M[i, i - 1] == -1.0
    assert M[i, i - 8] == pytest.approx(-1 - h * abs(wy)) and M[i, i + 8] == -1.0  # wy > 0: y- upwind


def test_q1_element_rigid_body_modes():
    """The element stiffness annihilates the 6 rigid-body modes and is PSD of
    rank 18."""
    Kl, Km = _q1_reference(0.5)
    K = 3.0 * Kl + 2.0 * Km
    pts = np.array([[(a & 1), (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], float) * 0.5
    modes = []
    for c in range(3):
        m = np.zeros((8, 3)); m[:, c] = 1; modes.append(m.ravel())
    for (i, j) in [(0, 1), (1, 2), (0, 2)]:
        m = np.zeros((8, 3)); m[:, i] = -pts[:, j]; m[:, j] = pts[:, i]; modes.append(m.ravel())
    for m in modes:
        assert np.abs(K @ m).max() < 1e-12 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev > 1e-10 * ev.max()) == 18 and ev.min() > -1e-12 * ev.max()


def test_elasticity_spd_after_dirichlet():
    A = elasticity_q1(4, 4, 4, seed=2)
    M = A.dense()
    assert np.allclose(M, M.T, rtol=1e-12, atol=1e-12 * np.abs(M).max())
    np.linalg.cholesky(M)


def test_batch_shapes_deterministic():
    m1, r1 = convdiff_batch(6, seed=5)
    m2, r2 = convdiff_batch(6, seed=5)
    assert [a.n for a in m1] == [a.n for a in m2]
    assert all(np.array_equal(a, b) for a, b in zip(r1, r2))
    assert all(16 <= int(np.sqrt(a.n)) <= 256 and r.shape == (a.n, 4) for a, r in zip(m1, r1))


def test_config_rhs_consistent():
    p = config_problem(1)
    np.testing.assert_allclose(p["A"].to_scipy() @ p["x_true"], p["b"])
    assert np.abs(p["x_true"]).max() <= 1.0
