"""Pins of the oracle's hybrid (block-Jacobi) GS2 sweeps (Section 3: local
relaxation on each process's diagonal block with a frozen halo)."""
import numpy as np
import pytest

import oracle
from gen import poisson2d, vardiff3d, random_sparse

F, B, S = oracle.FORWARD, oracle.BACKWARD, oracle.SYMMETRIC


def split(A, blocks):
    M = A.dense()
    n = A.n
    bs = -(-n // blocks)
    blk = np.arange(n) // bs
    same = blk[:, None] == blk[None, :]
    Aloc = np.where(same, M, 0.0)
    return M, Aloc, M - Aloc


@pytest.mark.parametrize("variant,sweeps,inner,nk", [(F, 1, 1, 1), (S, 2, 2, 1), (B, 1, 0, 3), (S, 2, 1, 2)])
def test_one_block_is_plain_gs2_bitwise(variant, sweeps, inner, nk):
    A = random_sparse(80, seed=3, avg_offdiag=5)
    rng = np.random.default_rng(0)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    x = oracle.gs2_block_sweep(A, b, x0, 1, variant, sweeps, nk, inner, 0.9)
    ref = oracle.gs2_sweep(A, b, x0, variant, sweeps * nk, inner, 0.9)
    assert np.array_equal(x, ref)


def test_row_blocks_reduce_to_jacobi_bitwise():
    A = poisson2d(6)
    rng = np.random.default_rng(1)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    x = oracle.gs2_block_sweep(A, b, x0, A.n, F, 3, 1, 2, 0.8)
    assert np.array_equal(x, oracle.jr_sweep(A, b, x0, 3, 0.8))


@pytest.mark.parametrize("blocks", [2, 3, 5])
@pytest.mark.parametrize("nk", [1, 2])
def test_block_sweep_closed_form(blocks, nk):
    """Each local half is x += w N_s(T_loc) (b - E y - A_loc x) with the
    degree-s Neumann sum of the block's own triangle and y frozen at the
    start of the global sweep."""
    A = vardiff3d(4, seed=5)
    M, Aloc, E = split(A, blocks)
    D = np.diag(np.diag(M))
    Di = np.diag(1 / np.diag(M))
    Lloc, Uloc = np.tril(Aloc, -1), np.triu(Aloc, 1)
    rng = np.random.default_rng(2)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    w, s = 0.9, 2

    def N(T):
        return sum(np.linalg.matrix_power(-w * Di @ T, k) for k in range(s + 1)) @ Di

    x, y = x0.copy(), x0.copy()
    for _ in range(nk):
        x = x + w * N(Lloc) @ (b - E @ y - Aloc @ x)
        x = x + w * N(Uloc) @ (b - E @ y - Aloc @ x)
    got = oracle.gs2_block_sweep(A, b, x0, blocks, S, 1, nk, s, w)
    np.testing.assert_allclose(got, x, rtol=1e-11, atol=1e-11)
    _ = D


def test_exact_local_solves_give_block_jacobi():
    """With exact inner solves and many local sweeps, one global sweep solves
    every block system: x1 = A_loc^{-1} (b - E x0) (block Jacobi)."""
    A = vardiff3d(3, seed=7)
    M, Aloc, E = split(A, 3)
    rng = np.random.default_rng(3)
    b, x0 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    got = oracle.gs2_block_sweep(A, b, x0, 3, S, 1, 200, A.n, 1.0)
    np.testing.assert_allclose(got, np.linalg.solve(Aloc, b - E @ x0), rtol=1e-10, atol=1e-10)
