"""GPU parity of the hybrid (block-Jacobi) relaxation emulated on one GPU:
P contiguous row blocks, local triangles in the inner sweeps, off-block
couplings on values frozen once per global sweep (Section 3).  FP64 bar:
1e-12 per half sweep (relative, infinity norm)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2104_01196_amd as g  # noqa: E402
from gen import laplace3d, poisson2d, random_sparse, vardiff3d, config_problem  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"

MATS = {
    "laplace3d_16": lambda: laplace3d(16),
    "poisson2d_50": lambda: poisson2d(50),
    "vardiff3d_10": lambda: vardiff3d(10, seed=4),
    "random_nonsym": lambda: random_sparse(900, seed=21, avg_offdiag=6, long_rows=4, long_len=100),
}


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("blocks,variant,sweeps,nk,inner,w", [
    (4, g.FORWARD, 1, 1, 1, 1.0), (8, g.SYMMETRIC, 2, 1, 2, 0.9), (3, g.FORWARD, 1, 4, 1, 1.0),
    (5, g.SYMMETRIC, 2, 2, 1, 0.8), (7, g.BACKWARD, 2, 3, 0, 1.0)])
def test_hybrid_gs2_apply(name, blocks, variant, sweeps, nk, inner, w):
    A = MATS[name]()
    dA = g.DeviceCSR.from_host(A)
    v = np.random.default_rng(3).standard_normal(A.n)
    ref = oracle.gs2_block_sweep(A, v, np.zeros(A.n), blocks, variant, sweeps, nk, inner, w)
    h = g.gs2_setup(dA, sweeps, inner, w, variant, blocks=blocks, local_sweeps=nk)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    g.gs2_apply(h, torch.as_tensor(v, device=DEV), z)
    torch.cuda.synchronize()
    halves = sweeps * nk * (2 if variant == g.SYMMETRIC else 1)
    zh = z.cpu().numpy()
    assert np.abs(zh - ref).max() <= 1e-12 * halves * np.abs(ref).max()


@pytest.mark.parametrize("blocks,sweeps,nk", [(4, 4, 1), (4, 1, 4), (6, 2, 2)])
def test_hybrid_jr_global_vs_local(blocks, sweeps, nk):
    """JR(n_t, n_k): global sweeps with n_k local sweeps each (the paper's
    JR(4,1) vs JR(1,4) comparison)."""
    A = MATS["laplace3d_16"]()
    dA = g.DeviceCSR.from_host(A)
    v = np.random.default_rng(4).standard_normal(A.n)
    ref = oracle.gs2_block_sweep(A, v, np.zeros(A.n), blocks, g.FORWARD, sweeps, nk, 0, 0.9)
    h = g.gs2_setup(dA, 1, 1, 1.0, g.FORWARD, blocks=blocks, local_sweeps=nk)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    g.jr_apply(h, sweeps, 0.9, torch.as_tensor(v, device=DEV), z)
    torch.cuda.synchronize()
    assert np.abs(z.cpu().numpy() - ref).max() <= 1e-12 * sweeps * nk * np.abs(ref).max()


@pytest.mark.parametrize("blocks,nk,kind", [(1, 1, g.PREC_GS2), (8, 1, g.PREC_GS2), (8, 3, g.PREC_GS2),
                                             (16, 2, g.PREC_JR)])
def test_hybrid_preconditioned_gmres(blocks, nk, kind):
    """GMRES with the hybrid preconditioner matches the oracle's iteration
    count (the same block sweep inside the oracle's GMRES)."""
    p = config_problem(2, size=20)
    A, b = p["A"], p["b"]
    dA = g.DeviceCSR.from_host(A)
    prec = "gs2" if kind == g.PREC_GS2 else "jr"
    _, io = oracle.gmres(A, b, restart=50, rtol=1e-8, prec=prec, sweeps=2, inner=1, blocks=blocks,
                         local_sweeps=nk)
    h = g.gs2_setup(dA, 2, 1, 1.0, g.FORWARD, blocks=blocks, local_sweeps=nk)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    info = g.gmres_solve(dA, torch.as_tensor(b, device=DEV), x, 50, 1e-8, 5000, kind, h)
    assert info["converged"] and abs(info["iterations"] - io["iterations"]) <= 1, (info, io)
    xh = x.cpu().numpy()
    assert np.linalg.norm(b - A.to_scipy() @ xh) / np.linalg.norm(b) <= 1e-8
