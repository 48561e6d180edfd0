"""GPU parity of the multicolor Gauss-Seidel comparison path (mtgs_apply and
as a GMRES / CG preconditioner) against the oracle.  Same coloring
definition on both sides; FP64 bar 1e-11 relative (rounding order only)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2104_01196_amd as g  # noqa: E402
from gen import poisson2d, laplace3d, vardiff3d, elasticity_q1, random_sparse, convdiff2d, config_problem  # noqa

pytestmark = pytest.mark.gpu
DEV = "cuda"

MATS = {
    "poisson2d_40": lambda: poisson2d(40),
    "laplace3d_12": lambda: laplace3d(12),
    "vardiff3d_9": lambda: vardiff3d(9, seed=2),
    "elasticity_4": lambda: elasticity_q1(4, 4, 4, seed=3),
    "random_nonsym": lambda: random_sparse(500, seed=14, avg_offdiag=5, long_rows=3, long_len=90),
    "convdiff_30": lambda: convdiff2d(30, 20.0, 2.0),
}


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("variant,sweeps,w", [(g.FORWARD, 1, 1.0), (g.BACKWARD, 2, 0.9), (g.SYMMETRIC, 1, 1.2)])
def test_mtgs_apply(name, variant, sweeps, w):
    A = MATS[name]()
    dA = g.DeviceCSR.from_host(A)
    v = np.random.default_rng(5).standard_normal(A.n)
    ref = oracle.mtgs_sweep(A, v, np.zeros(A.n), variant, sweeps, w)
    h = g.gs2_setup(dA, sweeps, 1, 1.0, g.FORWARD, build_levels=True)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    g.mtgs_apply(h, variant, w, torch.as_tensor(v, device=DEV), z)
    torch.cuda.synchronize()
    zh = z.cpu().numpy()
    assert np.abs(zh - ref).max() <= 1e-11 * np.abs(ref).max()


def test_mtgs_needs_colors():
    A = poisson2d(10)
    h = g.gs2_setup(g.DeviceCSR.from_host(A), 1, 1, 1.0, g.FORWARD)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    with pytest.raises(g.Gs2Error) as e:
        g.mtgs_apply(h, g.FORWARD, 1.0, torch.ones(A.n, dtype=torch.float64, device=DEV), z)
    assert e.value.status == -8


@pytest.mark.parametrize("solver", ["gmres", "cg"])
def test_mtgs_preconditioned_solve(solver):
    p = config_problem(4, size=12)
    A, b = p["A"], p["b"]
    dA = g.DeviceCSR.from_host(A)
    h = g.gs2_setup(dA, 1, 1, 1.0, g.SYMMETRIC, build_levels=True)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    if solver == "gmres":
        _, io = oracle.gmres(A, b, restart=30, prec="mtgs", variant=oracle.SYMMETRIC)
        info = g.gmres_solve(dA, torch.as_tensor(b, device=DEV), x, 30, 1e-8, 5000, g.PREC_MTGS, h)
    else:
        _, io = oracle.pcg(A, b, prec="mtgs", variant=oracle.SYMMETRIC)
        info = g.cg_solve(dA, torch.as_tensor(b, device=DEV), x, 1e-8, 5000, g.PREC_MTGS, h)
    assert info["converged"] and abs(info["iterations"] - io["iterations"]) <= 1, (info, io)
    xh = x.cpu().numpy()
    assert np.linalg.norm(b - A.to_scipy() @ xh) / np.linalg.norm(b) <= 1e-8
