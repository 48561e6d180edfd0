"""GMRES restart cycles replayed from a captured HIP graph must give exactly
what the same kernels give when launched one by one: several replays, with
unrelated GPU work and synchronisations in between, each compared bitwise
with the eager result.  Profiling on inside the graph must not change the
result (profiling launches the kernels one by one)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2104_01196_amd as g  # noqa: E402
from gen import config_problem  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"
M = 8  # restart length: short, so that every solve restarts several times


def _eager(dA, db, n, kind, h):
    prev = g.gs2_graphs(False)
    try:
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        info = g.gmres_solve(dA, db, x, M, 1e-8, 5000, kind, h)
    finally:
        g.gs2_graphs(prev)
    return x, info


@pytest.mark.parametrize("orth,kind,variant", [(0, g.PREC_GS2, g.FORWARD), (1, g.PREC_GS2, g.SYMMETRIC),
                                               (0, g.PREC_JR, g.FORWARD)])
def test_graph_replays_equal_eager(orth, kind, variant):
    p = config_problem(2, size=20)
    A, b = p["A"], p["b"]
    dA = g.DeviceCSR.from_host(A)
    db = torch.as_tensor(b, device=DEV)
    h = g.gs2_setup(dA, 2, 1, 1.0, variant, orthogonalization=orth)
    x_ref, info_ref = _eager(dA, db, A.n, kind, h)
    assert info_ref["converged"] and info_ref["restarts"] >= 1
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    for rep in range(3):
        junk = torch.randn(1 << 20, device=DEV, dtype=torch.float64)
        _ = float((junk * junk).sum())  # unrelated eager work + synchronisation
        x.zero_()
        info = g.gmres_solve(dA, db, x, M, 1e-8, 5000, kind, h)
        torch.cuda.synchronize()
        assert info["iterations"] == info_ref["iterations"] and info["restarts"] == info_ref["restarts"]
        assert torch.equal(x, x_ref), f"replay {rep} differs"
    # a different output buffer invalidates the captured graph (pointers are baked in)
    x2 = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    info2 = g.gmres_solve(dA, db, x2, M, 1e-8, 5000, kind, h)
    assert info2["iterations"] == info_ref["iterations"] and torch.equal(x2, x_ref)
    assert np.linalg.norm(b - A.to_scipy() @ x2.cpu().numpy()) / np.linalg.norm(b) <= 1e-8


def test_profiling_launches_eagerly_with_equal_results():
    """Per-kernel event profiling runs the cycle kernel by kernel (graph
    replay off) and gives the same bits as the replayed solve; every executed
    Arnoldi step is counted once, skipped ones not at all."""
    p = config_problem(2, size=20)
    A, b = p["A"], p["b"]
    dA = g.DeviceCSR.from_host(A)
    db = torch.as_tensor(b, device=DEV)
    h = g.gs2_setup(dA, 2, 1, 1.0, g.FORWARD)
    x_ref = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    info_ref = g.gmres_solve(dA, db, x_ref, M, 1e-8, 5000, g.PREC_GS2, h)  # graph replay
    g.gs2_profile(True)
    try:
        x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
        info = g.gmres_solve(dA, db, x, M, 1e-8, 5000, g.PREC_GS2, h)
    finally:
        g.gs2_profile(False)
    prof = g.gs2_profile_read()
    assert info["iterations"] == info_ref["iterations"] and torch.equal(x, x_ref)
    assert prof["spmv_dot"]["launches"] == info["iterations"]
    assert prof["true_resid"]["launches"] == info["restarts"] + 2
    assert all(v["ms"] > 0 for v in prof.values()), prof
