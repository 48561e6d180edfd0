"""GMRES restart cycles replayed from a captured HIP graph must give exactly
what the same kernels give when launched one by one: several replays, with
unrelated GPU work and synchronisations in between, each compared bitwise
with the eager result.  Profiling on inside the graph must not change the
result and must report every executed kernel."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2104_01196_amd as g  # noqa: E402
from gen import config_problem  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _eager(dA, db, n, kind, h):
    prev = g.gs2_graphs(False)
    try:
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        info = g.gmres_solve(dA, db, x, 30, 1e-8, 5000, kind, h)
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
        info = g.gmres_solve(dA, db, x, 30, 1e-8, 5000, kind, h)
        torch.cuda.synchronize()
        assert info["iterations"] == info_ref["iterations"] and info["restarts"] == info_ref["restarts"]
        assert torch.equal(x, x_ref), f"replay {rep} differs"
    # a different output buffer invalidates the captured graph (pointers are baked in)
    x2 = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    info2 = g.gmres_solve(dA, db, x2, 30, 1e-8, 5000, kind, h)
    assert info2["iterations"] == info_ref["iterations"] and torch.equal(x2, x_ref)
    assert np.linalg.norm(b - A.to_scipy() @ x2.cpu().numpy()) / np.linalg.norm(b) <= 1e-8


def test_profiled_graph_counts_executed_launches():
    p = config_problem(2, size=20)
    A, b = p["A"], p["b"]
    dA = g.DeviceCSR.from_host(A)
    db = torch.as_tensor(b, device=DEV)
    h = g.gs2_setup(dA, 2, 1, 1.0, g.FORWARD)
    x_ref, info_ref = _eager(dA, db, A.n, g.PREC_GS2, h)
    counts = []
    for graphs in (False, True, True):  # eager, graph capture + replay, replay of the same graph
        prev = g.gs2_graphs(graphs)
        try:
            g.gs2_profile(True)
            x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
            info = g.gmres_solve(dA, db, x, 30, 1e-8, 5000, g.PREC_GS2, h)
            g.gs2_profile(False)
            prof = g.gs2_profile_read()
        finally:
            g.gs2_graphs(prev)
        assert info["iterations"] == info_ref["iterations"] and torch.equal(x, x_ref)
        counts.append({k: v["launches"] for k, v in prof.items()})
        its = info["iterations"]
        # one SpMV per executed Arnoldi step
        assert prof["spmv_dot"]["launches"] == its
        assert sum(prof.get(k, {}).get("launches", 0) for k in ("gs2_inner", "gs2_first_jr")) > 0
        assert all(v["ms"] > 0 for v in prof.values() if v["launches"] > 0)
    assert counts[0] == counts[1] == counts[2]
