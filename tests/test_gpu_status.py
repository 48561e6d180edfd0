"""Solve-status paths of gmres_solve on the GPU: stagnation (GS2_STAGNATED).

Restarted GMRES(1) makes no progress at all on a skew-symmetric matrix:
(r, A r) = 0 for every r, so the one-step minimal residual correction is
zero and the residual never changes.  The solve must stop with
GS2_STAGNATED once the true residual has not halved for the stagnation
window (50 restart cycles by default, or the handle's stagnation_cycles),
instead of running to maxit; a window < 0 turns the test off."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2104_01196_amd as g  # noqa: E402
from gen import CSR  # noqa: E402

pytestmark = pytest.mark.gpu


def skew_tridiag(n):
    rows, cols, vals = [], [], []
    for i in range(n):
        if i > 0:
            rows.append(i), cols.append(i - 1), vals.append(-1.0)
        if i + 1 < n:
            rows.append(i), cols.append(i + 1), vals.append(1.0)
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, np.array(rows) + 1, 1)
    return CSR(n, np.cumsum(rp).astype(np.int32), np.array(cols, np.int32), np.array(vals))


def identity(n):
    return CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))


def test_gmres_stagnation_status():
    n = 200
    A = skew_tridiag(n)
    dA = g.DeviceCSR.from_host(A)
    b = torch.as_tensor(np.random.default_rng(3).standard_normal(n), device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    info = g.gmres_solve(dA, b, x, 1, 1e-8, 10000, g.PREC_NONE, None)
    assert info["status"] == g.STAGNATED and not info["converged"]
    assert info["iterations"] == 50 and info["restarts"] == 49
    assert info["relres"] == pytest.approx(1.0, rel=1e-12)
    # the window comes from the handle passed along (a handle of any matrix of the same size)
    dI = g.DeviceCSR.from_host(identity(n))
    h = g.gs2_setup(dI, 1, 1, 1.0, g.FORWARD, stagnation_cycles=10)
    x.zero_()
    info = g.gmres_solve(dA, b, x, 1, 1e-8, 10000, g.PREC_NONE, h)
    assert info["status"] == g.STAGNATED and info["iterations"] == 10
    h = g.gs2_setup(dI, 1, 1, 1.0, g.FORWARD, stagnation_cycles=-1)
    x.zero_()
    info = g.gmres_solve(dA, b, x, 1, 1e-8, 300, g.PREC_NONE, h)
    assert info["status"] == g.NOT_CONVERGED and info["iterations"] == 300
