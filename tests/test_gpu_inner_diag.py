"""GPU parity of the inner-iteration diagnostic (Section 8: convergence of
the inner JR sweeps for the lower triangular system (wL + D) g = r) against
the oracle's or_inner_residuals, through the C ABI.  Float64 handles:
relative 1e-9 per value, or 1e-13 absolute once the residual has fallen to
rounding level (the nilpotent limit j >= depth); float32 handles: 1e-4
relative or 1e-6 absolute (the inner steps run in binary32)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2104_01196_amd as g  # noqa: E402
from gen import poisson2d, random_sparse, vardiff3d, laplace3d  # noqa: E402

pytestmark = pytest.mark.gpu

MATS = {
    "rand_nonsym": lambda: random_sparse(600, seed=41, avg_offdiag=5, long_rows=3, long_len=90, neg_diag_rows=7),
    "poisson2d_9": lambda: poisson2d(9),  # depth 17: the residual vanishes from j = 17 on
    "vardiff3d_13": lambda: vardiff3d(13, seed=6),
    "laplace3d_20": lambda: laplace3d(20),
}


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("w", [0.8, 1.0, 1.2])
@pytest.mark.parametrize("fmt", [g.FORMAT_SELL, g.FORMAT_DIA])
def test_inner_residuals_fp64(name, w, fmt):
    A = MATS[name]()
    if fmt == g.FORMAT_DIA and name == "rand_nonsym":
        pytest.skip("a random pattern has too many distinct offsets for the diagonal layout")
    dA = g.DeviceCSR.from_host(A)
    r = np.random.default_rng(21).standard_normal(A.n)
    J = 20
    ref = oracle.inner_residuals(A, r, J, omega=w)
    h = g.gs2_setup(dA, 1, J, w, g.FORWARD, format=fmt)
    out = g.gs2_inner_residuals(h, torch.as_tensor(r, device="cuda"), J)
    assert out.shape == (J + 1,)
    np.testing.assert_allclose(out, ref, rtol=1e-9, atol=1e-13)


@pytest.mark.parametrize("name", ["vardiff3d_13", "rand_nonsym"])
def test_inner_residuals_fp32(name):
    A = MATS[name]()
    dA = g.DeviceCSR.from_host(A)
    r = np.random.default_rng(22).standard_normal(A.n)
    J = 8
    ref = oracle.inner_residuals(A, r, J, omega=0.9)
    h = g.gs2_setup(dA, 1, J, 0.9, g.FORWARD, precision=g.FP32)
    out = g.gs2_inner_residuals(h, torch.as_tensor(r, device="cuda"), J)
    np.testing.assert_allclose(out, ref, rtol=1e-4, atol=1e-6)


def test_inner_residuals_arguments():
    A = poisson2d(5)
    dA = g.DeviceCSR.from_host(A)
    h = g.gs2_setup(dA, 1, 1, 1.0, g.FORWARD)
    r = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(g.Gs2Error):
        g.gs2_inner_residuals(h, r, -1)
    hb = g.gs2_setup(dA, 1, 1, 1.0, g.FORWARD, blocks=2)
    with pytest.raises(g.Gs2Error):
        g.gs2_inner_residuals(hb, r, 3)
