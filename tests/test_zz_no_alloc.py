"""The allocation-free variant of the inner-iteration diagnostic,
gs2_inner_residuals_noalloc (partial sums in the library's fixed per-device
scratch array, output in device memory, no allocation and no host
synchronisation), against the allocating entry point gs2_inner_residuals,
through the C ABI.

Both enqueue the same kernels in the same order on the same handle, so the
values must be bitwise equal.  Two calls in a row, the second with a smaller
input (the scratch array keeps the first call's contents, which the second
must not read), each also checked against the CPU oracle's diagnostic at the
bar of the allocating entry point's own test (float64: 1e-9 relative or
1e-13 absolute; float32: 1e-4 relative or 1e-6 absolute).  An input beyond
the scratch limit is refused with GS2_ERR_SCRATCH before anything is
enqueued."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2104_01196_amd as g  # noqa: E402
from gen import poisson2d, vardiff3d  # noqa: E402

pytestmark = pytest.mark.gpu

# (matrix, precision, inner sweeps, damping, rtol, atol): the second is smaller in rows and steps
CALLS = [
    (lambda: vardiff3d(23, seed=9), g.FP64, 6, 0.8, 1e-9, 1e-13),   # 12167 rows: 48 workgroups of partials
    (lambda: poisson2d(20), g.FP32, 3, 1.1, 1e-4, 1e-6),            # 400 rows: 2 workgroups
]


def test_noalloc_matches_allocating_entry_two_calls():
    for mk, prec, J, w, rtol, atol in CALLS:
        A = mk()
        dA = g.DeviceCSR.from_host(A)
        h = g.gs2_setup(dA, 1, J, w, g.FORWARD, precision=prec)
        r_h = np.random.default_rng(A.n).standard_normal(A.n)
        r = torch.as_tensor(r_h, device="cuda")
        ref = g.gs2_inner_residuals(h, r, J)  # allocating entry point, host output
        out = torch.full((J + 1,), float("nan"), dtype=torch.float64, device="cuda")
        g.gs2_inner_residuals_noalloc(h, r, J, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print(f"n={A.n} prec={prec} inner={J}: noalloc {got}")
        assert got.tobytes() == ref.tobytes(), (got, ref)
        np.testing.assert_allclose(got, oracle.inner_residuals(A, r_h, J, omega=w), rtol=rtol, atol=atol)
        del h


def test_noalloc_refuses_inputs_beyond_the_scratch():
    A = poisson2d(20)  # 400 rows: 2 workgroups of partial sums
    dA = g.DeviceCSR.from_host(A)
    h = g.gs2_setup(dA, 1, 1, 1.0, g.FORWARD)
    r = torch.ones(A.n, dtype=torch.float64, device="cuda")
    nb = (A.n + 255) // 256
    J = g.native.NOALLOC_SCRATCH_DOUBLES // (nb + 1) - 1  # (nb + 1) (J + 2) > limit
    assert (nb + 1) * (J + 2) > g.native.NOALLOC_SCRATCH_DOUBLES >= (nb + 1) * (J + 1)
    out = torch.full((J + 1,), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(g.Gs2Error) as e:
        g.gs2_inner_residuals_noalloc(h, r, J, out)
    assert e.value.status == g.ERR_SCRATCH
    torch.cuda.synchronize()
    assert torch.isnan(out).all()  # nothing was enqueued
