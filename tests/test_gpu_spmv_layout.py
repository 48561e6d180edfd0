"""GPU parity of the layouts of the GMRES solver's copy of A (the product
w = A z of every Arnoldi step and the true residual): sliced ELL, the
diagonal-interleaved copy (no column indices, two rows per lane) and the
3-row block copy (3 unknowns per node, blocks along node offsets, one or
two nodes per lane), forced
through the handle's spmv_format, and the timed automatic choice.  Each
GS2-preconditioned GMRES solve is compared with the CPU oracle's solve of
the same system: iteration count within one step (the two orthogonalise in
different orders), true relative residual <= rtol recomputed on the host,
solution within 1e-6 (relative) of the oracle's.

The matrices span several 1024-row workgroups with a ragged last one and
offsets inside and beyond a block of rows (so the clamped and the direct
gathers both run); a random pattern has far more than 32 distinct offsets
and must fall back to sliced ELL when the diagonal copy is requested."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2104_01196_amd as g  # noqa: E402
from gen import convdiff2d, elasticity_q1, laplace3d, make_rhs, poisson2d, random_sparse, vardiff3d  # noqa: E402

pytestmark = pytest.mark.gpu

MATS = {
    "laplace3d_20": (lambda: laplace3d(20), True),              # 8000 rows: 8 workgroups, ragged
    "vardiff3d_23": (lambda: vardiff3d(23, seed=4), True),       # 12167 rows, offsets 1, 23, 529
    "poisson2d_45": (lambda: poisson2d(45), True),              # 2025 rows: 2 workgroups
    "convdiff_71": (lambda: convdiff2d(71, 30.0, 4.0), True),    # nonsymmetric, 5041 rows
    "random_3000": (lambda: random_sparse(3000, seed=5, avg_offdiag=6), False),  # scattered offsets: sliced ELL
}


def solve(A, fmt, variant=g.SYMMETRIC):
    dA = g.DeviceCSR.from_host(A)
    b = make_rhs(A, "normal", seed=11)[1]
    h = g.gs2_setup(dA, 1, 1, 1.0, variant, spmv_format=fmt)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    info = g.gmres_solve(dA, torch.as_tensor(b, device="cuda"), x, 30, 1e-8, 5000, g.PREC_GS2, h)
    return h, dA, b, x, info


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("fmt", [g.FORMAT_SELL, g.FORMAT_DIA])
def test_gmres_copy_layout_matches_oracle(name, fmt):
    mk, qualifies = MATS[name]
    A = mk()
    h, dA, b, x, info = solve(A, fmt)
    sched = g.gs2_gmres_schedule(h)
    want_dia = fmt == g.FORMAT_DIA and qualifies
    assert sched["format"] == (g.FORMAT_DIA if want_dia else g.FORMAT_SELL), sched
    assert sched["tuned"] == 0
    # small bases keep the wide load groups, untimed
    assert g.gs2_gmres_basis_schedule(h) == {"dot_narrow_from": -1, "update_narrow_from": -1, "tuned": 0}
    if want_dia:
        assert sched["rows_per_lane"] == 2 and sched["ndiag"] == len(np.unique(A.colind - np.repeat(
            np.arange(A.n), np.diff(A.rowptr))))
    xo, io = oracle.gmres(A, b, restart=30, rtol=1e-8, prec="gs2", variant=oracle.SYMMETRIC, sweeps=1, inner=1)
    xs = x.cpu().numpy()
    rel = np.linalg.norm(b - A.to_scipy() @ xs) / np.linalg.norm(b)
    print(f"{name} fmt {fmt}: {sched}, GPU {info['iterations']} its, oracle {io['iterations']}, relres {rel:.2e}")
    assert info["converged"] and rel <= 1e-8
    assert abs(info["iterations"] - io["iterations"]) <= 1
    assert np.linalg.norm(xs - xo) / np.linalg.norm(xo) <= 1e-6


def test_diagonal_copy_follows_values_changed_in_place():
    """The copy's values are refreshed at every solve: with A's values
    scaled by 2 in place (same arrays, same pattern, same handle, whose
    preconditioner built from A is then a scaled one for 2A, to which
    flexible GMRES is invariant), the solve of 2A x = b gives half the
    solution."""
    A = vardiff3d(17, seed=8)
    h, dA, b, x, info = solve(A, g.FORMAT_DIA)
    assert g.gs2_gmres_schedule(h)["format"] == g.FORMAT_DIA
    x1 = x.cpu().numpy()
    dA.val.mul_(2.0)
    x.zero_()
    info2 = g.gmres_solve(dA, torch.as_tensor(b, device="cuda"), x, 30, 1e-8, 5000, g.PREC_GS2, h)
    assert info2["converged"] and abs(info2["iterations"] - info["iterations"]) <= 1
    xs = x.cpu().numpy()
    assert np.linalg.norm(b - 2.0 * (A.to_scipy() @ xs)) / np.linalg.norm(b) <= 1e-8
    assert np.linalg.norm(2.0 * xs - x1) / np.linalg.norm(x1) <= 1e-6


@pytest.mark.parametrize("name", ["vardiff3d_23", "laplace3d_20"])
def test_basis_load_groups_bitwise_equal(name):
    """The basis passes' narrow and wide load groups (forced through
    basis_loads) change only how the loads are issued, not the order of any
    sum: GMRES(40) gives bit-identical iterates and iteration counts, and
    matches the oracle.  12,167 rows (odd: the paired second pass does not
    apply, wide throughout) and 8,000 rows (even: narrow from steps 8 and
    12), both with a partial last workgroup in both passes."""
    A = MATS[name][0]() if name != "vardiff3d_24" else vardiff3d(24, seed=4)
    dA = g.DeviceCSR.from_host(A)
    b = make_rhs(A, "normal", seed=24)[1]
    xs = []
    for mode in (1, 2):
        h = g.gs2_setup(dA, 1, 1, 1.0, g.SYMMETRIC, basis_loads=mode)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        info = g.gmres_solve(dA, torch.as_tensor(b, device="cuda"), x, 40, 1e-8, 5000, g.PREC_GS2, h)
        bs = g.gs2_gmres_basis_schedule(h)
        narrow = mode == 2 and A.n % 2 == 0
        assert bs == {"dot_narrow_from": 8 if narrow else -1, "update_narrow_from": 12 if narrow else -1,
                      "tuned": 0}, bs
        xs.append((x.cpu().numpy(), info["iterations"]))
    assert xs[0][1] == xs[1][1] and np.array_equal(xs[0][0], xs[1][0])
    xo, io = oracle.gmres(A, b, restart=40, rtol=1e-8, prec="gs2", variant=oracle.SYMMETRIC, sweeps=1, inner=1)
    assert abs(xs[0][1] - io["iterations"]) <= 1
    assert np.linalg.norm(xs[0][0] - xo) / np.linalg.norm(xo) <= 1e-6


def test_basis_load_groups_even_ragged():
    """The same on an even row count with partial last workgroups (24^3 =
    13,824 rows: 6.75 workgroups of the second pass, 13.5 of the first),
    where the narrow groups run from steps 8 and 12."""
    test_basis_load_groups_bitwise_equal("vardiff3d_24")


@pytest.mark.slow
def test_timed_layout_choice_matches_oracle():
    """Automatic choice on a matrix large enough to be timed: the schedule
    says tuned, and the solve matches the oracle."""
    A = laplace3d(48)  # 110592 rows
    h, dA, b, x, info = solve(A, g.FORMAT_AUTO, variant=g.FORWARD)
    sched = g.gs2_gmres_schedule(h)
    print(f"laplace3d_48 automatic: {sched}")
    assert sched["tuned"] == 1 and sched["format"] in (g.FORMAT_SELL, g.FORMAT_DIA)
    xo, io = oracle.gmres(A, b, restart=30, rtol=1e-8, prec="gs2", variant=oracle.FORWARD, sweeps=1, inner=1)
    assert info["converged"] and abs(info["iterations"] - io["iterations"]) <= 1
    xs = x.cpu().numpy()
    assert np.linalg.norm(xs - xo) / np.linalg.norm(xo) <= 1e-6


ELA = {"elasticity_12x11x10": lambda: elasticity_q1(12, 11, 10, seed=3),   # 3960 rows: 4 workgroups, ragged
       "elasticity_7x6x5": lambda: elasticity_q1(7, 6, 5, seed=4)}       # 630 rows: one partial workgroup


@pytest.mark.parametrize("name", list(ELA))
@pytest.mark.parametrize("fmt", [g.FORMAT_SELL, g.FORMAT_BLOCK3])
def test_block3_copy_matches_oracle(name, fmt):
    """The 3-row block copy on 3-dof elasticity (27 node offsets, 81 scalar
    offsets: too many for the diagonal copy), against the oracle's GMRES(30)
    with the damped SGS2(1,3) of the elasticity study (omega 0.7, inner
    damping 0.5): iterations within one, true residual, solution within
    1e-6."""
    A = ELA[name]()
    dA = g.DeviceCSR.from_host(A)
    b = make_rhs(A, "normal", seed=21)[1]
    h = g.gs2_setup(dA, 1, 3, 0.7, g.SYMMETRIC, inner_damping=0.5, spmv_format=fmt)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    info = g.gmres_solve(dA, torch.as_tensor(b, device="cuda"), x, 30, 1e-8, 5000, g.PREC_GS2, h)
    sched = g.gs2_gmres_schedule(h)
    assert sched["format"] == fmt and sched["tuned"] == 0, sched
    if fmt == g.FORMAT_BLOCK3:
        nodes = A.n // 3
        rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
        assert sched["rows_per_lane"] == 2
        assert sched["ndiag"] == len(np.unique(A.colind // 3 - rows // 3)) == 27 and nodes * 3 == A.n
    xo, io = oracle.gmres(A, b, restart=30, rtol=1e-8, prec="gs2", variant=oracle.SYMMETRIC, sweeps=1, inner=3,
                          omega=0.7, gamma=0.5)
    xs = x.cpu().numpy()
    rel = np.linalg.norm(b - A.to_scipy() @ xs) / np.linalg.norm(b)
    print(f"{name} fmt {fmt}: {sched}, GPU {info['iterations']} its, oracle {io['iterations']}, relres {rel:.2e}")
    assert info["converged"] and rel <= 1e-8
    assert abs(info["iterations"] - io["iterations"]) <= 1
    assert np.linalg.norm(xs - xo) / np.linalg.norm(xo) <= 1e-6


@pytest.mark.parametrize("name", list(ELA))
def test_block3_copy_without_delay_matches_oracle(name):
    """The block copy inside the fused product-and-dots kernels (the
    orthogonalisation without delayed reorthogonalisation forms w = A z one
    1024-row workgroup at a time, one node per thread over the nodes that
    meet its rows, the boundary nodes formed by both neighbours): iterations
    within one of the oracle's GMRES(30), solution within 1e-6, and the same
    iterations as the sliced-ELL copy on the same path."""
    A = ELA[name]()
    dA = g.DeviceCSR.from_host(A)
    b = make_rhs(A, "normal", seed=23)[1]
    its = {}
    for fmt in (g.FORMAT_SELL, g.FORMAT_BLOCK3):
        h = g.gs2_setup(dA, 1, 3, 0.7, g.SYMMETRIC, inner_damping=0.5, spmv_format=fmt, orthogonalization=1)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        info = g.gmres_solve(dA, torch.as_tensor(b, device="cuda"), x, 30, 1e-8, 5000, g.PREC_GS2, h)
        assert g.gs2_gmres_schedule(h)["format"] == fmt
        its[fmt] = info["iterations"]
        xs = x.cpu().numpy()
        rel = np.linalg.norm(b - A.to_scipy() @ xs) / np.linalg.norm(b)
        assert info["converged"] and rel <= 1e-8
    xo, io = oracle.gmres(A, b, restart=30, rtol=1e-8, prec="gs2", variant=oracle.SYMMETRIC, sweeps=1, inner=3,
                          omega=0.7, gamma=0.5)
    print(f"{name} without delay: GPU {its}, oracle {io['iterations']}")
    assert abs(its[g.FORMAT_BLOCK3] - io["iterations"]) <= 1 and abs(its[g.FORMAT_SELL] - its[g.FORMAT_BLOCK3]) <= 1
    assert np.linalg.norm(xs - xo) / np.linalg.norm(xo) <= 1e-6


def test_block3_refused_where_it_does_not_apply():
    """Forced block copy on matrices that do not qualify falls back to sliced
    ELL: a row count not divisible by 3, and scattered columns with far more
    than 32 node offsets (3000 rows)."""
    for A in (laplace3d(10), random_sparse(3000, seed=5, avg_offdiag=6)):
        dA = g.DeviceCSR.from_host(A)
        b = make_rhs(A, "normal", seed=22)[1]
        h = g.gs2_setup(dA, 1, 1, 1.0, g.SYMMETRIC, spmv_format=g.FORMAT_BLOCK3)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        info = g.gmres_solve(dA, torch.as_tensor(b, device="cuda"), x, 30, 1e-8, 5000, g.PREC_GS2, h)
        assert g.gs2_gmres_schedule(h)["format"] == g.FORMAT_SELL
        xo, io = oracle.gmres(A, b, restart=30, rtol=1e-8, prec="gs2", variant=oracle.SYMMETRIC, sweeps=1, inner=1)
        assert info["converged"] and abs(info["iterations"] - io["iterations"]) <= 1


@pytest.mark.slow
def test_block3_timed_choice_on_elasticity():
    """Automatic choice on an elasticity matrix large enough to be timed
    (98,304 rows): every candidate (sliced ELL at two lane counts, the block
    copy at one and two nodes per lane) builds and runs; the solve matches the
    oracle."""
    A = elasticity_q1(32, 32, 32, seed=5)
    dA = g.DeviceCSR.from_host(A)
    b = make_rhs(A, "normal", seed=23)[1]
    h = g.gs2_setup(dA, 1, 3, 0.7, g.SYMMETRIC, inner_damping=0.5)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    info = g.gmres_solve(dA, torch.as_tensor(b, device="cuda"), x, 50, 1e-8, 20000, g.PREC_GS2, h)
    sched = g.gs2_gmres_schedule(h)
    print(f"elasticity 32^3 automatic: {sched}, {info['iterations']} its")
    assert sched["tuned"] == 1
    xo, io = oracle.gmres(A, b, restart=50, rtol=1e-8, prec="gs2", variant=oracle.SYMMETRIC, sweeps=1, inner=3,
                          omega=0.7, gamma=0.5)
    assert info["converged"] and abs(info["iterations"] - io["iterations"]) <= 1
    xs = x.cpu().numpy()
    assert np.linalg.norm(xs - xo) / np.linalg.norm(xo) <= 1e-6
