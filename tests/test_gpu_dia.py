"""GPU parity of the diagonal-interleaved layout of the triangles (every rows-
per-lane candidate, with and without LDS staging of the source vector, with
workgroups walked in per-XCD ranges and in dispatch order)
against the CPU oracle, through the C ABI.  Same bars as the sliced-ELL
applies (tests/test_gpu_parity.py): 1e-12 per half sweep in float64 (the
scaled-space kernels and the textbook oracle differ only in rounding
order), 2e-5 / 1e-4 against the oracle's float32 / scaled-float16 forms
(same stored values, different summation order), GMRES within one
iteration of the oracle.

The matrices span several workgroups with a ragged last one (a workgroup
covers 256 R rows), and have offsets both inside the LDS halo (|col - row|
<= 64) and beyond it."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2104_01196_amd as g  # noqa: E402
from gen import laplace3d, poisson2d, vardiff3d, convdiff2d, elasticity_q1, random_sparse, config_problem  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"
MATS = {
    "laplace3d_17": lambda: laplace3d(17),        # offsets 1, 17 (staged) and 289 (not)
    "vardiff3d_23": lambda: vardiff3d(23, seed=5),  # 12167 rows: several workgroups at every R, ragged
    "poisson2d_45": lambda: poisson2d(45),        # 2025 rows: fewer than one workgroup at R >= 8
    "convdiff_71": lambda: convdiff2d(71, 35.0, 2.2),  # nonsymmetric, offsets 1 and 71 (beyond the halo)
}
_cache = {}

R_OF = {g.FP64: [1, 2], g.FP32: [1, 2, 4], g.FP16_SCALED: [1, 2, 4, 8]}
TOL = {g.FP64: None, g.FP32: 2e-5, g.FP16_SCALED: 1e-4}


def mat(name):
    if name not in _cache:
        A = MATS[name]()
        _cache[name] = (A, g.DeviceCSR.from_host(A))
    return _cache[name]


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_inf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def reference(A, v, prec, variant, sweeps, inner, w, gamma=1.0):
    if prec == g.FP64:
        return oracle.gs2_apply(A, v, variant, sweeps, inner, w, gamma)
    return oracle.gs2_apply_lp(A, v, prec, variant, sweeps, inner, w, gamma)


def schedules():
    for prec, Rs in R_OF.items():
        for R in Rs:
            for lds in (g.LDS_OFF, g.LDS_ON):
                for xcd in (g.XCD_RANGES, g.XCD_DISPATCH_ORDER):
                    yield prec, R, lds, xcd


CASES = [(g.FORWARD, 2, 1, 1.0), (g.SYMMETRIC, 1, 2, 0.9), (g.BACKWARD, 1, 3, 0.8), (g.FORWARD, 3, 0, 0.7)]


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("prec,R,lds,xcd", list(schedules()))
def test_dia_apply_every_schedule(name, prec, R, lds, xcd):
    A, dA = mat(name)
    v = np.random.default_rng(11).standard_normal(A.n)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    for variant, sweeps, inner, w in CASES:
        h = g.gs2_setup(dA, sweeps, inner, w, variant, precision=prec, format=g.FORMAT_DIA, rows_per_lane=R,
                        lds_staging=lds, xcd_ranges=xcd)
        sch = g.gs2_handle_schedule(h)
        assert (sch["format"], sch["rows_per_lane"], sch["lds_staging"], sch["xcd_ranges"]) == \
            (g.FORMAT_DIA, R, lds == g.LDS_ON, xcd == g.XCD_RANGES)
        assert sch["vector_bytes"] == R * {g.FP64: 8, g.FP32: 4, g.FP16_SCALED: 2}[prec]
        g.gs2_apply(h, dev(v), z)
        ref = reference(A, v, prec, variant, sweeps, inner, w)
        halves = sweeps * (2 if variant == g.SYMMETRIC else 1)
        tol = TOL[prec] or 1e-12 * halves
        assert rel_inf(host(z), ref) <= tol, (variant, sweeps, inner, w)


@pytest.mark.parametrize("name", ["vardiff3d_23", "convdiff_71"])
@pytest.mark.parametrize("lds", [g.LDS_OFF, g.LDS_ON])
def test_dia_damping_compact_and_jr(name, lds):
    """Inner damping gamma, the compact form and the JR entry point on the
    diagonal layout (float64)."""
    A, dA = mat(name)
    v = np.random.default_rng(12).standard_normal(A.n)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    h = g.gs2_setup(dA, 2, 3, 0.9, g.SYMMETRIC, inner_damping=0.6, format=g.FORMAT_DIA, lds_staging=lds)
    g.gs2_apply(h, dev(v), z)
    assert rel_inf(host(z), oracle.gs2_apply(A, v, g.SYMMETRIC, 2, 3, 0.9, 0.6)) <= 4e-12
    h = g.gs2_setup(dA, 2, 1, 0.8, g.FORWARD, compact=True, format=g.FORMAT_DIA, lds_staging=lds)
    g.gs2_apply(h, dev(v), z)
    assert rel_inf(host(z), oracle.gs2c_sweep(A, v, np.zeros(A.n), g.FORWARD, 2, 1, 0.8)) <= 4e-12
    g.jr_apply(h, 3, 0.7, dev(v), z)
    assert rel_inf(host(z), oracle.jr_sweep(A, v, np.zeros(A.n), 3, 0.7)) <= 3e-12


@pytest.mark.parametrize("prec", [g.FP32, g.FP16_SCALED])
def test_dia_prep_four_rows_per_thread(prec):
    """A row count divisible by 4 (24^3 = 13,824) takes the pass that forms
    S_l v four rows per thread (16-byte loads); the other matrices here have
    odd row counts and take the one-row pass.  Apply against the oracle's
    reduced-precision apply, and GMRES(30) within one iteration of the
    oracle (its first preconditioner pass then also closes the previous
    Arnoldi step)."""
    A = vardiff3d(24, seed=6)
    assert A.n % 4 == 0
    dA = g.DeviceCSR.from_host(A)
    v = np.random.default_rng(15).standard_normal(A.n)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    for variant, sweeps, inner, w in ((g.SYMMETRIC, 2, 2, 0.9), (g.FORWARD, 1, 1, 1.0)):
        h = g.gs2_setup(dA, sweeps, inner, w, variant, precision=prec, format=g.FORMAT_DIA)
        g.gs2_apply(h, dev(v), z)
        ref = oracle.gs2_apply_lp(A, v, prec, variant, sweeps, inner, w)
        assert rel_inf(host(z), ref) <= TOL[prec], (variant, sweeps, inner, w)
    b = np.random.default_rng(16).standard_normal(A.n)
    _, io = oracle.gmres(A, b, restart=30, rtol=1e-8, prec="gs2", variant=oracle.SYMMETRIC, sweeps=1, inner=1,
                         precision=prec)
    h = g.gs2_setup(dA, 1, 1, 1.0, g.SYMMETRIC, precision=prec, format=g.FORMAT_DIA)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    info = g.gmres_solve(dA, dev(b), x, 30, 1e-8, 5000, g.PREC_GS2, h)
    assert info["converged"] and abs(info["iterations"] - io["iterations"]) <= 1, (info, io)


@pytest.mark.parametrize("prec", [g.FP32, g.FP16_SCALED])
@pytest.mark.parametrize("lds", [g.LDS_OFF, g.LDS_ON])
def test_dia_reduced_precision_damping_and_compact(prec, lds):
    """Inner damping gamma and the compact form in the 32- and 16-bit forms on
    the diagonal layout, where S_l v is formed once per apply in the working
    precision and read by the first inner pass and every residual pass.
    Damped: against the oracle's reduced-precision apply with gamma at the
    forms' bars (2e-5 / 1e-4).  Compact: the oracle's reduced-precision forms
    have no compact sweep, so against its float64 compact sweep with the
    rounding of the form (float32: 1e-5; scaled float16, whose stored entries
    carry 2^-11 relative error: 3e-3).  Both also against the sliced-ELL
    layout of the same form (same stored values and arithmetic, another
    summation order: 2e-5 / 1e-4)."""
    A, dA = mat("vardiff3d_23")
    v = np.random.default_rng(14).standard_normal(A.n)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    zs = torch.empty(A.n, dtype=torch.float64, device=DEV)
    bar_or = {g.FP32: 1e-5, g.FP16_SCALED: 3e-3}[prec]
    bar_sell = TOL[prec]
    for kw, ref, bar in ((dict(sweeps=2, inner=3, w=0.9, var=g.SYMMETRIC, inner_damping=0.6),
                          oracle.gs2_apply_lp(A, v, prec, g.SYMMETRIC, 2, 3, 0.9, 0.6), TOL[prec]),
                         (dict(sweeps=2, inner=1, w=0.8, var=g.FORWARD, compact=True),
                          oracle.gs2c_sweep(A, v, np.zeros(A.n), g.FORWARD, 2, 1, 0.8), bar_or)):
        extra = {k: kw[k] for k in ("inner_damping", "compact") if k in kw}
        h = g.gs2_setup(dA, kw["sweeps"], kw["inner"], kw["w"], kw["var"], precision=prec, format=g.FORMAT_DIA,
                        lds_staging=lds, **extra)
        g.gs2_apply(h, dev(v), z)
        hs = g.gs2_setup(dA, kw["sweeps"], kw["inner"], kw["w"], kw["var"], precision=prec, format=g.FORMAT_SELL,
                         **extra)
        g.gs2_apply(hs, dev(v), zs)
        zd = host(z)
        assert rel_inf(zd, ref) <= bar, (kw, rel_inf(zd, ref))
        assert rel_inf(zd, host(zs)) <= bar_sell, (kw, rel_inf(zd, host(zs)))


@pytest.mark.parametrize("prec", [g.FP64, g.FP32, g.FP16_SCALED])
@pytest.mark.parametrize("lds,xcd", [(g.LDS_OFF, g.XCD_RANGES), (g.LDS_ON, g.XCD_RANGES),
                                     (g.LDS_OFF, g.XCD_DISPATCH_ORDER)])
def test_dia_gmres_iterations(prec, lds, xcd):
    """GMRES(30) with an SGS2(1,1) preconditioner on the diagonal layout: the
    first preconditioner pass of each step also closes the previous step
    (the fused variant of the pass)."""
    A, dA = mat("vardiff3d_23")
    b = np.random.default_rng(13).standard_normal(A.n)
    _, io = oracle.gmres(A, b, restart=30, rtol=1e-8, prec="gs2", variant=oracle.SYMMETRIC, sweeps=1, inner=1,
                         precision=prec)
    h = g.gs2_setup(dA, 1, 1, 1.0, g.SYMMETRIC, precision=prec, format=g.FORMAT_DIA, lds_staging=lds,
                    xcd_ranges=xcd)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    info = g.gmres_solve(dA, dev(b), x, 30, 1e-8, 5000, g.PREC_GS2, h)
    assert info["converged"] and info["relres"] <= 1e-8
    assert abs(info["iterations"] - io["iterations"]) <= 1, (info, io)


B3MATS = {"elasticity_12x11x10": lambda: elasticity_q1(12, 11, 10, seed=7),  # 3960 rows, ragged workgroups
          "elasticity_5x6x7": lambda: elasticity_q1(5, 6, 7, seed=8)}       # 630 rows: one partial workgroup


def b3_schedules():
    for prec, Rs in R_OF.items():
        for R in Rs:
            for xcd in (g.XCD_RANGES, g.XCD_DISPATCH_ORDER):
                yield prec, R, xcd


@pytest.mark.parametrize("name", list(B3MATS))
@pytest.mark.parametrize("prec,R,xcd", list(b3_schedules()))
def test_block3_apply_every_schedule(name, prec, R, xcd):
    """The 3-row block layout of the triangles (3-dof elasticity: 81 scalar
    offsets, too many for the diagonal layout; 14 node offsets per triangle,
    the diagonal block's strictly lower / upper entries included; nine
    node-major planes per offset, a lane owning R nodes and their three rows)
    at every nodes-per-lane R and both workgroup walks, against the oracle at
    the same bars as the diagonal layout."""
    A = B3MATS[name]()
    dA = g.DeviceCSR.from_host(A)
    v = np.random.default_rng(17).standard_normal(A.n)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    for variant, sweeps, inner, w in CASES:
        h = g.gs2_setup(dA, sweeps, inner, w, variant, precision=prec, format=g.FORMAT_BLOCK3, rows_per_lane=R,
                        xcd_ranges=xcd)
        sch = g.gs2_handle_schedule(h)
        assert (sch["format"], sch["rows_per_lane"], sch["lds_staging"], sch["xcd_ranges"]) == \
            (g.FORMAT_BLOCK3, R, False, xcd == g.XCD_RANGES)
        assert sch["ndiag_l"] == 14 and sch["ndiag_u"] == 14, sch
        g.gs2_apply(h, dev(v), z)
        ref = reference(A, v, prec, variant, sweeps, inner, w)
        halves = sweeps * (2 if variant == g.SYMMETRIC else 1)
        tol = TOL[prec] or 1e-12 * halves
        assert rel_inf(host(z), ref) <= tol, (variant, sweeps, inner, w, rel_inf(host(z), ref))


@pytest.mark.parametrize("prec", [g.FP64, g.FP32, g.FP16_SCALED])
@pytest.mark.parametrize("fmt,name", [(g.FORMAT_BLOCK3, "elasticity_12x11x10"), (g.FORMAT_DIA, "vardiff3d_23")])
def test_forced_layout_untimed_takes_widest_load(prec, fmt, name):
    """A forced layout without timing (autotune off, rows per lane free)
    takes the widest value load the precision allows (16 bytes: 2 float64,
    4 float32 or 8 float16 values per lane), in either layout, and applies
    as the oracle does at the layouts' usual bars."""
    if fmt == g.FORMAT_BLOCK3:
        A = B3MATS[name]()
        dA = g.DeviceCSR.from_host(A)
    else:
        A, dA = mat(name)
    v = np.random.default_rng(19).standard_normal(A.n)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    h = g.gs2_setup(dA, 1, 2, 0.9, g.SYMMETRIC, precision=prec, format=fmt, autotune=False)
    sch = g.gs2_handle_schedule(h)
    assert (sch["format"], sch["rows_per_lane"], sch["vector_bytes"], sch["tuned"]) == \
        (fmt, max(R_OF[prec]), 16, 0), sch
    g.gs2_apply(h, dev(v), z)
    ref = reference(A, v, prec, g.SYMMETRIC, 1, 2, 0.9)
    assert rel_inf(host(z), ref) <= (TOL[prec] or 2e-12)


@pytest.mark.parametrize("prec", [g.FP64, g.FP32, g.FP16_SCALED])
def test_block3_damping_compact_and_gmres(prec):
    """On the block layout: inner damping gamma (against the oracle's apply in
    the same form) and the compact form (against the oracle's float64
    compact sweep, with the reduced-precision bars of
    test_dia_reduced_precision_damping_and_compact), and GMRES(30) within
    one iteration of the oracle's solve in the same form: with SGS2(2,3) at
    omega 0.4 and with the elasticity study's SGS2(1,3), omega 0.7, gamma 0.5
    (undamped SGS2 at omega 1 stagnates on elasticity)."""
    A = B3MATS["elasticity_12x11x10"]()
    dA = g.DeviceCSR.from_host(A)
    v = np.random.default_rng(18).standard_normal(A.n)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    bar = {g.FP64: 4e-12, g.FP32: 1e-5, g.FP16_SCALED: 3e-3}[prec]
    h = g.gs2_setup(dA, 2, 3, 0.9, g.SYMMETRIC, precision=prec, inner_damping=0.6, format=g.FORMAT_BLOCK3)
    g.gs2_apply(h, dev(v), z)
    ref = reference(A, v, prec, g.SYMMETRIC, 2, 3, 0.9, 0.6)
    assert rel_inf(host(z), ref) <= (TOL[prec] or 4e-12), rel_inf(host(z), ref)
    h = g.gs2_setup(dA, 2, 1, 0.8, g.FORWARD, precision=prec, compact=True, format=g.FORMAT_BLOCK3)
    g.gs2_apply(h, dev(v), z)
    assert rel_inf(host(z), oracle.gs2c_sweep(A, v, np.zeros(A.n), g.FORWARD, 2, 1, 0.8)) <= bar
    b = np.random.default_rng(19).standard_normal(A.n)
    settings = [(2, 3, 0.4, 1.0), (1, 3, 0.7, 0.5)]
    for sweeps, inner, w, gamma in settings:
        _, io = oracle.gmres(A, b, restart=30, rtol=1e-8, prec="gs2", variant=oracle.SYMMETRIC, sweeps=sweeps,
                             inner=inner, omega=w, gamma=gamma, precision=prec)
        h = g.gs2_setup(dA, sweeps, inner, w, g.SYMMETRIC, precision=prec, inner_damping=gamma,
                        format=g.FORMAT_BLOCK3)
        x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
        info = g.gmres_solve(dA, dev(b), x, 30, 1e-8, 5000, g.PREC_GS2, h)
        assert io["converged"] and info["converged"], (info, io)
        assert abs(info["iterations"] - io["iterations"]) <= 1, (sweeps, inner, w, gamma, info, io)


def test_dia_eligibility():
    """The diagonal layout is refused where it does not apply: too many
    distinct offsets (3-dof elasticity), hybrid blocks, or a rows-per-lane
    whose load would exceed 16 bytes; the automatic choice then keeps the
    sliced-ELL layout."""
    A = elasticity_q1(5, 5, 5, seed=4)
    dA = g.DeviceCSR.from_host(A)
    with pytest.raises(g.Gs2Error) as e:
        g.gs2_setup(dA, 1, 1, 1.0, g.FORWARD, format=g.FORMAT_DIA)
    assert e.value.status == -1
    sch = g.gs2_handle_schedule(g.gs2_setup(dA, 1, 1, 1.0, g.FORWARD))
    assert sch["format"] == g.FORMAT_SELL and sch["ndiag_l"] == 0
    L, dL = mat("laplace3d_17")
    with pytest.raises(g.Gs2Error):
        g.gs2_setup(dL, 1, 1, 1.0, g.FORWARD, blocks=4, format=g.FORMAT_DIA)
    with pytest.raises(g.Gs2Error):
        g.gs2_setup(dL, 1, 1, 1.0, g.FORWARD, format=g.FORMAT_DIA, rows_per_lane=4)  # 32-byte float64 load
    sch = g.gs2_handle_schedule(g.gs2_setup(dL, 1, 1, 1.0, g.FORWARD, format=g.FORMAT_SELL))
    assert sch["format"] == g.FORMAT_SELL and sch["ndiag_l"] == 0
    R = random_sparse(500, seed=3, avg_offdiag=6)
    sch = g.gs2_handle_schedule(g.gs2_setup(g.DeviceCSR.from_host(R), 1, 1, 1.0, g.FORWARD))
    assert sch["format"] == g.FORMAT_SELL
    # the 3-row block layout: refused for a row count not divisible by 3, for
    # scattered columns (far more than 32 node offsets), for hybrid blocks
    for M in (dL, g.DeviceCSR.from_host(random_sparse(600, seed=4, avg_offdiag=6))):
        with pytest.raises(g.Gs2Error):
            g.gs2_setup(M, 1, 1, 1.0, g.FORWARD, format=g.FORMAT_BLOCK3)
    with pytest.raises(g.Gs2Error):
        g.gs2_setup(dA, 1, 1, 1.0, g.FORWARD, blocks=2, format=g.FORMAT_BLOCK3)
    sch = g.gs2_handle_schedule(g.gs2_setup(dA, 1, 1, 1.0, g.FORWARD, format=g.FORMAT_BLOCK3))
    assert sch["format"] == g.FORMAT_BLOCK3 and sch["ndiag_l"] == sch["ndiag_u"] == 14


@pytest.mark.parametrize("prec", [g.FP64, g.FP32, g.FP16_SCALED])
def test_tuned_schedule_matches_oracle(prec):
    """The timed choice (automatic format, rows per lane and staging) on a
    stencil matrix of 35,937 rows: reported as tuned, and its apply matches
    the oracle whichever candidate won."""
    A = laplace3d(33)
    dA = g.DeviceCSR.from_host(A)
    h = g.gs2_setup(dA, 1, 1, 1.0, g.SYMMETRIC, precision=prec)
    sch = g.gs2_handle_schedule(h)
    assert sch["tuned"] == 1 and sch["ndiag_l"] == 3 and sch["ndiag_u"] == 3
    v = np.random.default_rng(14).standard_normal(A.n)
    z = torch.empty(A.n, dtype=torch.float64, device=DEV)
    g.gs2_apply(h, dev(v), z)
    assert rel_inf(host(z), reference(A, v, prec, g.SYMMETRIC, 1, 1, 1.0)) <= (TOL[prec] or 2e-12)
    print(f"tuned schedule ({prec}): {sch}")
