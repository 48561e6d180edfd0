"""Benchmark: GS2-preconditioned GMRES time to solution on one MI355X.

Workload (default, --config 4): the precision-form study on the 3D
variable-coefficient diffusion problem, 192^3 cells (n = 7,077,888,
nnz = 49,324,032), kappa log-uniform over [1e-2, 1e2], CSR float64 in
natural ordering, b = A x_true with x_true ~ N(0,1) from a fixed seed,
x0 = 0.  GMRES(50) to ||b - A x|| / ||b|| <= 1e-8, right-preconditioned by
symmetric GS2 with 1 outer and 1 inner sweep (SGS2(1,1), damping 1.0, the
paper's mixed-precision setting), preconditioner stored and computed in
float64, float32 and diagonally scaled float16 (float32 arithmetic); the
Krylov loop is float64 in every form.
One "step" is one complete solve (the whole preconditioned Krylov path:
setup excluded, done once before timing).  `value` is the mean time to
solution of the float64-preconditioner solve over the timed steps (median and
spread reported with it); the float32 and scaled-float16 preconditioner
solves are timed the same way and reported under `forms`, each with its
iteration count, its error against the float64 CPU oracle's solution (stored
by tests/golden/make_oracle_solves.py, which calls only the oracle) and the
algorithmic bandwidth of its sweep kernels from a profiled pass.

--config 2 runs the same measurement on the 128^3 Laplacian with forward
GS2(2 sweeps, 1 inner); --config 5 times the batched persistent solver (512
uneven convection-diffusion systems x 4 right-hand sides, GS2(2,2),
GMRES(20), FP32 and FP64 preconditioner) against the plain FP64 path that
solves the 2048 systems one gmres_solve at a time.

--compare times GMRES(50) on the 128^3 Laplacian with each preconditioner of
the paper's comparison (GS2, SGS2, JR, exact level-scheduled GS/SGS,
multicolor GS, none).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--size N] [--config 2|4|5] [--compare]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=None, help="grid side (default: the configuration's)")
    ap.add_argument("--config", type=int, default=4, choices=[2, 3, 4, 5],
                    help="4: precision forms on the 192^3 variable-coefficient problem (default); 2: the 128^3 "
                         "Laplacian; 3: Q1 elasticity on 64^3 free nodes (damped SGS2 with inner damping, "
                         "and Jacobi); 5: batched form on 512 convection-diffusion systems x 4 right-hand sides")
    ap.add_argument("--compare", action="store_true",
                    help="GMRES(50) on the 128^3 Laplacian with each preconditioner of the comparison (GS2, SGS2, JR, "
                         "exact level-scheduled GS, multicolor GS) instead of the default measurement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sequential", action="store_true",
                    help="config 5: skip the one-solve-per-pair comparison (e.g. under a kernel tracer)")
    ap.add_argument("--no-forms", action="store_true", help="skip the float32 / float16 preconditioner solves")
    ap.add_argument("--schedule", default=None,
                    help="force the sweep kernels' schedule per form instead of timing it at setup, e.g. "
                         "'fp64=1/0/0,fp32=4/0/0,fp16_scaled=8/0/1' (diagonal layout, rows per lane / LDS staging "
                         "0 or 1 / per-XCD row ranges 0 or 1; the solver's copy of A then uses the diagonal layout "
                         "too; a 'b3:' prefix, e.g. 'fp64=b3:2/0/1', names the 3-row block layout, nodes per lane "
                         "instead of rows): for counter runs, whose "
                         "serialised launches would time the candidates differently")
    ap.add_argument("--profile", choices=["on", "off"], default="on",
                    help="per-kernel HIP-event timing of the float64 solves (a second pass of the same solves)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_digest():
    """sha256 of the HIP sources and the ABI header: counter-based traffic
    figures are used only when they were taken on the kernels built now."""
    import glob
    import hashlib

    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2104_01196_amd", "csrc", "*.hip")) +
                   glob.glob(os.path.join(ROOT, "paper_2104_01196_amd", "csrc", "*.hpp")) +
                   [os.path.join(ROOT, "include", "gs2.h")])
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def stream_ceiling(torch, nbytes=1 << 31, reps=5):
    """Measured HBM ceiling: device-to-device copy of nbytes (read + write
    counted), best of reps, timed with events on torch's stream."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def oracle_reference(wname, x_true, np):
    """The float64 oracle's solution of the workload and its iteration counts,
    from the record tests/golden/make_oracle_solves.py writes (it calls only
    the CPU oracle): x_oracle = x_true + the stored float32 difference.
    (None, record or None) when the record or its array is missing or stale."""
    import hashlib

    rec_path = os.path.join(ROOT, "tests", "golden", f"{wname}_oracle.json")
    if not os.path.exists(rec_path):
        log(f"[bench] no oracle record {rec_path}: errors against the oracle reported as null")
        return None, None
    rec = json.load(open(rec_path))
    f64 = rec["solves"]["fp64"]
    dx_path = os.path.join(ROOT, "tests", "golden", f64["dx_file"])
    if not os.path.exists(dx_path):
        log(f"[bench] {dx_path} is missing (python tests/golden/make_oracle_solves.py {wname} writes it)")
        return None, rec
    raw = open(dx_path, "rb").read()
    if hashlib.sha256(raw).hexdigest() != f64["dx_sha256"]:
        log(f"[bench] {dx_path} does not match its record: errors against the oracle reported as null")
        return None, rec
    dx = np.load(dx_path)
    return x_true + dx.astype(np.float64), rec


def forced_schedule(args, form, g):
    """gs2_setup keyword arguments that force the schedule --schedule names
    for this form (none: the setup times its candidates)."""
    if not args.schedule:
        return {}
    for item in args.schedule.split(","):
        name, val = item.split("=")
        if name == form:
            fmt = g.FORMAT_DIA
            if val.startswith("b3:"):  # the 3-row block layout (rows per lane then counts nodes)
                fmt, val = g.FORMAT_BLOCK3, val[3:]
            rows, lds, *xcd = val.split("/")
            return {"format": fmt, "rows_per_lane": int(rows), "lds_staging": g.LDS_ON if int(lds) else g.LDS_OFF,
                    "xcd_ranges": (g.XCD_RANGES if int(xcd[0]) else g.XCD_DISPATCH_ORDER) if xcd else g.XCD_AUTO,
                    "spmv_format": fmt}
    return {}


def oracle_sampled_error(rec, xs, np):
    """||x - x_oracle|| / ||x_oracle|| over the seeded sample of solution
    entries the oracle record stores (its float64 values, written by the
    oracle-only script), or None without a record."""
    if not rec:
        return None
    f64 = rec["solves"]["fp64"]
    if "sample_values" not in f64:
        return None
    rng = np.random.default_rng(rec["sample_seed"])
    idx = np.sort(rng.choice(len(xs), size=min(rec["nsample"], len(xs)), replace=False))
    xo = np.asarray(f64["sample_values"])
    return {"value": float(np.linalg.norm(xs[idx] - xo) / np.linalg.norm(xo)), "entries": int(len(idx))}


def oracle_cpu_baseline(A, b, restart, rtol, pv, psw, pin, gpu_iterations, np, omega=1.0, gamma=1.0):
    """The oracle (one host thread, as written) on a bounded sample of the
    same float64 solve: its first 4 and first 12 Arnoldi steps, timed apart.
    A step's cost is modelled as c0 + c1 (j + 1) (preconditioner and product,
    plus one Gram-Schmidt pass per basis vector), fitted to the two samples
    and summed over the GPU's steps (cycles of `restart` steps)."""
    import oracle

    k1, k2 = 4, 12
    t = {}
    for k in (k1, k2):
        _, oi = oracle.gmres(A, b, restart=restart, rtol=rtol, maxit=k, prec="gs2", variant=pv, sweeps=psw, inner=pin,
                             omega=omega, gamma=gamma)
        t[k] = oi["seconds"]
    # steps 0..k1-1 and k1..k2-1: mean (j + 1) is (k1 + 1) / 2 and (k1 + k2 + 1) / 2
    m1, m2 = (k1 + 1) / 2.0, (k1 + k2 + 1) / 2.0
    p1, p2 = t[k1] / k1, (t[k2] - t[k1]) / (k2 - k1)
    c1 = max((p2 - p1) / (m2 - m1), 0.0)
    c0 = p1 - c1 * m1
    steps = [j % restart for j in range(gpu_iterations)]
    total = sum(c0 + c1 * (j + 1) for j in steps)
    return {"value": total, "unit": "s", "cores": 1, "kind": "oracle", "host": cpu_model(),
            "sample": f"oracle float64 solve cut at its first {k1} and {k2} Arnoldi steps ({t[k1]:.1f} s, "
                      f"{t[k2]:.1f} s); per-step cost c0 + c1 (j + 1) fitted to them (c0 {c0:.3f} s, c1 "
                      f"{c1 * 1e3:.2f} ms) and summed over the GPU's {gpu_iterations} steps"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2104_01196_amd as g
    from gen import config_problem

    if args.config == 5:
        return bench_batched(args, g, torch, np)
    if args.compare:
        return bench_compare(args, g, torch, np)
    dev = torch.device("cuda:0")
    t0 = time.time()
    cfg = args.config
    size = args.size or {2: 128, 3: 64}.get(cfg, 192)
    p = config_problem(cfg, size=size)
    A, b = p["A"], p["b"]
    log(f"[bench] generated config {cfg}, side {size}: n={A.n} nnz={A.nnz} ({time.time() - t0:.1f}s)")
    # preconditioner: forward GS2(2 sweeps, 1 inner) for the benchmark workload;
    # symmetric GS2(1, 1) for the precision forms (the paper's mixed-precision setting)
    pv, psw, pin = (g.FORWARD, 2, 1) if cfg == 2 else (g.SYMMETRIC, 1, 1)
    # elasticity: SGS2(1 sweep, 3 inner) with damping 0.7 and inner damping 0.5 (undamped inner
    # sweeps stagnate GMRES on this problem, in the oracle as on the GPU)
    omega, gamma = 1.0, 1.0
    if cfg == 3:
        pv, psw, pin, omega, gamma = g.SYMMETRIC, 1, 3, 0.7, 0.5
    dA = g.DeviceCSR.from_host(A, dev)
    db = torch.as_tensor(b, device=dev)
    restart, rtol, maxit = 50, 1e-8, 20000
    if cfg == 2:
        wname = f"laplace3d_{size}"
        workload = f"laplace3d_7pt_{size}^3 GS2-forward(2 sweeps,1 inner) GMRES(50) rtol 1e-8"
    elif cfg == 3:
        wname = f"elasticity_{size}"
        workload = (f"elasticity_q1_27pt_{size}^3nodes_3dof E logU[1,100] nu U[0.2,0.45] SGS2(1 sweep,3 inner) "
                    f"damping 0.7 inner damping 0.5 GMRES(50) rtol 1e-8")
    else:
        wname = f"vardiff3d_{size}"
        workload = f"vardiff3d_7pt_{size}^3 kappa logU[1e-2,1e2] SGS2(1 sweep,1 inner) GMRES(50) rtol 1e-8"

    def solve(h, x):
        x.zero_()
        return g.gmres_solve(dA, db, x, restart, rtol, maxit, g.PREC_GS2, h)

    forms = [("fp64", g.FP64)] + ([] if args.no_forms else [("fp32", g.FP32), ("fp16_scaled", g.FP16_SCALED)])
    results = {}
    x = torch.zeros(A.n, dtype=torch.float64, device=dev)
    x_or, orec = oracle_reference(wname, p["x_true"], np)
    xref = None
    prof = None
    prof_solve_s = None
    for name, prec in forms:
        ts = time.time()
        h = g.gs2_setup(dA, psw, pin, omega, pv, precision=prec, inner_damping=gamma, **forced_schedule(args, name, g))
        torch.cuda.synchronize()
        setup_s = time.time() - ts
        lanes = g.gs2_handle_query(h)["lanes_per_row"]
        sched = g.gs2_handle_schedule(h)
        for _ in range(args.warmup):
            solve(h, x)
        torch.cuda.synchronize()
        headline = name == "fp64"
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        infos, each = [], []
        for _ in range(args.steps):  # gmres_solve synchronises its stream before returning
            te = time.perf_counter()
            infos.append(solve(h, x))
            each.append(time.perf_counter() - te)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        form_prof = None
        if args.profile == "on":
            # the same solves again with every launch bracketed by HIP events on
            # its stream (kernel by kernel: events do not time graph replays)
            g.gs2_profile(True)
            torch.cuda.synchronize()
            tp = time.perf_counter()
            for _ in range(args.steps):
                solve(h, x)
            torch.cuda.synchronize()
            g.gs2_profile(False)
            form_prof = g.gs2_profile_read()
            if headline:
                prof_solve_s = (time.perf_counter() - tp) / args.steps
                prof = form_prof
        xs = x.cpu().numpy()
        if xref is None:
            xref = xs
        info = infos[-1]
        rel = float(np.linalg.norm(b - A.to_scipy() @ xs) / np.linalg.norm(b))
        results[name] = {"time_to_solution_s": dt, "median_s": float(np.median(each)), "min_s": min(each),
                         "max_s": max(each), "iterations": info["iterations"], "restarts": info["restarts"],
                         "converged": info["converged"], "relres_true": rel, "setup_s": setup_s, "lanes_per_row": lanes,
                         "schedule": sched, "gmres_schedule": g.gs2_gmres_schedule(h),
                         "basis_schedule": g.gs2_gmres_basis_schedule(h),
                         "rel_err_vs_oracle_fp64": (float(np.linalg.norm(xs - x_or) / np.linalg.norm(x_or))
                                                    if x_or is not None else None),
                         "rel_err_vs_oracle_fp64_sampled": oracle_sampled_error(orec, xs, np),
                         "oracle_iterations": (orec["solves"][name]["iterations"]
                                               if orec and name in orec["solves"] else None),
                         "rel_err_vs_fp64_gpu_solution": float(np.linalg.norm(xs - xref) / np.linalg.norm(xref)),
                         "rel_err_vs_x_true": float(np.linalg.norm(xs - p["x_true"]) / np.linalg.norm(p["x_true"]))}
        if form_prof:  # the sweep kernels' roofline in this form
            sweep = {}
            for k, r in form_prof.items():
                if k not in ("gs2_prep", "gs2_inner", "gs2_resid", "gs2_first_jr") or not r["bytes"]:
                    continue
                ach = (r["bytes"] / r["launches"]) / ((r["ms"] / r["launches"]) * 1e-3) / 1e9
                sweep[k] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": ach / HBM_PEAK_GBS, "avg_launch_us": r["ms"] / r["launches"] * 1e3,
                            "algorithmic_bytes_per_launch": r["bytes"] / r["launches"],
                            "traffic": traffic_of(k, wname, name)}
            results[name]["sweep_roofline"] = sweep
            apply_ms = sum(form_prof[k]["ms"] for k in sweep) / max(info["iterations"] * args.steps, 1)
            results[name]["precond_us_per_apply"] = apply_ms * 1e3
            log(f"[bench] {name} sweep kernels: " + ", ".join(
                f"{k} {v['achieved']:.0f} GB/s ({100 * v['frac']:.1f}%, {v['avg_launch_us']:.1f} us)"
                for k, v in sweep.items()) + f"; preconditioner {apply_ms * 1e3:.1f} us per apply")
        eo = results[name]["rel_err_vs_oracle_fp64"]
        es = results[name]["rel_err_vs_oracle_fp64_sampled"]
        log(f"[bench] {name}: {dt * 1e3:.2f} ms/solve (median {np.median(each) * 1e3:.2f}, spread "
            f"{min(each) * 1e3:.2f}-{max(each) * 1e3:.2f}), its={info['iterations']} (oracle "
            f"{results[name]['oracle_iterations']}), relres={rel:.2e}, err vs oracle "
            f"{'n/a' if eo is None else f'{eo:.2e}'} (on {es['entries'] if es else 0} sampled entries: "
            f"{'n/a' if es is None else format(es['value'], '.2e')}), setup {setup_s:.2f}s, schedule {sched}")
        del h
    head = results["fp64"]

    # roofline of the dominant kernel (largest summed time in the timed region)
    roof = None
    kernels = {}
    if prof:
        for k, r in prof.items():
            avg_ms = r["ms"] / r["launches"]
            kernels[k] = {"launches": r["launches"], "avg_us": avg_ms * 1e3, "total_ms": r["ms"],
                          "GBps": (r["bytes"] / r["launches"]) / (avg_ms * 1e-3) / 1e9 if r["bytes"] else None}
        dom = max(prof, key=lambda k: prof[k]["ms"])
        r = prof[dom]
        ach = (r["bytes"] / r["launches"]) / ((r["ms"] / r["launches"]) * 1e-3) / 1e9
        traffic = traffic_of(dom, wname, "fp64")
        ceiling = stream_ceiling(torch)
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                "stream_copy_GBps": ceiling, "frac_of_stream_copy": ach / ceiling,
                "algorithmic_bytes_per_launch": r["bytes"] / r["launches"],
                "avg_launch_us": r["ms"] / r["launches"] * 1e3,
                "measured": f"HIP events around every launch in {args.steps} profiled solves (kernel by kernel, "
                            f"{prof_solve_s * 1e3:.2f} ms/solve) after the timed graph-replayed solves"}
        log(f"[bench] dominant kernel {dom}: {ach:.0f} GB/s ({100 * ach / HBM_PEAK_GBS:.1f}% of peak, "
            f"{100 * ach / ceiling:.1f}% of the measured {ceiling:.0f} GB/s copy)")

    comparison = None
    if cfg == 3:
        # Jacobi-Richardson, one sweep, as the paper's comparison on elasticity
        hj = g.gs2_setup(dA, 1, 0, 1.0, g.FORWARD)
        for _ in range(args.warmup):
            x.zero_()
            g.gmres_solve(dA, db, x, restart, rtol, maxit, g.PREC_JR, hj)
        torch.cuda.synchronize()
        each = []
        for _ in range(args.steps):
            x.zero_()
            te = time.perf_counter()
            ij = g.gmres_solve(dA, db, x, restart, rtol, maxit, g.PREC_JR, hj)
            each.append(time.perf_counter() - te)
        comparison = {"jr1": {"time_to_solution_s": float(np.mean(each)), "median_s": float(np.median(each)),
                              "iterations": ij["iterations"], "converged": ij["converged"], "relres": ij["relres"]}}
        log(f"[bench] JR(1): {np.mean(each) * 1e3:.2f} ms/solve, its={ij['iterations']}, relres={ij['relres']:.2e}")
        del hj

    cpu = None
    if not args.no_cpu_baseline:
        cpu = oracle_cpu_baseline(A, b, restart, rtol, pv, psw, pin, head["iterations"], np, omega, gamma)
        log(f"[bench] cpu oracle: {cpu['value']:.1f} s extrapolated ({cpu['sample']})")

    out = {
        "metric": "GS2-GMRES time-to-solution (s) + sweep HBM GB/s, FP64 vs FP32/FP16 precond",
        "value": head["time_to_solution_s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["time_to_solution_s"] * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "n": A.n, "nnz": A.nnz, "restart": restart, "rtol": rtol},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": results,
        "kernels": kernels,
    }
    if comparison:
        out["comparison"] = comparison
    print(json.dumps(out), flush=True)


def traffic_of(kernel, wname, form):
    """HBM bytes per launch of a kernel from the counter record
    profiles/traffic_<kernel>_<workload>[_<form>].json (FETCH_SIZE and
    WRITE_SIZE runs, scaled by a copy kernel's calibration), or None when no
    record exists or it was measured on other kernel sources."""
    for tf in (os.path.join(ROOT, "profiles", f"traffic_{kernel}_{wname}_{form}.json"),
               os.path.join(ROOT, "profiles", f"traffic_{kernel}_{wname}.json") if form == "fp64" else None):
        if tf and os.path.exists(tf):
            rec = json.load(open(tf))
            if rec.get("source_sha256") == source_digest():
                return rec.get("hbm_bytes_per_launch")
            log(f"[bench] {tf} was measured on other kernel sources: traffic reported as null")
            return None
    return None


def cpu_model():
    """The host CPU's model name and logical CPU count, for the baseline records."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name}, {os.cpu_count()} logical CPUs visible"


def bench_compare(args, g, torch, np):
    """GMRES(50) on the 128^3 Laplacian with each preconditioner of the
    paper's comparison: time to solution (graph-replayed), iterations, and
    the preconditioner's share from a profiled pass (events per launch)."""
    from gen import config_problem

    size = args.size or 128
    p = config_problem(2, size=size)
    A, b = p["A"], p["b"]
    dA = g.DeviceCSR.from_host(A)
    db = torch.as_tensor(b, device="cuda")
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    # name, kind, setup (sweeps, inner, damping, variant, build_levels)
    cases = [("GS2-FWD(2,1)", g.PREC_GS2, (2, 1, 1.0, g.FORWARD, False)),
             ("GS2-FWD(2,2)", g.PREC_GS2, (2, 2, 1.0, g.FORWARD, False)),
             ("GS2-FWD(2,3)", g.PREC_GS2, (2, 3, 1.0, g.FORWARD, False)),
             ("SGS2(1,1)", g.PREC_GS2, (1, 1, 1.0, g.SYMMETRIC, False)),
             ("SGS2(2,1)", g.PREC_GS2, (2, 1, 1.0, g.SYMMETRIC, False)),
             ("SGS2(2,2)", g.PREC_GS2, (2, 2, 1.0, g.SYMMETRIC, False)),
             ("JR(3)", g.PREC_JR, (3, 1, 1.0, g.FORWARD, False)),
             ("GS-FWD(2) exact, level-scheduled", g.PREC_GS_TRISOLVE, (2, 1, 1.0, g.FORWARD, True)),
             ("SGS(1) exact, level-scheduled", g.PREC_GS_TRISOLVE, (1, 1, 1.0, g.SYMMETRIC, True)),
             ("MT-GS-FWD(2) multicolor", g.PREC_MTGS, (2, 1, 1.0, g.FORWARD, True)),
             ("none", g.PREC_NONE, None)]
    pre_kinds = ("gs2_prep", "gs2_inner", "gs2_resid", "gs2_first_jr", "trisolve_level")
    res = {}
    for name, kind, cfg in cases:
        h = None
        if cfg:
            sw, inner, w, var, lev = cfg
            h = g.gs2_setup(dA, sw, inner, w, var, build_levels=lev)
        solve = lambda: (x.zero_(), g.gmres_solve(dA, db, x, 50, 1e-8, 20000, kind, h))[1]
        solve()
        torch.cuda.synchronize()
        each = []
        for _ in range(args.steps):
            te = time.perf_counter()
            info = solve()
            each.append(time.perf_counter() - te)
        g.gs2_profile(True)
        solve()
        g.gs2_profile(False)
        prof = g.gs2_profile_read()
        pre_ms = sum(r["ms"] for k, r in prof.items() if k in pre_kinds)
        rel = float(np.linalg.norm(b - A.to_scipy() @ x.cpu().numpy()) / np.linalg.norm(b))
        its = info["iterations"]
        res[name] = {"time_s": float(np.median(each)), "iterations": its, "converged": info["converged"],
                     "relres_true": rel, "precond_ms_per_apply": pre_ms / max(its, 1) if kind != g.PREC_NONE else 0.0}
        log(f"[bench] {name:34s} {res[name]['time_s'] * 1e3:8.2f} ms  its {its:4d}  "
            f"precond {res[name]['precond_ms_per_apply'] * 1e3:8.1f} us/apply  relres {rel:.2e}")
        del h
    out = {"metric": "GS2-GMRES time-to-solution (s) by preconditioner", "value": res["GS2-FWD(2,1)"]["time_s"],
           "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "higher_is_better": False,
           "data": "synthetic", "dtype": "f64",
           "config": {"workload": f"laplace3d_7pt_{size}^3 GMRES(50) rtol 1e-8, preconditioner comparison",
                      "n": A.n, "nnz": A.nnz},
           "preconditioners": res}
    print(json.dumps(out), flush=True)


def bench_batched(args, g, torch, np):
    """Batched form: every (system, right-hand side) pair of the 512-system
    workload in one persistent launch, against the plain FP64 path (one
    gs2_setup per system, one gmres_solve per pair)."""
    from gen import config_problem

    t0 = time.time()
    p = config_problem(5, size=args.size)
    mats, rhs = p["mats"], p["rhs"]
    nrhs, restart, rtol, maxit = rhs[0].shape[1], 20, 1e-8, 20000
    log(f"[bench] generated {len(mats)} systems, {sum(A.n for A in mats)} rows ({time.time() - t0:.1f}s)")
    dm = [g.DeviceCSR.from_host(A) for A in mats]
    B = torch.as_tensor(np.concatenate([r.ravel() for r in rhs]), device="cuda")
    X = torch.zeros_like(B)
    S = [A.to_scipy() for A in mats]

    def check(Xh):
        worst, off = 0.0, 0
        for A, Sa, r in zip(mats, S, rhs):
            x = Xh[off:off + A.n * nrhs].reshape(A.n, nrhs)
            off += A.n * nrhs
            worst = max(worst, float(np.max(np.linalg.norm(r - Sa @ x, axis=0) / np.linalg.norm(r, axis=0))))
        return worst

    res = {}
    for name, prec in (("batched_fp32", g.FP32), ("batched_fp64", g.FP64)):
        ts = time.time()
        bh = g.gs2_setup_batched(dm, sweeps=2, inner=2, precision=prec, restart=restart, nrhs=nrhs)
        torch.cuda.synchronize()
        setup_s = time.time() - ts
        for _ in range(args.warmup):
            X.zero_()
            g.gmres_solve_batched(bh, nrhs, B, X, rtol, maxit)
        each = []
        for _ in range(args.steps):
            X.zero_()
            torch.cuda.synchronize()
            te = time.perf_counter()
            st, infos = g.gmres_solve_batched(bh, nrhs, B, X, rtol, maxit)
            torch.cuda.synchronize()
            each.append(time.perf_counter() - te)
        its = [f["iterations"] for f in infos]
        res[name] = {"time_s": float(np.mean(each)), "median_s": float(np.median(each)), "min_s": min(each),
                     "max_s": max(each), "setup_s": setup_s, "status": st, "iterations": its,
                     "iterations_max": max(its),
                     "iterations_mean": float(np.mean(its)), "worst_relres_true": check(X.cpu().numpy()),
                     "schedule": g.gs2_batched_schedule(bh)}
        log(f"[bench] {name}: {res[name]['time_s'] * 1e3:.1f} ms for all {len(its)} pairs, its mean "
            f"{res[name]['iterations_mean']:.0f} max {max(its)}, worst relres {res[name]['worst_relres_true']:.2e}")
        del bh

    seq = None
    if not args.no_sequential:
        seq = sequential_pairs(g, torch, np, mats, dm, B, nrhs, restart, rtol, maxit, check, res)
    head = res["batched_fp32"]
    cpu = None
    if not args.no_cpu_baseline:
        cpu = batched_cpu_baseline(mats, rhs, res["batched_fp32"]["iterations"], restart, rtol, maxit, np)
    for r in res.values():
        r.pop("iterations", None)
    out = {
        "metric": "GS2-GMRES time-to-solution (s), batched form vs plain FP64 form",
        "value": head["time_s"], "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["time_s"] * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 preconditioner / f64 Krylov", "data": "synthetic",
        "config": {"workload": "512 convdiff2d upwind systems (sides U{16..256}, Pe U(0,50)) x 4 RHS, GS2(2,2) "
                               "FP32 preconditioner, GMRES(20) FP64, rtol 1e-8, one persistent launch",
                   "systems": len(mats), "rows": sum(A.n for A in mats), "nrhs": nrhs},
        "cpu_baseline": cpu,
        "forms": res,
        "speedup_vs_sequential_fp64": seq / head["time_s"] if seq else None,
    }
    print(json.dumps(out), flush=True)


def sequential_pairs(g, torch, np, mats, dm, B, nrhs, restart, rtol, maxit, check, res):
    """The plain FP64 path: one handle per system, one solve per pair
    (per-system b/x buffers so each system's captured restart cycle is
    replayed for all its pairs).  Returns the wall time of all pairs."""
    ts = time.time()
    hs = [g.gs2_setup(d, 2, 2, 1.0, g.FORWARD, precision=g.FP64) for d in dm]
    bb = [torch.empty(A.n, dtype=torch.float64, device="cuda") for A in mats]
    xb = [torch.empty(A.n, dtype=torch.float64, device="cuda") for A in mats]
    torch.cuda.synchronize()
    setup_s = time.time() - ts
    Xs = torch.zeros_like(B)

    def sequential():
        its, off = [], 0
        for i, A in enumerate(mats):
            blk = B[off:off + A.n * nrhs].view(A.n, nrhs)
            out = Xs[off:off + A.n * nrhs].view(A.n, nrhs)
            for r in range(nrhs):
                bb[i].copy_(blk[:, r])
                xb[i].zero_()
                its.append(g.gmres_solve(dm[i], bb[i], xb[i], restart, rtol, maxit, g.PREC_GS2, hs[i])["iterations"])
                out[:, r].copy_(xb[i])
            off += A.n * nrhs
        return its

    sequential()  # warmup: captures each system's cycle graph
    torch.cuda.synchronize()
    te = time.perf_counter()
    its = sequential()
    torch.cuda.synchronize()
    seq = time.perf_counter() - te
    res["sequential_fp64"] = {"time_s": seq, "setup_s": setup_s, "iterations_max": max(its),
                              "iterations_mean": float(np.mean(its)), "worst_relres_true": check(Xs.cpu().numpy())}
    log(f"[bench] sequential_fp64: {seq * 1e3:.1f} ms, its mean {np.mean(its):.0f} max {max(its)}, worst relres "
        f"{res['sequential_fp64']['worst_relres_true']:.2e}")
    return seq


def batched_cpu_baseline(mats, rhs, gpu_its, restart, rtol, maxit, np):
    """The oracle on a bounded sample of the batch: one right-hand side of
    every 16th system (sizes across the whole range), the float32-form GS2(2,2)
    GMRES(20) solves run by host threads at once (each oracle solve is one C
    call, outside the interpreter lock).  Extrapolated to all pairs by rows x
    iterations (the GPU's counts for the pairs not in the sample)."""
    import concurrent.futures as cf

    import oracle

    nrhs = rhs[0].shape[1]
    sample = list(range(0, len(mats), 16))
    threads = max(1, min(16, os.cpu_count() or 1, len(sample)))

    def one(i):
        _, oi = oracle.gmres(mats[i], rhs[i][:, 0], restart=restart, rtol=rtol, maxit=maxit, prec="gs2",
                             sweeps=2, inner=2, precision=oracle.FP32)
        return i, oi["iterations"], oi["seconds"]

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        done = list(ex.map(one, sample))
    wall = time.perf_counter() - t0
    busy = sum(t for *_, t in done)
    work_sample = sum(mats[i].n * its for i, its, _ in done)
    work_all = sum(mats[i].n * gpu_its[i * nrhs + r] for i in range(len(mats)) for r in range(nrhs))
    # the threads kept perfectly busy: the CPU's best case for the whole batch
    value = busy / threads * work_all / max(work_sample, 1)
    log(f"[bench] cpu oracle: {len(sample)} pairs in {wall:.1f}s on {threads} threads "
        f"(thread time {busy:.1f}s) -> {value:.1f} s extrapolated")
    return {"value": value, "unit": "s", "cores": threads, "kind": "oracle", "host": cpu_model(),
            "sample": f"{len(sample)} pairs (right-hand side 0 of every 16th system), {busy:.1f}s of oracle time on "
                      f"{threads} host threads ({wall:.1f}s wall); extrapolated to all {len(mats) * nrhs} pairs by "
                      f"rows x iterations, the threads assumed perfectly busy"}


if __name__ == "__main__":
    main()
