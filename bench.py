"""Benchmark: GS2-preconditioned GMRES time to solution on one MI355X.

Workload (default): 3D 7-point Dirichlet Laplacian on a 128^3 grid
(n = 2,097,152, nnz = 14,581,760), CSR float64 in natural ordering,
b = A x_true with x_true ~ N(0,1) from a fixed seed, x0 = 0.
GMRES(50) to ||b - A x|| / ||b|| <= 1e-8, right-preconditioned by forward GS2
with 2 outer sweeps and 1 inner Jacobi-Richardson sweep (damping 1.0).
One "step" is one complete solve (the whole preconditioned Krylov path:
setup excluded, done once before timing).  `value` is the mean time to
solution of the float64-preconditioner solve over the timed steps (median and
spread reported with it); the float32 and scaled-float16 preconditioner
solves are timed the same way and reported next to it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--size 128]
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
    ap.add_argument("--size", type=int, default=128, help="grid side of the 3D Laplacian")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the float32 / float16 preconditioner solves")
    ap.add_argument("--profile", choices=["on", "off"], default="on",
                    help="per-kernel HIP-event timing of the float64 solves (a second pass of the same solves)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2104_01196_amd as g
    from gen import config_problem

    dev = torch.device("cuda:0")
    t0 = time.time()
    p = config_problem(2, size=args.size)
    A, b = p["A"], p["b"]
    log(f"[bench] generated laplace3d {args.size}^3: n={A.n} nnz={A.nnz} ({time.time() - t0:.1f}s)")
    dA = g.DeviceCSR.from_host(A, dev)
    db = torch.as_tensor(b, device=dev)
    restart, rtol, maxit = 50, 1e-8, 20000

    def solve(h, x):
        x.zero_()
        return g.gmres_solve(dA, db, x, restart, rtol, maxit, g.PREC_GS2, h)

    forms = [("fp64", g.FP64)] + ([] if args.no_forms else [("fp32", g.FP32), ("fp16_scaled", g.FP16_SCALED)])
    results = {}
    x = torch.zeros(A.n, dtype=torch.float64, device=dev)
    xref = None
    prof = None
    prof_solve_s = None
    for name, prec in forms:
        ts = time.time()
        h = g.gs2_setup(dA, 2, 1, 1.0, g.FORWARD, precision=prec)
        torch.cuda.synchronize()
        setup_s = time.time() - ts
        lanes = g.gs2_handle_query(h)["lanes_per_row"]
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
        if headline and args.profile == "on":
            # the same solves again with every launch bracketed by HIP events on
            # its stream (kernel by kernel: events do not time graph replays)
            g.gs2_profile(True)
            torch.cuda.synchronize()
            tp = time.perf_counter()
            for _ in range(args.steps):
                solve(h, x)
            torch.cuda.synchronize()
            prof_solve_s = (time.perf_counter() - tp) / args.steps
            g.gs2_profile(False)
            prof = g.gs2_profile_read()
        xs = x.cpu().numpy()
        if xref is None:
            xref = xs
        info = infos[-1]
        rel = float(np.linalg.norm(b - A.to_scipy() @ xs) / np.linalg.norm(b))
        results[name] = {"time_to_solution_s": dt, "median_s": float(np.median(each)), "min_s": min(each),
                         "max_s": max(each), "iterations": info["iterations"], "restarts": info["restarts"],
                         "converged": info["converged"], "relres_true": rel, "setup_s": setup_s, "lanes_per_row": lanes,
                         "rel_err_vs_fp64_solution": float(np.linalg.norm(xs - xref) / np.linalg.norm(xref)),
                         "rel_err_vs_x_true": float(np.linalg.norm(xs - p["x_true"]) / np.linalg.norm(p["x_true"]))}
        log(f"[bench] {name}: {dt * 1e3:.2f} ms/solve (median {np.median(each) * 1e3:.2f}, spread "
            f"{min(each) * 1e3:.2f}-{max(each) * 1e3:.2f}), its={info['iterations']}, relres={rel:.2e}, "
            f"setup {setup_s:.2f}s, {lanes} lanes/row")
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
        traffic = None
        tf = os.path.join(ROOT, "profiles", f"traffic_{dom}_laplace3d_{args.size}.json")
        if os.path.exists(tf):
            traffic = json.load(open(tf)).get("hbm_bytes_per_launch")
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

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        nthreads = 1
        sample_steps = restart
        _, oi = oracle.gmres(A, b, restart=restart, rtol=rtol, maxit=sample_steps, prec="gs2",
                             variant=oracle.FORWARD, sweeps=2, inner=1)
        per_step = oi["seconds"] / max(oi["iterations"], 1)
        cpu = {"value": per_step * head["iterations"], "unit": "s", "cores": nthreads, "kind": "oracle",
               "sample": f"first GMRES(50) cycle ({oi['iterations']} Arnoldi steps, {oi['seconds']:.1f}s) of the "
                         f"same float64 solve, extrapolated to the GPU's {head['iterations']} iterations"}
        log(f"[bench] cpu oracle: {per_step:.3f} s/step -> {cpu['value']:.1f} s extrapolated")

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
        "config": {"workload": f"laplace3d_7pt_{args.size}^3 GS2-forward(2 sweeps,1 inner) GMRES(50) rtol 1e-8",
                   "n": A.n, "nnz": A.nnz, "restart": restart, "rtol": rtol},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": results,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
