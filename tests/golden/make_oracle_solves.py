"""Write the stored oracle results for the full-size workloads.

Calls only the CPU oracle (oracle/) and the seeded generators (gen/); nothing
here touches the HIP library.  Each record holds the oracle's GMRES iteration
count, restart count and final true relative residual, plus, for the float64
solve, sampled solution entries and weighted sums that the GPU tests compare
against, and the full solution difference x_oracle - x_true in float32
(a .npy file next to the record, kept out of version control for its size:
x_true is regenerated from the seed, and float32 keeps ~1e-7 of a difference
that is itself small, so the reconstructed x_oracle carries a relative error
far below the differences being measured).  The record stores that file's
sha256 so a stale file is detected.

The orthogonalisation study reruns the float64 solve with classical
Gram-Schmidt applied twice (CGS2) instead of modified Gram-Schmidt: both build
the same Krylov space in exact arithmetic, so the spread between their
iteration counts and solutions (rel_diff_vs_fp64) is the spread the oracle
itself shows under a change of rounding order.

Usage (CPU, minutes per solve at 192^3):
    python tests/golden/make_oracle_solves.py vardiff3d_192 [laplace3d_128] ...
Each workload runs its solves in parallel worker processes.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# workload -> (config, grid side, preconditioner parameters)
WORKLOADS = {
    # 192^3 variable-coefficient diffusion, SGS2(1,1), GMRES(50): the precision-form workload
    "vardiff3d_192": dict(config=4, size=192, variant=2, sweeps=1, inner=1, restart=50),
    # 128^3 Laplacian, forward GS2(2 sweeps, 1 inner), GMRES(50)
    "laplace3d_128": dict(config=2, size=128, variant=0, sweeps=2, inner=1, restart=50),
    # Q1 elasticity on 64^3 free nodes, SGS2(1 sweep, 3 inner) with damping 0.7 and inner damping 0.5,
    # GMRES(50), in the three preconditioner forms
    "elasticity_64": dict(config=3, size=64, variant=2, sweeps=1, inner=3, omega=0.7, gamma=0.5, restart=50),
}
RTOL = 1e-8
MAXIT = 20000
NSAMPLE = 4096  # sampled solution entries
NWEIGHT = 4  # weighted sums with seeded N(0,1) weights
SAMPLE_SEED = 7


def sample_plan(n: int):
    """Seeded row indices and weight vectors shared by the record and the tests."""
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = np.sort(rng.choice(n, size=min(NSAMPLE, n), replace=False))
    return idx, rng


def weights(n: int, rng):
    return [rng.standard_normal(n) for _ in range(NWEIGHT)]


def _solve(args):
    name, precision, cgs2 = args
    import oracle
    from gen import config_problem

    w = WORKLOADS[name]
    p = config_problem(w["config"], size=w["size"])
    x, info = oracle.gmres(p["A"], p["b"], restart=w["restart"], rtol=RTOL, maxit=MAXIT, prec="gs2",
                           variant=w["variant"], sweeps=w["sweeps"], inner=w["inner"], omega=w.get("omega", 1.0),
                           gamma=w.get("gamma", 1.0), precision=precision, cgs2=cgs2)
    out = {k: info[k] for k in ("iterations", "restarts", "relres", "converged", "status", "seconds")}
    if precision == 0:
        xt = p["x_true"]
        d = (x - xt).astype(np.float32)
        path = os.path.join(HERE, f"{name}_oracle{'_cgs2' if cgs2 else ''}_dx.npy")
        np.save(path, d)
        out["dx_file"] = os.path.basename(path)
        out["dx_sha256"] = hashlib.sha256(open(path, "rb").read()).hexdigest()
    if precision == 0 and not cgs2:
        out["x_norm"] = float(np.linalg.norm(x))
        out["rel_err_vs_x_true"] = float(np.linalg.norm(x - xt) / np.linalg.norm(xt))
        idx, rng = sample_plan(len(x))
        out["sample_idx_count"] = int(len(idx))
        out["sample_values"] = [float(v) for v in x[idx]]
        out["weighted_sums"] = [float(wk @ x) for wk in weights(len(x), rng)]
    return name, precision, cgs2, out


def main(names):
    jobs = []
    for name in names:
        for precision in WORKLOADS[name].get("precisions", (0, 1, 2)):
            jobs.append((name, precision, False))
        jobs.append((name, 0, True))
    results = {}
    with ProcessPoolExecutor(max_workers=min(4, len(jobs))) as ex:
        for name, precision, cgs2, out in ex.map(_solve, jobs):
            key = {0: "fp64", 1: "fp32", 2: "fp16_scaled"}[precision] + ("_cgs2" if cgs2 else "")
            results.setdefault(name, {})[key] = out
            print(f"{name} {key}: {out['iterations']} its, relres {out['relres']:.3e}, {out['seconds']:.0f} s",
                  flush=True)
    for name, recs in results.items():
        w = WORKLOADS[name]
        # how far the two orthogonalisations' float64 solutions lie apart
        from gen import config_problem

        xt = config_problem(w["config"], size=w["size"])["x_true"]
        xm = xt + np.load(os.path.join(HERE, recs["fp64"]["dx_file"])).astype(np.float64)
        xc = xt + np.load(os.path.join(HERE, recs["fp64_cgs2"]["dx_file"])).astype(np.float64)
        recs["fp64_cgs2"]["rel_diff_vs_fp64"] = float(np.linalg.norm(xc - xm) / np.linalg.norm(xm))
        rec = {"workload": name, **{k: v for k, v in w.items() if k != "precisions"}, "rtol": RTOL, "solves": recs,
               "sample_seed": SAMPLE_SEED, "nsample": NSAMPLE, "nweight": NWEIGHT,
               "written_by": "tests/golden/make_oracle_solves.py (CPU oracle only)"}
        with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or ["vardiff3d_192"])
