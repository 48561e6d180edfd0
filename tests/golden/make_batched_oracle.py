"""Write the stored oracle results for the full batched workload: 512
upwinded convection-diffusion systems (sides U{16..256}, Peclet U(0,50)) x 4
right-hand sides, GS2 (2 sweeps, 2 inner) with the float32 preconditioner
form, GMRES(20) to 1e-8 from x = 0.

Calls only the CPU oracle (oracle/) and the seeded generators (gen/).  Every
(system, right-hand side) pair is solved twice, with modified Gram-Schmidt
(the oracle's default) and with classical Gram-Schmidt applied twice (CGS2):
both build the same Krylov space in exact arithmetic, so the difference of
their iteration counts shows how far rounding order alone moves the count of
each pair (the spread a GPU solve, which orthogonalises in yet another
order, can be held to).  Per pair: both iteration counts, the final true
relative residual, ||x|| and x . w with w_i = sin(i + 1) (a fixed weight
vector, no random draw).

Usage (CPU; a few minutes on 8 cores):
    python tests/golden/make_batched_oracle.py [--workers N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

SWEEPS, INNER, RESTART, RTOL, MAXIT = 2, 2, 20, 1e-8, 20000
_P = None


def _problem():
    global _P
    if _P is None:
        from gen import config_problem

        _P = config_problem(5)
    return _P


def _solve(pair):
    import oracle

    i, r = pair
    p = _problem()
    A, b = p["mats"][i], p["rhs"][i][:, r]
    out = {"system": i, "rhs": r, "n": int(A.n)}
    for name, cgs2 in (("mgs", False), ("cgs2", True)):
        x, info = oracle.gmres(A, b, restart=RESTART, rtol=RTOL, maxit=MAXIT, prec="gs2", sweeps=SWEEPS, inner=INNER,
                               precision=oracle.FP32, cgs2=cgs2)
        out[f"iterations_{name}"] = info["iterations"]
        out[f"converged_{name}"] = bool(info["converged"])
        if name == "mgs":
            w = np.sin(np.arange(1, A.n + 1, dtype=np.float64))
            out["relres"] = info["relres"]
            out["x_norm"] = float(np.linalg.norm(x))
            out["x_dot_w"] = float(x @ w)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    p = _problem()
    nrhs = p["rhs"][0].shape[1]
    pairs = [(i, r) for i in range(len(p["mats"])) for r in range(nrhs)]
    # largest systems first, so the pool's tail is short
    pairs.sort(key=lambda q: -p["mats"][q[0]].n)
    with ProcessPoolExecutor(max_workers=args.workers) as ex:
        res = list(ex.map(_solve, pairs, chunksize=1))
    res.sort(key=lambda o: (o["system"], o["rhs"]))
    d = np.array([o["iterations_cgs2"] - o["iterations_mgs"] for o in res])
    rec = {"workload": "convdiff512x4", "sweeps": SWEEPS, "inner": INNER, "restart": RESTART, "rtol": RTOL,
           "precision": "fp32", "pairs": res,
           "mgs_vs_cgs2": {"max_abs_diff": int(np.abs(d).max()), "pairs_diff_gt_1": int((np.abs(d) > 1).sum()),
                           "pairs": len(res)},
           "written_by": "tests/golden/make_batched_oracle.py (CPU oracle only)"}
    with open(os.path.join(HERE, "convdiff512x4_oracle.json"), "w") as f:
        json.dump(rec, f, indent=0)
        f.write("\n")
    print(json.dumps(rec["mgs_vs_cgs2"]))


if __name__ == "__main__":
    main()
