"""Known-size copy for calibrating HBM byte counters.

Runs `reps` device-to-device copies of a `mib`-MiB float32 buffer (one read
and one write of `mib` MiB each), so that FETCH_SIZE / WRITE_SIZE read by
`rocprofv3 --pmc` for this copy kernel can be compared with the exact byte
count.  The ratio scales the counters read for the library's kernels.

Usage: python -m paper_2104_01196_amd.calibrate [--mib 1024] [--reps 3]
"""
from __future__ import annotations

import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    import torch

    n = a.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": a.reps}))


if __name__ == "__main__":
    main()
