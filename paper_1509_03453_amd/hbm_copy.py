"""Plain device-to-device copy of a known size, for calibrating HBM byte counters.

``python -m paper_1509_03453_amd.hbm_copy [--mib 2048] [--reps 3]`` copies a
buffer of the given size with torch's copy kernel; a profiler's fetch and
write byte counters for that kernel, divided into the known size, give the
factor that turns the same counters for the search kernels into bytes.
"""
from __future__ import annotations

import argparse
import json
import time

import torch


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=2048)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    n = args.mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.reps
    print(json.dumps({"bytes_per_copy": n, "reps": args.reps, "ms_per_copy": round(dt * 1e3, 3),
                      "GBps_read_plus_write": round(2 * n / dt / 1e9, 1)}), flush=True)


if __name__ == "__main__":
    main()
