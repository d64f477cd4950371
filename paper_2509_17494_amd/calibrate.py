"""Device copy of a known size, used to calibrate rocprofv3's FETCH_SIZE and
WRITE_SIZE counters (KiB per dispatch) against true HBM bytes.

Usage: python -m paper_2509_17494_amd.calibrate [--mib 1024] [--reps 3]
Each repetition copies --mib MiB from one device buffer to another (a plain
streaming copy: reads and writes the same number of bytes once).
"""
from __future__ import annotations

import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(a.reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}: {a.mib * 1024} KiB read and written per dispatch",
          flush=True)


if __name__ == "__main__":
    main()
