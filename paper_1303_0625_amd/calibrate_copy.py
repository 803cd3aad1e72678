"""Plain device copy of a known size, for calibrating HBM traffic counters.

Run under ``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``): the counters
read for this copy of ``--mib`` MiB in and out give the scale from counter
units to bytes that ``pmc_summary`` applies to the lattice kernels.
"""
from __future__ import annotations

import argparse

import torch


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--repeat", type=int, default=3)
    args = ap.parse_args()
    n = args.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.repeat):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {args.mib} MiB x {args.repeat}", flush=True)


if __name__ == "__main__":
    main()
