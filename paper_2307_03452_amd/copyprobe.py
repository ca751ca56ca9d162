"""Plain device copy of a known size, used to calibrate HBM byte counters.

    python -m paper_2307_03452_amd.copyprobe [--mib 1024] [--reps 3]

Runs `dst = src + 0.0` on float64 tensors of --mib MiB: one elementwise kernel
that reads and writes exactly that many bytes.  The FETCH_SIZE and WRITE_SIZE
counters of this kernel, divided by its known bytes, give the scale factor
applied to the counters of the integral kernel.
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        torch.add(src, 0.0, out=dst)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}", flush=True)


if __name__ == "__main__":
    main()
