"""Plain device-to-device copy of a known size, the reference for turning
rocprofv3 FETCH_SIZE / WRITE_SIZE counters into HBM bytes.

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2008_02478_amd.calibrate
copies `--mib` MiB (default 256) `--reps` times with torch's copy kernel; the
counter per dispatch divided by the copy size gives the scale factor.
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=256)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(a.reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps} (read {a.mib} MiB + write {a.mib} MiB per dispatch)", flush=True)


if __name__ == "__main__":
    main()
