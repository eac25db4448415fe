"""Plain device copy of a known size, used to calibrate HBM byte counters.

Runs `reps` copies of a `mib`-MiB float32 buffer into another with torch's
elementwise copy kernel; a profiler's FETCH_SIZE and WRITE_SIZE for one of
those dispatches, divided by the copied bytes, give the counters' scale.
"""
import argparse
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    import torch
    n = a.mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.reps
    print(f"copy {a.mib} MiB: {ms:.3f} ms per copy, {2 * n * 4 / ms / 1e6:.0f} GB/s (read+write)",
          file=sys.stderr)


if __name__ == "__main__":
    main()
