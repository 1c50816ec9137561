"""Plain device-to-device copy of a known size, for calibrating HBM byte
counters (FETCH_SIZE / WRITE_SIZE) against a kernel whose traffic is exact.

    python -m paper_1810_12707_amd.copy_probe [--mib 1024] [--reps 3]
"""
import argparse
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args(argv)
    import torch

    n = a.mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(a.reps):
        y.copy_(x)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / a.reps
    print(f"copy {a.mib} MiB: {ms:.4f} ms, {2 * a.mib * (1 << 20) / (ms * 1e-3) / 1e9:.1f} GB/s (read+write)",
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
