"""Plain device-to-device copy of a known size (PyTorch's copy kernel).

Used under `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` to calibrate the
HBM byte counters: the counters read for this copy, divided into the bytes it
must move (size read + size written), give the factor that converts the
counter values of the lattice kernels into bytes.
"""
import argparse
import json

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    n = args.mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.reps
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "reps": args.reps,
                      "ms_per_copy": ms, "gbs_read_plus_write": 2 * n * 4 / (ms * 1e-3) / 1e9}))


if __name__ == "__main__":
    main()
