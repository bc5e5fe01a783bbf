#!/usr/bin/env python3
"""HBM reference streams beside the lattice sweep (measurement only).

Times plain device copies of a known size: PyTorch's copy kernel and the
hand-written 16-byte copies of copy_probe.hip (grid-stride and one workgroup
per 16 KiB chunk, each with plain and with non-temporal loads and stores),
plus a read-only and a write-only stream.  The best read-plus-write rate is
the bandwidth a stream that reads and writes the same number of bytes (the
sweep: 36 B read and 36 B written per node in FP32) can reach on this part;
bench.py reports the sweep's rate against it beside the datasheet peak.

Under `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE`, `--torch-only`
gives the calibration copy of the HBM byte counters.

    python copy_probe.py [--mib 1024] [--reps 20] [--torch-only]
"""
import argparse
import ctypes
import json
import os
import subprocess

ROOT = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(ROOT, "copy_probe.hip")
LIB = os.path.join(ROOT, "libcopy_probe.so")
VARIANTS = {0: "copy16_loop", 1: "copy16_loop_nt", 2: "copy16_chunk", 3: "copy16_chunk_nt", 4: "read16_nt",
            5: "write16_nt"}


def build():
    """Compile copy_probe.hip for gfx950 (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", SRC, "-o", tmp]
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + proc.stdout)
    os.replace(tmp, LIB)
    return LIB


def _lib():
    import torch  # noqa: F401  (one HIP runtime for torch and the probe)
    if not os.path.exists(LIB):
        raise RuntimeError("libcopy_probe.so is not built; run copy_probe.build()")
    L = ctypes.CDLL(LIB)
    L.copy_probe_launch.restype = ctypes.c_int
    L.copy_probe_launch.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_void_p]
    return L


def _time(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def measure(mib=1024, reps=20, grids=(1024, 2048, 4096, 8192), torch_only=False):
    """Rates (GB/s, bytes moved per second counting reads and writes) of each
    stream; 'best_copy_gbs' is the fastest read-plus-write copy."""
    import torch
    n = mib * (1 << 20)
    x = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    out = {"mib": mib, "reps": reps}
    ms = _time(lambda: y.copy_(x), reps, torch)
    out["torch_copy_gbs"] = 2 * n / (ms * 1e-3) / 1e9
    if torch_only:
        return out
    L = _lib()
    scratch = torch.empty(max(grids) * 4, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rates = {}
    for v, name in VARIANTS.items():
        for g in (grids if v in (0, 1, 4, 5) else (0,)):
            def run():
                rc = L.copy_probe_launch(v, y.data_ptr(), x.data_ptr(), n, max(g, 1), scratch.data_ptr(), st)
                if rc != 0:
                    raise RuntimeError("copy_probe_launch(%d) returned %d" % (v, rc))
            t = _time(run, reps, torch)
            moved = n if v in (4, 5) else 2 * n
            rates["%s%s" % (name, "_g%d" % g if g else "")] = moved / (t * 1e-3) / 1e9
    out["rates_gbs"] = {k: round(r, 1) for k, r in rates.items()}
    copies = {k: r for k, r in rates.items() if k.startswith("copy")}
    best = max(copies, key=copies.get)
    out["best_copy"] = best
    out["best_copy_gbs"] = round(copies[best], 1)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--torch-only", action="store_true")
    args = ap.parse_args()
    print(json.dumps(measure(args.mib, args.reps, torch_only=args.torch_only)), flush=True)


if __name__ == "__main__":
    main()
