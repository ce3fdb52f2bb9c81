#!/usr/bin/env python3
"""Throughput of the MOFF imaging hot path on one MI355X.

One step = one epic_image_accumulate over the whole LWA-like workload: 256
dual-polarisation antennas, 132 channels, a 64 x 64 grid and 1000 samples per
channel, giving 132 accumulated 4-polarisation channel images.  Inputs are
synthetic (seeded) and resident in HBM before the timed region.

Prints one JSON line.  `value` is channel-images/s of the fused kernel path;
the plain float32 staged path (one kernel per stage, intermediates in HBM) is
reported beside it, and the FP64 CPU oracle is timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "channel-images/s (4-pol, 64² grid) vs plain FP32; % HBM/MFMA roofline"
PEAK_FP32_VALU = 157.3e12       # MI355X fp32 vector, FLOP/s
PEAK_HBM = 8.0e12               # MI355X HBM3E, B/s


def flops_per_tc(N: int, P: int, A: int, K: int = 3) -> int:
    """Algorithmic float work of one (time, channel) image.

    transform: 5 n_g log2 n_g per polarisation (radix-2 count of a complex FFT)
    gridding:  4 flops (complex x real weight, add) per tap per antenna per pol
    gain:      6 flops per complex multiply per antenna per pol
    products:  XX 3, YY 3, XY 6 and 4 accumulating adds per pixel (P = 2);
               XX 3 + 1 add (P = 1)
    """
    ng = N * N
    fft = P * 5 * ng * int(round(math.log2(ng)))
    grid = 4 * K * K * P * A
    gain = 6 * P * A
    prod = 16 * ng if P == 2 else 4 * ng
    return fft + grid + gain + prod


def cpu_baseline(inp, n_chan: int):
    """The FP64 oracle as it stands, on the first n_chan channels, all samples."""
    import oracle
    import synth
    sub = synth.Inputs(inp.grid_n, n_chan, inp.n_pol, inp.n_ant, inp.kernel_support,
                       inp.kernel_sigma_cells, inp.cell_wavelengths, inp.xy_m,
                       inp.freq_hz[:n_chan], inp.gains[:n_chan],
                       np.ascontiguousarray(inp.efield[:, :n_chan]))
    t0 = time.perf_counter()
    oracle.image_from(sub)
    dt = time.perf_counter() - t0
    return {"value": n_chan / dt, "unit": "channel-images/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_chan} of {inp.n_chan} channels x all {inp.n_time} samples "
                      f"({dt:.1f} s, numpy float64, one thread)",
            "tc_images_per_s": n_chan * inp.n_time / dt}


def copy_calibration(mib: int) -> int:
    """A device-to-device copy of known size: its profiler counters read
    mib MiB fetched and mib MiB written per dispatch when the counters are exact."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "bytes_read_per_copy": n * 4, "bytes_written_per_copy": n * 4}))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-channels", type=int, default=16,
                    help="channels of the workload the CPU oracle is timed on")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-staged", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (five times), to "
                         "scale the FETCH_SIZE / WRITE_SIZE counters of a profiler run")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the imager shards by channel with no communication; see the design notes)",
              file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_1904_11422_amd import Imager

    print("bench: generating the LWA-like workload", file=sys.stderr, flush=True)
    inp = synth.config2()
    N, C, P, A, T = inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.n_time
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ef = torch.from_numpy(inp.efield).to(dev)
    g = torch.from_numpy(inp.gains).to(dev)

    im = Imager(N, C, P, A, timing=True)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    img = torch.empty(im.image_shape(), dtype=torch.complex128, device=dev)
    for _ in range(args.warmup):
        im.accumulate(ef, g, image=img, reset=True)
    torch.cuda.synchronize()
    print("bench: timing the fused path", file=sys.stderr, flush=True)

    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        im.accumulate(ef, g, image=img, reset=True)
        kernel_ms.append(im.last_timing()[0])      # HIP events around the main kernel
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = C * args.steps / dt
    kname = im.last_kernel_name()

    k_ms = float(np.mean(kernel_ms))
    fl = flops_per_tc(N, P, A) * C * T
    achieved = fl / (k_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU, "traffic": None,
                "kernel": kname, "kernel_ms": k_ms,
                "flops_per_launch": fl, "flops_per_tc_image": flops_per_tc(N, P, A)}
    im.close()

    staged = None
    if not args.no_staged:
        print("bench: timing the plain staged path", file=sys.stderr, flush=True)
        ims = Imager(N, C, P, A, staged=True, timing=True)
        ims.set_antennas(inp.xy_m, inp.freq_hz)
        ims.accumulate(ef, g, image=img, reset=True)
        torch.cuda.synchronize()
        n_st = max(2, args.steps // 5)
        t1 = time.perf_counter()
        for _ in range(n_st):
            ims.accumulate(ef, g, image=img, reset=True)
        torch.cuda.synchronize()
        dts = time.perf_counter() - t1
        staged = {"value": C * n_st / dts, "unit": "channel-images/s",
                  "ms_per_step": dts * 1e3 / n_st, "steps": n_st,
                  "speedup_of_fused": value / (C * n_st / dts)}
        ims.close()

    cpu = None
    if not args.no_cpu:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(inp, args.cpu_channels)

    out = {
        "metric": METRIC, "value": value, "unit": "channel-images/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "LWA-like: 256 dual-pol antennas, 132 x 25 kHz channels at "
                               "38 MHz, 64x64 grid at lambda/2, 3x3 Gaussian kernel, "
                               "1000 samples per channel image",
                   "grid_n": N, "n_chan": C, "n_pol": P, "n_ant": A, "n_time": T,
                   "accumulate": "f64"},
        "tc_images_per_s": value * T,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain_fp32_staged": staged,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
