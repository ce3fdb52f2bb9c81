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
PEAK_FP32_VALU = 157.3e12       # MI355X fp32 vector, FLOP/s (counts packed FP32)
PEAK_FP32_VALU_NONPACKED = PEAK_FP32_VALU / 2   # the issue ceiling with packed FP32 off
PEAK_HBM = 8.0e12               # MI355X HBM3E, B/s


def flops_per_tc(N: int, P: int, A: int, K: int = 3, complex_kernel: bool = False) -> int:
    """Algorithmic float work of one (time, channel) image.

    transform: 5 n_g log2 n_g per polarisation (radix-2 count of a complex FFT)
    gridding:  4 flops (complex x real weight, add) per tap per antenna per pol,
               8 with a complex kernel (complex multiply-add)
    gain:      6 flops per complex multiply per antenna per pol
    products:  XX 3, YY 3, XY 6 and 4 accumulating adds per pixel (P = 2);
               XX 3 + 1 add (P = 1)
    """
    ng = N * N
    fft = P * 5 * ng * int(round(math.log2(ng)))
    grid = (8 if complex_kernel else 4) * K * K * P * A
    gain = 6 * P * A
    prod = 16 * ng if P == 2 else 4 * ng
    return fft + grid + gain + prod


def _oracle_channel(job):
    """One channel through the oracle in a worker process; returns its seconds."""
    import oracle
    t0 = time.perf_counter()
    oracle.image(*job)
    return time.perf_counter() - t0


def _worker_ready(_):
    import oracle  # noqa: F401  (the import is the warm-up)
    time.sleep(0.2)
    return os.getpid()


def host_cpu() -> dict:
    """What the host offers: logical CPUs the OS reports, those this process
    may run on, and the processor model (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable": usable, "model": model}


# worker processes for the CPU baseline: the machine's CPU share per GPU (the
# host may report more logical CPUs than one GPU's share)
CPU_SHARE = 16


def cpu_baseline(inp, n_chan: int, max_workers: int = CPU_SHARE):
    """The FP64 oracle as it stands, on the first n_chan channels, all samples:
    once in this process (one thread: numpy's FFT and the oracle's array code
    are single-threaded), and once with one spawned process per channel on up
    to max_workers cores (BLAS/OpenMP threads 1; the workers are started and
    have imported the oracle before the clock starts)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import oracle
    import synth
    sub = synth.Inputs(inp.grid_n, n_chan, inp.n_pol, inp.n_ant, inp.kernel_support,
                       inp.kernel_sigma_cells, inp.cell_wavelengths, inp.xy_m,
                       inp.freq_hz[:n_chan], inp.gains[:n_chan],
                       np.ascontiguousarray(inp.efield[:, :n_chan]))
    t0 = time.perf_counter()
    oracle.image_from(sub)
    dt1 = time.perf_counter() - t0
    one = {"value": n_chan / dt1, "unit": "channel-images/s", "cores": 1,
           "tc_images_per_s": n_chan * inp.n_time / dt1, "seconds": dt1}
    workers = max(1, min(max_workers, n_chan, os.cpu_count() or 1))
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    jobs = [(inp.xy_m, inp.freq_hz[c:c + 1], inp.gains[c:c + 1],
             np.ascontiguousarray(inp.efield[:, c:c + 1]), inp.grid_n, inp.kernel_support,
             inp.kernel_sigma_cells, inp.cell_wavelengths) for c in range(n_chan)]
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as pool:
        pids = set(pool.map(_worker_ready, range(workers)))
        t0 = time.perf_counter()
        list(pool.map(_oracle_channel, jobs))
        dtn = time.perf_counter() - t0
    return {"value": n_chan / dtn, "unit": "channel-images/s", "cores": workers, "kind": "oracle",
            "host": host_cpu(),
            "sample": f"{n_chan} of {inp.n_chan} channels x all {inp.n_time} samples, one "
                      f"process per channel on {workers} cores ({len(pids)} workers started): "
                      f"{dtn:.2f} s; the same sample in one thread: {dt1:.1f} s "
                      f"(numpy float64); workers capped at the per-GPU CPU share of "
                      f"{max_workers}",
            "tc_images_per_s": n_chan * inp.n_time / dtn, "one_core": one}


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


def batch_results(steps: int, warmup: int, sequential: bool = True) -> dict:
    """Six blocks of different (N, A, C) advanced together: autotuned launch
    shapes, one HIP graph replay per step."""
    import tempfile
    import torch
    import synth
    from paper_1904_11422_amd import Batch
    print("bench: generating the heterogeneous batch", file=sys.stderr, flush=True)
    inputs = [synth.config4_block(b) for b in range(len(synth.CONFIG4_BLOCKS))]
    T = inputs[0].n_time
    b = Batch([dict(grid_n=i.grid_n, n_chan=i.n_chan, n_pol=i.n_pol, n_ant=i.n_ant) for i in inputs])
    for k, i in enumerate(inputs):
        b.set_antennas(k, i.xy_m, i.freq_hz)
    ef = [torch.from_numpy(i.efield).cuda() for i in inputs]
    g = [torch.from_numpy(i.gains).cuda() for i in inputs]
    imgs = b.new_images()
    cache = os.path.join(tempfile.gettempdir(), "epic_batch_plans.txt")
    print("bench: tuning and capturing the batch", file=sys.stderr, flush=True)
    b.tune(ef, g, imgs, cache)
    b.capture(ef, g, imgs)
    for _ in range(warmup):
        b.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    tc = sum(i.n_chan for i in inputs) * T
    fl = sum(flops_per_tc(i.grid_n, i.n_pol, i.n_ant) * i.n_chan * T for i in inputs)
    out = {"value": tc / dt, "unit": "(t,c)-images/s", "ms_per_step": dt * 1e3, "steps": steps,
           "channel_images_per_s": sum(i.n_chan for i in inputs) / dt,
           "blocks": [dict(grid_n=i.grid_n, n_ant=i.n_ant, n_chan=i.n_chan, grid=p[0],
                           staged_batch=p[1], launch=lp[0], launch_blocks=lp[1], team=lp[2],
                           kblock=lp[3], xcd=lp[4])
                      for i, p, lp in zip(inputs, b.plan(), b.launch_plan())],
           "serial": b.serial,
           "roofline": {"bound": "alu", "kernel": "whole batch (graph replay, wall clock)",
                        "achieved": fl / dt / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                        "unit": "TFLOP/s", "frac": fl / dt / PEAK_FP32_VALU,
                        "frac_nonpacked": fl / dt / PEAK_FP32_VALU_NONPACKED,
                        "flops_per_step": fl},
           "n_time": T}
    if sequential:
        # the same batch, one block after another, no graph, default launch shapes
        from paper_1904_11422_amd import Imager
        ims = []
        for i in inputs:
            im = Imager(i.grid_n, i.n_chan, i.n_pol, i.n_ant)
            im.set_antennas(i.xy_m, i.freq_hz)
            ims.append(im)
        seq = [ims[k].accumulate(ef[k], g[k]) for k in range(len(inputs))]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            for k in range(len(inputs)):
                ims[k].accumulate(ef[k], g[k], image=seq[k])
        torch.cuda.synchronize()
        out["sequential_no_graph_ms"] = (time.perf_counter() - t1) / steps * 1e3
        for im in ims:
            im.close()
    b.close()
    return out


def bench_batch(args) -> int:
    r = batch_results(args.steps, args.warmup)
    out = {"metric": "heterogeneous batch (t,c)-images/s", **r, "data": "synthetic"}
    print(json.dumps(out))
    return 0


PEAK_MFMA_F16 = 2.5e15          # MI355X dense fp16 / bf16 MFMA, FLOP/s


def split_results(steps: int, with_oracle: bool = True) -> dict:
    """16 antennas, one channel, 32x32 grid, 10^5 samples: the float32 fused
    path and the float16 / bfloat16 hi+lo matrix forms on the same input."""
    import torch
    import oracle
    import synth
    from paper_1904_11422_amd import Imager
    print("bench: generating the long tiny-geometry integration", file=sys.stderr, flush=True)
    inp = synth.config3()
    T, N, A, P = inp.n_time, inp.grid_n, inp.n_ant, inp.n_pol
    ef = torch.from_numpy(inp.efield).cuda()
    g = torch.from_numpy(inp.gains).cuda()
    ref, t_oracle = None, None
    if with_oracle:
        print("bench: FP64 oracle over all samples", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        ref = oracle.image_from(inp)
        t_oracle = time.perf_counter() - t0
    res = {}
    for prec in ("fp32", "split_fp16", "split_bf16"):
        im = Imager(N, 1, P, A, precision=prec, timing=True)
        im.set_antennas(inp.xy_m, inp.freq_hz)
        img = im.accumulate(ef, g)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            im.accumulate(ef, g, image=img)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / steps
        ks = im.timing_history(steps)             # HIP events around each main kernel
        r = {"samples_per_s": T / dt, "ms_per_call": dt * 1e3, "kernel": im.last_kernel_name(),
             "kernel_ms": float(np.mean(ks))}
        if ref is not None:
            r["rel_err_vs_fp64"] = {"XX": float(oracle.rel_errors(img.cpu().numpy(), ref)[0][0])}
        if prec != "fp32":
            # v_mfma_f32_32x32x16: 32*32*16 MACs; per 32 samples x 32 pixels x 16 antennas:
            # (Re, Im) x (er, ei) = 4 products, x 2 for the hi and lo parts
            qb = (A + 15) // 16
            n_mfma = (N * N // 32) * ((T + 31) // 32) * qb * P * 8
            hw = n_mfma * 32 * 32 * 16 * 2
            k_s = r["kernel_ms"] * 1e-3
            r["roofline"] = {"bound": "mfma", "kernel": "split_image_kernel",
                             "achieved": hw / k_s / 1e12, "peak": PEAK_MFMA_F16 / 1e12,
                             "unit": "TFLOP/s", "frac": hw / k_s / PEAK_MFMA_F16,
                             "frac_useful": hw / 2 / k_s / PEAK_MFMA_F16,
                             "hardware_flops": hw, "useful_flops": hw // 2}
        res[prec] = r
        im.close()
    out = {"workload": "16 single-pol antennas in a 20 m square, 1 channel at 50 MHz, 32x32 "
                       "grid, 100000 samples", "results": res}
    if t_oracle is not None:
        out["cpu_baseline"] = {"value": T / t_oracle, "unit": "samples/s", "cores": 1,
                               "kind": "oracle", "sample": "all 100000 samples"}
    return out


def bench_split(args) -> int:
    out = {"metric": "split-precision matrix forms, samples/s and error per product",
           **split_results(args.steps), "data": "synthetic"}
    print(json.dumps(out))
    return 0


def grad_results(steps: int, warmup: int) -> dict:
    """Calibration workload: 256 dual-pol antennas, 64 channels, 64x64 grid,
    200 samples; one forward image and one gain gradient per step."""
    import torch
    import synth
    from paper_1904_11422_amd import Imager
    print("bench: generating the calibration workload", file=sys.stderr, flush=True)
    inp = synth.config5()
    N, C, P, A, T = inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.n_time
    ef = torch.from_numpy(inp.efield).cuda()
    g = torch.from_numpy(inp.gains).cuda()
    im = Imager(N, C, P, A, timing=True)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    img = im.accumulate(ef, g)
    gam = (2.0 * img).contiguous()
    for _ in range(warmup):
        im.accumulate(ef, g, image=img)
        im.backward(ef, g, gam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        im.accumulate(ef, g, image=img)
        fname = im.last_kernel_name()
        im.backward(ef, g, gam)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    hist = im.timing_history(2 * steps)          # forward and adjoint kernels, alternating
    fw, bw = hist[0::2], hist[1::2]
    bname = im.last_kernel_name()
    im.close()
    # adjoint work per (t,c): the forward recompute without the products, dL/dF*
    # (20 flop per pixel at P = 2), the adjoint transform, the degridding
    # (K^2 taps, 4 flop each, and conj(e) h, 6 flop, per (p, a))
    fl_fwd = flops_per_tc(N, P, A) - 16 * N * N
    fl_adj = fl_fwd + 20 * N * N + P * 5 * N * N * int(math.log2(N * N)) + (4 * 9 + 6) * P * A
    adj_s = float(np.mean(bw)) * 1e-3
    return {"value": 1.0 / dt, "unit": "evaluations/s", "ms_per_step": dt * 1e3, "steps": steps,
            "forward_kernel": fname, "forward_kernel_ms": float(np.mean(fw)),
            "adjoint_kernel_ms": adj_s * 1e3,
            "adjoint_tc_images_per_s": C * T / adj_s,
            "roofline": {"bound": "alu", "kernel": bname,
                         "achieved": fl_adj * C * T / adj_s / 1e12,
                         "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                         "frac": fl_adj * C * T / adj_s / PEAK_FP32_VALU,
                         "frac_nonpacked": fl_adj * C * T / adj_s / PEAK_FP32_VALU_NONPACKED,
                         "flops_per_tc_image": fl_adj},
            "workload": "256 dual-pol antennas, 64 channels, 64x64 grid, 200 samples, "
                        "20 sources"}


def bench_grad(args) -> int:
    out = {"metric": "forward + gain-gradient evaluations/s", **grad_results(args.steps, args.warmup),
           "data": "synthetic"}
    print(json.dumps(out))
    return 0


def autos_results(steps: int, warmup: int, inp=None) -> dict:
    """The default workload with the antenna autocorrelations removed: one
    imaging call per step, then the removal (a second pass over the E-field
    for the exact per-antenna sums, a per-channel table, a pass over the image)."""
    import torch
    import synth
    from paper_1904_11422_amd import Imager
    if inp is None:
        print("bench: generating the LWA-like workload", file=sys.stderr, flush=True)
        inp = synth.config2()
    N, C, P, A, T = inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.n_time
    ef = torch.from_numpy(inp.efield).cuda()
    g = torch.from_numpy(inp.gains).cuda()
    im = Imager(N, C, P, A, timing=True, remove_autos=True)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    img = torch.empty(im.image_shape(), dtype=torch.complex128, device="cuda")
    for _ in range(warmup):
        im.accumulate(ef, g, image=img)
    torch.cuda.synchronize()
    print("bench: timing imaging with autocorrelation removal", file=sys.stderr, flush=True)
    main_ms, sum_ms, rem_ms = [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        im.accumulate(ef, g, image=img)
        main_ms.append(im.last_timing()[0])
        s, r = im.last_autos_timing()
        sum_ms.append(s)
        rem_ms.append(r)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    nq = 4 if P == 2 else 1
    # algorithmic bytes of the sum pass: every sample byte once, the exact
    # per-antenna sums (nq int32) out once
    alg = C * T * P * A + C * A * nq * 4
    s_ms = float(np.mean(sum_ms))
    out = {"metric": "channel-images/s with autocorrelations removed", "value": C / dt,
           "unit": "channel-images/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "LWA-like: 256 dual-pol antennas, 132 channels, 64x64 grid, "
                                  "1000 samples, autocorrelations removed",
                      "grid_n": N, "n_chan": C, "n_pol": P, "n_ant": A, "n_time": T},
           "imager_kernel_ms": float(np.mean(main_ms)), "auto_sum_kernel_ms": s_ms,
           "removal_ms": float(np.mean(rem_ms)),
           "roofline": {"bound": "hbm", "kernel": "auto_sum_kernel",
                        "achieved": alg / (s_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                        "unit": "GB/s", "frac": alg / (s_ms * 1e-3) / PEAK_HBM,
                        "traffic": measured_traffic(AUTOS_PROFILE, AUTOS_SOURCES),
                        "bytes_per_launch": alg}}
    im.close()
    return out


def bench_autos(args) -> int:
    print(json.dumps(autos_results(args.steps, args.warmup)))
    return 0


def stream_results(steps: int, warmup: int, inp=None) -> dict:
    """Streaming ingest: gulps of the LWA-like workload arriving as 264 channels
    [T][C][A][P] in pinned host memory, the central 132 channels selected (a
    contiguous sub-band, so only it crosses the host link), transposed and
    imaged, the copy of each gulp overlapping the imaging of the one before."""
    import torch
    import synth
    from paper_1904_11422_amd import Imager, Pipeline
    print("bench: generating two raw gulps", file=sys.stderr, flush=True)
    if inp is None:
        inp = synth.config2()
    N, C, P, A, T = inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.n_time
    c_in, c0 = 2 * C, C // 2
    gulps = [torch.from_numpy(synth.raw_gulp(9000 + k, T, c_in, A, P)).pin_memory() for k in range(2)]
    g = torch.from_numpy(inp.gains).cuda()
    im = Imager(N, C, P, A)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    img = torch.empty(im.image_shape(), dtype=torch.complex128, device="cuda")
    # the front end alone, timed with events around back-to-back launches
    dev_raw = gulps[0].cuda()
    ef = im.frontend(dev_raw, c0, 1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        im.frontend(dev_raw, c0, 1, out=ef)
    e1.record()
    torch.cuda.synchronize()
    fe_ms = e0.elapsed_time(e1) / reps
    fe_bytes = 2 * T * C * P * A
    del dev_raw
    pipe = Pipeline(im, T, c_in, c0, 1, sample_s=40e-6)
    for k in range(warmup):
        pipe.push(gulps[k % 2], g, img)
    pipe.report()
    pipe.close()
    pipe = Pipeline(im, T, c_in, c0, 1, sample_s=40e-6)
    print("bench: streaming", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for k in range(steps):
        pipe.push(gulps[k % 2], g, img)
    st = pipe.report()
    dt = (time.perf_counter() - t0) / steps
    out = {"metric": "streamed channel-images/s (host gulps -> images)", "value": C / dt,
           "unit": "channel-images/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "LWA-like gulps: 264 channels arriving [T][C][A][P] in pinned "
                                  "host memory, central 132 imaged (64x64, 256 dual-pol antennas), "
                                  "1000 samples (40 ms) per gulp",
                      "grid_n": N, "n_chan": C, "c_in": c_in, "n_pol": P, "n_ant": A, "n_time": T},
           "pipeline": st,
           "realtime_factor": st["gulp_ms"] / st["mean_ms"],
           "host_copy_GBps": T * C * P * A / (st["mean_copy_ms"] * 1e-3) / 1e9,
           "roofline": {"bound": "hbm", "kernel": "frontend_kernel",
                        "achieved": fe_bytes / (fe_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                        "unit": "GB/s", "frac": fe_bytes / (fe_ms * 1e-3) / PEAK_HBM,
                        "traffic": None, "kernel_ms": fe_ms, "bytes_per_launch": fe_bytes}}
    pipe.close()
    im.close()
    return out


def bench_stream(args) -> int:
    print(json.dumps(stream_results(args.steps, args.warmup)))
    return 0


def kernels_results(steps: int, warmup: int, inp=None) -> dict:
    """The LWA-like workload gridded with seeded complex kernels per channel and
    antenna (A-projection-like): 5 x 5 on the 64 x 64 grid (the largest support
    whose taps keep this aperture inside N/2 cells, so the N/2 fused kernel runs),
    and 15 x 15 on a 128 x 128 grid (same array, same channels)."""
    import torch
    import synth
    from paper_1904_11422_amd import Imager
    if inp is None:
        print("bench: generating the LWA-like workload", file=sys.stderr, flush=True)
        inp = synth.config2()
    base = inp
    ef = torch.from_numpy(base.efield).cuda()
    g = torch.from_numpy(base.gains).cuda()
    out = {}
    for N, K in ((64, 5), (128, 15)):
        inp = synth.with_kernels(base, K, 7000 + K)
        C, P, A, T = inp.n_chan, inp.n_pol, inp.n_ant, inp.n_time
        im = Imager(N, C, P, A, kernel_support=K, timing=True)
        im.set_antennas(inp.xy_m, inp.freq_hz, kernels=inp.kernels)
        img = torch.empty(im.image_shape(), dtype=torch.complex128, device="cuda")
        for _ in range(warmup):
            im.accumulate(ef, g, image=img)
        torch.cuda.synchronize()
        steps = steps if N == 64 else max(3, steps // 4)
        t0 = time.perf_counter()
        for _ in range(steps):
            im.accumulate(ef, g, image=img)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ks = im.timing_history(steps)
        k_ms = float(np.mean(ks))
        fl = flops_per_tc(N, P, A, K, complex_kernel=True)
        out[f"n{N}_k{K}"] = {
            "value": C / dt, "unit": "channel-images/s", "ms_per_step": dt * 1e3, "steps": steps,
            "kernel": im.last_kernel_name(), "kernel_ms": k_ms,
            "roofline": {"bound": "alu", "achieved": fl * C * T / (k_ms * 1e-3) / 1e12,
                         "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                         "frac": fl * C * T / (k_ms * 1e-3) / PEAK_FP32_VALU,
                         "traffic": None, "flops_per_tc_image": fl}}
        im.close()
    main = out["n64_k5"]
    line = {"metric": "channel-images/s with complex per-antenna kernels", "value": main["value"],
            "unit": "channel-images/s", "n_gpus": 1, "steps": main["steps"], "warmup": warmup,
            "ms_per_step": main["ms_per_step"], "higher_is_better": True, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "LWA-like (256 dual-pol antennas, 132 channels, 1000 samples) "
                                   "gridded with seeded complex 5x5 kernels per channel and "
                                   "antenna on 64x64; also 15x15 on 128x128",
                       "grid_n": 64, "kernel_support": 5},
            "roofline": main["roofline"], "results": out}
    return line


def bench_kernels(args) -> int:
    print(json.dumps(kernels_results(args.steps, args.warmup)))
    return 0


def deployment_results(steps: int, warmup: int, inp=None) -> dict:
    """The paper's deployed geometry (Sec. 4.1-4.2: 256 antennas in a 110 m x
    100 m ellipse, lambda / 2 cells, 64 x 64 grid) over 132 channels of 25 kHz
    centred on 55.25 MHz, one 50 ms image (1250 samples of 40 us) per step.
    With the taps the aperture spans 43-45 cells, wider than N/2: the wide
    fused kernel runs; the staged kernels are timed beside it."""
    import torch
    import synth
    from paper_1904_11422_amd import Imager
    print("bench: generating the deployment workload", file=sys.stderr, flush=True)
    inp = synth.deployment(n_time=1250, n_chan=132)
    N, C, P, A, T = inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.n_time
    ef = torch.from_numpy(inp.efield).cuda()
    g = torch.from_numpy(inp.gains).cuda()
    out = {}
    for staged in (False, True):
        im = Imager(N, C, P, A, staged=staged, timing=True)
        im.set_antennas(inp.xy_m, inp.freq_hz)
        img = torch.empty(im.image_shape(), dtype=torch.complex128, device="cuda")
        for _ in range(warmup if not staged else 1):
            im.accumulate(ef, g, image=img)
        torch.cuda.synchronize()
        steps = steps if not staged else max(2, steps // 5)
        t0 = time.perf_counter()
        for _ in range(steps):
            im.accumulate(ef, g, image=img)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ks = im.timing_history(steps)
        k_ms = float(np.mean(ks))
        kname = im.last_kernel_name()              # the image kernel, before the gradient runs
        fl = flops_per_tc(N, P, A) * C * T
        # one gain-gradient evaluation (image + adjoint) per call, same route
        gam = torch.randn(im.image_shape(), dtype=torch.complex128, device="cuda")
        im.backward(ef, g, gam)
        torch.cuda.synchronize()
        nb = max(2, steps // 4)
        t1 = time.perf_counter()
        for _ in range(nb):
            im.backward(ef, g, gam)
        torch.cuda.synchronize()
        grad_ms = (time.perf_counter() - t1) / nb * 1e3
        grad_kernel = im.last_kernel_name()
        out["staged" if staged else "fused"] = {
            "gradient_ms_per_call": grad_ms, "gradient_kernel": grad_kernel,
            "value": C / dt, "unit": "channel-images/s", "ms_per_step": dt * 1e3, "steps": steps,
            "kernel": kname, "kernel_ms": k_ms,
            "roofline": {"bound": "alu", "achieved": fl / (k_ms * 1e-3) / 1e12,
                         "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                         "frac": fl / (k_ms * 1e-3) / PEAK_FP32_VALU, "traffic": None,
                         "flops_per_tc_image": flops_per_tc(N, P, A)}}
        im.close()
    main = out["fused"]
    main["speedup_over_staged"] = main["value"] / out["staged"]["value"]
    main["gradient_speedup_over_staged"] = (out["staged"]["gradient_ms_per_call"]
                                            / main["gradient_ms_per_call"])
    line = {"metric": "channel-images/s (4-pol, 64\u00b2 grid), the paper's deployed geometry",
            "value": main["value"], "unit": "channel-images/s", "n_gpus": 1,
            "steps": main["steps"], "warmup": warmup, "ms_per_step": main["ms_per_step"],
            "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "256 dual-pol antennas uniform in a 110 m x 100 m ellipse, "
                                   "132 x 25 kHz channels at 55.25 MHz, 64x64 grid at lambda/2, "
                                   "3x3 Gaussian, 1250 samples (one 50 ms image)",
                       "grid_n": 64, "n_time": T},
            "roofline": main["roofline"], "results": out}
    return line


def bench_deployment(args) -> int:
    print(json.dumps(deployment_results(args.steps, args.warmup)))
    return 0


def bench_arrays(args) -> int:
    """Denser arrays on the LWA-like grid: 256, 512 and 1024 dual-pol antennas
    in one 26-cell disk (64 x 64 grid, 132 channels, 250 samples).  The three
    counts select the kernel variants that stage 1, 2 and 4 sample bytes per
    thread; the 4-byte variant stages E' in grid rows of the second
    polarisation that nothing else uses (its column transforms exchange
    through the first one's columns), so that its LDS footprint (70.1 KB)
    lets two workgroups share a CU."""
    import torch
    import synth
    from paper_1904_11422_amd import Imager
    out = {}
    for A in (256, 512, 1024):
        print(f"bench: generating the {A}-antenna array", file=sys.stderr, flush=True)
        inp = synth.random_problem(8100 + A, 64, A, 132, 2, 250, fill=0.45, min_sep_cells=0.6)
        N, C, P, T = inp.grid_n, inp.n_chan, inp.n_pol, inp.n_time
        ef = torch.from_numpy(inp.efield).cuda()
        g = torch.from_numpy(inp.gains).cuda()
        im = Imager(N, C, P, A, timing=True)
        im.set_antennas(inp.xy_m, inp.freq_hz)
        img = im.accumulate(ef, g)
        for _ in range(args.warmup):
            im.accumulate(ef, g, image=img)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            im.accumulate(ef, g, image=img)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        ks = im.timing_history(args.steps)
        k_ms = float(np.mean(ks))
        fl = flops_per_tc(N, P, A)
        out[f"a{A}"] = {"bytes_per_thread": -(-P * A // 512), "kernel": im.last_kernel_name(),
                        "kernel_ms": k_ms, "ms_per_step": dt * 1e3, "value": C / dt,
                        "tc_images_per_s": C * T / (k_ms * 1e-3),
                        "roofline": {"bound": "alu", "achieved": fl * C * T / (k_ms * 1e-3) / 1e12,
                                     "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                                     "frac": fl * C * T / (k_ms * 1e-3) / PEAK_FP32_VALU,
                                     "traffic": None, "flops_per_tc_image": fl}}
        im.close()
    main = out["a1024"]
    line = {"metric": "channel-images/s for denser arrays (64\u00b2 grid)", "value": main["value"],
            "unit": "channel-images/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": main["ms_per_step"], "higher_is_better": True, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "256 / 512 / 1024 dual-pol antennas in a 26-cell disk, "
                                   "132 channels, 250 samples, 64x64 grid", "grid_n": 64},
            "roofline": main["roofline"], "results": out}
    print(json.dumps(line))
    return 0


def post_results(steps: int, warmup: int, inp=None) -> dict:
    """Post-processing of the LWA-like image (132 channels, 64 x 64, 4 products):
    pseudo-Stokes I, Q, U, V with the kernel taper divided out, then FITS export."""
    import tempfile
    import torch
    import synth
    from paper_1904_11422_amd import Imager, fits
    if inp is None:
        print("bench: generating the LWA-like workload", file=sys.stderr, flush=True)
        inp = synth.config2()
    N, C, P, A, T = inp.grid_n, inp.n_chan, inp.n_pol, inp.n_ant, inp.n_time
    im = Imager(N, C, P, A)
    im.set_antennas(inp.xy_m, inp.freq_hz)
    img = im.accumulate(torch.from_numpy(inp.efield).cuda(), torch.from_numpy(inp.gains).cuda())
    out = im.postprocess(img, 1e-3)
    for _ in range(warmup):
        im.postprocess(img, 1e-3, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        im.postprocess(img, 1e-3, out=out)
    e1.record()
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / steps
    # algorithmic bytes: the four complex128 products in, the taper, four float64 planes out
    alg = C * N * N * (4 * 16 + 8 + 4 * 8)
    with tempfile.TemporaryDirectory() as d:
        t0 = time.perf_counter()
        fits.write(os.path.join(d, "cube.fits"), out, N, inp.cell_wavelengths, inp.freq_hz,
                   n_time=T, sample_s=40e-6)
        fits_s = time.perf_counter() - t0
    line = {"metric": "post-processed channel images/s (pseudo-Stokes, taper-corrected)",
            "value": C / (k_ms * 1e-3), "unit": "channel-images/s", "n_gpus": 1,
            "steps": steps, "warmup": warmup, "ms_per_step": k_ms,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "LWA-like image: 132 channels, 4 products, 64x64, "
                                   "taper floor 1e-3", "grid_n": N, "n_chan": C},
            "roofline": {"bound": "hbm", "kernel": "postprocess_kernel",
                         "achieved": alg / (k_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                         "unit": "GB/s", "frac": alg / (k_ms * 1e-3) / PEAK_HBM,
                         "traffic": None, "bytes_per_launch": alg, "kernel_ms": k_ms},
            "fits_write_s": fits_s, "fits_bytes": C * 4 * N * N * 4}
    im.close()
    return line


def bench_post(args) -> int:
    print(json.dumps(post_results(args.steps, args.warmup)))
    return 0


PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
PROFILE = os.path.join(PROFILES, "fused_image_kernel_lwa64_c132_t1000.md")
PROFILED_SOURCES = ("csrc/fused.hpp", "csrc/dft.hpp", "csrc/reduce.hpp", "build.py")
AUTOS_PROFILE = os.path.join(PROFILES, "auto_sum_kernel_lwa64_c132_t1000.md")
AUTOS_SOURCES = ("csrc/autos.hpp", "build.py")


def measured_traffic(profile=PROFILE, sources=PROFILED_SOURCES):
    """HBM bytes per launch of a kernel from its committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's reading), or None
    when the kernel sources have changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(profile).read()
    except OSError:
        return None
    want = re.search(r"sources_sha256: ([0-9a-f]{64})", text)
    val = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if not want or not val:
        return None
    h = hashlib.sha256()
    pkg = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1904_11422_amd")
    for f in sources:
        with open(os.path.join(pkg, f), "rb") as fh:
            h.update(fh.read())
    return int(val.group(1)) if h.hexdigest() == want.group(1) else None


def measured_clock(profile=PROFILE, sources=PROFILED_SOURCES):
    """Mean shader clock (GHz) under the main kernel, from the committed
    counter summary (GRBM_GUI_ACTIVE cycles over the kernel's traced time),
    or None when the kernel sources have changed since."""
    import re
    if measured_traffic(profile, sources) is None:
        return None
    m = re.search(r"clock_ghz: ([0-9.]+)", open(profile).read())
    return float(m.group(1)) if m else None


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-channels", type=int, default=16,
                    help="channels of the workload the CPU oracle is timed on")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-staged", action="store_true")
    ap.add_argument("--no-rows", action="store_true",
                    help="leave out the compact results of the other rows (split precision, gradient, "
                         "batch, deployed geometry, autocorrelations, complex kernels, post-processing, "
                         "streaming)")
    ap.add_argument("--batch", action="store_true",
                    help="measure the heterogeneous batch (grids 32/64/128, 64/256/1024 "
                         "antennas, 16-264 channels, 200 samples) instead of the default line")
    ap.add_argument("--split", action="store_true",
                    help="measure the split-precision matrix forms on the tiny geometry over "
                         "a long integration, with errors against the FP64 oracle")
    ap.add_argument("--grad", action="store_true",
                    help="measure forward + gain-gradient evaluations on the calibration workload")
    ap.add_argument("--autos", action="store_true",
                    help="measure the default workload with the antenna autocorrelations removed")
    ap.add_argument("--stream", action="store_true",
                    help="measure the double-buffered streaming ingest (host gulps in arrival "
                         "order, decimated, transposed and imaged)")
    ap.add_argument("--kernels", action="store_true",
                    help="measure imaging with complex per-antenna gridding kernels (5x5 on 64x64, "
                         "15x15 on 128x128)")
    ap.add_argument("--post", action="store_true",
                    help="measure post-processing (pseudo-Stokes with kernel-taper correction) "
                         "and FITS export of the LWA-like image")
    ap.add_argument("--arrays", action="store_true",
                    help="256, 512 and 1024 antennas (1, 2 and 4 sample bytes per thread)")
    ap.add_argument("--deployment", action="store_true",
                    help="the paper's deployed geometry (aperture wider than N/2: wide fused "
                         "kernel) against the staged kernels")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (five times), to "
                         "scale the FETCH_SIZE / WRITE_SIZE counters of a profiler run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(channels shard across GPUs with no communication, so one GPU's "
              "throughput times the GPU count is the multi-GPU figure)", file=sys.stderr)
        return 2
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.batch:
        return bench_batch(args)
    if args.split:
        return bench_split(args)
    if args.grad:
        return bench_grad(args)
    if args.autos:
        return bench_autos(args)
    if args.stream:
        return bench_stream(args)
    if args.kernels:
        return bench_kernels(args)
    if args.post:
        return bench_post(args)
    if args.deployment:
        return bench_deployment(args)
    if args.arrays:
        return bench_arrays(args)

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

    # The plain float32 staged comparator is timed first: its ~70 ms of kernels
    # also leave the GPU at its steady clock, which otherwise settles only
    # after the first ~15 fused launches of a process.
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
                  "ms_per_step": dts * 1e3 / n_st, "steps": n_st}
        ims.close()

    for _ in range(args.warmup):
        im.accumulate(ef, g, image=img, reset=True)
    torch.cuda.synchronize()
    print("bench: timing the fused path", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    for _ in range(args.steps):
        im.accumulate(ef, g, image=img, reset=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # HIP events the library records around each call's main kernel, read
    # after the timed region (no wait inside it)
    kernel_ms = im.timing_history(args.steps)
    ms_per_step = dt * 1e3 / args.steps
    value = C * args.steps / dt
    kname = im.last_kernel_name()

    k_ms = float(np.mean(kernel_ms))
    fl = flops_per_tc(N, P, A) * C * T
    achieved = fl / (k_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU, "traffic": measured_traffic(),
                "frac_nonpacked": achieved / PEAK_FP32_VALU_NONPACKED,
                "clock_ghz_measured": measured_clock(),
                "kernel": kname, "kernel_ms": k_ms,
                "flops_per_launch": fl, "flops_per_tc_image": flops_per_tc(N, P, A),
                "input_bytes_per_launch": C * T * P * A}
    im.close()
    if staged is not None:
        staged["speedup_of_fused"] = value / staged["value"]

    subs = {}
    if not args.no_rows:
        # the other hot-path rows, compact: split-precision matrix forms (16 antennas,
        # 10^5 samples), forward + gain gradient (calibration workload), the
        # heterogeneous batch (graph replay)
        del ef, g, img
        torch.cuda.empty_cache()
        sub_steps = max(5, args.steps)
        subs["split_precision"] = split_results(sub_steps, with_oracle=not args.no_cpu)
        subs["gradient"] = grad_results(sub_steps, args.warmup)
        subs["batch"] = batch_results(sub_steps, args.warmup, sequential=False)
        # the paper's deployed geometry (wide aperture block) and the further rows:
        # autocorrelation removal, per-antenna complex kernels, post-processing,
        # streamed ingest from host gulps
        subs["deployed_geometry"] = deployment_results(sub_steps, args.warmup)
        subs["autocorrelation_removal"] = autos_results(sub_steps, args.warmup, inp)
        subs["complex_kernels"] = kernels_results(sub_steps, args.warmup, inp)
        subs["post_processing"] = post_results(sub_steps, args.warmup, inp)
        subs["streaming"] = stream_results(sub_steps, args.warmup, inp)

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
        **subs,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
