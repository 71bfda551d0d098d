#!/usr/bin/env python3
"""Benchmark of the MDC forward + adjoint hot path on one MI355X.

Workload (single virtual point, GEMV form, FP32/complex64): nt = 512, dt = 4 ms,
nfmax = 150 of 257 bins, ns = nr = 40 x 40 = 1600 traces on a 20 m grid;
synthetic hyperbolic-event kernel with 20 reflectors and 5% noise (3.07 GB
complex64) generated on the device, input = time-reversed direct arrival of a
20 Hz Ricker from a point at 650 m depth.

One step = one forward and one adjoint apply (rFFT, per-frequency product,
inverse rFFT each).  `value` = algorithmic bytes of a step (kernel read twice,
input and output vectors once per apply) / step time, in GB/s, with every
input already resident in HBM.

The JSON line also carries
  roofline      -- the product kernels (the dominant cost): algorithmic bytes
                   per launch / average launch duration from HIP events on the
                   apply stream, against the 8 TB/s HBM peak; `traffic` is the
                   counter-measured HBM bytes per launch from a committed
                   rocprofv3 summary when its source hash still matches;
  cpu_baseline  -- the FP64 oracle timed on the host on a bounded frequency
                   sample of the same workload, scaled by bins (the bins are
                   independent, so work scales exactly).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = dict(nt=512, nfmax=150, nx=40, nv=1, dt=0.004, dx=20.0)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gemv_c2.json")
PRODUCT_SRC = os.path.join(ROOT, "paper_2011_11120_amd", "csrc", "gemv.hip")


def source_hash(path: str) -> str:
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def algorithmic_bytes(nt, nfmax, n, nv):
    kernel = 8 * nfmax * n * n
    spectra = 8 * nfmax * n * nv * 2       # product: spectrum in + spectrum out
    vectors = 4 * nt * n * nv * 2          # apply: time vector in + out
    return kernel, kernel + spectra, kernel + vectors


def host_cpu():
    """CPU model and core counts of the host the baseline runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def cpu_baseline(spec, x, y, target_s: float = 8.0):
    """FP64 oracle on a frequency subset; time scaled to all bins.  Timed with the BLAS library's
    own thread count and again on one thread; the figure per run is the median repeat."""
    import statistics

    import numpy as np
    from oracle import mdc as om
    from paper_2011_11120_amd import synth
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    nsub = 10
    bins = np.linspace(0, spec.nfmax - 1, nsub).astype(int)
    idx = np.arange(spec.n)
    Ksub = synth.kernel_block(spec, bins, idx, idx)  # input generation, not timed

    def one():
        # the oracle's forward and adjoint on a kernel of nsub bins: the same work per bin as the
        # full apply (DFT rows, per-bin product, inverse), so the time scales by nfmax / nsub
        om.mdc_forward(Ksub, x)
        om.mdc_adjoint(Ksub, y)

    def timed(budget_s):
        reps, t0 = [], time.perf_counter()
        while True:
            a = time.perf_counter()
            one()
            reps.append(time.perf_counter() - a)
            if time.perf_counter() - t0 >= budget_s or len(reps) >= 200:
                break
        return statistics.median(reps) * spec.nfmax / nsub, statistics.mean(reps) * spec.nfmax / nsub, len(reps)

    med_all, mean_all, n_all = timed(target_s)
    with threadpool_limits(limits=1):
        med_one, mean_one, n_one = timed(target_s)
    return {"median_s": med_all, "mean_s": mean_all, "repeats": n_all, "threads": threads,
            "one_thread": {"median_s": med_one, "mean_s": mean_one, "repeats": n_one},
            "sample": f"{nsub} of {spec.nfmax} bins (FP64), scaled by bins", "host": host_cpu()}


COPY_BYTES = 256 * 1024 * 1024
TRAFFIC_COMMANDS = [
    "cd /tmp && export TMPDIR=/tmp && timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -d $REPO/gpurun_out/pmc_fetch "
    "-o fetch -- python3 $REPO/bench.py --steps 2 --warmup 1 --no-cpu-baseline --copy-calibration",
    "cd /tmp && export TMPDIR=/tmp && timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d $REPO/gpurun_out/pmc_write "
    "-o write -- python3 $REPO/bench.py --steps 2 --warmup 1 --no-cpu-baseline --copy-calibration",
    "python3 bench.py --write-traffic gpurun_out/pmc_fetch/fetch_results.db gpurun_out/pmc_write/write_results.db",
]


def write_traffic(fetch_db: str, write_db: str) -> None:
    """Counter-calibrated HBM traffic of the matrix-vector kernels, from two rocprofv3 --pmc runs.

    Each counter (KiB per dispatch) is scaled by bytes / reading of the plain device copies of
    COPY_BYTES bytes in the same run; the record carries the product source hash so that a
    changed kernel reports no traffic until the counters are taken again.
    """
    import sqlite3
    import statistics

    def per_kernel(db, counter):
        out = {}
        con = sqlite3.connect(db)
        for name, cn, v in con.execute("select kernel_name, counter_name, value from counters_collection"):
            if cn == counter:
                short = name.replace("void ", "").replace("mdc::(anonymous namespace)::", "").split("(")[0]
                out.setdefault(short, []).append(float(v))
        return out

    fetch, write = per_kernel(fetch_db, "FETCH_SIZE"), per_kernel(write_db, "WRITE_SIZE")
    copy = "__amd_rocclr_copyBuffer"
    ff = COPY_BYTES / (statistics.median(sorted(fetch[copy])[-3:]) * 1024)
    wf = COPY_BYTES / (statistics.median(sorted(write[copy])[-3:]) * 1024)
    kernels, per_launch = {}, []
    for name in sorted(fetch):
        if not name.startswith(("gemv_fwd_kernel", "gemv_adj_kernel")):
            continue
        fk, wk = statistics.mean(fetch[name]), statistics.mean(write[name])
        kernels[name] = {"fetch_KiB_raw": round(fk, 1), "write_KiB_raw": round(wk, 1),
                         "fetch_bytes": round(fk * 1024 * ff), "write_bytes": round(wk * 1024 * wf)}
        per_launch.append(fk * 1024 * ff + wk * 1024 * wf)
    alg = algorithmic_bytes(WORKLOAD["nt"], WORKLOAD["nfmax"], WORKLOAD["nx"] ** 2, WORKLOAD["nv"])[1]
    rec = {"workload": WORKLOAD, "source": os.path.relpath(PRODUCT_SRC, ROOT),
           "source_sha256_16": source_hash(PRODUCT_SRC),
           "copy_calibration": {"bytes_copied": COPY_BYTES, "fetch_factor": round(ff, 4), "write_factor": round(wf, 4)},
           "kernels": kernels, "bytes_per_launch": round(statistics.mean(per_launch)),
           "algorithmic_bytes_per_launch": alg,
           "traffic_over_algorithmic": round(statistics.mean(per_launch) / alg, 4), "commands": TRAFFIC_COMMANDS}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({k: rec[k] for k in ("bytes_per_launch", "traffic_over_algorithmic", "copy_calibration")}))


def main():
    if len(sys.argv) == 4 and sys.argv[1] == "--write-traffic":
        return write_traffic(sys.argv[2], sys.argv[3])
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: c2 100 forward + adjoint steps, c3 20, c4 3 solves per grid)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default: c2 10, c3 2, c4 1)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["c2", "c3", "c4", "c5"], default="c2",
                    help="c2: single-point GEMV workload (default line); c3: 64-point matrix-core workload; "
                         "c4: Marchenko LSQR solves (full, 2x, 4x decimated); c5: served stream of solves")
    ap.add_argument("--requests", type=int, default=64, help="c5: requests per run")
    ap.add_argument("--skip", type=int, default=8, help="c5: first completions left out of the latency stats")
    ap.add_argument("--c5-precs", default="fp32,fp16s", help="c5: kernel formats to serve, in order")
    ap.add_argument("--c5-max-cols", type=int, default=384, help="c5: column budget (2 per focusing point)")
    ap.add_argument("--c5-sublattice", type=int, default=6,
                    help="c5: decimation levels solved on their own lattice (0, 2, 4 or 6)")
    ap.add_argument("--c5-rate", type=float, default=None,
                    help="c5: Poisson rate (solves/s) measured as 0.7 x the FP32 capacity in an earlier run")
    ap.add_argument("--c5-light", type=float, default=0.0,
                    help="c5: light-load Poisson stream at this fraction of the format's capacity (0: none)")
    ap.add_argument("--c5-light-requests", type=int, default=24, help="c5: requests of the light-load stream")
    ap.add_argument("--c5-alone", type=int, default=0,
                    help="c5: solve this many sampled requests of a closed-loop run again alone and compare")
    ap.add_argument("--c5-closed-only", action="store_true", help="c5: closed loop only (no Poisson streams)")
    ap.add_argument("--prec", choices=["fp32", "fp16s", "bf16", "bf16x2", "fp16"], default="fp32",
                    help="kernel storage format for the c3/c4 workloads")
    ap.add_argument("--no-legs", action="store_true",
                    help="default workload: skip the matrix-core and served-stream legs of the line")
    ap.add_argument("--leg-requests", type=int, default=12, help="served-stream leg: requests per format")
    ap.add_argument("--leg-skip", type=int, default=2, help="served-stream leg: first completions excluded")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    # c2: forward and adjoint each applied 100 times after 10 warm-up steps; c3: 20 steps
    defaults = {"c2": (100, 10), "c3": (20, 2), "c4": (3, 1), "c5": (1, 0)}[args.workload]
    if args.steps is None:
        args.steps = defaults[0]
    if args.warmup is None:
        args.warmup = defaults[1]
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the MDC path here is single-GPU "
              "(frequency sharding across GPUs is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2011_11120_amd import mdc, synth

    torch.cuda.set_device(0)
    if args.workload == "c3":
        return bench_c3(args)
    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "c5":
        return bench_c5(args)
    W = WORKLOAD
    spec = synth.KernelSpec(nt=W["nt"], nfmax=W["nfmax"], nx=W["nx"], dt=W["dt"], dx=W["dx"])
    n, nv = spec.n, W["nv"]
    op = mdc.MdcOp(spec.nt, spec.nfmax, n, n, max_cols=nv)
    op.synth_kernel(spec)
    gx, gy = synth.grid_xy(spec.nx, spec.nx, spec.dx)
    c = (spec.nx - 1) * spec.dx / 2
    td = synth.direct_traveltime(gx, gy, np.full(nv, c), np.full(nv, c), np.full(nv, 650.0), 2400.0)
    x_h = synth.direct_focusing(spec.nt, td, spec.dt)
    y_h = synth.gaussian((spec.nt, n, nv))
    x = torch.as_tensor(x_h, dtype=torch.float32).cuda()
    y = torch.as_tensor(y_h, dtype=torch.float32).cuda()
    yo = torch.empty_like(x)
    xo = torch.empty_like(y)
    torch.cuda.synchronize()
    print(f"setup done: kernel {8 * spec.nfmax * n * n / 1e9:.3f} GB resident", file=sys.stderr, flush=True)

    def step():
        mdc.mdc_forward(op.handle, x, yo, nv)
        mdc.mdc_adjoint(op.handle, y, xo, nv)

    for _ in range(args.warmup):
        step()
    if args.copy_calibration:
        a = torch.empty(256 * 1024 * 1024, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copy calibration: 3 copies of 268435456 bytes", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    # Timed steps: the workload alone.  The library's per-stage events put about 10 us of idle
    # time at every kernel boundary, so the per-launch kernel durations come from the same number
    # of steps run again right after, with those events recorded on the apply stream.
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    mdc.mdc_profile_read(op.handle)  # drop anything recorded so far
    mdc.mdc_profile(op.handle, True)
    ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev2.record()
    for _ in range(args.steps):
        step()
    ev3.record()
    torch.cuda.synchronize()
    mdc.mdc_profile(op.handle, False)
    ms_stage, cnt = mdc.mdc_profile_read(op.handle)
    ms_step_profiled = ev2.elapsed_time(ev3) / args.steps
    # third pass: one event pair per step, for the median and spread of the step time
    per_step = []
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a, b in evs:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    per_step = sorted(a.elapsed_time(b) for a, b in evs)
    ms_median = per_step[len(per_step) // 2] if len(per_step) % 2 else 0.5 * (
        per_step[len(per_step) // 2 - 1] + per_step[len(per_step) // 2])

    kbytes, prod_bytes, apply_bytes = algorithmic_bytes(spec.nt, spec.nfmax, n, nv)
    step_bytes = 2 * apply_bytes
    value = step_bytes / (ms_step * 1e-3) / 1e9
    prod_ms = (ms_stage[1] + ms_stage[2]) / max(1, cnt[1] + cnt[2])
    achieved = prod_bytes / (prod_ms * 1e-3) / 1e9

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("source_sha256_16") == source_hash(PRODUCT_SRC) and tr.get("workload") == W:
            traffic = round(tr["bytes_per_launch"] / 1e9, 4)

    cpu = None
    if not args.no_cpu_baseline:
        cb = cpu_baseline(spec, x_h, y_h)
        cpu = {"value": round(step_bytes / cb["median_s"] / 1e9, 4), "unit": "GB/s", "cores": cb["threads"],
               "kind": "oracle", "sample": cb["sample"] + f", median of {cb['repeats']} repeats",
               "s_per_step_median": round(cb["median_s"], 3), "s_per_step_mean": round(cb["mean_s"], 3),
               "one_core": {"value": round(step_bytes / cb["one_thread"]["median_s"] / 1e9, 4), "unit": "GB/s",
                            "s_per_step_median": round(cb["one_thread"]["median_s"], 3),
                            "repeats": cb["one_thread"]["repeats"]},
               "host": cb["host"]}

    out = {
        "metric": "MDC fwd/adj HBM GB/s & MFMA % peak; served LSQR solves/s, p50/p99 latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_median": round(ms_median, 4),
        "ms_per_step_min_max": [round(per_step[0], 4), round(per_step[-1], 4)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (device-generated hyperbolic-event kernel, 20 reflectors + 5% noise)",
        "config": {"workload": "MDC GEMV nt=512 nfmax=150 ns=nr=1600 nv=1 (40x40 grid, dt=4ms), fwd+adj per step",
                   "kernel_GB": round(kbytes / 1e9, 4), "prec": "fp32", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_GB_per_launch": round(prod_bytes / 1e9, 4),
                     "kernel": "gemv_fwd_kernel / gemv_adj_kernel",
                     "avg_launch_ms": round(prod_ms, 5),
                     "stage_ms_per_launch": {k: round(ms_stage[i] / max(1, cnt[i]), 5) for i, k in
                                             enumerate(["rfft", "product_fwd", "product_adj", "irfft"])},
                     "timing": "per-launch durations from HIP events on the apply stream over a second "
                               "pass of the same steps (events add idle time at kernel boundaries)",
                     "ms_per_step_with_events": round(ms_step_profiled, 4)},
        "cpu_baseline": cpu,
        "wall_s": round(wall, 3),
    }
    op.close()
    del op, x, y, xo, yo
    torch.cuda.empty_cache()
    if not args.no_legs and not args.copy_calibration:
        out["legs"] = headline_legs(args)
    print(json.dumps(out), flush=True)


def headline_legs(args):
    """The other two legs of the headline metric, measured in the same run at reduced counts:
    the matrix-core product of the 64-point workload (FP32 MFMA fraction of peak) and the served
    stream (closed-loop solves/s and p50/p99 per format).  The full-count records of both are
    produced by --workload c3 / c5."""
    import argparse as _ap
    legs = {}
    print("leg: 64-point matrix-core product", file=sys.stderr, flush=True)
    c3 = bench_c3(_ap.Namespace(prec="fp32", steps=5, warmup=1), emit=False)
    legs["mfma_64_points_fp32"] = {"workload": c3["workload"], "product_ms": c3["product_ms"],
                                   "roofline": c3["roofline"], "steps": 5}
    print("leg: served stream", file=sys.stderr, flush=True)
    ns = _ap.Namespace(requests=args.leg_requests, skip=args.leg_skip, c5_precs="fp32,fp16s", c5_max_cols=384,
                       c5_sublattice=6, c5_rate=None, c5_light=0.0, c5_light_requests=0, c5_closed_only=True,
                       c5_alone=0)
    c5 = bench_c5(ns, emit=False)
    legs["served_lsqr"] = {"workload": c5["workload"],
                           "closed_loop": {p: {k: v["closed"][k] for k in ("solves_per_s", "p50_s", "p99_s",
                                                                            "latency_samples", "max_active")}
                                           for p, v in c5["results"].items()},
                           "solution_rel_diff_fp16s_vs_fp32": c5["solution_rel_diff_vs_fp32"].get("fp16s")}
    return legs


def bench_c3(args, emit=True):
    """64 virtual points: nt=1024, nfmax=300, ns=nr=60x60=3600, complex64 kernel (31.1 GB), FP32 MFMA."""
    import numpy as np
    import torch
    from paper_2011_11120_amd import mdc, synth
    spec = synth.KernelSpec(nt=1024, nfmax=300, nx=60)
    n, nv = spec.n, 64
    op = mdc.MdcOp(spec.nt, spec.nfmax, n, n, max_cols=nv, prec=args.prec)
    op.synth_kernel(spec)
    mdc.mdc_autotune(op.handle)
    tune = mdc.mdc_tune_table(op.handle)
    x = torch.as_tensor(synth.ricker_spikes(spec.nt, n, nv, dt=spec.dt), dtype=torch.float32).cuda()
    y = torch.as_tensor(synth.gaussian((spec.nt, n, nv)), dtype=torch.float32).cuda()
    yo, xo = torch.empty_like(x), torch.empty_like(y)
    torch.cuda.synchronize()
    print("setup done", file=sys.stderr, flush=True)

    def step():
        mdc.mdc_forward(op.handle, x, yo, nv)
        mdc.mdc_adjoint(op.handle, y, xo, nv)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    mdc.mdc_profile_read(op.handle)
    mdc.mdc_profile(op.handle, True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    mdc.mdc_profile(op.handle, False)
    ms_stage, cnt = mdc.mdc_profile_read(op.handle)
    ms_step = ev0.elapsed_time(ev1) / args.steps
    flops = 8.0 * spec.nfmax * n * n * nv
    prod_ms = (ms_stage[1] + ms_stage[2]) / max(1, cnt[1] + cnt[2])
    tf = flops / (prod_ms * 1e-3) / 1e12
    kbytes = {"fp32": 8, "bf16x2": 8, "fp16s": 4, "bf16": 4, "fp16": 4}[args.prec] * spec.nfmax * n * n
    if args.prec == "fp32":
        roof = {"bound": "mfma", "achieved": round(tf, 2), "peak": 157.3, "unit": "TFLOP/s", "frac": round(tf / 157.3, 4)}
    else:  # split bf16 products: HBM-bound on the stored kernel bytes
        gbs = kbytes / (prod_ms * 1e-3) / 1e9
        nprod = {"bf16x2": 3, "fp16": 1}.get(args.prec, 2)  # products on the 16-bit matrix cores
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4),
                "mfma_16bit_TFLOPs": round(nprod * tf, 1), "mfma_16bit_frac": round(nprod * tf / 2500.0, 4)}
    # transforms (HBM-bound): time samples 4 B, retained bins 8 B per trace, Q = n * nv traces
    q_tr = n * nv
    fft_bytes = 4.0 * spec.nt * q_tr + 8.0 * spec.nfmax * q_tr
    fft_roof = {}
    for i, k in ((0, "rfft"), (3, "irfft")):
        ms = ms_stage[i] / max(1, cnt[i])
        gb = fft_bytes / (ms * 1e-3) / 1e9
        fft_roof[k] = {"bound": "hbm", "achieved": round(gb, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(gb / HBM_PEAK_GBS, 4), "algorithmic_GB_per_launch": round(fft_bytes / 1e9, 4)}
    out = {"workload": "MDC GEMM nt=1024 nfmax=300 ns=nr=3600 nv=64, fwd+adj per step", "prec": args.prec,
           "tuning_table_ncols_fwd_adj": tune,
           "ms_per_step": round(ms_step, 3), "product_ms": round(prod_ms, 3),
           "complex_TFLOPs": round(tf, 2), "roofline": roof,
           "hbm_GBs_product": round(kbytes / (prod_ms * 1e-3) / 1e9, 1),
           "stage_ms_per_launch": {k: round(ms_stage[i] / max(1, cnt[i]), 4) for i, k in
                                   enumerate(["rfft", "product_fwd", "product_adj", "irfft"])},
           "fft_roofline": fft_roof}
    if emit:
        print(json.dumps(out), flush=True)
    op.close()
    del op, x, y, xo, yo
    torch.cuda.empty_cache()
    return out


def bench_c4(args, niter=30):
    """Marchenko LSQR: nt=1024, nfmax=250, 50x50 traces, 32 points, 30 iterations, d = 1, 2, 4."""
    import numpy as np
    import torch
    from paper_2011_11120_amd import mdc, workloads
    res = {}
    for d in (1, 2, 4):
        case = workloads.marchenko_case(d=d, kappa_value=workloads.kappa("c4"))
        op = mdc.MdcOp(case.spec.nt, case.spec.nfmax, case.n, case.n, max_cols=2 * case.nv, prec=args.prec)
        op.synth_kernel(case.spec, s_index=case.idx, r_index=case.idx)
        mdc.mdc_autotune(op.handle)
        on = torch.as_tensor(case.onset, dtype=torch.int32).cuda()
        fd = torch.as_tensor(case.fd, dtype=torch.float32).cuda()
        dg = op.marchenko_data(on, fd)
        x = torch.empty((2, case.spec.nt, case.n, case.nv), dtype=torch.float32, device="cuda")
        hist = torch.empty(niter + 1, dtype=torch.float64, device="cuda")
        op.lsqr(dg, niter, kind=mdc.MDC_OP_MARCHENKO, nv=case.nv, onset=on, out=(x, hist))  # warm-up + graph capture
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(max(1, args.steps)):  # timed solves: iterations replay the captured graph
            ev0.record()
            op.lsqr(dg, niter, kind=mdc.MDC_OP_MARCHENKO, nv=case.nv, onset=on, out=(x, hist))
            ev1.record()
            torch.cuda.synchronize()
            times.append(ev0.elapsed_time(ev1) / 1e3)
        mdc.mdc_profile_read(op.handle)
        mdc.mdc_profile(op.handle, True)  # one more solve with per-stage events (eager, no graph)
        op.lsqr(dg, niter, kind=mdc.MDC_OP_MARCHENKO, nv=case.nv, onset=on, out=(x, hist))
        torch.cuda.synchronize()
        mdc.mdc_profile(op.handle, False)
        ms_stage, cnt = mdc.mdc_profile_read(op.handle)
        h = hist.cpu().numpy()
        n = case.n
        prod_ms = (ms_stage[1] + ms_stage[2]) / max(1, cnt[1] + cnt[2])
        flops = 8.0 * case.spec.nfmax * n * n * 2 * case.nv
        res[f"d{d}"] = {"n": n, "s_per_solve": round(float(np.median(times)), 4),
                        "solves_per_s": round(1.0 / float(np.median(times)), 3),
                        "rel_residual": float(h[-1] / h[0]),
                        "product_ms": round(prod_ms, 4), "product_TFLOPs": round(flops / prod_ms / 1e9, 2),
                        "stage_ms_total": [round(v, 2) for v in ms_stage], "stage_counts": cnt}
        op.close()
        del op
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "Marchenko LSQR nt=1024 nfmax=250 50x50 grid nv=32 (N=64 fused) 30 it",
                      "prec": f"kernel {args.prec}, fp32 vectors, fp64 scalars", "results": res}), flush=True)


def c5_requests(R, seed=3):
    """Seeded request mix: nv in [1, 64], iterations in [10, 60], decimation in {1, 2, 4};
    focusing points are the first nv of an 8 x 8 grid (20 m) centred under the array at 650 m."""
    import numpy as np
    from paper_2011_11120_amd import synth
    u = synth.rng_uniform(seed, synth.STREAM_SERVE, np.arange(4 * R)).reshape(R, 4)
    vx, vy, vz = synth.virtual_points(100, 100, 20.0, 8, 8)
    reqs = []
    for k in range(R):
        nv = 1 + int(u[k, 0] * 64)
        niter = 10 + int(u[k, 1] * 51)
        decim = (1, 2, 4)[int(u[k, 2] * 3)]
        reqs.append(dict(nv=nv, niter=niter, decim=decim, vx=vx[:nv], vy=vy[:nv], vz=vz[:nv], u=float(u[k, 3])))
    return reqs


def serve_run(srv, reqs, rate=None, cap=6, keep=()):
    """Submit requests (closed loop with at most `cap` outstanding, or Poisson arrivals at `rate`/s),
    poll until all finish; returns per-request latencies and the kept solutions (host copies)."""
    import numpy as np
    import torch
    t0 = time.perf_counter()
    arrivals = []
    if rate is not None:
        acc = 0.0
        for r in reqs:
            acc += -np.log(1.0 - r["u"]) / rate  # exponential inter-arrival times from the seeded draw
            arrivals.append(acc)
    pending, out, kept = list(range(len(reqs))), {}, {}
    live = {}
    while pending or live:
        now = time.perf_counter() - t0
        while pending and (len(live) < cap if rate is None else arrivals[pending[0]] <= now):
            k = pending.pop(0)
            r = reqs[k]
            rid = srv.submit(r["vx"], r["vy"], r["vz"], r["niter"], r["decim"], hist=False)
            live[rid] = k
        for rid in list(live):
            done, lat = srv.poll(rid)
            if done != 0:
                k = live.pop(rid)
                out[k] = lat
                if k in keep:
                    kept[k] = srv.result(rid)[0].cpu()
                srv.release(rid)
                print(f"  request {k}: nv={reqs[k]['nv']} it={reqs[k]['niter']} d={reqs[k]['decim']} "
                      f"latency {lat:.2f} s", file=sys.stderr, flush=True)
        time.sleep(0.002)
    torch.cuda.empty_cache()
    return out, kept


def c5_leg(mdc, op, spec, reqs, arena_t, args, rate=None, keep=()):
    """One served stream; every figure comes from the server's own statistics: solves/s = completions /
    (last completion - first submission), p50/p99 over the completions after the first `skip`."""
    srv = mdc.Server(op, spec.nx, dx=spec.dx, dt=spec.dt, arena=arena_t, sublattice=args.c5_sublattice)
    lat, kept = serve_run(srv, reqs, rate=rate, keep=keep)
    st, gs, ps = srv.stats(skip=args.skip), srv.graph_stats(), srv.phase_stats()
    srv.close()
    return {"requests": len(reqs), "solves_per_s": round(st["solves_per_s"], 4),
            "p50_s": round(st["p50_s"], 3), "p99_s": round(st["p99_s"], 3),
            "latency_samples": st["completed"] - min(args.skip, st["completed"]),
            "mean_latency_s": round(float(sum(lat.values()) / max(1, len(lat))), 3),
            "max_active": st["max_active"], "steps": st["steps"],
            "graph_steps": {"captured": gs["captured"], "replayed": gs["replayed"]},
            "lockstep": {"request_steps": ps["request_steps"], "deferred_requests": ps["deferred"],
                         "deferred_wait_s": round(ps["deferred_s"], 3)}}, kept


def bench_c5(args, emit=True):
    """Served stream: 100 x 100 traces, nfmax=200, nt=1024; FP32 vs 16-bit kernel storage.

    Per format: a closed loop (6 outstanding requests) gives the capacity; a Poisson stream at 0.7 x
    the FP32 capacity (the same rate for every format), and for the 16-bit formats a second one at
    0.7 x their own capacity; optionally a light-load stream (--c5-light, a fraction of the format's
    capacity) on the first requests, where the lockstep statistics show what a pass serving both
    directions at once could save."""
    import numpy as np
    import torch
    from paper_2011_11120_amd import mdc, workloads
    spec = workloads.marchenko_spec(nx=100, nt=1024, nfmax=200, kappa_value=workloads.kappa("c5"))
    reqs = c5_requests(args.requests)
    results, sols = {}, {}
    rate32 = args.c5_rate
    precs = args.c5_precs.split(",")
    for prec in precs:
        op = mdc.MdcOp(spec.nt, spec.nfmax, spec.n, spec.n, max_cols=args.c5_max_cols, prec=prec)
        op.synth_kernel(spec)
        mdc.mdc_autotune(op.handle)
        torch.cuda.synchronize()
        free = torch.cuda.mem_get_info()[0]
        outs = sorted((2 * spec.nt * spec.n * r["nv"] * 4 for r in reqs), reverse=True)
        out_bytes = sum(outs[:6])  # outputs of the (at most) 6 outstanding requests
        levels = sum(mdc.serve_level_bytes(op.handle, d) for d in (2, 4) if args.c5_sublattice & d)
        arena = int(max(free - out_bytes - (4 << 30), levels + (1 << 30)))
        arena_t = torch.empty(arena, dtype=torch.uint8, device="cuda")
        print(f"{prec}: kernel {op.resident.numel() / 1e9:.1f} GB, arena {arena / 1e9:.1f} GB "
              f"({levels / 1e9:.1f} GB lattice levels)", file=sys.stderr, flush=True)
        res = {"kernel_GB": round(op.resident.numel() / 1e9, 1), "arena_GB": round(arena / 1e9, 1),
               "lattice_levels_GB": round(levels / 1e9, 1)}
        picks = list(range(0, len(reqs), max(1, len(reqs) // args.c5_alone)))[:args.c5_alone] if args.c5_alone else []
        res["closed"], kept = c5_leg(mdc, op, spec, reqs, arena_t, args, keep=tuple(sorted({0, 1, *picks})))
        sols[prec] = {k: kept[k] for k in (0, 1)}
        cap = res["closed"]["solves_per_s"]
        if prec == "fp32" and rate32 is None:
            rate32 = 0.7 * cap
        if getattr(args, "c5_closed_only", False):
            pass
        elif rate32 is not None:
            res["poisson_fp32_rate"], _ = c5_leg(mdc, op, spec, reqs, arena_t, args, rate=rate32)
            res["poisson_fp32_rate"]["rate_per_s"] = round(rate32, 4)
        if prec != "fp32" and not getattr(args, "c5_closed_only", False):
            res["poisson_own_rate"], _ = c5_leg(mdc, op, spec, reqs, arena_t, args, rate=0.7 * cap)
            res["poisson_own_rate"]["rate_per_s"] = round(0.7 * cap, 4)
        if picks:  # sampled requests of the closed loop solved again alone
            errs = {}
            for k in picks:
                _, alone = c5_leg(mdc, op, spec, [reqs[k]], arena_t, args, keep=(0,))
                a, m = alone[0], kept[k]
                errs[k] = float(torch.linalg.vector_norm(m - a) / torch.linalg.vector_norm(a))
            res["alone_vs_mix"] = {"requests": picks, "rel_diff": errs, "max_rel_diff": max(errs.values())}
        del kept
        if args.c5_light > 0:
            light = reqs[:args.c5_light_requests]
            res["poisson_light"], _ = c5_leg(mdc, op, spec, light, arena_t, args, rate=args.c5_light * cap)
            res["poisson_light"]["rate_per_s"] = round(args.c5_light * cap, 4)
        results[prec] = res
        op.close()
        del op, arena_t
        torch.cuda.empty_cache()
    diff = {}
    for p in precs[1:]:
        diff[p] = {k: float(torch.linalg.vector_norm(sols[p][k] - sols[precs[0]][k]) /
                            torch.linalg.vector_norm(sols[precs[0]][k])) for k in sols[p]}
    out = {"workload": "served Marchenko LSQR, 100x100 traces, nfmax=200, nt=1024, "
                       f"{len(reqs)} requests (nv 1-64, 10-60 it, d 1/2/4), first {args.skip} "
                       "completions excluded from p50/p99",
           "sublattice": args.c5_sublattice, "column_budget": args.c5_max_cols,
           "requests": [{k: r[k] for k in ("nv", "niter", "decim")} for r in reqs],
           "results": results, "poisson_rate_fp32_capacity_x0.7": rate32,
           "solution_rel_diff_vs_" + precs[0]: diff}
    if emit:
        print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
