"""Benchmark: MPDATA steps on one MI355X, grid-point updates per second.

Default workload: the 1024x512x80 lat-lon grid, FP64, 3 passes per step with
the non-oscillatory limiter, divergence-free streamfunction winds (max
Courant 0.6), lognormal tracer.  One "step" advances every cell by one full
MPDATA time step (all passes).  Inputs are resident in HBM before timing.

Prints ONE JSON line.  Besides the headline value it carries
  roofline      the dominant kernel's algorithmic HBM bytes per launch over its
                average launch time (HIP events on the stream it runs on),
                against the 8 TB/s HBM peak;
  cpu_baseline  the CPU oracle (plain C, OpenMP, FP64) timed on this host on a
                bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "grid-point updates/s per MPDATA step (FP64 vs FP32, HBM %); adjoint/forward time"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name, dtype):
    import numpy as np

    import workloads

    if name == "latlon-1024x512x80":
        w = workloads.config3()
        if dtype == "f32":
            w = workloads.config3_fp32_inputs(w)
    elif name == "latlon-256x128x60":
        w = workloads.config2()
    elif name == "2d-64x64":
        w = workloads.config1()
    else:
        raise SystemExit(f"unknown workload {name}")
    return w


def bytes_per_cell_step(elem, with_cz=True):
    # algorithmic HBM traffic of one step: read psi, Cx, Cy, (Cz), G; write psi
    return elem * ((5 if with_cz else 4) + 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="latlon-1024x512x80")
    ap.add_argument("--dtype", default="f64", choices=("f64", "f32"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the domain-decomposition design is described, not built)", file=sys.stderr)
        raise SystemExit(2)

    import numpy as np
    import torch

    import paper_1908_06094_amd as mp

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    mp.lib()  # fail loudly if the HIP library is missing

    w = make_workload(args.workload, args.dtype)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    elem = 8 if args.dtype == "f64" else 4
    log(f"[bench] workload {w.name} shape={w.shape} iters={w.iters} limiter={w.limiter} dtype={args.dtype}")
    dev = torch.device("cuda:0")
    psi = torch.from_numpy(w.psi).to(dev, tdt)
    cx, cy, cz, g = (torch.from_numpy(a).to(dev, tdt) for a in (w.cx, w.cy, w.cz, w.g))
    p = mp.problem_for(w.shape, w.bc, w.iters, w.limiter, args.dtype)
    ws = torch.empty(mp.workspace_bytes(p, mp.MPDATA_OP_RUN), dtype=torch.uint8, device=dev)
    kw = dict(iters=w.iters, limiter=w.limiter, bc=w.bc, workspace=ws)

    stream = torch.cuda.current_stream(dev)
    if args.warmup:
        mp.run(psi, cx, cy, cz, g, args.warmup, **kw)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps done")

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    mp.run(psi, cx, cy, cz, g, args.steps, **kw)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    log(f"[bench] {args.steps} steps: wall {wall*1e3:.2f} ms, events {ev_ms:.2f} ms")

    ms_per_step = wall * 1e3 / args.steps
    updates = w.cells * args.steps / wall
    step_bytes = bytes_per_cell_step(elem) * w.cells
    ev_step_s = ev_ms * 1e-3 / args.steps
    achieved = step_bytes / ev_step_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "whole step (all stage kernels)", "bytes_per_launch": step_bytes,
            "avg_launch_us": round(ev_step_s * 1e6, 2)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        if not os.path.exists(oracle.lib_path()):
            oracle.build()
        rp = oracle.RefProblem(w.shape[2], w.shape[1], w.shape[0], bc=w.bc, iters=w.iters, limiter=w.limiter)
        # bounded sample: whole-grid steps of the same workload, as many as fit
        # the time target (at least one)
        src = w.psi.astype(np.float64)
        t1 = time.perf_counter()
        out = oracle.step(rp, src, w.cx, w.cy, w.cz, w.g)
        one = time.perf_counter() - t1
        n = 1
        while (n + 1) * one <= args.cpu_seconds:
            out = oracle.step(rp, out, w.cx, w.cy, w.cz, w.g)
            n += 1
        cpu_s = time.perf_counter() - t1
        cpu = {"value": round(w.cells * n / cpu_s, 1), "unit": "grid-point updates/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{n} full step(s) of {w.name} (FP64, plain C, OpenMP over levels), {cpu_s:.1f} s"}
        log(f"[bench] cpu oracle: {n} steps in {cpu_s:.1f} s")

    line = {
        "metric": METRIC,
        "value": round(updates, 1),
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.shape[2], "ny": w.shape[1], "nz": w.shape[0],
                   "iters": w.iters, "limiter": w.limiter, "bc": list(w.bc), "parallelism": "single-gpu"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
