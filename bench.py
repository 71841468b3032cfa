"""Benchmark: MPDATA steps on one MI355X, grid-point updates per second.

Default workload: the 1024x512x80 lat-lon grid, FP64, 3 passes per step with
the non-oscillatory limiter, divergence-free streamfunction winds (max
Courant 0.6), lognormal tracer.  One "step" advances every cell by one full
MPDATA time step (all passes).  Inputs are resident in HBM before timing.

Inputs are generated in FP64 and rounded to FP32 once, and the FP64 and
FP32 runs both start from those values, so that their difference measures
arithmetic precision only.

Prints ONE JSON line.  Besides the headline value (FP64) it carries
  roofline      the algorithmic HBM bytes of one cell-step (read psi, Cx, Cy,
                Cz, G, write psi: 48 B in FP64, 24 B in FP32) times the cells
                one launch of the dominant kernel processes, over that
                kernel's mean launch time (HIP events on the stream it runs
                on), against the 8 TB/s HBM peak; the step-level fraction
                (the same bytes over the whole step's time) is beside it;
  fp32          the same workload in FP32 storage and arithmetic: throughput,
                the same roofline figures, and its error against the FP64
                oracle (max and RMS, mass drift, min psi);
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

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
METRIC = "grid-point updates/s per MPDATA step (FP64 vs FP32, HBM %); adjoint/forward time"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name, dtype):
    import workloads

    if name == "latlon-1024x512x80":
        w = workloads.rounded_to_fp32(workloads.latlon_wave())
    elif name == "latlon-256x128x60":
        w = workloads.latlon_solid_body()
    elif name == "2d-64x64":
        w = workloads.gaussian_2d()
    else:
        raise SystemExit(f"unknown workload {name}")
    return w


def bytes_per_cell_step(elem, with_cz=True):
    # algorithmic HBM traffic of one step: read psi, Cx, Cy, (Cz), G; write psi
    return elem * ((5 if with_cz else 4) + 1)


def traffic_record(kernel_src_sha, dtype, workload, kernel):
    """Counter-derived HBM bytes per launch of `kernel`, if the committed
    record was taken on this workload, on this kernel and on the kernel
    source as it is now (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_fused_pass_{dtype}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != kernel_src_sha or rec.get("kernel_kind") != kernel:
        return None
    grid = rec.get("workload", "").split(" ")[0]     # e.g. latlon-1024x512x80
    if not grid or not workload.startswith(grid):
        return None
    return rec.get("bytes_per_launch")


# Kernel kinds the library times, with the words per cell one launch moves
# by this library's own accounting (the pass's reads and writes).
KERNEL_KINDS = {
    "pass_donor": "first corrective pass with the donor-cell pass folded in (k_pass, DONOR)",
    "pass": "fused corrective pass (k_pass)",
    "donor": "donor-cell pass (k_donor_march)",
    "stage": "per-stage kernels of one step",
}


def model_words(kind, w, last):
    from paper_1908_06094_amd import model

    if kind == "pass_donor":
        return 5 + (1 if last else 4)          # psi^n, Cx, Cy, Cz, G; new iterate (+ 3 velocities)
    if kind == "pass":
        return model.pass_kernel_words(not last, True)
    if kind == "donor":
        return model.donor_kernel_words(True)
    return model.STEP_WORDS


def roofline(w, elem, dtype, fw, steps):
    """Roofline of the dominant kernel (the timed kernel kind with the largest
    total time; one whole step under a graph replay): the algorithmic bytes
    of one cell-step (6 words) times the cells one launch processes, over the
    mean launch time.  Returns that record, the same launch time against this
    library's per-launch word model, and the ALU figure."""
    from paper_1908_06094_amd import model, profsum

    step_bytes = bytes_per_cell_step(elem) * w.cells
    timed = {k: fw[k] for k in KERNEL_KINDS if fw[k][1]}
    breakdown = {k: {"launches": n, "avg_launch_us": round(ms * 1e3 / n, 2), "ms_per_step": round(ms / steps, 4)}
                 for k, (ms, n) in timed.items()}
    if timed:
        dom = max(timed, key=lambda k: timed[k][0])
        ms, n = timed[dom]
        avg_s = ms * 1e-3 / n
        kernel = KERNEL_KINDS[dom]
        traffic = traffic_record(profsum.kernel_source_sha(), dtype, w.name, dom) if dom.startswith("pass") else None
        # which pass of the step the kind is: the donor-fused pass is pass 2, the plain ones 3 .. iters
        last = (dom == "pass_donor" and w.iters == 2) or (dom == "pass" and w.iters == 3)
        model_bytes = model_words(dom, w, last) * elem * w.cells
        ops = model.corrective_pass_ops(w.limiter) if dom.startswith("pass") else model.step_ops(w.iters, w.limiter)
    else:
        avg_s = fw["ev_ms"] * 1e-3 / steps
        kernel = "one whole step (HIP events around the replay)"
        traffic = None
        model_bytes = step_bytes
        ops = model.step_ops(w.iters, w.limiter)
    achieved = step_bytes / avg_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_source": (f"committed counter record profiles/traffic_fused_pass_{dtype}.json "
                               "(FETCH_SIZE x copy factor + WRITE_SIZE per launch; its kernel and kernel-source "
                               "hash match)" if traffic is not None else None),
            "kernel": kernel, "bytes_per_launch": int(step_bytes),
            "bytes_rule": f"{bytes_per_cell_step(elem)} B per cell (read psi, Cx, Cy, Cz, G; write psi) x {w.cells} cells",
            "avg_launch_us": round(avg_s * 1e6, 2),
            "step_frac": round(step_bytes * steps / (fw["ev_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernels": breakdown}
    pass_model = {"bytes_per_launch": int(model_bytes),
                  "rule": "the dominant kernel's own reads and writes per cell",
                  "achieved_GBps": round(model_bytes / avg_s / 1e9, 1),
                  "frac": round(model_bytes / avg_s / 1e9 / HBM_PEAK_GBS, 4)}
    ops_s = ops.total * w.cells / avg_s
    alu = {"bound": "alu", "achieved": round(ops_s / 1e12, 3), "peak": round(model.FP64_VALU_OPS_PEAK / 1e12, 2),
           "unit": "T FP64 ops/s", "frac": round(ops_s / model.FP64_VALU_OPS_PEAK, 4),
           "ops_per_cell": ops.total, "divisions_per_cell": ops.divisions}
    return roof, pass_model, alu


def time_forward(mp, torch, dev, w, dtype, steps, warmup, use_graph=False):
    """`steps` steps of workload w in `dtype` after `warmup` steps, inputs
    resident in HBM: wall and HIP-event times and the per-kernel launch times
    recorded on the launch stream."""
    tdt = torch.float64 if dtype == "f64" else torch.float32
    psi = torch.from_numpy(w.psi).to(dev, tdt)
    cx, cy, cz, g = (torch.from_numpy(a).to(dev, tdt) for a in (w.cx, w.cy, w.cz, w.g))
    p = mp.problem_for(w.shape, w.bc, w.iters, w.limiter, dtype)
    ws = torch.empty(mp.workspace_bytes(p, mp.MPDATA_OP_RUN), dtype=torch.uint8, device=dev)
    kw = dict(iters=w.iters, limiter=w.limiter, bc=w.bc, workspace=ws)
    stream = torch.cuda.current_stream(dev)
    if warmup:
        mp.run(psi, cx, cy, cz, g, warmup, **kw)
    torch.cuda.synchronize()
    log(f"[bench] {dtype}: warmup {warmup} steps done")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    graph = None
    if use_graph:
        # the K steps captured once on a side stream, then replayed
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                mp.run(psi, cx, cy, cz, g, steps, **kw)
        stream.wait_stream(side)
        graph.replay()               # one untimed replay
        torch.cuda.synchronize()
        log(f"[bench] captured {steps} steps in one graph")
    torch.cuda.synchronize()
    mp.timing_enable(True)          # HIP events around every kernel launch, on the launch stream
    t0 = time.perf_counter()
    ev0.record(stream)
    if graph is not None:
        graph.replay()
    else:
        mp.run(psi, cx, cy, cz, g, steps, **kw)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mp.timing_enable(False)
    r = {"wall": wall, "ev_ms": ev0.elapsed_time(ev1), "graph": graph is not None}
    r["pass_donor"] = mp.timing_read(mp.MPDATA_KERNEL_PASS_DONOR)
    r["pass"] = mp.timing_read(mp.MPDATA_KERNEL_PASS)
    r["donor"] = mp.timing_read(mp.MPDATA_KERNEL_DONOR)
    r["stage"] = mp.timing_read(mp.MPDATA_KERNEL_STAGE)
    log(f"[bench] {dtype}: {steps} steps: wall {wall*1e3:.2f} ms, events {r['ev_ms']:.2f} ms; " +
        ", ".join(f"{k} {r[k][1]} x {r[k][0] / r[k][1]:.3f} ms" for k in KERNEL_KINDS if r[k][1]))
    del psi, cx, cy, cz, g, ws
    return r


def gpu_accuracy(mp, torch, dev, w, dtype, n, want):
    """n steps on the GPU in `dtype` from the workload's start against the
    FP64 oracle's result `want` from the same start."""
    import numpy as np

    tdt = torch.float64 if dtype == "f64" else torch.float32
    x = torch.from_numpy(w.psi).to(dev, tdt)
    cx, cy, cz, g = (torch.from_numpy(a).to(dev, tdt) for a in (w.cx, w.cy, w.cz, w.g))
    m0 = mp.mass(x, g, bc=w.bc)
    mp.run(x, cx, cy, cz, g, n, iters=w.iters, limiter=w.limiter, bc=w.bc)
    m1 = mp.mass(x, g, bc=w.bc)
    got = x.double().cpu().numpy()
    diff = got - want
    return {"steps": n, "max_abs_err_rel": float(np.max(np.abs(diff)) / np.max(np.abs(want))),
            "rms_err_rel": float(np.sqrt(np.mean(diff * diff)) / np.sqrt(np.mean(want * want))),
            "mass_drift_rel": float(abs(m1 - m0) / m0), "min_psi": float(got.min()),
            "against": "the CPU oracle (FP64) from the same (FP32-representable) start"}


def time_adjoint(mp, torch, dev, steps=20, checkpoint_every=5, reps=3):
    """Adjoint/forward time on the 256x128x60 lat-lon workload (FP64, 2 passes,
    limiter, solid-body winds): mpdata_adjoint over `steps` steps with
    checkpoints every `checkpoint_every` steps (its forward recomputation
    included) against `steps` forward steps."""
    import numpy as np

    import workloads

    w = workloads.latlon_solid_body()
    wt = torch.from_numpy(workloads.cost_weights(w.shape)).to(dev)
    psi0, cx, cy, cz, g = (torch.from_numpy(a).to(dev) for a in (w.psi, w.cx, w.cy, w.cz, w.g))
    kw = dict(iters=2, limiter=True, bc=w.bc)
    out = psi0.clone()
    mp.run(out, cx, cy, cz, g, steps, **kw)
    seed = 2 * wt * out
    mp.adjoint(psi0, cx, cy, cz, g, seed, steps, checkpoint_every=checkpoint_every, **kw)   # warm-up
    torch.cuda.synchronize()
    fwd, adj = [], []
    for _ in range(reps):
        t = psi0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mp.run(t, cx, cy, cz, g, steps, **kw)
        torch.cuda.synchronize()
        fwd.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        mp.adjoint(psi0, cx, cy, cz, g, seed, steps, checkpoint_every=checkpoint_every, **kw)
        torch.cuda.synchronize()
        adj.append(time.perf_counter() - t0)
    f, a = float(np.median(fwd)), float(np.median(adj))
    log(f"[bench] adjoint: forward {f*1e3:.2f} ms, adjoint {a*1e3:.2f} ms for {steps} steps")
    return {"workload": f"{w.name} FP64, {steps} steps, checkpoint every {checkpoint_every}",
            "forward_ms": round(f * 1e3, 3), "adjoint_ms": round(a * 1e3, 3), "ratio": round(a / f, 2)}


def time_batched(mp, torch, dev, steps=20, reps=3):
    """The batched workload: 64 lat-lon problems of uneven sizes with 1-8
    tracers each (FP32, 2 passes, limiter), 20 steps per call, one persistent
    launch per pass, replayed from a captured HIP graph (autotuned variant)."""
    import numpy as np

    import workloads

    probs_h = workloads.batched_problems()
    probs = [{k: torch.from_numpy(v).to(dev) for k, v in p.items()} for p in probs_h]
    del probs_h
    start = [p["psi"].clone() for p in probs]
    tracer_cells = sum(p["psi"].numel() for p in probs)
    _, _, nb = mp.batch_problem(probs, iters=2)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream(dev)
    # the tuner appends its choice to the file MPDATA_TUNE_CACHE names
    import tempfile

    old_cache = os.environ.get("MPDATA_TUNE_CACHE")
    cache = tempfile.NamedTemporaryFile(prefix="mpdata_tune_", suffix=".txt", delete=False)
    cache.close()
    os.environ["MPDATA_TUNE_CACHE"] = cache.name
    with torch.cuda.stream(stream):
        mp.run_batched(probs, steps, iters=2, graph=True, tune=True, workspace=ws, stream=stream)  # tune + capture
        stream.synchronize()
    if old_cache is None:
        del os.environ["MPDATA_TUNE_CACHE"]
    else:
        os.environ["MPDATA_TUNE_CACHE"] = old_cache
    with open(cache.name) as f:
        lines = [ln.rstrip("\n").split("\t") for ln in f if ln.strip()]
    os.unlink(cache.name)
    tuned = None
    if lines and lines[-1][-1].isdigit():
        v = int(lines[-1][-1])
        lanes, threads, wgs, donor = mp.BATCH_VARIANTS_F32[v]
        tuned = {"index": v, "row_lanes": lanes, "threads": threads, "workgroups_per_cu": wgs,
                 "donor_cell_pass": donor}
    with torch.cuda.stream(stream):
        times = []
        for _ in range(reps):
            for p, s0 in zip(probs, start):
                p["psi"].copy_(s0)
            stream.synchronize()
            t0 = time.perf_counter()
            mp.run_batched(probs, steps, iters=2, graph=True, tune=True, workspace=ws, stream=stream)
            stream.synchronize()
            times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    log(f"[bench] batched: {tracer_cells / 1e6:.0f} M tracer-cells x {steps} steps in {t * 1e3:.1f} ms")
    return {"workload": f"64 lat-lon problems (nx 64-512, ny 32-256, nz 20-80), 1-8 tracers, FP32, 2 passes, "
                        f"limiter, {steps} steps, HIP graph",
            "tracer_cells": tracer_cells, "value": round(tracer_cells * steps / t, 1),
            "unit": "tracer-cell updates/s", "ms_per_step": round(t * 1e3 / steps, 4), "tuned_variant": tuned}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _urun_timed(mp, torch, dev, u, steps):
    """Wall and mean kernel time of `steps` unstructured steps of workload u."""
    import numpy as np

    dm = mp.DeviceMesh.from_octa(u.mesh, u.nz, pivbz=u.pivbz)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    psi, vn, w, rho = t(u.psi), t(u.vn), t(u.w), t(u.rho)
    ws = torch.empty(u.points * 8 + 256, dtype=torch.uint8, device=dev)
    mp.urun(dm, psi, vn, w, rho, 2, workspace=ws)
    torch.cuda.synchronize()
    mp.timing_enable(True)
    t0 = time.perf_counter()
    mp.urun(dm, psi, vn, w, rho, steps, workspace=ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mp.timing_enable(False)
    kms, kn = mp.timing_read(mp.MPDATA_KERNEL_USTEP)
    return wall, kms * 1e-3 / max(kn, 1)


def time_unstructured(mp, torch, dev, steps=20, cpu=True):
    """The paper's own dwarf: the edge-based donor-cell step on an octahedral
    grid of 70 144 nodes (O128: 209 864 edges) x 80 levels, FP64 (solid-body
    winds through the dual faces, a zero vertical wind read all the same,
    unit density, a cosine bell plus noise), `steps` steps; and the same
    mesh with its nodes and edges numbered at random and along a Hilbert
    curve, against the row-by-row numbering (the kernel and the arithmetic
    are the same; only the memory locality of the gathers differs)."""
    from workloads import octahedral as octa

    u = octa.octahedral_workload(128, 80)
    m = u.mesh
    wall, avg_s = _urun_timed(mp, torch, dev, u, steps)
    _, avg_r = _urun_timed(mp, torch, dev, octa.renumbered_workload(u), steps)
    _, avg_h = _urun_timed(mp, torch, dev, octa.renumbered_workload(u, numbering="hilbert"), steps)
    # algorithmic traffic per step: read psi, w, rho and write psi per node
    # and level, read vn per edge and level (the edge fluxes and the vertical
    # fluxes stay on chip)
    nbytes = (4 * m.n_nodes + m.n_edges) * u.nz * 8
    res = {"workload": f"{u.name}: {m.n_nodes} nodes, {m.n_edges} edges, {u.nz} levels, FP64, {steps} steps",
           "value": round(u.points * steps / wall, 1), "unit": "grid-point updates/s",
           "ms_per_step": round(wall * 1e3 / steps, 4), "kernel_us": round(avg_s * 1e6, 2),
           "bytes_per_step": nbytes, "hbm_GBps": round(nbytes / avg_s / 1e9, 1),
           "hbm_frac": round(nbytes / avg_s / 1e9 / HBM_PEAK_GBS, 4),
           "table2_accesses_per_plane_fused": 5 * m.n_nodes,
           "numbering": {"row_by_row_kernel_us": round(avg_s * 1e6, 2), "random_kernel_us": round(avg_r * 1e6, 2),
                         "hilbert_kernel_us": round(avg_h * 1e6, 2),
                         "random_over_row_by_row": round(avg_r / avg_s, 3),
                         "hilbert_over_row_by_row": round(avg_h / avg_s, 3)}}
    if cpu:
        import oracle

        t1 = time.perf_counter()
        oracle.ustep(m.edges, m.node_ptr, m.node_edges, m.node_sign, m.dual_volume, u.psi, u.vn, u.w, u.rho,
                     u.pivbz)
        cs = time.perf_counter() - t1
        res["cpu_oracle"] = {"value": round(u.points / cs, 1), "unit": "grid-point updates/s", "cores": 1,
                             "sample": f"1 step of {u.name}, {cs:.2f} s"}
    log(f"[bench] unstructured: {res}")
    return res


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
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched 64-problem FP32 measurement")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward timing on the 256x128x60 workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, run a plain device copy of one field (for counter calibration)")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the FP32 leg of the default FP64 run")
    ap.add_argument("--no-unstructured", action="store_true",
                    help="skip the edge-based step on the octahedral grid")
    ap.add_argument("--graph", action="store_true",
                    help="time the steps as replays of one captured HIP graph (launch-bound small grids)")
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
    elem = 8 if args.dtype == "f64" else 4
    log(f"[bench] workload {w.name} shape={w.shape} iters={w.iters} limiter={w.limiter} dtype={args.dtype}")
    dev = torch.device("cuda:0")
    fw = time_forward(mp, torch, dev, w, args.dtype, args.steps, args.warmup, args.graph)
    wall, ev_ms = fw["wall"], fw["ev_ms"]
    ms_per_step = wall * 1e3 / args.steps
    updates = w.cells * args.steps / wall
    roof, pass_model, alu = roofline(w, elem, args.dtype, fw, args.steps)

    # the FP32 leg of the same workload (inputs already FP32-representable)
    fp32 = None
    if args.dtype == "f64" and not args.no_fp32:
        f3 = time_forward(mp, torch, dev, w, "f32", args.steps, args.warmup, args.graph)
        r32, m32, _ = roofline(w, 4, "f32", f3, args.steps)
        fp32 = {"value": round(w.cells * args.steps / f3["wall"], 1), "unit": "grid-point updates/s",
                "ms_per_step": round(f3["wall"] * 1e3 / args.steps, 4),
                "ms_per_step_events": round(f3["ev_ms"] / args.steps, 4),
                "roofline": r32, "roofline_pass_model": m32,
                "speedup_vs_f64": round(wall / f3["wall"], 3)}

    adjoint = None
    if not args.no_adjoint and args.dtype == "f64":
        adjoint = time_adjoint(mp, torch, dev)
    batched = None
    if not args.no_batched:
        batched = time_batched(mp, torch, dev)
    unstructured = None
    if not args.no_unstructured:
        unstructured = time_unstructured(mp, torch, dev, cpu=not args.no_cpu_baseline)

    # practical HBM ceiling: a plain device copy of one field, read + write
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    stream = torch.cuda.current_stream(dev)
    csrc = torch.empty(w.cells, dtype=tdt, device=dev).fill_(1.0)
    cdst = torch.empty_like(csrc)
    cdst.copy_(csrc)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    copy_ms = []
    for _ in range(5):
        c0.record(stream)
        cdst.copy_(csrc)
        c1.record(stream)
        torch.cuda.synchronize()
        copy_ms.append(c0.elapsed_time(c1))
    copy_gbs = 2 * w.cells * elem / (float(np.median(copy_ms)) * 1e-3) / 1e9
    del csrc, cdst

    if args.copy_calibration:
        src = torch.empty(w.cells, dtype=tdt, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 copies of {src.numel() * elem} bytes")

    cpu = None
    accuracy = None
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
               "sample": f"{n} full step(s) of {w.name} (FP64, plain C, OpenMP over levels), {cpu_s:.1f} s",
               "cpu_model": cpu_model(), "cpus_visible": len(os.sched_getaffinity(0))}
        log(f"[bench] cpu oracle: {n} steps in {cpu_s:.1f} s")
        # one thread, on the lowest levels of the same grid (same winds and
        # tracer; the oracle's cost per cell does not depend on the level count)
        nz1 = min(w.shape[0], 4)
        rp1 = oracle.RefProblem(w.shape[2], w.shape[1], nz1, bc=w.bc, iters=w.iters, limiter=w.limiter)
        threads = oracle.num_threads()
        oracle.set_num_threads(1)
        try:
            sl = (slice(0, nz1),)
            t1 = time.perf_counter()
            oracle.step(rp1, src[sl], w.cx[sl], w.cy[sl], w.cz[sl], w.g[sl])
            one_s = time.perf_counter() - t1
        finally:
            oracle.set_num_threads(threads)
        cells1 = w.shape[2] * w.shape[1] * nz1
        cpu["one_thread"] = {"value": round(cells1 / one_s, 1), "unit": "grid-point updates/s",
                             "sample": f"1 step of levels 0-{nz1 - 1} of {w.name}, {one_s:.2f} s"}
        log(f"[bench] cpu oracle, 1 thread: {cells1} cells in {one_s:.2f} s")
        # the same n steps on the GPU from the same start: errors against the oracle
        accuracy = gpu_accuracy(mp, torch, dev, w, args.dtype, n, out)
        log(f"[bench] accuracy ({args.dtype}) after {n} steps: {accuracy}")
        if fp32 is not None:
            fp32["accuracy"] = gpu_accuracy(mp, torch, dev, w, "f32", n, out)
            log(f"[bench] accuracy (f32) after {n} steps: {fp32['accuracy']}")

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
        "roofline_pass_model": pass_model,
        "roofline_alu": alu,
        "fp32": fp32,
        "step": {"ms_per_step_events": round(ev_ms / args.steps, 4),
                 "hbm_frac_step": roof["step_frac"]},
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "hbm_copy": {"GBps": round(copy_gbs, 1), "frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4),
                     "pass_frac_of_copy": round(roof["achieved"] / copy_gbs, 4),
                     "what": "torch device copy of one field (read + write), median of 5"},
        "graph": fw["graph"],
        "adjoint": adjoint,
        "batched": batched,
        "unstructured": unstructured,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
