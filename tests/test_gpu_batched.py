"""Batched runs (mpdata_run_batched): many problems and tracers in one
persistent launch per pass, with and without a captured HIP graph (needs a
GPU).  Checked per problem and tracer against the CPU oracle, and bitwise
against the single-problem fused path."""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

P, C = "periodic", "closed"


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


SHAPES = [(5, 19, 70, 2), (3, 40, 131, 1), (7, 13, 64, 3), (1, 1, 1, 2), (4, 25, 61, 1), (6, 30, 1, 2), (90, 2, 5, 1)]


def _batch(dtype, seed=0):
    torch = _torch()
    probs, host = [], []
    for n, (nz, ny, nx, nt) in enumerate(SHAPES):
        psi, cx, cy, cz, g = workloads.random_problem((nz, ny, nx), (P, C, C), seed=seed + n, courant=0.8)
        tr = np.stack([psi * (1.0 + 0.5 * t) for t in range(nt)])
        tr, cx, cy, cz, g = (a.astype(np.float32).astype(np.float64) for a in (tr, cx, cy, cz, g))
        host.append((tr, cx, cy, cz, g))
        tdt = torch.float64 if dtype == "f64" else torch.float32
        probs.append({k: torch.from_numpy(np.ascontiguousarray(v)).to("cuda", tdt)
                      for k, v in zip(("psi", "cx", "cy", "cz", "g"), (tr, cx, cy, cz, g))})
    return probs, host


@pytest.mark.parametrize("dtype,iters,graph", [("f64", 2, False), ("f64", 3, True), ("f32", 2, True),
                                                 ("f32", 3, False)])
def test_batched_matches_oracle(dtype, iters, graph):
    torch = _torch()
    import paper_1908_06094_amd as mp

    _say(f"[batched] dtype={dtype} iters={iters} graph={graph}")
    probs, host = _batch(dtype)
    steps = 5   # odd: the final state comes back through the copy kernel
    mp.run_batched(probs, steps, iters=iters, limiter=True, bc=(P, C, C), graph=graph)
    torch.cuda.synchronize()
    tol = 1e-12 if dtype == "f64" else 3e-5
    for (tr, cx, cy, cz, g), pr in zip(host, probs):
        nz, ny, nx = g.shape
        p = oracle.RefProblem(nx, ny, nz, bc=(P, C, C), iters=iters, limiter=True)
        got = pr["psi"].double().cpu().numpy()
        for t in range(tr.shape[0]):
            want = oracle.run(p, steps, tr[t], cx, cy, cz, g)
            assert np.max(np.abs(got[t] - want)) <= tol * np.max(np.abs(want))


def test_batched_equals_single_problem_path():
    torch = _torch()
    import paper_1908_06094_amd as mp

    probs, host = _batch("f64", seed=10)
    ref = []
    for (tr, cx, cy, cz, g), pr in zip(host, probs):
        outs = []
        for t in range(tr.shape[0]):
            x = pr["psi"][t].clone()
            mp.run(x, pr["cx"], pr["cy"], pr["cz"], pr["g"], 4, iters=3, limiter=True, bc=(P, C, C))
            outs.append(x)
        ref.append(torch.stack(outs))
    mp.run_batched(probs, 4, iters=3, limiter=True, bc=(P, C, C), graph=False)
    torch.cuda.synchronize()
    for pr, r in zip(probs, ref):
        assert torch.equal(pr["psi"], r)


def test_batched_f32_matches_single_problem_path():
    """FP32, 3 passes: the batched kernels (per-tracer velocity fields in the
    tile layout) against the single-problem path, tracer by tracer."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    _say("[batched] f32, 3 passes, against the single-problem path")
    probs, _ = _batch("f32", seed=11)
    ref = []
    for pr in probs:
        outs = []
        for t in range(pr["psi"].shape[0]):
            x = pr["psi"][t].clone()
            mp.run(x, pr["cx"], pr["cy"], pr["cz"], pr["g"], 3, iters=3, limiter=True, bc=(P, C, C))
            outs.append(x)
        ref.append(torch.stack(outs))
    mp.run_batched(probs, 3, iters=3, limiter=True, bc=(P, C, C), graph=False)
    torch.cuda.synchronize()
    for pr, r in zip(probs, ref):
        assert torch.max(torch.abs(pr["psi"] - r)).item() <= 1e-6 * torch.max(torch.abs(r)).item()


def test_graph_replays_match_eager():
    """Replays of the cached graph, with eager work and synchronisations in
    between, each equal the eager (uncaptured) result."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    probs, _ = _batch("f32", seed=20)
    start = [pr["psi"].clone() for pr in probs]
    eager = [pr.copy() for pr in probs]
    for pr, s0 in zip(eager, start):
        pr["psi"] = s0.clone()
    mp.run_batched(eager, 3, iters=2, graph=False)
    torch.cuda.synchronize()
    side = torch.zeros(1 << 20, device="cuda")
    ws = None
    for rep in range(3):
        run = [dict(pr) for pr in probs]
        for pr, s0 in zip(run, start):
            pr["psi"].copy_(s0)
        _, _, nb = mp.batch_problem(run, iters=2)
        if ws is None:
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        mp.run_batched(run, 3, iters=2, graph=True, workspace=ws)
        side.add_(1.0)                      # the program's own eager work between replays
        torch.cuda.synchronize()
        for a, b in zip(run, eager):
            assert torch.equal(a["psi"], b["psi"]), rep


def test_tuner_writes_cache(tmp_path, monkeypatch):
    torch = _torch()
    import paper_1908_06094_amd as mp

    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MPDATA_TUNE_CACHE", str(path))
    probs, _ = _batch("f32", seed=30)
    before = [pr["psi"].clone() for pr in probs]
    mp.run_batched(probs, 2, iters=2, graph=False, tune=True)
    torch.cuda.synchronize()
    # the tuning step does not touch the fields; the run advanced them
    assert any(not torch.equal(a, b["psi"]) for a, b in zip(before, probs))


def test_64_problem_batch_sampled():
    """The batched workload (64 problems, 1-8 tracers, FP32, 2 passes,
    limiter, 20 steps, graph): the three smallest problems checked tracer by
    tracer against the FP64 oracle; every tracer stays positive."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    probs_h = workloads.batched_problems()
    _say(f"[batched] 64-problem batch: {len(probs_h)} problems, "
         f"{sum(p['psi'].size for p in probs_h) / 1e6:.0f} M tracer-cells")
    probs = [{k: torch.from_numpy(v).cuda() for k, v in p.items()} for p in probs_h]
    mp.run_batched(probs, 20, iters=2, limiter=True, graph=True)
    torch.cuda.synchronize()
    sizes = [p["g"].size for p in probs_h]
    for i in np.argsort(sizes)[:3]:
        h = probs_h[i]
        nz, ny, nx = h["g"].shape
        p = oracle.RefProblem(nx, ny, nz, bc=(P, C, C), iters=2, limiter=True)
        got = probs[i]["psi"].double().cpu().numpy()
        for t in range(h["psi"].shape[0]):
            want = oracle.run(p, 20, h["psi"][t].astype(np.float64), *(h[k].astype(np.float64)
                                                                       for k in ("cx", "cy", "cz", "g")))
            assert np.max(np.abs(got[t] - want)) <= 3e-5 * np.max(np.abs(want))
    for pr in probs:
        assert float(pr["psi"].min()) >= 0.0
