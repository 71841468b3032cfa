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
    tol = 1e-12 if dtype == "f64" else 7e-7
    worst = 0.0
    for (tr, cx, cy, cz, g), pr in zip(host, probs):
        nz, ny, nx = g.shape
        p = oracle.RefProblem(nx, ny, nz, bc=(P, C, C), iters=iters, limiter=True)
        got = pr["psi"].double().cpu().numpy()
        for t in range(tr.shape[0]):
            want = oracle.run(p, steps, tr[t], cx, cy, cz, g)
            worst = max(worst, float(np.max(np.abs(got[t] - want)) / np.max(np.abs(want))))
    _say(f"[batched]   worst rel err vs oracle {worst:.3e}")
    assert worst <= tol


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


# The batched kernel variants (FP32): tile row width x threads per workgroup
# (the tile's rows: threads / row width) x workgroups per CU x donor-cell pass
# folded into the first corrective pass or separate.
VARIANTS_F32 = [(32, 768, 1, "fold"), (32, 768, 2, "fold"), (64, 768, 1, "fold"), (64, 768, 2, "fold"),
                (16, 768, 1, "fold"), (16, 768, 2, "fold"), (32, 768, 1, "split"), (32, 768, 2, "split"),
                (64, 768, 1, "split"), (64, 768, 2, "split"), (16, 768, 1, "split"), (16, 768, 2, "split"),
                (32, 1024, 1, "fold"), (64, 1024, 1, "fold"), (16, 1024, 1, "fold"),
                (32, 1024, 1, "split"), (64, 1024, 1, "split"), (16, 1024, 1, "split")]


def test_variant_table_matches_binding():
    """The binding's table of variants (which bench.py reports the tuner's
    choice from) lists the same variants in the same order."""
    import paper_1908_06094_amd as mp

    names = {"fold": "folded", "split": "separate"}
    assert mp.BATCH_VARIANTS_F32 == [(l, t, w, names[f]) for l, t, w, f in VARIANTS_F32]


@pytest.mark.parametrize("variant", range(len(VARIANTS_F32)))
@pytest.mark.parametrize("iters", [2, 3])
def test_every_f32_variant_matches_oracle_and_single_path(variant, iters, monkeypatch):
    """Each tile variant the tuner can pick, forced with MPDATA_BATCH_VARIANT:
    every tracer against the FP64 oracle and against the single-problem path
    (the same arithmetic per cell whatever the tile)."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    lanes, threads, wgs, fold = VARIANTS_F32[variant]
    _say(f"[batched] variant {variant} ({lanes} lanes, {threads} threads, {wgs} workgroup(s) per CU, {fold}) "
         f"iters={iters}")
    monkeypatch.setenv("MPDATA_BATCH_VARIANT", str(variant))
    probs, host = _batch("f32", seed=40 + variant)
    single = []
    for pr in probs:
        outs = []
        for t in range(pr["psi"].shape[0]):
            x = pr["psi"][t].clone()
            mp.run(x, pr["cx"], pr["cy"], pr["cz"], pr["g"], 3, iters=iters, limiter=True, bc=(P, C, C))
            outs.append(x)
        single.append(torch.stack(outs))
    mp.run_batched(probs, 3, iters=iters, limiter=True, bc=(P, C, C), graph=(variant % 2 == 0))
    torch.cuda.synchronize()
    worst = 0.0
    for (tr, cx, cy, cz, g), pr, r in zip(host, probs, single):
        nz, ny, nx = g.shape
        p = oracle.RefProblem(nx, ny, nz, bc=(P, C, C), iters=iters, limiter=True)
        got = pr["psi"].double().cpu().numpy()
        for t in range(tr.shape[0]):
            want = oracle.run(p, 3, tr[t], cx, cy, cz, g)
            worst = max(worst, float(np.max(np.abs(got[t] - want)) / np.max(np.abs(want))))
        assert torch.max(torch.abs(pr["psi"] - r)).item() <= 1e-6 * torch.max(torch.abs(r)).item()
    _say(f"[batched]   worst rel err vs oracle {worst:.3e}")
    assert worst <= 7e-7


@pytest.mark.parametrize("variant", [0, 1])
def test_f64_variants_equal_single_path(variant, monkeypatch):
    """FP64's two variants (donor-cell pass folded or separate) equal the
    single-problem path bitwise; a third index is refused."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    probs, _ = _batch("f64", seed=50)
    monkeypatch.setenv("MPDATA_BATCH_VARIANT", "2")
    with pytest.raises(mp.MpdataError) as ei:
        mp.run_batched(probs, 1, iters=2, graph=False)
    assert "MPDATA_BATCH_VARIANT" in str(ei.value)
    monkeypatch.setenv("MPDATA_BATCH_VARIANT", str(variant))
    if variant == 1:
        monkeypatch.setenv("MPDATA_KERNELS", "split")   # the single path's split layout
    ref = []
    for pr in probs:
        outs = []
        for t in range(pr["psi"].shape[0]):
            x = pr["psi"][t].clone()
            mp.run(x, pr["cx"], pr["cy"], pr["cz"], pr["g"], 3, iters=3, limiter=True, bc=(P, C, C))
            outs.append(x)
        ref.append(torch.stack(outs))
    monkeypatch.delenv("MPDATA_KERNELS", raising=False)
    mp.run_batched(probs, 3, iters=3, limiter=True, bc=(P, C, C), graph=False)
    torch.cuda.synchronize()
    for pr, r in zip(probs, ref):
        assert torch.equal(pr["psi"], r)


def _cache_lines(path):
    return [ln.rstrip("\n").split("\t") for ln in open(path) if ln.strip()]


def test_tuner_writes_cache(tmp_path, monkeypatch):
    """Tuning times every variant on the batch, writes its choice (batch
    shape, tab, variant) to the file MPDATA_TUNE_CACHE names, and reuses it;
    a new cache path within the same process is read afresh (its file knows
    nothing of this shape, so the batch is tuned again and the choice lands
    in the new file)."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    monkeypatch.delenv("MPDATA_BATCH_VARIANT", raising=False)
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MPDATA_TUNE_CACHE", str(path))
    probs, _ = _batch("f32", seed=30)
    before = [pr["psi"].clone() for pr in probs]
    mp.run_batched(probs, 2, iters=2, graph=False, tune=True)
    torch.cuda.synchronize()
    # the tuning steps do not touch the fields; the run advanced them
    assert any(not torch.equal(a, b["psi"]) for a, b in zip(before, probs))
    lines = _cache_lines(path)
    assert len(lines) == 1, lines
    key, variant = lines[0]
    assert key.startswith("d1 i2 l1 b011 n%d;" % len(probs))
    for nz, ny, nx, nt in SHAPES:
        assert f"{nx}x{ny}x{nz}t{nt}" in key
    assert 0 <= int(variant) < len(VARIANTS_F32)
    _say(f"[batched] tuned variant {variant}: {VARIANTS_F32[int(variant)]}")
    # the same shape again: answered from the cache, nothing appended
    mp.run_batched(probs, 2, iters=2, graph=False, tune=True)
    torch.cuda.synchronize()
    assert len(_cache_lines(path)) == 1
    # another cache file, same process
    path2 = tmp_path / "tune2.txt"
    monkeypatch.setenv("MPDATA_TUNE_CACHE", str(path2))
    mp.run_batched(probs, 2, iters=2, graph=False, tune=True)
    torch.cuda.synchronize()
    lines2 = _cache_lines(path2)
    assert len(lines2) == 1 and lines2[0][0] == key


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
            err = float(np.max(np.abs(got[t] - want)) / np.max(np.abs(want)))
            _say(f"[batched]   problem {i} tracer {t}: rel err vs oracle {err:.3e}")
            assert err <= 3e-6
    for pr in probs:
        assert float(pr["psi"].min()) >= 0.0
