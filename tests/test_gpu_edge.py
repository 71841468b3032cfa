"""Degenerate and edge inputs of the scheme on the GPU, forward (FP64 and
FP32) and adjoint (FP64), against the oracle or an exact property (needs a
GPU).

Cases (each pinned on the oracle side in test_oracle_pins.py):
  * exactly zero blocks of the tracer, limiter on and off, default and
    smallest accepted eps (guarded denominators at their minimum);
  * exactly uniform patches in exactly non-divergent winds with the limiter
    on: inside them A = B = 0, in = out = 0 and beta = 0 * G / eps = 0;
  * Courant number +1 or -1 on one axis, G = 1, dyadic tracer: every pass
    after the donor cell has a zero antidiffusive velocity, and the step is
    the exact one-cell shift, bitwise, for any pass count, limiter on;
  * psi = 1 in exactly non-divergent winds stays 1 bitwise;
  * non-default eps;
  * psi scaled by 1e100 and 1e-100 (FP64) or 1e30 and 1e-30 (FP32), the
    ends of the documented range: finite results at the parity bar;
  * a NaN in the input stays in its own cell (it is not silently lost);
  * MPDATA_DEBUG refuses negative, NaN and out-of-range inputs.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

P, C = "periodic", "closed"
TOL64 = 1e-12


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _mp():
    import paper_1908_06094_amd as mp

    return mp


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a, dtype=None):
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _zero_block(shape, bc, seed):
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=seed, courant=0.8)
    nz, ny, nx = shape
    psi[:, ny // 4: ny // 4 + max(ny // 2, 1), nx // 5: nx // 5 + max(nx // 2, 1)] = 0.0
    psi[: max(nz // 3, 1)] = np.where(psi[: max(nz // 3, 1)] < 0.3, 0.0, psi[: max(nz // 3, 1)])
    return psi, cx, cy, cz, g


def _uniform_patch(nx, ny, nz, seed, value=1.0):
    """Exactly non-divergent lat-lon winds, a uniform patch in a noisy field."""
    rng = np.random.default_rng(seed)
    cx, cy, cz, _ = workloads.stream_winds(nx, ny, nz, "solid", 0.5)
    g = workloads.metric(nx, ny, nz)
    psi = 0.5 + 0.2 * rng.uniform(size=(nz, ny, nx))
    psi[:, ny // 4: 3 * ny // 4, nx // 6: nx // 2] = value
    return psi, cx, cy, cz, g


def _fp32_inputs(arrs):
    return [a.astype(np.float32).astype(np.float64) for a in arrs]


def _forward_case(arrs, shape, bc, iters, lim, eps, steps, dtype):
    torch = _torch()
    mp = _mp()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        arrs = _fp32_inputs(arrs)
    psi, cx, cy, cz, g = arrs
    p = oracle.RefProblem(shape[2], shape[1], shape[0], bc=bc, iters=iters, limiter=lim, eps=eps)
    want = oracle.run(p, steps, psi, cx, cy, cz, g)
    t = _dev(psi, tdt)
    mp.run(t, *[_dev(a, tdt) for a in (cx, cy, cz, g)], steps, iters=iters, limiter=lim, bc=bc, eps=eps)
    torch.cuda.synchronize()
    got = t.double().cpu().numpy()
    assert np.all(np.isfinite(got))
    return got, want


# FP32 bound for these short runs (2 steps): the measured errors of the cases
# (printed by the tests) lie in 6.9e-8 .. 1.8e-7 relative to max|psi|, the
# FP32 rounding unit being 6e-8; the bound is at most 10x each of them.  The
# exact-zero blocks at eps = 1e-30 also pin that beta's ratio is taken in
# FP64: (in + eps)(out + eps) = 1e-60 there would underflow in FP32.
TOL32_EDGE = 6e-7


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("lim", [True, False])
@pytest.mark.parametrize("eps", [0.0, 1e-30, 1e-8])
def test_zero_blocks(dtype, lim, eps):
    shape, bc = (6, 26, 131), (P, C, C)
    _say(f"[edge] zero blocks dtype={dtype} limiter={lim} eps={eps}")
    got, want = _forward_case(_zero_block(shape, bc, 21), shape, bc, 3, lim, eps, 2, dtype)
    err = _rel(got, want)
    _say(f"[edge]   rel err {err:.3e}")
    assert err <= (TOL64 if dtype == "f64" else TOL32_EDGE)
    if lim:
        assert got.min() >= 0.0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("iters", [2, 3])
def test_uniform_patch_with_limiter(dtype, iters):
    nx, ny, nz = 128, 64, 3
    bc = (P, C, C)
    _say(f"[edge] uniform patch dtype={dtype} iters={iters}")
    arrs = _uniform_patch(nx, ny, nz, 22)
    got, want = _forward_case(arrs, (nz, ny, nx), bc, iters, True, 0.0, 2, dtype)
    err = _rel(got, want)
    _say(f"[edge]   rel err {err:.3e}")
    assert err <= (TOL64 if dtype == "f64" else TOL32_EDGE)
    # deep inside the patch every velocity is 0 and the field stays exactly 1
    # (the step's stencil reaches 1 + 2 (iters - 1) cells; 2 steps)
    m = 2 * (1 + 2 * (iters - 1)) + 1
    inner = got[:, ny // 4 + m: 3 * ny // 4 - m, nx // 6 + m: nx // 2 - m]
    assert inner.size and np.all(inner == 1.0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("iters", [1, 2, 3])
def test_courant_one_is_an_exact_shift(dtype, axis, sign, iters):
    torch = _torch()
    mp = _mp()
    shape = (6, 19, 70)
    rng = np.random.default_rng(30 + axis)
    psi = rng.integers(0, 64, size=shape) / 8.0
    c = [np.zeros(shape) for _ in range(3)]          # x, y, z
    c[2 - axis][...] = float(sign)                   # axis 0 = z ... 2 = x in (nz, ny, nx)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    bc = (P, P, P)
    _say(f"[edge] Courant {sign:+d} on array axis {axis} dtype={dtype} iters={iters}")
    t = _dev(psi, tdt)
    mp.run(t, *[_dev(a, tdt) for a in c], _dev(np.ones(shape), tdt), 3, iters=iters, limiter=True, bc=bc)
    torch.cuda.synchronize()
    got = t.double().cpu().numpy()
    assert np.array_equal(got, np.roll(psi, 3 * sign, axis=axis))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("iters,lim", [(2, True), (3, True), (3, False)])
def test_constant_field_stays_constant(dtype, iters, lim):
    torch = _torch()
    mp = _mp()
    nx, ny, nz = 96, 48, 4
    cx, cy, cz, _ = workloads.stream_winds(nx, ny, nz, "wave", 0.6)
    g = workloads.metric(nx, ny, nz)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    _say(f"[edge] psi = 1 in non-divergent winds dtype={dtype} iters={iters} limiter={lim}")
    t = _dev(np.ones((nz, ny, nx)), tdt)
    mp.run(t, *[_dev(a, tdt) for a in (cx, cy, cz, g)], 5, iters=iters, limiter=lim, bc=(P, C, C))
    torch.cuda.synchronize()
    assert bool(torch.all(t == 1.0))


@pytest.mark.parametrize("dtype,scale", [("f64", 1e100), ("f64", 1e-100), ("f32", 1e30), ("f32", 1e-30)])
def test_range_ends(dtype, scale):
    shape, bc = (5, 21, 70), (P, C, C)
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=41, courant=0.8)
    _say(f"[edge] psi scaled by {scale:g} dtype={dtype}")
    got, want = _forward_case([psi * scale, cx, cy, cz, g], shape, bc, 3, True, 0.0, 2, dtype)
    err = _rel(got, want)
    _say(f"[edge]   rel err {err:.3e}")
    assert err <= (TOL64 if dtype == "f64" else TOL32_EDGE)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_nan_stays_in_its_cell(dtype):
    torch = _torch()
    mp = _mp()
    shape, bc = (4, 17, 70), (P, C, C)
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=42, courant=0.8)
    psi[2, 8, 33] = np.nan
    tdt = torch.float64 if dtype == "f64" else torch.float32
    _say(f"[edge] NaN at (2, 8, 33) dtype={dtype}")
    out = mp.step(*[_dev(a, tdt) for a in (psi, cx, cy, cz, g)], iters=3, limiter=True, bc=bc)
    torch.cuda.synchronize()
    assert bool(torch.isnan(out[2, 8, 33]))
    p = oracle.RefProblem(shape[2], shape[1], shape[0], bc=bc, iters=3, limiter=True)
    assert np.isnan(oracle.step(p, psi, cx, cy, cz, g)[2, 8, 33])


def test_debug_mode_refuses_bad_inputs(monkeypatch):
    torch = _torch()
    mp = _mp()
    shape, bc = (3, 9, 40), (P, C, C)
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=43)
    monkeypatch.setenv("MPDATA_DEBUG", "1")
    dv = [_dev(a) for a in (psi, cx, cy, cz, g)]
    mp.step(*dv, iters=2)                                   # in range: accepted
    for name, idx, val in (("psi", 0, -1e-3), ("psi", 0, np.nan), ("psi", 0, 1e101), ("g", 4, 0.0),
                           ("g", 4, 1e7)):
        bad = [t.clone() for t in dv]
        bad[idx][1, 2, 3] = val
        _say(f"[edge] MPDATA_DEBUG: {name}[1,2,3] = {val}")
        with pytest.raises(mp.MpdataError) as ei:
            mp.step(*bad, iters=2)
        assert ei.value.code == mp._lib.MPDATA_EINVAL and "MPDATA_DEBUG" in str(ei.value)
    x = dv[0].clone()
    x[0, 0, 0] = -1.0
    with pytest.raises(mp.MpdataError):
        mp.run(x, *dv[1:], 2, iters=2)
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# Adjoint (FP64) on the same degenerate inputs, against the oracle's reverse
# sweep.  At the kinks both follow the branch rules of the header (the
# forward values there are exact on both sides).
# ---------------------------------------------------------------------------

def _adjoint_case(arrs, shape, bc, iters, lim, eps, steps, k):
    torch = _torch()
    mp = _mp()
    psi, cx, cy, cz, g = arrs
    w = np.random.default_rng(9).uniform(0, 1, size=shape)
    p = oracle.RefProblem(shape[2], shape[1], shape[0], bc=bc, iters=iters, limiter=lim, eps=eps)
    out = oracle.run(p, steps, psi, cx, cy, cz, g)
    seed = 2.0 * w * out
    want = oracle.adjoint(p, steps, psi, cx, cy, cz, g, seed)
    got = mp.adjoint(*[_dev(a) for a in (psi, cx, cy, cz, g)], _dev(seed), steps, checkpoint_every=k, iters=iters,
                     limiter=lim, bc=bc, eps=eps)
    torch.cuda.synchronize()
    for which in range(4):
        gw, ww = got[which].cpu().numpy(), want[which]
        assert np.all(np.isfinite(gw)), which
        scale = max(np.max(np.abs(ww)), np.max(np.abs(want[0])), 1e-300)
        err = np.max(np.abs(gw - ww)) / scale
        _say(f"[edge-adj]   gradient {which}: rel err {err:.3e}")
        assert err <= 1e-11, which


@pytest.mark.parametrize("lim,eps", [(True, 0.0), (False, 0.0), (True, 1e-30), (True, 1e-8)])
def test_adjoint_zero_blocks(lim, eps):
    shape, bc = (4, 17, 70), (P, C, C)
    _say(f"[edge-adj] zero blocks limiter={lim} eps={eps}")
    _adjoint_case(_zero_block(shape, bc, 23), shape, bc, 3, lim, eps, 3, 2)


def test_adjoint_uniform_patch():
    nx, ny, nz = 96, 32, 3
    _say("[edge-adj] uniform patch, limiter")
    _adjoint_case(_uniform_patch(nx, ny, nz, 24), (nz, ny, nx), (P, C, C), 2, True, 0.0, 3, 2)


@pytest.mark.parametrize("axis,sign", [(2, 1), (2, -1), (1, 1), (0, -1)])
def test_adjoint_courant_one(axis, sign):
    shape = (5, 12, 70)
    rng = np.random.default_rng(31)
    psi = rng.integers(1, 64, size=shape) / 8.0
    c = [np.zeros(shape) for _ in range(3)]
    c[2 - axis][...] = float(sign)
    _say(f"[edge-adj] Courant {sign:+d} on array axis {axis}")
    _adjoint_case([psi, *c, np.ones(shape)], shape, (P, P, P), 2, True, 0.0, 2, 1)


def test_adjoint_constant_field():
    nx, ny, nz = 64, 32, 3
    cx, cy, cz, _ = workloads.stream_winds(nx, ny, nz, "solid", 0.5)
    g = workloads.metric(nx, ny, nz)
    _say("[edge-adj] psi = 1 in non-divergent winds")
    _adjoint_case([np.ones((nz, ny, nx)), cx, cy, cz, g], (nz, ny, nx), (P, C, C), 3, True, 0.0, 2, 1)
