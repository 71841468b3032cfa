"""GPU adjoint (mpdata_adjoint) against the oracle's reverse sweep and central
finite differences of the GPU forward path (needs a GPU)."""
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


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("shape,bc,iters,lim,steps,k", [
    ((4, 9, 70), (P, C, C), 2, True, 4, 2),
    ((5, 11, 33), (C, C, C), 3, True, 3, 0),
    ((3, 8, 21), (P, P, P), 2, False, 5, 3),
    ((4, 7, 66), (C, P, C), 1, False, 3, 1),
    ((6, 13, 17), (P, C, P), 3, True, 4, 4),
    ((1, 3, 2), (P, P, P), 3, True, 2, 1),
    ((5, 10, 24), (P, C, C), 3, False, 3, 2),
    ((3, 1, 40), (P, C, C), 2, True, 3, 2),    # one row: every y face a wall, dJ/dCy = 0
    ((4, 20, 1), (C, P, C), 3, True, 3, 1),    # one column
    ((2, 2, 3), (C, C, C), 3, True, 3, 2),     # every cell next to a closed end
    ((40, 4, 6), (P, C, C), 2, True, 4, 2),    # tall column over a tiny plane
    ((3, 6, 16), (P, C, C), 8, True, 2, 1),    # the largest pass count
])
def test_adjoint_matches_oracle(shape, bc, iters, lim, steps, k):
    torch = _torch()
    import paper_1908_06094_amd as mp

    _say(f"[adjoint] shape={shape} bc={bc} iters={iters} limiter={lim} steps={steps} k={k}")
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=sum(shape), courant=0.8)
    psi = psi + 0.2
    w = np.random.default_rng(3).uniform(0, 1, size=shape)
    p = oracle.RefProblem(shape[2], shape[1], shape[0], bc=bc, iters=iters, limiter=lim)
    out = oracle.run(p, steps, psi, cx, cy, cz, g)
    seed = 2.0 * w * out
    want = oracle.adjoint(p, steps, psi, cx, cy, cz, g, seed)
    got = mp.adjoint(_dev(psi), _dev(cx), _dev(cy), _dev(cz), _dev(g), _dev(seed), steps, checkpoint_every=k,
                     iters=iters, limiter=lim, bc=bc)
    torch.cuda.synchronize()
    for which in range(4):
        gw = got[which].cpu().numpy()
        ww = want[which]
        scale = max(np.max(np.abs(ww)), 1e-300)
        assert np.max(np.abs(gw - ww)) / scale <= 1e-11, which
    assert np.max(np.abs(got[4].cpu().numpy() - out)) <= 1e-12 * np.max(np.abs(out))


@pytest.mark.parametrize("shape,bc,iters,steps,k", [
    ((9, 40, 70), (P, C, C), 2, 3, 2),     # several tiles in x and y, ragged ends
    ((8, 33, 95), (P, P, P), 3, 2, 1),     # all periodic: every cell on the k-marching path
    ((7, 23, 31), (C, C, C), 3, 2, 0),     # all closed: general-path bands on every side
    ((5, 4, 4), (P, P, P), 2, 2, 1),       # the smallest periodic extents of the fast path
    ((6, 3, 33), (P, P, C), 2, 2, 1),      # a periodic axis of 3 cells: every cell general
    ((60, 128, 256), (P, C, C), 2, 2, 1),  # the configured grid
])
def test_adjoint_march_equals_gather_kernels(shape, bc, iters, steps, k, monkeypatch):
    """The antidiffusive-velocity adjoint of a limited pass as one k-marching
    kernel (MPDATA_ADJOINT=march) gives the same gradients, bit for bit, as
    its two gather kernels with the slot fields in HBM."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    _say(f"[adjoint-march] shape={shape} bc={bc} iters={iters} steps={steps} k={k}")
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=7 + sum(shape), courant=0.8)
    args = [_dev(a) for a in (psi, cx, cy, cz, g)]
    seed = _dev(np.random.default_rng(4).uniform(-1, 1, size=shape))
    monkeypatch.delenv("MPDATA_ADJOINT", raising=False)
    want = mp.adjoint(*args, seed, steps, checkpoint_every=k, iters=iters, limiter=True, bc=bc)
    monkeypatch.setenv("MPDATA_ADJOINT", "march")
    got = mp.adjoint(*args, seed, steps, checkpoint_every=k, iters=iters, limiter=True, bc=bc)
    torch.cuda.synchronize()
    for which in range(5):
        assert torch.equal(got[which], want[which]), which


def test_adjoint_deterministic():
    torch = _torch()
    import paper_1908_06094_amd as mp

    shape = (5, 17, 40)
    psi, cx, cy, cz, g = workloads.random_problem(shape, (P, C, C), seed=9)
    args = [_dev(a) for a in (psi, cx, cy, cz, g)] + [_dev(np.ones(shape))]
    a = mp.adjoint(*args, 3, checkpoint_every=2, iters=2, limiter=True)
    b = mp.adjoint(*args, 3, checkpoint_every=1, iters=2, limiter=True)
    torch.cuda.synchronize()
    for x, y in zip(a[:4], b[:4]):
        assert torch.equal(x, y)


def test_autograd_function_matches_adjoint():
    torch = _torch()
    import paper_1908_06094_amd as mp

    shape = (3, 9, 30)
    psi, cx, cy, cz, g = workloads.random_problem(shape, (P, C, C), seed=2)
    t = [_dev(a).requires_grad_(True) for a in (psi, cx, cy, cz)]
    gd = _dev(g)
    w = _dev(np.random.default_rng(0).uniform(0, 1, size=shape))
    out = mp.MPDATAFunction.apply(t[0], t[1], t[2], t[3], gd, 4, 2, 2, True)
    J = (w * out * out).sum()
    J.backward()
    ref = mp.adjoint(*[x.detach() for x in t], gd, (2 * w * out).detach(), 4, checkpoint_every=2)
    for x, r in zip(t, ref[:4]):
        assert torch.allclose(x.grad, r, rtol=0, atol=0)


def test_adjoint_256x128x60_matches_oracle_reverse_sweep():
    """The exact check at scale: on the full 256x128x60 lat-lon grid (solid-body
    winds, limiter, 2 passes) the GPU adjoint over 3 steps with checkpoints
    every 2 equals the oracle's reverse sweep to 1e-11."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    w0 = workloads.latlon_solid_body()
    steps = 3
    p = oracle.RefProblem(w0.shape[2], w0.shape[1], w0.shape[0], bc=w0.bc, iters=2, limiter=True)
    out = oracle.run(p, steps, w0.psi, w0.cx, w0.cy, w0.cz, w0.g)
    seed = 2.0 * workloads.cost_weights(w0.shape) * out
    _say("[adjoint] 256x128x60, 3 steps: oracle reverse sweep")
    want = oracle.adjoint(p, steps, w0.psi, w0.cx, w0.cy, w0.cz, w0.g, seed)
    got = mp.adjoint(*[_dev(a) for a in (w0.psi, w0.cx, w0.cy, w0.cz, w0.g)], _dev(seed), steps,
                     checkpoint_every=2, iters=2, limiter=True, bc=w0.bc)
    torch.cuda.synchronize()
    for which in range(3):       # dJ/dcz: Cz = 0 everywhere, compared below
        gw, ww = got[which].cpu().numpy(), want[which]
        assert np.max(np.abs(gw - ww)) / np.max(np.abs(ww)) <= 1e-11, which
    gz = got[3].cpu().numpy()
    assert np.max(np.abs(gz - want[3])) <= 1e-11 * max(np.max(np.abs(want[3])), np.max(np.abs(want[0])))


def test_adjoint_configured_20_steps_matches_oracle_reverse_sweep():
    """The configured adjoint run: 20 limited steps (2 passes) with checkpoints
    every 5, solid-body winds on the 256x128 lat-lon plane, J = sum(w psi_T^2),
    against the oracle's reverse sweep at 1e-11 (16 of the 60 levels, so that
    the oracle finishes in seconds; every level carries the same plane
    problem up to its noise)."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    w0 = workloads.latlon_solid_body(nz=16)
    steps, k = 20, 5
    p = oracle.RefProblem(w0.shape[2], w0.shape[1], w0.shape[0], bc=w0.bc, iters=2, limiter=True)
    out = oracle.run(p, steps, w0.psi, w0.cx, w0.cy, w0.cz, w0.g)
    seed = 2.0 * workloads.cost_weights(w0.shape) * out
    _say("[adjoint] 256x128x16, 20 steps, checkpoints every 5: oracle reverse sweep")
    want = oracle.adjoint(p, steps, w0.psi, w0.cx, w0.cy, w0.cz, w0.g, seed)
    got = mp.adjoint(*[_dev(a) for a in (w0.psi, w0.cx, w0.cy, w0.cz, w0.g)], _dev(seed), steps,
                     checkpoint_every=k, iters=2, limiter=True, bc=w0.bc)
    torch.cuda.synchronize()
    for which in range(4):
        gw, ww = got[which].cpu().numpy(), want[which]
        scale = max(np.max(np.abs(ww)), np.max(np.abs(want[0])))
        err = np.max(np.abs(gw - ww)) / scale
        _say(f"[adjoint]   gradient {which}: rel err {err:.3e}")
        assert err <= 1e-11, which
    assert np.max(np.abs(got[4].cpu().numpy() - out)) <= 1e-12 * np.max(np.abs(out))


def _fd_setup(mp, torch, w0, psi0, steps, iters, limiter, k=5):
    w = workloads.cost_weights(w0.shape)
    dev = [_dev(a) for a in (psi0, w0.cx, w0.cy, w0.cz, w0.g)]
    wd = _dev(w)
    kw = dict(iters=iters, limiter=limiter, bc=w0.bc)

    def cost(psi, cx, cy, cz):
        t = psi.clone()
        mp.run(t, cx, cy, cz, dev[4], steps, **kw)
        return float(torch.sum(wd * t * t))

    out = dev[0].clone()
    mp.run(out, *dev[1:4], dev[4], steps, **kw)
    grads = mp.adjoint(*dev, 2 * wd * out, steps, checkpoint_every=k, **kw)
    return dev, cost, grads


def _direction(rng, dev):
    """A direction that keeps x +- eps d inside the scheme's domain for eps
    well below 1: the psi0 block is psi0 times N(0, 1) (psi0 +- eps d stays
    > 0) and each Courant block is |C| times N(0, 1) (no Courant number
    changes sign or leaves 0; zero faces, the closed walls and Cz, get 0)."""
    return [_dev(rng.standard_normal(tuple(dev[0].shape))) * x.abs() for x in dev[:4]]


def _fd_mismatch(cost, dev, grads, d, eps):
    plus = [x + eps * y for x, y in zip(dev[:4], d)]
    minus = [x - eps * y for x, y in zip(dev[:4], d)]
    fd = (cost(*plus) - cost(*minus)) / (2 * eps)
    ad = sum(float((gr * y).sum()) for gr, y in zip(grads[:4], d))
    return fd, ad, abs(fd - ad) / max(abs(fd), 1e-30)


def test_adjoint_256x128x60_finite_differences():
    """The configured check: 256x128x60, solid-body winds, limiter, 2 passes,
    20 steps, J = sum(w psi_T^2), checkpoints every 5 steps, central
    differences with eps 1e-6 on 16 random directions in (psi0, C), each
    scaled so that x +- eps d stays in the domain (psi > 0, no Courant sign
    change).

    J is piecewise smooth: the limiter's min/max and the [U~]+- switches put
    kinks in it, and every kink between x - eps d and x + eps d costs the
    central difference a slope jump of that term, whatever eps.  Their
    number grows with eps, so the mismatch falls with eps (about linearly
    down to eps 1e-6, then as sqrt(eps), a random walk over fewer and fewer
    crossings) instead of at the O(eps^2) of a smooth function.  The test
    shows that convergence on a sweep over eps on 4 directions, then bounds
    the 16 configured directions at eps 1e-6 by what the sweep measured
    there: |fd - adjoint| <= 10 x the sweep's median at 1e-6, both taken
    relative to the RMS of the directional derivatives (a direction whose
    projection happens to be near 0 would otherwise inflate its relative
    error without any larger absolute error)."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    w0 = workloads.latlon_solid_body()
    dev, cost, grads = _fd_setup(mp, torch, w0, w0.psi, 20, 2, True)
    rng = np.random.default_rng(50)
    dirs = [_direction(rng, dev) for _ in range(16)]
    sweep = {}
    for eps in (1e-4, 1e-5, 1e-6, 1e-7, 1e-8):
        res = [_fd_mismatch(cost, dev, grads, d, eps) for d in dirs[:4]]
        scale = float(np.sqrt(np.mean([r[1] ** 2 for r in res])))     # RMS of the adjoint's projections
        sweep[eps] = float(np.median([abs(fd - ad) for fd, ad, _ in res])) / scale
        _say(f"[fd] eps={eps:.0e}: |fd - adjoint| / rms " + " ".join(f"{abs(fd - ad) / scale:.2e}"
                                                                       for fd, ad, _ in res)
             + "; relative " + " ".join(f"{r:.2e}" for _, _, r in res))
    # convergence: the mismatch falls by >= 30x from eps 1e-4 to 1e-6 and keeps falling to 1e-8
    assert sweep[1e-6] <= sweep[1e-4] / 30.0, sweep
    assert sweep[1e-8] <= sweep[1e-6], sweep
    res = [_fd_mismatch(cost, dev, grads, d, 1e-6) for d in dirs]
    scale = float(np.sqrt(np.mean([r[1] ** 2 for r in res])))
    norm = []
    for i, (fd, ad, r) in enumerate(res):
        norm.append(abs(fd - ad) / scale)
        _say(f"[fd] direction {i}: fd={fd:.10e} adjoint={ad:.10e} rel={r:.2e} |fd-ad|/rms={norm[-1]:.2e}")
    bound = 10.0 * sweep[1e-6]
    _say(f"[fd] eps=1e-6: max {max(norm):.2e}, median {np.median(norm):.2e}, bound {bound:.2e}")
    assert max(norm) <= bound


def test_smooth_field_finite_differences():
    """Where J is smooth at the difference scale (no limiter, a smooth tracer
    bounded away from 0: the cosine bell on a background of 0.5), the adjoint
    and central differences agree to the truncation error, with the
    directions kept in the domain as above (no Courant sign change, so no
    donor-flux kink is crossed)."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    w0 = workloads.latlon_solid_body()
    psi0 = 0.5 + np.broadcast_to(workloads.cosine_bell(w0.shape[2], w0.shape[1])[None], w0.shape).copy()
    dev, cost, grads = _fd_setup(mp, torch, w0, psi0, 10, 2, False)
    rng = np.random.default_rng(51)
    rels = []
    for i in range(6):
        fd, ad, r = _fd_mismatch(cost, dev, grads, _direction(rng, dev), 1e-6)
        rels.append(r)
        _say(f"[fd-smooth] direction {i}: fd={fd:.10e} adjoint={ad:.10e} rel={r:.2e}")
    assert max(rels) <= 1e-5
