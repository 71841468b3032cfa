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
    for a in range(3):
        # closed axes: the wall slot is unused; compare the rest
        pass
    for which in range(4):
        gw = got[which].cpu().numpy()
        ww = want[which]
        scale = max(np.max(np.abs(ww)), 1e-300)
        assert np.max(np.abs(gw - ww)) / scale <= 1e-11, which
    assert np.max(np.abs(got[4].cpu().numpy() - out)) <= 1e-12 * np.max(np.abs(out))


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


def test_config5_finite_differences():
    """256x128x60 lat-lon, solid-body winds, limiter, 2 passes, 20 steps,
    J = sum(w psi_T^2), checkpoints every 5 steps: the adjoint's directional
    derivatives against central differences (eps 1e-6) of the GPU forward on
    16 random directions in (psi0, C), C directions masked where C == 0."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    w0 = workloads.config2()
    steps = 20
    w = workloads.config5_weights(w0.shape)
    dev = [_dev(a) for a in (w0.psi, w0.cx, w0.cy, w0.cz, w0.g)]
    wd = _dev(w)
    kw = dict(iters=2, limiter=True, bc=w0.bc)

    def cost(psi, cx, cy, cz):
        t = psi.clone()
        mp.run(t, cx, cy, cz, dev[4], steps, **kw)
        return float(torch.sum(wd * t * t))

    out = dev[0].clone()
    mp.run(out, *dev[1:4], dev[4], steps, **kw)
    grads = mp.adjoint(*dev, 2 * wd * out, steps, checkpoint_every=5, **kw)
    rng = np.random.default_rng(50)
    eps = 1e-6
    cmax = float(max(np.max(np.abs(w0.cx)), np.max(np.abs(w0.cy))))
    worst = 0.0
    for d_i in range(16):
        d = [rng.standard_normal(w0.shape) for _ in range(4)]
        for a, base in zip(range(1, 4), (w0.cx, w0.cy, w0.cz)):
            d[a] = d[a] * cmax
            d[a][base == 0.0] = 0.0
        dd = [_dev(x) for x in d]
        plus = [x + eps * y for x, y in zip(dev[:4], dd)]
        minus = [x - eps * y for x, y in zip(dev[:4], dd)]
        fd = (cost(*plus) - cost(*minus)) / (2 * eps)
        ad = sum(float(torch.sum(gr * y)) for gr, y in zip(grads[:4], dd))
        rel = abs(fd - ad) / max(abs(fd), 1e-30)
        worst = max(worst, rel)
        _say(f"[fd] direction {d_i}: fd={fd:.10e} adjoint={ad:.10e} rel={rel:.2e}")
    assert worst <= 1e-5
