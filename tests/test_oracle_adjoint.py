"""Pins of the oracle's reverse sweep (no GPU): directional derivatives of
J = sum(w psi_T^2) from the adjoint must match central finite differences of
the forward oracle, for psi0 and for each Courant-number array, with and
without the limiter, on every boundary combination."""
import numpy as np
import pytest

import oracle
import workloads

P, C = "periodic", "closed"


def _cost(p, steps, psi, cx, cy, cz, g, w):
    out = oracle.run(p, steps, psi, cx, cy, cz, g)
    return float(np.sum(w * out * out))


def _mask_faces(a, bc, axis):
    """Zero the unused wall slot of a closed axis (the forward never reads it)."""
    a = a.copy()
    if bc[axis] == C:
        sl = [slice(None)] * 3
        sl[2 - axis] = -1
        a[tuple(sl)] = 0.0
    return a


@pytest.mark.parametrize("bc", [(P, C, C), (P, P, P), (C, C, C)])
@pytest.mark.parametrize("iters,lim", [(1, False), (2, False), (2, True), (3, True)])
def test_adjoint_matches_finite_differences(bc, iters, lim):
    shape = (4, 6, 7)
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=iters * 10 + len(bc[0]), courant=0.8)
    psi = psi + 0.2                      # keep clear of the psi = 0 corner of the ratios
    rng = np.random.default_rng(5)
    w = rng.uniform(0, 1, size=shape)
    p = oracle.RefProblem(shape[2], shape[1], shape[0], bc=bc, iters=iters, limiter=lim)
    steps = 3
    out = oracle.run(p, steps, psi, cx, cy, cz, g)
    grads = oracle.adjoint(p, steps, psi, cx, cy, cz, g, 2.0 * w * out)
    eps = 1e-6
    inputs = [psi, cx, cy, cz]
    for which in range(4):
        for trial in range(3):
            d = rng.standard_normal(shape)
            if which > 0:
                d = _mask_faces(d, bc, which - 1) * np.max(np.abs(inputs[which]))
                d[inputs[which] == 0.0] = 0.0
            plus = [x.copy() for x in inputs]
            minus = [x.copy() for x in inputs]
            plus[which] += eps * d
            minus[which] -= eps * d
            fd = (_cost(p, steps, *plus, g, w) - _cost(p, steps, *minus, g, w)) / (2 * eps)
            ad = float(np.sum(grads[which] * d))
            assert abs(fd - ad) <= 1e-6 * max(abs(fd), 1e-3), (which, trial, fd, ad)


def test_adjoint_of_linear_donor_is_transpose():
    """iters=1 is linear in psi: <A d1, d2> == <d1, A^T d2> to rounding."""
    shape = (3, 5, 6)
    bc = (P, C, C)
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=2, courant=0.8)
    p = oracle.RefProblem(shape[2], shape[1], shape[0], bc=bc, iters=1, limiter=False)
    rng = np.random.default_rng(1)
    d1, d2 = rng.standard_normal(shape), rng.standard_normal(shape)
    a_d1 = oracle.run(p, 4, d1, cx, cy, cz, g)
    at_d2 = oracle.adjoint(p, 4, psi, cx, cy, cz, g, d2)[0]
    assert abs(np.sum(a_d1 * d2) - np.sum(d1 * at_d2)) <= 1e-13 * np.sum(np.abs(a_d1 * d2))


def test_adjoint_zero_steps_is_identity():
    shape = (2, 3, 4)
    psi, cx, cy, cz, g = workloads.random_problem(shape, (P, C, C), seed=3)
    p = oracle.RefProblem(4, 3, 2, iters=2, limiter=True)
    seed = np.arange(24.0).reshape(shape)
    d = oracle.adjoint(p, 0, psi, cx, cy, cz, g, seed)
    assert np.array_equal(d[0], seed) and not d[1].any() and not d[2].any() and not d[3].any()


@pytest.mark.parametrize("iters", [2, 3])
def test_adjoint_exact_on_uniform_background(iters):
    """A cosine bell on an exactly uniform background (lat-lon metric,
    solid-body winds, no limiter): over the uniform region the antidiffusive
    velocities are exactly 0, where the donor flux [U]+ pL + [U]- pR is
    differentiable with slope pL = pR.  The adjoint must take that slope
    (the symmetric subgradient 1/2 of [c]+- at c = 0); central differences
    are smooth here and pin it."""
    nx, ny, nz = 32, 16, 3
    cx, cy, cz, _ = workloads.stream_winds(nx, ny, nz, "solid", 0.5)
    g = workloads.metric(nx, ny, nz)
    psi = 0.5 + np.broadcast_to(workloads.cosine_bell(nx, ny)[None], (nz, ny, nx)).copy()
    p = oracle.RefProblem(nx, ny, nz, bc=(P, C, C), iters=iters, limiter=False)
    w = np.random.default_rng(5).uniform(0, 1, size=psi.shape)
    steps = 5
    out = oracle.run(p, steps, psi, cx, cy, cz, g)
    grads = oracle.adjoint(p, steps, psi, cx, cy, cz, g, 2.0 * w * out)
    rng = np.random.default_rng(1)
    base = [psi, cx, cy, cz]
    for which in range(3):
        d = [np.zeros(psi.shape) for _ in range(4)]
        d[which] = rng.standard_normal(psi.shape) * (1.0 if which == 0 else 0.1)
        if which:
            d[which][base[which] == 0.0] = 0.0
        eps = 1e-6
        fd = (_cost(p, steps, *[x + eps * y for x, y in zip(base, d)], g, w)
              - _cost(p, steps, *[x - eps * y for x, y in zip(base, d)], g, w)) / (2 * eps)
        ad = sum(float(np.sum(a * b)) for a, b in zip(grads, d))
        assert abs(fd - ad) <= 1e-5 * abs(fd), (which, fd, ad)
