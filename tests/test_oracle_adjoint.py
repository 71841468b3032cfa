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
