"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test ties one part of the oracle to something other than itself: a
closed form, an exact special case, an invariant the scheme guarantees, an
observed convergence order, or a symmetry.  Together they are chosen so that a
dropped term, a wrong sign, a wrong index or a transposed operand in any stage
fails at least one of them.

Stages: C1-C2 donor cell (paper, Section 5, Listings 4-8); C3 antidiffusive
velocity, C4-C5 limiter (MPDATA literature the paper refers to); C7 mass.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import exact

P, C = "periodic", "closed"


def _prob(shape, bc=(P, P, P), iters=2, limiter=False):
    nz, ny, nx = shape
    return oracle.RefProblem(nx, ny, nz, bc=bc, iters=iters, limiter=limiter)


# ---------------------------------------------------------------------------
# C1-C2: donor cell
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("courant,gval", [((0.2, 0.15, 0.1), 1.0), ((-0.3, 0.1, -0.05), 1.0),
                                          ((0.4, -0.3, 0.2), 2.0)])
def test_donor_fourier_closed_form(courant, gval):
    """iters=1, constant C, constant G, periodic: the step is linear and
    shift-invariant, so a Fourier mode is multiplied by the donor-cell
    amplification factor every step."""
    nz, ny, nx = 6, 10, 12
    p_, q_, r_ = 2, 1, 1
    shape = (nz, ny, nx)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    theta = 2 * math.pi * (p_ * i / nx + q_ * j / ny + r_ * k / nz)
    psi0 = 1.0 + 0.5 * np.cos(theta)
    cx, cy, cz = (np.full(shape, c) for c in courant)
    g = np.full(shape, gval)
    amp = 1.0 + 0j
    for c, th in zip(courant, (2 * math.pi * p_ / nx, 2 * math.pi * q_ / ny, 2 * math.pi * r_ / nz)):
        c = c / gval
        if c >= 0:
            amp -= c * (1 - np.exp(-1j * th))        # upwind neighbour on the left
        else:
            amp -= -c * (1 - np.exp(1j * th))        # upwind neighbour on the right
    steps = 7
    want = 1.0 + 0.5 * np.real(amp ** steps * np.exp(1j * theta))
    got = oracle.run(_prob(shape, iters=1), steps, psi0, cx, cy, cz, g)
    assert np.max(np.abs(got - want)) < 1e-13


def test_zero_courant_is_identity():
    shape = (4, 5, 7)
    psi, _, _, _, g = workloads.random_problem(shape, (P, C, C), seed=11)
    z = np.zeros(shape)
    for iters, lim in ((1, False), (2, False), (2, True), (3, True)):
        for bc in ((P, P, P), (P, C, C), (C, C, C)):
            out = oracle.run(_prob(shape, bc, iters, lim), 3, psi, z, z, z, g)
            assert np.array_equal(out, psi)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [1.0, -1.0])
@pytest.mark.parametrize("iters,lim", [(1, False), (2, False), (2, True), (3, True)])
def test_courant_one_is_exact_shift(axis, sign, iters, lim):
    """C = +-1 on one axis, 0 elsewhere, G = 1: every pass moves the field by
    exactly one cell (the antidiffusive velocity (|C| - C^2) A - C (0 B + 0 B)
    is exactly 0), bitwise, with or without the limiter."""
    shape = (5, 6, 7)
    rng = np.random.default_rng(3)
    psi = rng.integers(0, 64, size=shape).astype(np.float64) / 8.0   # dyadic values
    vel = [np.zeros(shape) for _ in range(3)]
    vel[axis][:] = sign
    out = oracle.run(_prob(shape, (P, P, P), iters, lim), 2, psi, *vel, np.ones(shape))
    np_axis = 2 - axis
    want = np.roll(psi, int(2 * sign), axis=np_axis)
    assert np.array_equal(out, want)


def test_closed_vertical_boundary_flux_is_zero():
    """A closed axis is the paper's vertical boundary with factor 0 (Listing 7):
    no flux enters or leaves through the end faces, so with Cz > 0 the top cell
    only gains what the face below it carries."""
    shape = (5, 1, 1)
    psi = np.array([1.0, 2.0, 3.0, 4.0, 5.0]).reshape(shape)
    cz = np.full(shape, 0.25)
    z = np.zeros(shape)
    g = np.ones(shape)
    out = oracle.step(_prob(shape, (P, P, C), 1), psi, z, z, cz, g)
    flat = psi.ravel()
    want = flat.copy()
    want[0] = flat[0] - 0.25 * flat[0]
    for k in range(1, 4):
        want[k] = flat[k] - (0.25 * flat[k] - 0.25 * flat[k - 1])
    want[4] = flat[4] + 0.25 * flat[3]
    assert np.array_equal(out.ravel(), want)


# ---------------------------------------------------------------------------
# C3: antidiffusive velocity -- second order, the G terms, the cross terms
# ---------------------------------------------------------------------------

def _advect_error(n, axes, courants, iters, dims=3):
    """Max error after advecting 2 + sin*sin... over a fixed physical time."""
    shape = [1, 1, 1]
    for a in axes:
        shape[2 - a] = n
    shape = tuple(shape)
    coords = [np.zeros(1)] * 3
    for a in axes:
        coords[a] = (np.arange(n) + 0.5) / n
    k, j, i = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    xyz = [i, j, k]

    def field(shift):
        val = np.full(shape, 1.0)
        for a in axes:
            val = val * np.sin(2 * math.pi * (xyz[a] - shift[a]))
        return 2.0 + val

    steps = n // 2
    vel = [np.zeros(shape) for _ in range(3)]
    shift = [0.0, 0.0, 0.0]
    for a, c in zip(axes, courants):
        vel[a][:] = c
        shift[a] = c * steps / n
    out = oracle.run(_prob(shape, (P, P, P), iters), steps, field([0, 0, 0]), *vel, np.ones(shape))
    return float(np.max(np.abs(out - field(shift))))


def _order(errs):
    return [math.log2(errs[m] / errs[m + 1]) for m in range(len(errs) - 1)]


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_second_order_1d(axis):
    ns = (32, 64, 128)
    o2 = _order([_advect_error(n, (axis,), (0.4,), 2) for n in ns])
    o1 = _order([_advect_error(n, (axis,), (0.4,), 1) for n in ns])
    assert min(o2) >= 1.8, o2
    assert max(o1) <= 1.2, o1


@pytest.mark.parametrize("axes", [(0, 1), (0, 2), (1, 2)])
def test_second_order_oblique_2d(axes):
    """Oblique flow needs the cross terms of the antidiffusive velocity;
    without them (or with a wrong sign) the order drops to 1."""
    ns = (32, 64, 128)
    o2 = _order([_advect_error(n, axes, (0.3, -0.2), 2) for n in ns])
    assert min(o2) >= 1.8, o2


def test_second_order_oblique_3d():
    ns = (16, 32, 64)
    o2 = _order([_advect_error(n, (0, 1, 2), (0.2, -0.15, 0.1), 2) for n in ns])
    assert min(o2) >= 1.8, o2


def _variable_g_error(n, axis, amp=0.5, c=0.3):
    """1-D, constant C, G(x) = 1 + amp sin(2 pi x): psi is carried along the
    characteristics dx/dt = C h / G(x), so int_X^x G = C h S."""
    shape = [1, 1, 1]
    shape[2 - axis] = n
    shape = tuple(shape)
    x = (np.arange(n) + 0.5) / n
    G = 1.0 + amp * np.sin(2 * math.pi * x)

    def prim(s):
        return s - amp / (2 * math.pi) * np.cos(2 * math.pi * s)

    def psi0(s):
        return 2.0 + np.sin(2 * math.pi * s)

    steps = n // 2
    dist = c * steps / n
    # foot of the characteristic: prim(x) - prim(X) = dist, solved by Newton
    X = x - dist
    for _ in range(60):
        f = prim(x) - prim(X) - dist
        X = X + f / (1.0 + amp * np.sin(2 * math.pi * X))
    vel = [np.zeros(shape) for _ in range(3)]
    vel[axis][:] = c
    g = G.reshape(shape)
    out = oracle.run(_prob(shape, (P, P, P), 2), steps, psi0(x).reshape(shape), *vel, g)
    return float(np.max(np.abs(out.ravel() - psi0(X))))


@pytest.mark.parametrize("axis", [0, 2])
def test_second_order_variable_metric(axis):
    ns = (32, 64, 128)
    o = _order([_variable_g_error(n, axis) for n in ns])
    assert min(o) >= 1.8, o


def _small_stream_case(kind="solid", nx=48, ny=24, nz=5, courant=0.5):
    cx, cy, cz, _ = workloads.stream_winds(nx, ny, nz, kind, courant)
    g = workloads.metric(nx, ny, nz)
    return cx, cy, cz, g


@pytest.mark.parametrize("kind,iters", [("solid", 2), ("wave", 3)])
def test_constant_preserved_in_nondivergent_flow(kind, iters):
    cx, cy, cz, g = _small_stream_case(kind)
    # a vertical wind that is also divergence-free: constant in k per column is
    # not (closed ends), so keep Cz = 0 as in the lat-lon workloads
    psi = np.ones(g.shape)
    p = _prob(g.shape, (P, C, C), iters, True)
    out = oracle.run(p, 6, psi, cx, cy, cz, g)
    assert np.array_equal(out, psi)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("bc", [P, C])
def test_mirror_symmetry(axis, bc):
    """Reflecting one axis and negating its Courant numbers reflects the result."""
    shape = (6, 7, 9)
    psi, cx, cy, cz, g = workloads.random_problem(shape, (P, C, C), seed=5)
    vel = [cx, cy, cz]
    bcs = [P, P, P]
    bcs[axis] = bc
    p = _prob(shape, tuple(bcs), 3, True)
    ax = 2 - axis
    n = shape[ax]

    def refl(a):
        return np.flip(a, axis=ax)

    def refl_face(a):
        # face m+1/2 of the mirror is face (n-2-m)+1/2 of the original
        idx = [(n - 2 - m) % n for m in range(n)]
        out = -np.take(a, idx, axis=ax)
        if bc == C:
            sl = [slice(None)] * 3
            sl[ax] = n - 1
            out[tuple(sl)] = 0.0
        return out

    mv = [refl(v) if b != axis else refl_face(v) for b, v in enumerate(vel)]
    if bc == C:
        sl = [slice(None)] * 3
        sl[ax] = n - 1
        vel[axis] = vel[axis].copy()
        vel[axis][tuple(sl)] = 0.0
    a = oracle.run(p, 3, psi, *vel, g)
    b = oracle.run(p, 3, refl(psi), *mv, refl(g))
    assert np.max(np.abs(refl(b) - a)) <= 1e-14 * np.max(np.abs(a))


def test_axis_permutation_symmetry():
    """Swapping the roles of x and y (fields transposed) transposes the result:
    all three axes are coded alike."""
    shape = (5, 8, 8)
    psi, cx, cy, cz, g = workloads.random_problem(shape, (P, C, C), seed=8)
    p = _prob(shape, (C, C, P), 3, True)
    a = oracle.run(p, 3, psi, cx, cy, cz, g)
    t = lambda x: np.ascontiguousarray(np.swapaxes(x, 1, 2))
    b = oracle.run(p, 3, t(psi), t(cy), t(cx), t(cz), t(g))
    assert np.max(np.abs(t(b) - a)) <= 1e-14 * np.max(np.abs(a))
    # z <-> x as well
    u = lambda x: np.ascontiguousarray(np.swapaxes(x, 0, 2))
    shape3 = (6, 6, 6)
    psi, cx, cy, cz, g = workloads.random_problem(shape3, (P, C, C), seed=9)
    p3 = _prob(shape3, (C, P, C), 3, True)
    a = oracle.run(p3, 2, psi, cx, cy, cz, g)
    b = oracle.run(p3, 2, u(psi), u(cz), u(cy), u(cx), u(g))
    assert np.max(np.abs(u(b) - a)) <= 1e-14 * np.max(np.abs(a))


# ---------------------------------------------------------------------------
# C4-C6: limiter invariants
# ---------------------------------------------------------------------------

def _pass_by_pass(p, psin, cx, cy, cz, g):
    """Run one step stage by stage, checking every corrective pass against the
    local bounds it was limited with."""
    phi = oracle.donor(p, psin, cx, cy, cz, g)
    prev = (cx, cy, cz)
    worst = 0.0
    for _ in range(2, p.iters + 1):
        ut = oracle.antidiff(p, phi, *prev, g)
        mx, mn = oracle.bounds(p, psin, phi)
        bup, bdn = oracle.beta(p, phi, *ut, mx, mn, g)
        assert np.all(bup >= 0) and np.all(bdn >= 0)
        ul = oracle.limit(p, *ut, bup, bdn)
        nxt = oracle.donor(p, phi, *ul, g)
        scale = np.max(np.abs(nxt))
        worst = max(worst, float(np.max(nxt - mx) / scale), float(np.max(mn - nxt) / scale))
        phi, prev = nxt, ul
    return phi, worst


@pytest.mark.parametrize("bc", [(P, C, C), (P, P, P), (C, C, C)])
def test_limited_pass_stays_in_local_bounds(bc):
    shape = (6, 9, 11)
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=21, courant=0.9)
    p = _prob(shape, bc, 4, True)
    phi, worst = _pass_by_pass(p, psi, cx, cy, cz, g)
    assert worst <= 4 * np.finfo(float).eps
    # and the staged run equals the oracle's own step
    assert np.array_equal(phi, oracle.step(p, psi, cx, cy, cz, g))


def test_unlimited_pass_does_leave_bounds():
    """Control: without the limiter the same rough data over/undershoots."""
    shape = (6, 9, 11)
    psi, cx, cy, cz, g = workloads.random_problem(shape, (P, C, C), seed=21, courant=0.9)
    p = _prob(shape, (P, C, C), 3, False)
    out = oracle.step(p, psi, cx, cy, cz, g)
    mx, mn = oracle.bounds(p, psi, oracle.donor(p, psi, cx, cy, cz, g))
    assert np.max(out - mx) > 1e-6 or np.max(mn - out) > 1e-6


@pytest.mark.parametrize("kind,iters", [("solid", 2), ("wave", 3)])
def test_global_bounds_and_positivity(kind, iters):
    cx, cy, cz, g = _small_stream_case(kind)
    rng = np.random.default_rng(7)
    psi = np.exp(rng.standard_normal(g.shape))
    psi[:, 5:9, 10:20] = 0.0                    # a block of exact zeros
    p = _prob(g.shape, (P, C, C), iters, True)
    out = oracle.run(p, 20, psi, cx, cy, cz, g)
    assert out.min() >= 0.0
    assert out.min() >= psi.min() - 1e-14 * psi.max()
    assert out.max() <= psi.max() * (1 + 1e-14)


def test_step_function_no_overshoot():
    shape = (1, 1, 64)
    psi = np.zeros(shape)
    psi[..., 10:30] = 1.0
    z = np.zeros(shape)
    cx = np.full(shape, 0.37)
    lim = oracle.run(_prob(shape, (P, P, P), 3, True), 40, psi, cx, z, z, np.ones(shape))
    unl = oracle.run(_prob(shape, (P, P, P), 3, False), 40, psi, cx, z, z, np.ones(shape))
    assert lim.max() <= 1.0 + 1e-15 and lim.min() >= 0.0
    assert unl.max() > 1.0 + 1e-6            # the unlimited scheme does overshoot


# ---------------------------------------------------------------------------
# C7: mass
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bc", [(P, C, C), (P, P, P), (C, C, C)])
def test_mass_conserved(bc):
    shape = (5, 12, 16)
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=31)
    p = _prob(shape, bc, 3, True)
    m0 = oracle.mass(p, psi, g)
    out = oracle.run(p, 100, psi, cx, cy, cz, g)
    assert abs(oracle.mass(p, out, g) - m0) / m0 <= 1e-13


def test_mass_is_compensated_sum():
    shape = (3, 50, 70)
    rng = np.random.default_rng(2)
    psi = rng.uniform(0, 1e8, size=shape) * rng.choice([1e-8, 1.0], size=shape)
    g = rng.uniform(0.5, 1.0, size=shape)
    got = oracle.mass(_prob(shape), psi, g)
    assert got == math.fsum((g * psi).ravel().tolist())


# ---------------------------------------------------------------------------
# Transcription cross-check against the exact rational model
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bc", [(P, C, C), (P, P, P), (C, C, C), (C, P, C)])
@pytest.mark.parametrize("iters,lim", [(1, False), (2, False), (2, True), (3, True)])
def test_oracle_matches_exact_rational_model(bc, iters, lim):
    shape = (3, 3, 4)
    rng = np.random.default_rng(17)
    q = lambda a: np.round(a * 64) / 64
    psi = q(rng.random(shape) + 0.05)
    cx, cy, cz = (q((rng.random(shape) - 0.5) * 0.3) for _ in range(3))
    g = q(0.5 + rng.random(shape))
    a = oracle.run(_prob(shape, bc, iters, lim), 1, psi, cx, cy, cz, g)
    b = exact.run(shape, bc, psi, cx, cy, cz, g, iters, lim, 1)
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))


def test_degenerate_sizes():
    for shape in ((1, 1, 1), (1, 1, 5), (4, 1, 1), (1, 3, 1)):
        psi, cx, cy, cz, g = workloads.random_problem(shape, (P, C, C), seed=1)
        for bc in ((P, P, P), (C, C, C)):
            out = oracle.run(_prob(shape, bc, 3, True), 2, psi, cx, cy, cz, g)
            assert np.all(np.isfinite(out))
            if bc == (C, C, C) or shape == (1, 1, 1):
                pass
    # a single closed cell cannot change
    psi = np.full((1, 1, 1), 0.7)
    one = np.full((1, 1, 1), 0.3)
    out = oracle.run(_prob((1, 1, 1), (C, C, C), 3, True), 3, psi, one, one, one, np.ones((1, 1, 1)))
    assert np.array_equal(out, psi)


def test_invalid_arguments_rejected():
    shape = (2, 2, 2)
    a = np.ones(shape)
    with pytest.raises(ValueError):
        oracle.step(oracle.RefProblem(2, 2, 2, iters=0), a, a, a, a, a)
    with pytest.raises(ValueError):
        oracle.step(oracle.RefProblem(0, 2, 2), np.ones((2, 2, 0)), *(np.ones((2, 2, 0)),) * 4)


# ---------------------------------------------------------------------------
# Failure propagation: a NaN in the input is not silently lost
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("iters,limiter", [(1, False), (3, False), (3, True)])
def test_nan_in_input_reaches_its_cell(iters, limiter):
    """A NaN planted in psi^n stays in its own cell after a step (the update
    psi - div/G carries it) and after a run, whatever the max/min of the
    limiter do with it; cells outside its stencil stay finite."""
    shape, bc = (14, 9, 12), (P, C, C)
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=8, courant=0.8)
    psi[2, 4, 6] = np.nan
    p = oracle.RefProblem(shape[2], shape[1], shape[0], bc=bc, iters=iters, limiter=limiter)
    out = oracle.step(p, psi, cx, cy, cz, g)
    assert np.isnan(out[2, 4, 6])
    # 11 levels away: beyond one step's vertical reach (1 for the donor pass, 2 per corrective pass)
    assert np.all(np.isfinite(out[13]))
    assert np.isnan(oracle.run(p, 3, psi, cx, cy, cz, g)[2, 4, 6])
