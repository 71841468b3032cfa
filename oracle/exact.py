"""Exact rational model of one MPDATA step, for tiny grids (test infrastructure).

An independent second transcription of the scheme, written cell by cell with
``fractions.Fraction`` so that there is no rounding at all.  It cross-checks the
C oracle's indexing and offsets on 4x3x3-sized grids: a transposed index or a
wrong halo rule in either one shows up as a difference far above the C
oracle's rounding.  It is not a pin of the scheme itself (that is the job of
the invariant, closed-form and convergence tests).

Scheme (paper, Section 5, Listings 4-9 for the donor-cell stages; the
corrective passes and the limiter from the MPDATA literature):
  donor flux      F = [c]+ * psi_left + [c]- * psi_right
  update          psi' = psi - (sum over axes of F(+1/2) - F(-1/2)) / G
  antidiffusive   U~ = (|U| - U^2/Gf) A - (U/Gf) (sum_t Vbar_t B_t)
  limiter         beta_up = (max - psi) G / (in + eps), beta_dn = (psi - min) G / (out + eps)
  limited         U~lim = [U~]+ min(1, b_dn(L), b_up(R)) + [U~]- min(1, b_up(L), b_dn(R))
"""
from __future__ import annotations

from fractions import Fraction

HALF = Fraction(1, 2)
QUARTER = Fraction(1, 4)


class Grid:
    def __init__(self, nx, ny, nz, bc):
        self.n = (nx, ny, nz)
        self.closed = tuple(b == "closed" for b in bc)

    def cells(self):
        nx, ny, nz = self.n
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    yield (i, j, k)

    def wrap(self, axis, x):
        n = self.n[axis]
        if self.closed[axis]:
            return min(max(x, 0), n - 1)
        return x % n

    def cell(self, c):
        return tuple(self.wrap(a, c[a]) for a in range(3))

    def face_is_zero(self, axis, x):
        """Face x+1/2 on `axis` is a closed wall (or beyond)."""
        return self.closed[axis] and (x <= -1 or x >= self.n[axis] - 1)


def _shift(c, axis, d):
    c = list(c)
    c[axis] += d
    return tuple(c)


def _get(grid, fld, c):
    return fld[grid.cell(c)]


def _face(grid, vel, axis, c):
    """Velocity of face c[axis]+1/2 of the (halo-mapped) column c."""
    if grid.face_is_zero(axis, c[axis]):
        return Fraction(0)
    d = [grid.wrap(b, c[b]) if b != axis else c[b] % grid.n[axis] for b in range(3)]
    return vel[axis][tuple(d)]


def _pos(x):
    return x if x > 0 else Fraction(0)


def _neg(x):
    return x if x < 0 else Fraction(0)


def donor_pass(grid, psi, vel, g):
    out = {}
    for c in grid.cells():
        total = Fraction(0)
        for a in range(3):
            right = _shift(c, a, 1)
            left = _shift(c, a, -1)
            u_r = _face(grid, vel, a, c)
            u_l = _face(grid, vel, a, left)
            f_r = _pos(u_r) * _get(grid, psi, c) + _neg(u_r) * _get(grid, psi, right)
            f_l = _pos(u_l) * _get(grid, psi, left) + _neg(u_l) * _get(grid, psi, c)
            total += f_r - f_l
        out[c] = psi[c] - total / g[c]
    return out


def antidiffusive(grid, psi, vel, g, eps):
    res = [dict(), dict(), dict()]
    for c in grid.cells():
        for a in range(3):
            if grid.face_is_zero(a, c[a]):
                res[a][c] = Fraction(0)
                continue
            L, R = c, _shift(c, a, 1)
            pl, pr = _get(grid, psi, L), _get(grid, psi, R)
            A = (pr - pl) / (pr + pl + eps)
            cross = Fraction(0)
            for t in range(3):
                if t == a:
                    continue
                sp = _get(grid, psi, _shift(R, t, 1)) + _get(grid, psi, _shift(L, t, 1))
                sm = _get(grid, psi, _shift(R, t, -1)) + _get(grid, psi, _shift(L, t, -1))
                B = HALF * (sp - sm) / (sp + sm + eps)
                vbar = QUARTER * (_face(grid, vel, t, L) + _face(grid, vel, t, R)
                                  + _face(grid, vel, t, _shift(L, t, -1))
                                  + _face(grid, vel, t, _shift(R, t, -1)))
                cross += vbar * B
            gf = HALF * (_get(grid, g, L) + _get(grid, g, R))
            u = vel[a][c]
            res[a][c] = (abs(u) - u * u / gf) * A - (u / gf) * cross
    return res


def limited(grid, psin, psi, vt, g, eps):
    hi, lo = {}, {}
    for c in grid.cells():
        vals = []
        for fld in (psin, psi):
            vals.append(_get(grid, fld, c))
            for a in range(3):
                vals.append(_get(grid, fld, _shift(c, a, 1)))
                vals.append(_get(grid, fld, _shift(c, a, -1)))
        hi[c], lo[c] = max(vals), min(vals)
    bup, bdn = {}, {}
    for c in grid.cells():
        fin = Fraction(0)
        fout = Fraction(0)
        for a in range(3):
            left, right = _shift(c, a, -1), _shift(c, a, 1)
            u_r = _face(grid, vt, a, c)
            u_l = _face(grid, vt, a, left)
            fin += _pos(u_l) * _get(grid, psi, left) - _neg(u_r) * _get(grid, psi, right)
            fout += _pos(u_r) * _get(grid, psi, c) - _neg(u_l) * _get(grid, psi, c)
        bup[c] = (hi[c] - psi[c]) * g[c] / (fin + eps)
        bdn[c] = (psi[c] - lo[c]) * g[c] / (fout + eps)
    out = [dict(), dict(), dict()]
    one = Fraction(1)
    for c in grid.cells():
        for a in range(3):
            if grid.face_is_zero(a, c[a]):
                out[a][c] = Fraction(0)
                continue
            r = grid.cell(_shift(c, a, 1))
            u = vt[a][c]
            out[a][c] = (_pos(u) * min(one, bdn[c], bup[r])
                         + _neg(u) * min(one, bup[c], bdn[r]))
    return out


def step(grid, psin, vel, g, iters, limiter, eps):
    phi = donor_pass(grid, psin, vel, g)
    prev = vel
    for _ in range(2, iters + 1):
        vt = antidiffusive(grid, phi, prev, g, eps)
        if limiter:
            vt = limited(grid, psin, phi, vt, g, eps)
        phi = donor_pass(grid, phi, vt, g)
        prev = vt
    return phi


def from_numpy(arr):
    """(nz, ny, nx) float array -> {(i, j, k): Fraction} (exact conversion)."""
    nz, ny, nx = arr.shape
    return {(i, j, k): Fraction(float(arr[k, j, i]))
            for k in range(nz) for j in range(ny) for i in range(nx)}


def to_numpy(d, shape):
    import numpy as np

    out = np.empty(shape)
    for (i, j, k), v in d.items():
        out[k, j, i] = float(v)
    return out


def run(shape, bc, psi, cx, cy, cz, g, iters, limiter, nsteps, eps=1e-15):
    nz, ny, nx = shape
    grid = Grid(nx, ny, nz, bc)
    e = Fraction(eps)
    cur = from_numpy(psi)
    vel = [from_numpy(cx), from_numpy(cy), from_numpy(cz)]
    gg = from_numpy(g)
    for _ in range(nsteps):
        cur = step(grid, cur, vel, gg, iters, limiter, e)
    return to_numpy(cur, shape)
