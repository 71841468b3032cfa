"""Seeded synthetic inputs for the MPDATA step (shared by tests and benchmark).

This module holds none of the scheme's arithmetic: it only builds fields
(tracer, face Courant numbers, metric G) of the shapes and structure of the
paper's workloads.  The paper measures on octahedral meshes of 71 424 nodes x
80 levels and a 128x128x80 patch (Section 6.1, Table 1, Figures 13-14); those
meshes are not available, so lat-lon-shaped structured grids of similar and
larger size stand in for them.

Geometry of the lat-lon grids: cell centres at lambda_i = (i+1/2) 2pi/nx and
phi_j = -pi/2 + (j+1/2) pi/ny over the whole globe, G = cos(phi_j) at every
level, boundary conditions (periodic, closed, closed).

Winds come from a streamfunction Psi sampled at cell corners, so they are
discretely non-divergent: Cx = -s (Psi(i+1/2, j+1/2) - Psi(i+1/2, j-1/2)),
Cy = s (Psi(i+1/2, j+1/2) - Psi(i-1/2, j+1/2)), Cz = 0.  The scaled corner
values s*Psi are rounded to multiples of 2**-20 (one exact value per pole) so
that every face difference and every divergence sum is exact in FP64 and in
FP32.  The scale s makes the largest outflow Courant sum over G,
max_i (sum_axes [C_{i+1/2}]+ - [C_{i-1/2}]-) / G_i, equal the stated value.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

QUANTUM = 2.0 ** -20


@dataclass
class Workload:
    name: str
    shape: tuple            # (nz, ny, nx)
    bc: tuple               # per axis x, y, z
    iters: int
    limiter: bool
    steps: int
    psi: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    cz: np.ndarray
    g: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        nz, ny, nx = self.shape
        return nx * ny * nz

    def astype(self, dtype):
        out = Workload(self.name, self.shape, self.bc, self.iters, self.limiter, self.steps,
                       *(a.astype(dtype) for a in (self.psi, self.cx, self.cy, self.cz, self.g)),
                       meta=dict(self.meta))
        return out


def lat_lon(nx: int, ny: int):
    lam = (np.arange(nx) + 0.5) * (2.0 * math.pi / nx)
    phi = -0.5 * math.pi + (np.arange(ny) + 0.5) * (math.pi / ny)
    return lam, phi


def metric(nx: int, ny: int, nz: int) -> np.ndarray:
    _, phi = lat_lon(nx, ny)
    return np.ascontiguousarray(np.broadcast_to(np.cos(phi)[None, :, None], (nz, ny, nx)))


def _corner_coords(nx: int, ny: int):
    # corners (i+1/2, j+1/2) for i = -1..nx-1 and j = -1..ny-1
    lam_c = (np.arange(-1, nx) + 1.0) * (2.0 * math.pi / nx)
    phi_c = -0.5 * math.pi + (np.arange(-1, ny) + 1.0) * (math.pi / ny)
    return lam_c, phi_c


def solid_body_stream(lam, phi, alpha=0.05):
    return -(np.sin(phi) * math.cos(alpha) - np.cos(lam) * np.cos(phi) * math.sin(alpha))


def wave_stream(lam, phi):
    return -np.sin(phi) + 0.5 * np.cos(phi) ** 3 * np.sin(2.0 * lam)


def _faces_from_corners(psi_c):
    """psi_c[(j+1), (i+1)] at corners (i+1/2, j+1/2), i, j from -1; returns (cx, cy) 2-D."""
    # Cx(i, j) = -(Psi(i+1/2, j+1/2) - Psi(i+1/2, j-1/2))
    cx = -(psi_c[1:, 1:] - psi_c[:-1, 1:])
    # Cy(i, j) = Psi(i+1/2, j+1/2) - Psi(i-1/2, j+1/2)
    cy = psi_c[1:, 1:] - psi_c[1:, :-1]
    return cx, cy


def _outflow_over_g(cx, cy, g2):
    """Largest (sum over axes of outflow Courant) / G for x periodic, y closed."""
    cxl = np.roll(cx, 1, axis=1)                       # face i-1/2 (periodic)
    cyl = np.concatenate([np.zeros_like(cy[:1]), cy[:-1]], axis=0)  # face j-1/2, wall at j=0
    cyr = cy.copy()
    cyr[-1] = 0.0                                       # wall at j = ny-1/2
    out = (np.maximum(cx, 0) - np.minimum(cxl, 0)) + (np.maximum(cyr, 0) - np.minimum(cyl, 0))
    return float(np.max(out / g2))


def stream_winds(nx, ny, nz, kind="solid", max_courant=0.5, alpha=0.05):
    """Non-divergent face Courant numbers from a corner streamfunction."""
    lam_c, phi_c = _corner_coords(nx, ny)
    L, P = np.meshgrid(lam_c, phi_c)
    if kind == "solid":
        psi_c = solid_body_stream(L, P, alpha)
        pole_s, pole_n = math.cos(alpha), -math.cos(alpha)   # cos(lat) = 0 there
    elif kind == "wave":
        psi_c = wave_stream(L, P)
        pole_s, pole_n = 1.0, -1.0
    else:
        raise ValueError(kind)
    psi_c[0, :] = pole_s                  # corner row j = -1/2 is the south pole
    psi_c[-1, :] = pole_n                 # corner row j = ny-1/2 is the north pole
    psi_c[:, 0] = psi_c[:, -1]            # the corner i = -1/2 is the corner nx-1/2
    _, phi = lat_lon(nx, ny)
    g2 = np.broadcast_to(np.cos(phi)[:, None], (ny, nx))
    cx, cy = _faces_from_corners(psi_c)
    s = max_courant / _outflow_over_g(cx, cy, g2)
    psi_q = np.round(psi_c * s / QUANTUM) * QUANTUM
    cx, cy = _faces_from_corners(psi_q)
    cy[-1, :] = 0.0                        # closed north wall slot (unused)
    cx3 = np.ascontiguousarray(np.broadcast_to(cx[None], (nz, ny, nx)))
    cy3 = np.ascontiguousarray(np.broadcast_to(cy[None], (nz, ny, nx)))
    cz3 = np.zeros((nz, ny, nx))
    return cx3, cy3, cz3, {"scale": s, "max_outflow_over_g": _outflow_over_g(cx, cy, g2)}


def cosine_bell(nx, ny, centre=(1.5 * math.pi, 0.0), radius=1.0 / 3.0, h=1.0):
    lam, phi = lat_lon(nx, ny)
    L, P = np.meshgrid(lam, phi)
    lc, pc = centre
    cosr = np.sin(pc) * np.sin(P) + np.cos(pc) * np.cos(P) * np.cos(L - lc)
    r = np.arccos(np.clip(cosr, -1.0, 1.0))
    return np.where(r < radius, 0.5 * h * (1.0 + np.cos(math.pi * r / radius)), 0.0)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def gaussian_2d(n=64, steps=100):
    """2-D periodic n x n, constant Courant (0.25, 0.15), G = 1, Gaussian blob
    (amplitude 1, sigma 6 cells, background 0), 2 passes, no limiter."""
    shape = (1, n, n)
    i = np.arange(n)
    I, J = np.meshgrid(i, i)
    c = n // 2
    psi = np.exp(-((I - c) ** 2 + (J - c) ** 2) / (2.0 * 6.0 ** 2))[None].copy()
    return Workload("2d-periodic-64x64-gaussian", shape, ("periodic",) * 3, 2, False, steps,
                    psi, np.full(shape, 0.25), np.full(shape, 0.15), np.zeros(shape), np.ones(shape))


def latlon_solid_body(nx=256, ny=128, nz=60, steps=50, seed=2):
    """Lat-lon 256x128x60, 2 passes, limiter on, G = cos(lat), solid-body winds
    (tilt 0.05 rad) scaled to max Courant 0.5, Cz = 0, cosine bell + U[0, 0.1)."""
    rng = np.random.default_rng(seed)
    cx, cy, cz, meta = stream_winds(nx, ny, nz, "solid", 0.5)
    bell = cosine_bell(nx, ny)
    psi = bell[None] + rng.uniform(0.0, 0.1, size=(nz, ny, nx))
    return Workload(f"latlon-{nx}x{ny}x{nz}-solid-body", (nz, ny, nx),
                    ("periodic", "closed", "closed"), 2, True, steps,
                    np.ascontiguousarray(psi), cx, cy, cz, metric(nx, ny, nz), meta)


def latlon_wave(nx=1024, ny=512, nz=80, steps=50, seed=3, iters=3):
    """Lat-lon 1024x512x80, 3 passes, limiter on, streamfunction winds
    Psi = -sin(lat) + 0.5 cos^3(lat) sin(2 lon) scaled to max Courant 0.6,
    lognormal(0, 1) tracer."""
    rng = np.random.default_rng(seed)
    cx, cy, cz, meta = stream_winds(nx, ny, nz, "wave", 0.6)
    psi = np.exp(rng.standard_normal((nz, ny, nx)))
    return Workload(f"latlon-{nx}x{ny}x{nz}-wave", (nz, ny, nx),
                    ("periodic", "closed", "closed"), iters, True, steps,
                    psi, cx, cy, cz, metric(nx, ny, nz), meta)


def rounded_to_fp32(w: Workload) -> Workload:
    """Inputs rounded to FP32 once, so FP32 and FP64 runs start from the same values."""
    r = w.astype(np.float32).astype(np.float64)
    r.name = w.name
    return r


def random_problem(shape, bc, seed, courant=0.3, gmin=0.5, positive=True, cz=True):
    """Small random problem for parity tests: rough positive tracer, random
    (divergent) face velocities kept under the donor-cell stability bound."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    psi = rng.uniform(0.0, 1.0, size=shape) ** 3 + (0.0 if not positive else 1e-3)
    g = rng.uniform(gmin, 1.0, size=shape)
    lim = courant * gmin / 6.0
    cx = rng.uniform(-lim, lim, size=shape)
    cy = rng.uniform(-lim, lim, size=shape)
    czz = rng.uniform(-lim, lim, size=shape) if cz else np.zeros(shape)
    return psi, cx, cy, czz, g


def cost_weights(shape, seed=5):
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=shape)


def batched_problems(count=64, seed=4, dtype=np.float32, max_courant=0.5):
    """Batched workload: `count` lat-lon problems of uneven sizes, each with
    1-8 lognormal(0, 1) tracers sharing its winds (the 1024x512x80 workload's streamfunction
    family at max Courant 0.5) and metric; FP32, 2 passes, limiter, 20 steps.
    Returns a list of dicts: psi (ntracers, nz, ny, nx), cx, cy, cz, g."""
    rng = np.random.default_rng(seed + 1000)
    out = []
    for nx, ny, nz, nt in batch_sizes(count, seed):
        cx, cy, cz, _ = stream_winds(nx, ny, nz, "wave", max_courant)
        g = metric(nx, ny, nz)
        psi = np.exp(rng.standard_normal((nt, nz, ny, nx), dtype=np.float64)).astype(dtype)
        out.append({"psi": psi, "cx": cx.astype(dtype), "cy": cy.astype(dtype), "cz": cz.astype(dtype),
                    "g": g.astype(dtype)})
    return out


def batch_sizes(count=64, seed=4):
    """Sizes and tracer counts of the batched workload: nx in U{64..512},
    ny in U{32..256}, nz in U{20..80}, 1-8 tracers."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nx = int(rng.integers(64, 513))
        ny = int(rng.integers(32, 257))
        nz = int(rng.integers(20, 81))
        nt = int(rng.integers(1, 9))
        out.append((nx, ny, nz, nt))
    return out
