"""ctypes binding of the C oracle ``liboracle_mpdata.so`` (test infrastructure).

Every array is a C-contiguous float64 numpy array of shape (nz, ny, nx).
Boundary conditions are given per axis (x, y, z) as "periodic" or "closed".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpdata_ref.c")
_LIB = os.path.join(_HERE, "liboracle_mpdata.so")

PERIODIC, CLOSED = 0, 1
_BC = {"periodic": PERIODIC, "closed": CLOSED, PERIODIC: PERIODIC, CLOSED: CLOSED}


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, OpenMP."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 3), ("iters", ctypes.c_int32),
                ("limiter", ctypes.c_int32), ("eps", ctypes.c_double)]


@dataclass(frozen=True)
class RefProblem:
    nx: int
    ny: int
    nz: int
    bc: tuple = ("periodic", "closed", "closed")
    iters: int = 2
    limiter: bool = True
    eps: float = 0.0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def c(self) -> _Problem:
        s = _Problem()
        s.nx, s.ny, s.nz = self.nx, self.ny, self.nz
        for a in range(3):
            s.bc[a] = _BC[self.bc[a]]
        s.iters = self.iters
        s.limiter = 1 if self.limiter else 0
        s.eps = self.eps
        return s


class _UMesh(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_edges", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("pivbz", ctypes.c_double)]


_lib = None
_P = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        pp = ctypes.POINTER(_Problem)
        for name, nptr in (("ref_donor", 6), ("ref_bounds", 4), ("ref_limit", 8),
                           ("ref_antidiff", 8), ("ref_beta", 9)):
            f = getattr(lib, name)
            f.argtypes = [pp] + [_P] * nptr
            f.restype = ctypes.c_int
        lib.ref_step.argtypes = [pp] + [_P] * 6
        lib.ref_step.restype = ctypes.c_int
        lib.ref_run.argtypes = [pp, ctypes.c_int32] + [_P] * 5
        lib.ref_run.restype = ctypes.c_int
        lib.ref_mass.argtypes = [pp, _P, _P, _P]
        lib.ref_mass.restype = ctypes.c_int
        lib.ref_adjoint.argtypes = [pp, ctypes.c_int32] + [_P] * 10
        lib.ref_adjoint.restype = ctypes.c_int
        lib.ref_num_threads.argtypes = []
        lib.ref_num_threads.restype = ctypes.c_int
        lib.ref_set_num_threads.argtypes = [ctypes.c_int]
        lib.ref_set_num_threads.restype = None
        _I32 = ctypes.POINTER(ctypes.c_int32)
        _I8 = ctypes.POINTER(ctypes.c_int8)
        lib.ref_ustep.argtypes = [ctypes.POINTER(_UMesh), _I32, _I32, _I32, _I8] + [_P] * 6
        lib.ref_ustep.restype = ctypes.c_int
        _lib = lib
    return _lib


def _arr(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _call(name, *args):
    rc = getattr(_load(), name)(*args)
    if rc != 0:
        raise ValueError(f"{name} rejected its arguments (rc={rc})")


def donor(p: RefProblem, phi, u, v, w, g):
    s = p.shape
    phi, u, v, w, g = (_arr(x, s) for x in (phi, u, v, w, g))
    out = np.empty(s)
    _call("ref_donor", ctypes.byref(p.c()), _ptr(phi), _ptr(u), _ptr(v), _ptr(w), _ptr(g), _ptr(out))
    return out


def antidiff(p: RefProblem, phi, u, v, w, g):
    s = p.shape
    phi, u, v, w, g = (_arr(x, s) for x in (phi, u, v, w, g))
    ut, vt, wt = np.empty(s), np.empty(s), np.empty(s)
    _call("ref_antidiff", ctypes.byref(p.c()), _ptr(phi), _ptr(u), _ptr(v), _ptr(w), _ptr(g),
          _ptr(ut), _ptr(vt), _ptr(wt))
    return ut, vt, wt


def bounds(p: RefProblem, psin, phi):
    s = p.shape
    psin, phi = _arr(psin, s), _arr(phi, s)
    mx, mn = np.empty(s), np.empty(s)
    _call("ref_bounds", ctypes.byref(p.c()), _ptr(psin), _ptr(phi), _ptr(mx), _ptr(mn))
    return mx, mn


def beta(p: RefProblem, phi, ut, vt, wt, mx, mn, g):
    s = p.shape
    phi, ut, vt, wt, mx, mn, g = (_arr(x, s) for x in (phi, ut, vt, wt, mx, mn, g))
    bup, bdn = np.empty(s), np.empty(s)
    _call("ref_beta", ctypes.byref(p.c()), _ptr(phi), _ptr(ut), _ptr(vt), _ptr(wt), _ptr(mx),
          _ptr(mn), _ptr(g), _ptr(bup), _ptr(bdn))
    return bup, bdn


def limit(p: RefProblem, ut, vt, wt, bup, bdn):
    s = p.shape
    ut, vt, wt, bup, bdn = (_arr(x, s) for x in (ut, vt, wt, bup, bdn))
    ul, vl, wl = np.empty(s), np.empty(s), np.empty(s)
    _call("ref_limit", ctypes.byref(p.c()), _ptr(ut), _ptr(vt), _ptr(wt), _ptr(bup), _ptr(bdn),
          _ptr(ul), _ptr(vl), _ptr(wl))
    return ul, vl, wl


def step(p: RefProblem, psi, cx, cy, cz, g):
    s = p.shape
    psi, cx, cy, g = (_arr(x, s) for x in (psi, cx, cy, g))
    cz = None if cz is None else _arr(cz, s)
    out = np.empty(s)
    _call("ref_step", ctypes.byref(p.c()), _ptr(psi), _ptr(out), _ptr(cx), _ptr(cy), _ptr(cz), _ptr(g))
    return out


def run(p: RefProblem, nsteps: int, psi, cx, cy, cz, g):
    s = p.shape
    psi = np.array(_arr(psi, s), copy=True)
    cx, cy, g = (_arr(x, s) for x in (cx, cy, g))
    cz = None if cz is None else _arr(cz, s)
    _call("ref_run", ctypes.byref(p.c()), int(nsteps), _ptr(psi), _ptr(cx), _ptr(cy), _ptr(cz), _ptr(g))
    return psi


def mass(p: RefProblem, psi, g) -> float:
    s = p.shape
    psi, g = _arr(psi, s), _arr(g, s)
    out = np.zeros(1)
    _call("ref_mass", ctypes.byref(p.c()), _ptr(psi), _ptr(g), _ptr(out))
    return float(out[0])


def num_threads() -> int:
    return int(_load().ref_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later calls (its OpenMP loops)."""
    _load().ref_set_num_threads(int(n))


def adjoint(p: RefProblem, nsteps: int, psi0, cx, cy, cz, g, seed):
    """Reverse sweep: (dJ/dpsi0, dJ/dcx, dJ/dcy, dJ/dcz) for the seed dJ/dpsi_T."""
    s = p.shape
    psi0, cx, cy, g, seed = (_arr(x, s) for x in (psi0, cx, cy, g, seed))
    cz = None if cz is None else _arr(cz, s)
    out = [np.empty(s) for _ in range(4)]
    _call("ref_adjoint", ctypes.byref(p.c()), int(nsteps), _ptr(psi0), _ptr(cx), _ptr(cy), _ptr(cz), _ptr(g),
          _ptr(seed), *[_ptr(o) for o in out])
    return tuple(out)


def ustep(edges, node_ptr, node_edges, node_sign, vol, psi, vn, w, rho, pivbz=0.0):
    """Unstructured donor-cell step (see mpdata_ref.h): psi, w, rho are
    (nodes, nz), vn is (edges, nz), edges is (edges, 2)."""
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    nn, nz = psi.shape
    edges = np.ascontiguousarray(edges, dtype=np.int32)
    ne = edges.shape[0]
    node_ptr = np.ascontiguousarray(node_ptr, dtype=np.int32)
    node_edges = np.ascontiguousarray(node_edges, dtype=np.int32)
    node_sign = np.ascontiguousarray(node_sign, dtype=np.int8)
    vol = np.ascontiguousarray(vol, dtype=np.float64)
    vn = np.ascontiguousarray(vn, dtype=np.float64).reshape(ne, nz) if ne else np.zeros((1, nz))
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(nn, nz)
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(nn, nz)
    out = np.empty((nn, nz))
    m = _UMesh(nn, ne, nz, float(pivbz))
    i32 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    _call("ref_ustep", ctypes.byref(m), i32(edges), i32(node_ptr), i32(node_edges),
          node_sign.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), _ptr(vol), _ptr(psi), _ptr(vn), _ptr(w),
          _ptr(rho), _ptr(out))
    return out


def urun(nsteps, edges, node_ptr, node_edges, node_sign, vol, psi, vn, w, rho, pivbz=0.0):
    out = np.array(psi, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        out = ustep(edges, node_ptr, node_edges, node_sign, vol, out, vn, w, rho, pivbz)
    return out
