"""ctypes binding of the C ABI declared in include/mpdata.h."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libmpdata.so")

MPDATA_OK, MPDATA_EINVAL, MPDATA_ENOMEM, MPDATA_EDEVICE, MPDATA_EUNSUPPORTED = 0, -1, -2, -3, -4
MPDATA_F64, MPDATA_F32 = 0, 1
MPDATA_PERIODIC, MPDATA_CLOSED = 0, 1
MPDATA_OP_STEP, MPDATA_OP_RUN, MPDATA_OP_ADJOINT, MPDATA_OP_MASS = 0, 1, 2, 3

_BC = {"periodic": MPDATA_PERIODIC, "closed": MPDATA_CLOSED,
       MPDATA_PERIODIC: MPDATA_PERIODIC, MPDATA_CLOSED: MPDATA_CLOSED}


class MpdataError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mpdata error {code}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 3), ("iters", ctypes.c_int32), ("limiter", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32), ("eps", ctypes.c_double)]


class UMesh(ctypes.Structure):
    """mpdata_umesh: an unstructured mesh whose tables live in device memory."""
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_edges", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("pivbz", ctypes.c_double), ("edge_nodes", ctypes.c_void_p),
                ("node_ptr", ctypes.c_void_p), ("node_edges", ctypes.c_void_p), ("node_sign", ctypes.c_void_p),
                ("dual_volume", ctypes.c_void_p)]


_lib = None
_vp = ctypes.c_void_p
_pp = ctypes.POINTER(Problem)
_up = ctypes.POINTER(UMesh)

_SIGNATURES = {
    "mpdata_workspace_bytes": ([_pp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_size_t),
    "mpdata_step": ([_pp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "mpdata_run": ([_pp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "mpdata_step_noalloc": ([_pp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "mpdata_mass": ([_pp, _vp, _vp, ctypes.POINTER(ctypes.c_double), _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "mpdata_adjoint": ([_pp, ctypes.c_int32, ctypes.c_int32] + [_vp] * 11 + [_vp, ctypes.c_size_t, _vp],
                       ctypes.c_int),
    "mpdata_batch_workspace_bytes": ([_pp, ctypes.c_int32, _vp], ctypes.c_size_t),
    "mpdata_run_batched": ([_pp, ctypes.c_int32, _vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_size_t, _vp],
                           ctypes.c_int),
    "mpdata_ustep": ([_up, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "mpdata_uworkspace_bytes": ([_up], ctypes.c_size_t),
    "mpdata_urun": ([_up, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "mpdata_last_error": ([], ctypes.c_char_p),
    "mpdata_timing_enable": ([ctypes.c_int32], ctypes.c_int),
    "mpdata_timing_read": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
                           ctypes.c_int),
}

MPDATA_KERNEL_PASS, MPDATA_KERNEL_DONOR, MPDATA_KERNEL_STAGE, MPDATA_KERNEL_USTEP, MPDATA_KERNEL_PASS_DONOR = 0, 1, 2, 3, 4


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load libmpdata.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with paper_1908_06094_amd/build.py "
                               "(or __graft_entry__.build()) first")
        handle = ctypes.CDLL(_LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            f = getattr(handle, name)
            f.argtypes = args
            f.restype = res
        _lib = handle
    return _lib


def _check(rc):
    if rc != MPDATA_OK:
        msg = lib().mpdata_last_error()
        raise MpdataError(rc, msg.decode() if msg else "")


def problem_for(shape, bc=("periodic", "closed", "closed"), iters=2, limiter=True, dtype="f64", eps=0.0):
    nz, ny, nx = shape
    p = Problem()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    for a in range(3):
        p.bc[a] = _BC[bc[a]]
    p.iters = int(iters)
    p.limiter = 1 if limiter else 0
    p.dtype = {"f64": MPDATA_F64, "f32": MPDATA_F32}[dtype]
    p.reserved = 0
    p.eps = float(eps)
    return p


def workspace_bytes(p: Problem, op: int, nsteps: int = 0, checkpoint_every: int = 0) -> int:
    n = lib().mpdata_workspace_bytes(ctypes.byref(p), op, nsteps, checkpoint_every)
    if n == 0:
        _check(MPDATA_EINVAL)
    return int(n)


def _dtype_code(t):
    import torch

    if t.dtype == torch.float64:
        return "f64"
    if t.dtype == torch.float32:
        return "f32"
    raise TypeError(f"unsupported dtype {t.dtype}")


def _fields(psi, others):
    import torch

    if not psi.is_cuda:
        raise ValueError("fields must be device tensors")
    for t in (psi, *[o for o in others if o is not None]):
        if t.shape != psi.shape or t.dtype != psi.dtype or t.device != psi.device:
            raise ValueError("all fields must share shape, dtype and device")
        if not t.is_contiguous():
            raise ValueError("fields must be contiguous")
    if psi.dim() != 3:
        raise ValueError("fields must have shape (nz, ny, nx)")
    return torch.cuda.current_stream(psi.device).cuda_stream


def _workspace(nbytes, device):
    import torch

    # 256-byte aligned by the caching allocator
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def step(psi, cx, cy, cz, g, *, iters=2, limiter=True, bc=("periodic", "closed", "closed"), eps=0.0,
         out=None, workspace=None):
    """One MPDATA step on the current stream; returns psi^{n+1} (a new tensor
    unless `out` is given)."""
    import torch

    stream = _fields(psi, (cx, cy, cz, g, out))
    p = problem_for(tuple(psi.shape), bc, iters, limiter, _dtype_code(psi), eps)
    if out is None:
        out = torch.empty_like(psi)
    nb = workspace_bytes(p, MPDATA_OP_STEP)
    ws = workspace if workspace is not None else _workspace(nb, psi.device)
    _check(lib().mpdata_step(ctypes.byref(p), _ptr(psi), _ptr(out), _ptr(cx), _ptr(cy), _ptr(cz), _ptr(g),
                             _ptr(ws), ws.numel(), ctypes.c_void_p(stream)))
    return out


NOALLOC_SCRATCH_BYTES = 168 << 20   # MPDATA_NOALLOC_SCRATCH_BYTES


def step_noalloc(psi, cx, cy, cz, g, out, *, iters=2, limiter=True, bc=("periodic", "closed", "closed"), eps=0.0):
    """One MPDATA step into `out` through mpdata_step_noalloc (the library's
    fixed device scratch, no workspace): allocates nothing."""
    stream = _fields(psi, (cx, cy, cz, g, out))
    p = problem_for(tuple(psi.shape), bc, iters, limiter, _dtype_code(psi), eps)
    _check(lib().mpdata_step_noalloc(ctypes.byref(p), _ptr(psi), _ptr(out), _ptr(cx), _ptr(cy), _ptr(cz), _ptr(g),
                                     ctypes.c_void_p(stream)))
    return out


def run(psi, cx, cy, cz, g, nsteps, *, iters=2, limiter=True, bc=("periodic", "closed", "closed"), eps=0.0,
        workspace=None):
    """nsteps MPDATA steps in place on psi (enqueued on the current stream)."""
    stream = _fields(psi, (cx, cy, cz, g))
    p = problem_for(tuple(psi.shape), bc, iters, limiter, _dtype_code(psi), eps)
    nb = workspace_bytes(p, MPDATA_OP_RUN)
    ws = workspace if workspace is not None else _workspace(nb, psi.device)
    _check(lib().mpdata_run(ctypes.byref(p), int(nsteps), _ptr(psi), _ptr(cx), _ptr(cy), _ptr(cz), _ptr(g),
                            _ptr(ws), ws.numel(), ctypes.c_void_p(stream)))
    return psi


def mass(psi, g, *, bc=("periodic", "closed", "closed")) -> float:
    """sum(G psi) accumulated in FP64 on the device (synchronises the stream)."""
    stream = _fields(psi, (g,))
    p = problem_for(tuple(psi.shape), bc, 1, False, _dtype_code(psi))
    ws = _workspace(workspace_bytes(p, MPDATA_OP_MASS), psi.device)
    out = ctypes.c_double(0.0)
    _check(lib().mpdata_mass(ctypes.byref(p), _ptr(psi), _ptr(g), ctypes.byref(out), _ptr(ws), ws.numel(),
                             ctypes.c_void_p(stream)))
    return out.value


def timing_enable(on: bool = True) -> None:
    """Start (clearing earlier records) or stop event timing of kernel launches."""
    _check(lib().mpdata_timing_enable(1 if on else 0))


def timing_read(kind: int):
    """(total milliseconds, launches) of one kernel kind since timing_enable."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().mpdata_timing_read(kind, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def adjoint(psi0, cx, cy, cz, g, seed, nsteps, *, checkpoint_every=0, iters=2, limiter=True,
            bc=("periodic", "closed", "closed"), eps=0.0, want_dcz=True):
    """Reverse sweep of `run`: returns (dJ/dpsi0, dJ/dcx, dJ/dcy, dJ/dcz or None, psi_T)
    for the seed dJ/dpsi_T (FP64)."""
    import torch

    stream = _fields(psi0, (cx, cy, cz, g, seed))
    p = problem_for(tuple(psi0.shape), bc, iters, limiter, _dtype_code(psi0), eps)
    nb = lib().mpdata_workspace_bytes(ctypes.byref(p), MPDATA_OP_ADJOINT, int(nsteps), int(checkpoint_every))
    if nb == 0:
        _check(MPDATA_EINVAL)
    ws = _workspace(nb, psi0.device)
    dpsi0 = torch.empty_like(psi0)
    dcx, dcy = torch.empty_like(psi0), torch.empty_like(psi0)
    dcz = torch.empty_like(psi0) if want_dcz else None
    psiT = torch.empty_like(psi0)
    _check(lib().mpdata_adjoint(ctypes.byref(p), int(nsteps), int(checkpoint_every), _ptr(psi0), _ptr(cx),
                                _ptr(cy), _ptr(cz), _ptr(g), _ptr(seed), _ptr(dpsi0), _ptr(dcx), _ptr(dcy),
                                _ptr(dcz), _ptr(psiT), _ptr(ws), ws.numel(), ctypes.c_void_p(stream)))
    return dpsi0, dcx, dcy, dcz, psiT


def _make_function():
    import torch

    class MPDATAFunction(torch.autograd.Function):
        """(psi0, cx, cy, cz) -> psi_T after `nsteps` MPDATA steps; the backward
        runs the library's hand-written adjoint (mpdata_adjoint) with
        checkpoints every `checkpoint_every` steps.  g is a fixed metric."""

        @staticmethod
        def forward(ctx, psi0, cx, cy, cz, g, nsteps, checkpoint_every=0, iters=2, limiter=True,
                    bc=("periodic", "closed", "closed")):
            ctx.save_for_backward(psi0, cx, cy, cz, g)
            ctx.cfg = (int(nsteps), int(checkpoint_every), int(iters), bool(limiter), tuple(bc))
            out = psi0.detach().clone()
            run(out, cx.detach(), cy.detach(), cz.detach(), g.detach(), nsteps, iters=iters, limiter=limiter, bc=bc)
            return out

        @staticmethod
        def backward(ctx, grad_out):
            psi0, cx, cy, cz, g = ctx.saved_tensors
            nsteps, k, iters, limiter, bc = ctx.cfg
            d0, dx, dy, dz, _ = adjoint(psi0.detach(), cx.detach(), cy.detach(), cz.detach(), g.detach(),
                                        grad_out.contiguous(), nsteps, checkpoint_every=k, iters=iters,
                                        limiter=limiter, bc=bc)
            return d0, dx, dy, dz, None, None, None, None, None, None

    return MPDATAFunction


_fn_cache = []


def mpdata_function():
    if not _fn_cache:
        _fn_cache.append(_make_function())
    return _fn_cache[0]


MPDATA_BATCH_GRAPH, MPDATA_BATCH_TUNE = 1, 2

# The batched kernel variants by index (include/mpdata.h, MPDATA_BATCH_TUNE):
# (row lanes, threads per workgroup, workgroups per CU, donor-cell pass).
BATCH_VARIANTS_F32 = [(32, 768, 1, "folded"), (32, 768, 2, "folded"), (64, 768, 1, "folded"),
                      (64, 768, 2, "folded"), (16, 768, 1, "folded"), (16, 768, 2, "folded"),
                      (32, 768, 1, "separate"), (32, 768, 2, "separate"), (64, 768, 1, "separate"),
                      (64, 768, 2, "separate"), (16, 768, 1, "separate"), (16, 768, 2, "separate"),
                      (32, 1024, 1, "folded"), (64, 1024, 1, "folded"), (16, 1024, 1, "folded"),
                      (32, 1024, 1, "separate"), (64, 1024, 1, "separate"), (16, 1024, 1, "separate")]
BATCH_VARIANTS_F64 = [(64, 768, 1, "folded"), (64, 768, 1, "separate")]


class BatchItem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("ntracers", ctypes.c_int32), ("cx", ctypes.c_void_p), ("cy", ctypes.c_void_p),
                ("cz", ctypes.c_void_p), ("g", ctypes.c_void_p), ("psi", ctypes.c_void_p)]


def _batch_items(problems):
    import torch

    arr = (BatchItem * len(problems))()
    dtype = None
    for i, pr in enumerate(problems):
        psi, cx, cy, cz, g = pr["psi"], pr["cx"], pr["cy"], pr.get("cz"), pr["g"]
        if psi.dim() != 4:
            raise ValueError("psi of a batch item has shape (ntracers, nz, ny, nx)")
        for t in (psi, cx, cy, cz, g):
            if t is None:
                continue
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("batch fields must be contiguous device tensors")
            if dtype is None:
                dtype = t.dtype
            if t.dtype != dtype:
                raise ValueError("all batch fields must share one dtype")
        if tuple(cx.shape) != tuple(psi.shape[1:]) or tuple(g.shape) != tuple(psi.shape[1:]):
            raise ValueError("winds and metric must have the shape of one tracer field")
        nt, nz, ny, nx = psi.shape
        arr[i] = BatchItem(nx, ny, nz, nt, cx.data_ptr(), cy.data_ptr(), 0 if cz is None else cz.data_ptr(),
                           g.data_ptr(), psi.data_ptr())
    return arr, {torch.float64: "f64", torch.float32: "f32"}[dtype]


def batch_problem(problems, *, iters=2, limiter=True, bc=("periodic", "closed", "closed"), eps=0.0):
    """(items array, common problem, workspace bytes) for run_batched."""
    items, dt = _batch_items(problems)
    p = problem_for((1, 1, 1), bc, iters, limiter, dt, eps)
    nb = lib().mpdata_batch_workspace_bytes(ctypes.byref(p), len(problems), ctypes.cast(items, ctypes.c_void_p))
    if nb == 0:
        _check(MPDATA_EINVAL)
    return items, p, int(nb)


def run_batched(problems, nsteps, *, iters=2, limiter=True, bc=("periodic", "closed", "closed"), eps=0.0,
                graph=True, tune=False, workspace=None, stream=None):
    """nsteps steps of every problem in `problems` (dicts with psi of shape
    (ntracers, nz, ny, nx) and cx, cy, cz (or None), g of shape (nz, ny, nx)),
    in place, in one persistent launch per pass."""
    import torch

    items, p, nb = batch_problem(problems, iters=iters, limiter=limiter, bc=bc, eps=eps)
    dev = problems[0]["psi"].device
    ws = workspace if workspace is not None else _workspace(nb, dev)
    if ws.numel() < nb:
        raise ValueError("workspace too small")
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    flags = (MPDATA_BATCH_GRAPH if graph else 0) | (MPDATA_BATCH_TUNE if tune else 0)
    _check(lib().mpdata_run_batched(ctypes.byref(p), len(problems), ctypes.cast(items, ctypes.c_void_p),
                                    int(nsteps), flags, _ptr(ws), ws.numel(), ctypes.c_void_p(st.cuda_stream)))


# ---------------------------------------------------------------------------
# Unstructured (edge-based) donor-cell step
# ---------------------------------------------------------------------------

class DeviceMesh:
    """An unstructured mesh uploaded to the device: the connectivity is
    checked on the host (every index in range, the node table consistent
    with the edge table) before it is copied, so the kernels only ever see
    valid indices.  Keeps the device arrays alive as long as the mesh."""

    def __init__(self, edges, node_ptr, node_edges, node_sign, dual_volume, nz, *, dtype="f64", pivbz=0.0,
                 device="cuda"):
        import numpy as np
        import torch

        edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        node_ptr = np.ascontiguousarray(node_ptr, dtype=np.int32)
        node_edges = np.ascontiguousarray(node_edges, dtype=np.int32)
        node_sign = np.ascontiguousarray(node_sign, dtype=np.int8)
        vol = np.ascontiguousarray(dual_volume, dtype=np.float64)
        nn, ne = len(node_ptr) - 1, len(edges)
        if nn < 1 or nz < 1 or len(vol) != nn:
            raise ValueError("mesh sizes are inconsistent")
        if node_ptr[0] != 0 or node_ptr[-1] != len(node_edges) or np.any(np.diff(node_ptr) < 0):
            raise ValueError("node_ptr must start at 0, be non-decreasing and end at len(node_edges)")
        if len(node_sign) != len(node_edges) or not np.all(np.abs(node_sign) == 1):
            raise ValueError("node_sign must hold +1 / -1 for every node_edges entry")
        if ne and (edges.min() < 0 or edges.max() >= nn):
            raise ValueError("edge node index out of range")
        if len(node_edges) and (node_edges.min() < 0 or node_edges.max() >= ne):
            raise ValueError("node edge index out of range")
        if not np.all(vol > 0):
            raise ValueError("dual volumes must be positive")
        self.dtype = torch.float64 if dtype == "f64" else torch.float32
        dev = torch.device(device)
        as_dev = lambda a: torch.from_numpy(a).to(dev)
        self._keep = [as_dev(edges.reshape(-1)), as_dev(node_ptr), as_dev(node_edges if len(node_edges) else
                      np.zeros(1, np.int32)), as_dev(node_sign if len(node_sign) else np.zeros(1, np.int8)),
                      torch.from_numpy(vol).to(dev, self.dtype)]
        self.c = UMesh(nn, ne, int(nz), MPDATA_F64 if dtype == "f64" else MPDATA_F32, float(pivbz),
                       *[t.data_ptr() for t in self._keep])
        self.n_nodes, self.n_edges, self.nz, self.device = nn, ne, int(nz), dev

    @classmethod
    def from_octa(cls, mesh, nz, **kw):
        return cls(mesh.edges, mesh.node_ptr, mesh.node_edges, mesh.node_sign, mesh.dual_volume, nz, **kw)


def _ufields(m, psi, vn, w, rho):
    import torch

    for t, shape, what in ((psi, (m.n_nodes, m.nz), "psi"), (vn, (m.n_edges, m.nz), "vn"),
                           (w, (m.n_nodes, m.nz), "w"), (rho, (m.n_nodes, m.nz), "rho")):
        if t is None and what == "w":
            continue
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.dtype != m.dtype:
            raise ValueError(f"{what} must be a contiguous device tensor of the mesh's dtype")
        if tuple(t.shape) != shape:
            raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {shape}")
    return torch.cuda.current_stream(psi.device).cuda_stream


def ustep(m, psi, vn, w, rho, out=None):
    """One unstructured donor-cell step on the current stream; returns the new field."""
    import torch

    stream = _ufields(m, psi, vn, w, rho)
    out = torch.empty_like(psi) if out is None else out
    _check(lib().mpdata_ustep(ctypes.byref(m.c), _ptr(psi), _ptr(out), _ptr(vn), _ptr(w), _ptr(rho),
                              ctypes.c_void_p(stream)))
    return out


def urun(m, psi, vn, w, rho, nsteps, workspace=None):
    """nsteps unstructured steps in place on psi."""
    stream = _ufields(m, psi, vn, w, rho)
    nb = lib().mpdata_uworkspace_bytes(ctypes.byref(m.c))
    ws = workspace if workspace is not None else _workspace(nb, psi.device)
    _check(lib().mpdata_urun(ctypes.byref(m.c), int(nsteps), _ptr(psi), _ptr(vn), _ptr(w), _ptr(rho), _ptr(ws),
                             ws.numel(), ctypes.c_void_p(stream)))
    return psi
