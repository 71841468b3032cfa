"""No kernel writes outside the buffers it is given.

Every output and the workspace sit inside larger device allocations whose
margins hold a canary byte pattern; after each call the margins must be
unchanged (the forward step and run in FP64 and FP32, with and without the
limiter, the adjoint, and the edge-based step).  Inputs are ordinary
tensors.  The grids are small and ragged (several tiles, partial edge tiles).
"""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

PAD = 4096          # canary bytes on each side (keeps the inner buffer 256-byte aligned)
CANARY = 0xA5
P, C = "periodic", "closed"


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _padded(torch, nbytes):
    whole = torch.full((nbytes + 2 * PAD,), CANARY, dtype=torch.uint8, device="cuda")
    return whole, whole[PAD:PAD + nbytes]


def _typed(inner, dtype, shape):
    return inner.view(dtype).view(shape)


def _margins_intact(whole, nbytes):
    h = whole.cpu().numpy()
    return bool((h[:PAD] == CANARY).all() and (h[PAD + nbytes:] == CANARY).all())


@pytest.mark.parametrize("dtype,iters,lim,shape", [("f64", 3, True, (5, 37, 131)), ("f32", 3, True, (5, 37, 131)),
                                                   ("f64", 2, False, (5, 37, 131)), ("f64", 3, True, (5, 30, 1)),
                                                   ("f32", 2, True, (130, 3, 5))])
def test_step_and_run_write_only_their_buffers(dtype, iters, lim, shape):
    torch = _torch()
    import paper_1908_06094_amd as mp

    bc = (P, C, C)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    elem = 8 if dtype == "f64" else 4
    print(f"[canary] step/run {dtype} shape={shape} iters={iters} limiter={lim}", flush=True)
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=21, courant=0.8)
    dev = [torch.from_numpy(a).to("cuda", tdt) for a in (psi, cx, cy, cz, g)]
    nbytes = int(np.prod(shape)) * elem
    p = mp.problem_for(shape, bc, iters, lim, dtype)

    out_whole, out_inner = _padded(torch, nbytes)
    ws_bytes = mp.workspace_bytes(p, mp.MPDATA_OP_STEP)
    ws_whole, ws_inner = _padded(torch, ws_bytes)
    out = mp.step(*dev, iters=iters, limiter=lim, bc=bc, out=_typed(out_inner, tdt, shape), workspace=ws_inner)
    torch.cuda.synchronize()
    assert _margins_intact(out_whole, nbytes)
    assert _margins_intact(ws_whole, ws_bytes)
    assert torch.isfinite(out).all()

    run_bytes = mp.workspace_bytes(p, mp.MPDATA_OP_RUN)
    rws_whole, rws_inner = _padded(torch, run_bytes)
    psi_whole, psi_inner = _padded(torch, nbytes)
    x = _typed(psi_inner, tdt, shape)
    x.copy_(dev[0])
    mp.run(x, *dev[1:], 3, iters=iters, limiter=lim, bc=bc, workspace=rws_inner)
    torch.cuda.synchronize()
    assert _margins_intact(psi_whole, nbytes)
    assert _margins_intact(rws_whole, run_bytes)


def test_adjoint_writes_only_its_buffers():
    torch = _torch()
    import paper_1908_06094_amd as mp
    from paper_1908_06094_amd import _lib

    shape, bc, iters, steps, k = (4, 21, 70), (P, C, C), 2, 3, 2
    print(f"[canary] adjoint shape={shape} iters={iters} steps={steps} checkpoint_every={k}", flush=True)
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=22, courant=0.8)
    dev = [torch.from_numpy(a).cuda() for a in (psi + 0.2, cx, cy, cz, g, np.ones(shape))]
    nbytes = int(np.prod(shape)) * 8
    p = mp.problem_for(shape, bc, iters, True, "f64")
    ws_bytes = _lib.lib().mpdata_workspace_bytes(ctypes.byref(p), _lib.MPDATA_OP_ADJOINT, steps, k)
    bufs = [_padded(torch, nbytes) for _ in range(5)]          # dpsi0, dcx, dcy, dcz, psiT
    ws_whole, ws_inner = _padded(torch, ws_bytes)
    stream = torch.cuda.current_stream().cuda_stream
    rc = _lib.lib().mpdata_adjoint(ctypes.byref(p), steps, k, *[_lib._ptr(t) for t in dev],
                                   *[_lib._ptr(inner) for _, inner in bufs], _lib._ptr(ws_inner), ws_bytes,
                                   ctypes.c_void_p(stream))
    _lib._check(rc)
    torch.cuda.synchronize()
    for whole, _ in bufs:
        assert _margins_intact(whole, nbytes)
    assert _margins_intact(ws_whole, ws_bytes)


def test_unstructured_step_writes_only_its_buffer():
    torch = _torch()
    import paper_1908_06094_amd as mp
    from workloads import octahedral as octa

    u = octa.random_uproblem(4, 70, seed=23, pivbz=0.5)
    m = u.mesh
    print(f"[canary] unstructured O4 nodes={m.n_nodes} levels={u.nz}", flush=True)
    dm = mp.DeviceMesh.from_octa(m, u.nz, pivbz=0.5)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (u.psi, u.vn, u.w, u.rho)]
    nbytes = u.psi.size * 8
    out_whole, out_inner = _padded(torch, nbytes)
    mp.ustep(dm, *dev, out=_typed(out_inner, torch.float64, u.psi.shape))
    torch.cuda.synchronize()
    assert _margins_intact(out_whole, nbytes)
