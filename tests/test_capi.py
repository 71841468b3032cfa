"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/mpdata.h declares, and rejects invalid arguments
synchronously with the documented codes before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _mp():
    import paper_1908_06094_amd as mp

    if not os.path.exists(mp.lib_path()):
        from paper_1908_06094_amd import build

        build.build()
    return mp


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(mpdata_[a-z0-9_]+)\s*\(", text))
    return names


def test_exports_every_declared_symbol():
    mp = _mp()
    handle = ctypes.CDLL(mp.lib_path())
    declared = _declared()
    assert {"mpdata_step", "mpdata_run", "mpdata_mass", "mpdata_workspace_bytes", "mpdata_last_error"} <= declared
    for name in declared:
        assert hasattr(handle, name), name


def _no_device():
    """Calls below pass bogus device addresses that validation must reject;
    they are only made where no GPU could ever be reached."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("host-only argument checks (no device calls with bogus pointers where a GPU is present)")


def _call_step(mp, p, psi_in=8, psi_out=16, ws_bytes=None, ws=256):
    _no_device()
    lib = mp.lib()
    nb = ws_bytes if ws_bytes is not None else 1 << 40
    v = lambda x: ctypes.c_void_p(x) if x else None
    return lib.mpdata_step(ctypes.byref(p), v(psi_in), v(psi_out), v(24), v(32), None, v(40), v(ws), nb, None)


def test_invalid_problems_rejected():
    mp = _mp()
    bad = []
    p = mp.problem_for((4, 5, 6)); p.nx = 0; bad.append(p)
    p = mp.problem_for((4, 5, 6)); p.bc[1] = 7; bad.append(p)
    p = mp.problem_for((4, 5, 6), iters=0); bad.append(p)
    p = mp.problem_for((4, 5, 6), iters=9); bad.append(p)
    p = mp.problem_for((4, 5, 6)); p.limiter = 2; bad.append(p)
    p = mp.problem_for((4, 5, 6)); p.dtype = 5; bad.append(p)
    p = mp.problem_for((4, 5, 6)); p.reserved = 1; bad.append(p)
    p = mp.problem_for((4, 5, 6), eps=-1.0); bad.append(p)
    for p in bad:
        assert _call_step(mp, p) == mp._lib.MPDATA_EINVAL
        assert mp.lib().mpdata_last_error()
        assert mp.lib().mpdata_workspace_bytes(ctypes.byref(p), 0, 0, 0) == 0


def test_pointer_and_workspace_checks():
    mp = _mp()
    p = mp.problem_for((4, 5, 6))
    assert _call_step(mp, p, psi_in=None) == mp._lib.MPDATA_EINVAL
    assert _call_step(mp, p, psi_in=64, psi_out=64) == mp._lib.MPDATA_EINVAL        # aliasing
    assert b"alias" in mp.lib().mpdata_last_error()
    assert _call_step(mp, p, psi_in=12) == mp._lib.MPDATA_EINVAL                    # misaligned
    assert _call_step(mp, p, ws=None) == mp._lib.MPDATA_EINVAL
    assert _call_step(mp, p, ws=128) == mp._lib.MPDATA_EINVAL                       # ws alignment
    need = mp.workspace_bytes(p, mp.MPDATA_OP_STEP)
    assert need > 0
    assert _call_step(mp, p, ws_bytes=need - 1) == mp._lib.MPDATA_EINVAL
    lib = mp.lib()
    _no_device()
    assert lib.mpdata_run(ctypes.byref(p), -1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8),
                          None, ctypes.c_void_p(8), ctypes.c_void_p(256), 1 << 40, None) == mp._lib.MPDATA_EINVAL


def test_workspace_sizes_scale_with_dtype():
    mp = _mp()
    p64 = mp.problem_for((10, 20, 30), dtype="f64")
    p32 = mp.problem_for((10, 20, 30), dtype="f32")
    a = mp.workspace_bytes(p64, mp.MPDATA_OP_STEP)
    b = mp.workspace_bytes(p32, mp.MPDATA_OP_STEP)
    assert a > b > 0
    assert mp.workspace_bytes(p64, mp.MPDATA_OP_RUN) > a


def test_binding_refuses_host_tensors():
    torch = pytest.importorskip("torch")
    mp = _mp()
    x = torch.ones(2, 3, 4, dtype=torch.float64)
    with pytest.raises(ValueError):
        mp.step(x, x, x, x, x)


def _items(mp, shapes, ptr=256):
    """A batch item array with fake (aligned, never dereferenced) pointers."""
    arr = (mp.BatchItem * len(shapes))()
    for i, (nx, ny, nz, nt) in enumerate(shapes):
        arr[i].nx, arr[i].ny, arr[i].nz, arr[i].ntracers = nx, ny, nz, nt
        arr[i].cx = arr[i].cy = arr[i].g = arr[i].psi = ptr
        arr[i].cz = None
    return arr


def _batch_ws(mp, shapes, iters=2, ptr=256):
    p = mp.problem_for((1, 1, 1), iters=iters, dtype="f32")
    arr = _items(mp, shapes, ptr)
    return mp.lib().mpdata_batch_workspace_bytes(ctypes.byref(p), len(shapes), ctypes.cast(arr, ctypes.c_void_p))


def test_batched_workspace_and_validation():
    mp = _mp()
    small = _batch_ws(mp, [(64, 32, 20, 1)])
    assert small > 0
    assert _batch_ws(mp, [(64, 32, 20, 1), (128, 64, 40, 3)]) > small
    assert _batch_ws(mp, [(64, 32, 20, 0)]) == 0                       # no tracers
    assert b"ntracers" in mp.lib().mpdata_last_error()
    assert _batch_ws(mp, [(0, 32, 20, 1)]) == 0                        # empty grid
    assert _batch_ws(mp, [(64, 32, 70000, 1)]) == 0                    # nz beyond the grid limit
    assert _batch_ws(mp, [(64, 32, 20, 1)], ptr=258) == 0              # misaligned field
    # 2 x 2^30 donor-pass blocks (64 x 4 columns x 16 levels each) exceed one launch
    assert _batch_ws(mp, [(64, 4, 16, 1 << 30), (64, 4, 16, 1 << 30)]) == 0
    assert b"blocks" in mp.lib().mpdata_last_error()


def test_unstructured_validation():
    mp = _mp()
    lib = mp.lib()
    m = mp.UMesh(10, 15, 4, mp.MPDATA_F64, 0.0, 256, 256, 256, 256, 256)
    assert lib.mpdata_uworkspace_bytes(ctypes.byref(m)) == (10 * 4 * 8 + 255) // 256 * 256
    for field, val in (("n_nodes", 0), ("nz", 0), ("n_edges", -1), ("dtype", 7)):
        bad = mp.UMesh(10, 15, 4, mp.MPDATA_F64, 0.0, 256, 256, 256, 256, 256)
        setattr(bad, field, val)
        assert lib.mpdata_uworkspace_bytes(ctypes.byref(bad)) == 0
    bad = mp.UMesh(10, 15, 4, mp.MPDATA_F64, float("nan"), 256, 256, 256, 256, 256)
    assert lib.mpdata_uworkspace_bytes(ctypes.byref(bad)) == 0
    bad = mp.UMesh(10, 15, 4, mp.MPDATA_F64, 0.0, 0, 256, 256, 256, 256)      # edge table missing
    assert lib.mpdata_uworkspace_bytes(ctypes.byref(bad)) == 0
    _no_device()
    v = ctypes.c_void_p
    assert lib.mpdata_ustep(ctypes.byref(m), v(512), v(512), v(768), None, v(1024), None) == mp._lib.MPDATA_EINVAL
    assert b"alias" in lib.mpdata_last_error()
    assert lib.mpdata_ustep(ctypes.byref(m), v(512), v(2048), None, None, v(1024), None) == mp._lib.MPDATA_EINVAL
    assert lib.mpdata_urun(ctypes.byref(m), 2, v(512), v(768), None, v(1024), v(4096), 16, None) == \
        mp._lib.MPDATA_EINVAL


def test_unsupported_combinations():
    """FP32 adjoints and batched runs of more than 9 passes are refused with
    MPDATA_EUNSUPPORTED before anything is enqueued."""
    mp = _mp()
    lib = mp.lib()
    _no_device()
    v = ctypes.c_void_p
    p32 = mp.problem_for((8, 6, 4), dtype="f32")
    args = [v(256)] * 5 + [v(512)] + [v(768)] * 3 + [None, None, v(1024), 1 << 40, None]
    assert lib.mpdata_adjoint(ctypes.byref(p32), 2, 1, *args) == mp._lib.MPDATA_EUNSUPPORTED
    assert b"FP64" in lib.mpdata_last_error()
    p = mp.problem_for((1, 1, 1), iters=10)
    arr = _items(mp, [(64, 32, 20, 1)])
    assert lib.mpdata_run_batched(ctypes.byref(p), 1, ctypes.cast(arr, ctypes.c_void_p), 2, 0, v(4096), 1 << 40,
                                  None) in (mp._lib.MPDATA_EUNSUPPORTED, mp._lib.MPDATA_EINVAL)


def test_eps_floor():
    """eps is 0 (the default) or in [1e-30, 1e-3]: below the floor a guarded
    denominator could leave the normal range."""
    mp = _mp()
    lib = mp.lib()
    for eps, ok in ((0.0, True), (1e-30, True), (1e-15, True), (1e-3, True), (9e-31, False), (1e-100, False),
                    (2e-3, False), (float("nan"), False), (-1e-15, False)):
        p = mp.problem_for((4, 5, 6), eps=eps)
        assert (lib.mpdata_workspace_bytes(ctypes.byref(p), 0, 0, 0) > 0) == ok, eps
        if not ok:
            assert b"eps" in lib.mpdata_last_error()


def test_noalloc_refuses_grids_beyond_its_scratch():
    """mpdata_step_noalloc checks its fixed scratch's size before it touches
    the device."""
    mp = _mp()
    lib = mp.lib()
    big = mp.problem_for((80, 256, 256))
    assert mp.workspace_bytes(big, mp.MPDATA_OP_STEP) > mp.NOALLOC_SCRATCH_BYTES
    small = mp.problem_for((60, 128, 256))
    assert mp.workspace_bytes(small, mp.MPDATA_OP_STEP) <= mp.NOALLOC_SCRATCH_BYTES
    _no_device()
    v = ctypes.c_void_p
    assert lib.mpdata_step_noalloc(ctypes.byref(big), v(256), v(512), v(768), v(1024), None, v(1280), None) == \
        mp._lib.MPDATA_EINVAL
    assert b"scratch" in lib.mpdata_last_error()
    assert lib.mpdata_step_noalloc(ctypes.byref(small), v(256), v(256), v(768), v(1024), None, v(1280), None) == \
        mp._lib.MPDATA_EINVAL
    assert b"alias" in lib.mpdata_last_error()


def test_adjoint_rejects_aliased_outputs():
    """No adjoint output may alias an input, another output or the workspace."""
    mp = _mp()
    lib = mp.lib()
    _no_device()
    v = ctypes.c_void_p
    p = mp.problem_for((4, 5, 6))
    psi0, cx, cy, cz, g, seed = 1 << 12, 2 << 12, 3 << 12, 4 << 12, 5 << 12, 6 << 12
    d0, dx, dy, dz, pt, ws = 7 << 12, 8 << 12, 9 << 12, 10 << 12, 11 << 12, 1 << 20

    def call(**kw):
        a = dict(psi0=psi0, cx=cx, cy=cy, cz=cz, g=g, seed=seed, d0=d0, dx=dx, dy=dy, dz=dz, pt=pt)
        a.update(kw)
        return lib.mpdata_adjoint(ctypes.byref(p), 2, 1, v(a["psi0"]), v(a["cx"]), v(a["cy"]), v(a["cz"]),
                                  v(a["g"]), v(a["seed"]), v(a["d0"]), v(a["dx"]), v(a["dy"]), v(a["dz"]),
                                  v(a["pt"]), v(ws), 1 << 40, None)

    for kw in (dict(pt=seed), dict(dx=cx), dict(dy=cy), dict(dz=cz), dict(d0=psi0), dict(d0=seed), dict(dy=dx),
               dict(pt=d0), dict(dz=g), dict(pt=ws)):
        assert call(**kw) == mp._lib.MPDATA_EINVAL, kw
        assert b"alias" in lib.mpdata_last_error()
