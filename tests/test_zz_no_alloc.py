"""The allocation-free step (mpdata_step_noalloc) against mpdata_step, through
the C ABI (needs a GPU).

mpdata_step_noalloc runs the step's kernels on the library's fixed device
scratch instead of a caller's workspace.  Two calls in a row on one GPU,
the second on a smaller grid (so it runs over what the first left in the
scratch), must each give mpdata_step's result to the FP64 parity bar
(1e-12 relative; both run the same kernels, so the values are equal), and
FP32 likewise.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

P, C = "periodic", "closed"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(torch, mp, shape, bc, iters, dtype, seed, with_cz=True):
    tdt = torch.float64 if dtype == "f64" else torch.float32
    psi, cx, cy, cz, g = workloads.random_problem(shape, bc, seed=seed, courant=0.8)
    dv = [torch.from_numpy(a).to("cuda", tdt) for a in (psi, cx, cy, cz, g)]
    if not with_cz:
        dv[3] = None
    want = mp.step(*dv, iters=iters, limiter=True, bc=bc)
    out = torch.full_like(dv[0], float("nan"))
    mp.step_noalloc(*dv, out, iters=iters, limiter=True, bc=bc)
    torch.cuda.synchronize()
    return out, want


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_two_calls_match_step(dtype):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_06094_amd as mp

    tol = 1e-12 if dtype == "f64" else 0.0
    # a large call first, then a smaller one over the same scratch
    for shape, bc, iters, seed, with_cz in (((60, 128, 256), (P, C, C), 3, 11, True),
                                            ((5, 19, 131), (C, C, C), 2, 12, False)):
        _say(f"[noalloc] dtype={dtype} shape={shape} bc={bc} iters={iters} cz={with_cz}")
        out, want = _case(torch, mp, shape, bc, iters, dtype, seed, with_cz)
        err = float((out.double() - want.double()).abs().max() / want.double().abs().max())
        assert err <= tol, (shape, err)
        assert torch.equal(out, want), shape


def test_noalloc_refuses_grids_beyond_the_scratch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_06094_amd as mp

    shape = (80, 256, 256)      # 10 fields of 5.2 M FP64 cells: above the fixed scratch
    p = mp.problem_for(shape, (P, C, C), 2, True, "f64")
    assert mp.workspace_bytes(p, mp.MPDATA_OP_STEP) > mp.NOALLOC_SCRATCH_BYTES
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    with pytest.raises(mp.MpdataError) as ei:
        mp.step_noalloc(x, x, x, x, x + 1.0, torch.empty_like(x), iters=2)
    assert ei.value.code == mp._lib.MPDATA_EINVAL
