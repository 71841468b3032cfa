"""MPDATA advection step on MI355X: Python binding of libmpdata.so.

Argument marshalling only: every stage of the scheme runs in the library's
HIP kernels.  PyTorch supplies device memory and the current stream.  The
binding fails loudly if the built library is missing; there is no fallback.

Fields are contiguous torch tensors of shape (nz, ny, nx), dtype float64 or
float32, on a ROCm device.  Boundary conditions are per axis (x, y, z):
"periodic" or "closed".  The unstructured (edge-based) step takes
(nodes, levels) and (edges, levels) tensors and a DeviceMesh.
"""
from __future__ import annotations

from ._lib import (  # noqa: F401
    MPDATA_CLOSED,
    MPDATA_F32,
    MPDATA_F64,
    MPDATA_KERNEL_DONOR,
    MPDATA_KERNEL_PASS,
    MPDATA_KERNEL_PASS_DONOR,
    MPDATA_KERNEL_STAGE,
    MPDATA_KERNEL_USTEP,
    MPDATA_OP_ADJOINT,
    MPDATA_OP_MASS,
    MPDATA_OP_RUN,
    MPDATA_OP_STEP,
    MPDATA_PERIODIC,
    MPDATA_BATCH_GRAPH,
    MPDATA_BATCH_TUNE,
    BATCH_VARIANTS_F32,
    BATCH_VARIANTS_F64,
    BatchItem,
    DeviceMesh,
    UMesh,
    urun,
    ustep,
    MpdataError,
    batch_problem,
    run_batched,
    adjoint,
    mpdata_function,
    Problem,
    lib,
    lib_path,
    mass,
    problem_for,
    run,
    step,
    step_noalloc,
    NOALLOC_SCRATCH_BYTES,
    timing_enable,
    timing_read,
    workspace_bytes,
)


def __getattr__(name):
    if name == "MPDATAFunction":
        return mpdata_function()
    raise AttributeError(name)
