"""CPU FP64 oracle of the MPDATA step -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
``paper_1908_06094_amd``: the C oracle (``mpdata_ref.c``) and the exact
rational model (``exact.py``) are written independently of the HIP kernels.
"""
from .ref import (  # noqa: F401
    ustep, urun,
    RefProblem,
    adjoint,
    antidiff,
    beta,
    bounds,
    build,
    donor,
    limit,
    lib_path,
    mass,
    num_threads,
    set_num_threads,
    run,
    step,
)
