"""Algorithmic traffic and operation counts of the MPDATA kernels.

The paper counts main-memory accesses of the MPDATA flux stages per vertical
plane, with and without fusion (Section 6.1, Table 2), and defines bandwidth
as required data transfer over run time (Table 1).  The same accounting,
applied to this library's kernels, gives the algorithmic bytes behind the
benchmark's roofline figures.
"""
from __future__ import annotations

from dataclasses import dataclass


def plane_accesses(edge_reads, edge_writes, node_reads, node_writes, n_edges, n_nodes):
    """Main-memory accesses per vertical plane for an edge/node access pattern
    (the accounting of the paper's Table 2)."""
    return (edge_reads + edge_writes) * n_edges + (node_reads + node_writes) * n_nodes


# Per cell and step, the minimum traffic of a whole MPDATA step: read psi, the
# three face Courant arrays and G; write psi.
STEP_WORDS = 6
STEP_WORDS_NO_CZ = 5


def pass_kernel_words(write_velocities: bool, with_cz: bool = True) -> int:
    """Words per cell one fused corrective pass moves: read the iterate,
    psi^n, the three previous-pass velocities and G; write the new iterate
    (and its three limited velocities when another pass follows)."""
    reads = 6 if with_cz else 5
    return reads + (4 if write_velocities else 1)


def donor_kernel_words(with_cz: bool = True) -> int:
    """Words per cell of the donor-cell pass: read psi, Cx, Cy, (Cz), G; write psi^(1)."""
    return (5 if with_cz else 4) + 1


@dataclass(frozen=True)
class OpCount:
    """FP64 operations one cell needs, counted from the scheme's formulas:
    every add, subtract, multiply, divide, max, min and absolute value is one
    operation (an IEEE division is one operation here, although gfx950 has no
    divide instruction and expands it into about ten)."""
    total: int
    divisions: int


def antidiffusive_face_ops() -> OpCount:
    # A: difference, pair sum, + eps, divide                         -> 4 (1 div)
    # per transverse axis: two pair sums, difference, sum, + eps,
    #   divide, times 1/2                                            -> 7 (1 div) x 2
    # per transverse axis: velocity average (3 adds, times 1/4)      -> 4 x 2
    # face metric: add, times 1/2                                    -> 2
    # combination: |U|, U*U, /Gf, -, *A, U/Gf, 2 products, +, *, -   -> 11 (2 div)
    return OpCount(4 + 14 + 8 + 2 + 11, 1 + 2 + 2)


def donor_pass_ops() -> OpCount:
    # three own-face fluxes ([c]+, [c]-, two products, add), the
    # divergence (3 differences, 2 adds), divide by G, subtract
    return OpCount(3 * 5 + 5 + 1 + 1, 1)


def corrective_pass_ops(limiter: bool = True) -> OpCount:
    face = antidiffusive_face_ops()
    total = 3 * face.total
    div = 3 * face.divisions
    if limiter:
        total += 26        # max and min over the 14 values of the 7-point cross of psi^n and phi
        total += 3 * 10 + 4  # in/out: per axis 4 parts (max/min + product) and 2 differences; 4 adds
        total += 2 * 4     # beta_up, beta_dn: difference, times G, + eps, divide
        div += 2
        total += 3 * 9     # limited velocity per face: [U]+, [U]-, 4 mins, 2 products, add
    d = donor_pass_ops()
    return OpCount(total + d.total, div + d.divisions)


def step_ops(iters: int, limiter: bool) -> OpCount:
    d = donor_pass_ops()
    c = corrective_pass_ops(limiter)
    return OpCount(d.total + (iters - 1) * c.total, d.divisions + (iters - 1) * c.divisions)


# MI355X peaks used for the roofline figures
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz: one FP64 operation per lane
# and cycle (the 78.6 TFLOP/s FP64 vector figure counts an FMA as two)
FP64_VALU_OPS_PEAK = 256 * 4 * 16 * 2.4e9
