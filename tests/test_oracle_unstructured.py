"""Pins of the oracle's unstructured (edge-based) donor-cell step, the
paper's own MPDATA operator sequence (Section 5, Listings 4-9): a reduction
to the structured oracle, invariants of the scheme and properties of the
generated octahedral mesh."""
import numpy as np
import pytest

import oracle
from workloads import octahedral as octa


def _ring(nx):
    """nx nodes on a ring, edge i from node i to node i+1 (mod nx)."""
    edges = np.array([[i, (i + 1) % nx] for i in range(nx)], dtype=np.int32)
    inc = [[] for _ in range(nx)]
    for e, (a, b) in enumerate(edges):
        inc[a].append((e, 1))
        inc[b].append((e, -1))
    ptr = np.zeros(nx + 1, dtype=np.int32)
    ptr[1:] = np.cumsum([len(x) for x in inc])
    ne = np.array([e for x in inc for e, _ in sorted(x)], dtype=np.int32)
    sg = np.array([s for x in inc for _, s in sorted(x)], dtype=np.int8)
    return edges, ptr, ne, sg


@pytest.mark.parametrize("nx,nz", [(7, 5), (12, 1), (3, 9)])
def test_ring_reduces_to_the_structured_donor_step(nx, nz):
    """A ring of nodes with unit dual volumes is the structured grid with
    ny = 1: the edge step must equal the structured oracle's donor-cell pass
    (one pass, no limiter; x periodic, z closed <-> pivbz = 0) bit for bit."""
    rng = np.random.default_rng(nx * 10 + nz)
    shape = (nz, 1, nx)
    psi = rng.uniform(0, 1, shape)
    cx = rng.uniform(-0.4, 0.4, shape)
    cz = rng.uniform(-0.4, 0.4, shape)
    g = rng.uniform(0.7, 1.3, shape)
    p = oracle.RefProblem(nx, 1, nz, bc=("periodic", "closed", "closed"), iters=1, limiter=False)
    want = oracle.step(p, psi, cx, np.zeros(shape), cz, g)

    edges, ptr, ne, sg = _ring(nx)
    # node-major, level-fastest fields; w[n, k] sits at the interface k-1 / k = the structured face k-1/2
    upsi = psi[:, 0, :].T.copy()
    urho = g[:, 0, :].T.copy()
    vn = cx[:, 0, :].T.copy()
    w = np.zeros((nx, nz))
    w[:, 1:] = cz[:-1, 0, :].T
    got = oracle.ustep(edges, ptr, ne, sg, np.ones(nx), upsi, vn, w, urho, pivbz=0.0)
    assert np.array_equal(got, want[:, 0, :].T)


def test_mesh_is_a_closed_sphere():
    m = octa.build(6)
    assert m.n_nodes == 4 * 6 * 6 + 36 * 6          # 2 * sum over rows of (16 + 4 i)
    assert m.n_nodes - m.n_edges + len(m.faces) == 2
    assert (m.edge_faces >= 0).all()
    assert abs(m.dual_volume.sum() - 4 * np.pi) < 0.05 * 4 * np.pi
    deg = np.diff(m.node_ptr)
    assert deg.min() >= 3 and deg.sum() == 2 * m.n_edges
    # every node's signed edge fluxes of a streamfunction flow telescope to 0
    vn = octa.streamfunction_flux(m, 1, 0.5)[:, 0]
    s = np.zeros(m.n_nodes)
    np.add.at(s, m.edges[:, 0], vn)
    np.add.at(s, m.edges[:, 1], -vn)
    assert np.all(s == 0.0)


def test_constant_field_is_preserved_exactly():
    """A uniform tracer in a discretely non-divergent flow (no vertical wind)
    does not change: every node's signed flux sum is exactly zero."""
    u = octa.random_uproblem(5, 4, seed=3)
    m = u.mesh
    psi = np.full((m.n_nodes, u.nz), 0.75)
    out = oracle.ustep(m.edges, m.node_ptr, m.node_edges, m.node_sign, m.dual_volume, psi, u.vn,
                       np.zeros_like(psi), u.rho)
    assert np.all(out == 0.75)


def test_mass_is_conserved_with_closed_top_and_bottom():
    """sum(vol rho psi) is conserved: each edge flux leaves one node and
    enters the other, and with pivbz = 0 no vertical flux crosses the ends."""
    u = octa.random_uproblem(5, 6, seed=4)
    m = u.mesh
    mass = lambda f: float(np.sum(m.dual_volume[:, None] * u.rho * f))
    out = oracle.urun(3, m.edges, m.node_ptr, m.node_edges, m.node_sign, m.dual_volume, u.psi, u.vn, u.w, u.rho)
    assert abs(mass(out) - mass(u.psi)) <= 1e-13 * mass(u.psi)


def test_boundary_factor_of_the_vertical_flux():
    """pivbz = 1 copies the nearest interior interface flux to the top and
    bottom (Listing 7): a uniform column in a uniform vertical wind then
    stays uniform.  With pivbz = 0 the ends are closed: an upward wind
    empties the bottom level and fills the top one."""
    m = octa.build(3)
    nz = 6
    psi = np.full((m.n_nodes, nz), 2.0)
    w = np.full((m.n_nodes, nz), 0.25)
    vn = np.zeros((m.n_edges, nz))
    rho = np.ones((m.n_nodes, nz))
    args = (m.edges, m.node_ptr, m.node_edges, m.node_sign, m.dual_volume)
    open_ = oracle.ustep(*args, psi, vn, w, rho, pivbz=1.0)
    assert np.all(open_ == 2.0)
    closed = oracle.ustep(*args, psi, vn, w, rho, pivbz=0.0)
    assert np.all(closed[:, 0] < 2.0) and np.all(closed[:, -1] > 2.0)
    assert np.all(closed[:, 1:-1] == 2.0)


def test_positivity_below_unit_outflow_courant():
    """The upwind step keeps psi >= 0 while each node's outflow Courant sum
    stays below 1."""
    u = octa.random_uproblem(6, 5, seed=5, courant=0.4)
    m = u.mesh
    out = oracle.urun(5, m.edges, m.node_ptr, m.node_edges, m.node_sign, m.dual_volume, u.psi, u.vn, u.w, u.rho)
    assert out.min() >= 0.0


def test_rejects_bad_connectivity():
    m = octa.build(2)
    nz = 2
    f = np.ones((m.n_nodes, nz))
    bad = m.edges.copy()
    bad[0, 0] = m.n_nodes
    with pytest.raises(ValueError):
        oracle.ustep(bad, m.node_ptr, m.node_edges, m.node_sign, m.dual_volume, f, np.zeros((m.n_edges, nz)), f, f)


def test_hilbert_index_walks_the_grid():
    """The Hilbert numbering's curve: on a 2^k x 2^k grid it visits every
    point once, and consecutive points are grid neighbours (a wrong rotation
    or reflection of a quadrant breaks the second property)."""
    for k in (1, 2, 3, 4, 6):
        n = 1 << k
        x, y = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        d = octa.hilbert_index(x.ravel(), y.ravel(), k)
        assert np.array_equal(np.sort(d), np.arange(n * n))
        order = np.argsort(d)
        steps = np.abs(np.diff(x.ravel()[order])) + np.abs(np.diff(y.ravel()[order]))
        assert np.all(steps == 1), k


@pytest.mark.parametrize("numbering", ["random", "hilbert"])
def test_renumbered_mesh_gives_the_same_step_any_numbering(numbering):
    """The same octahedral mesh numbered at random or along a Hilbert curve:
    the step gives every node the same value up to the order of its edge sum."""
    u = octa.random_uproblem(6, 5, seed=3, pivbz=0.5)
    r = octa.renumbered_workload(u, 11, numbering=numbering)
    perms = octa.hilbert_order(u.mesh) if numbering == "hilbert" else None
    _, (node_perm, edge_perm) = octa.renumbered(u.mesh, 11, perms)
    assert sorted(node_perm) == list(range(u.mesh.n_nodes)) and sorted(edge_perm) == list(range(u.mesh.n_edges))
    m, mr = u.mesh, r.mesh
    a = oracle.ustep(m.edges, m.node_ptr, m.node_edges, m.node_sign, m.dual_volume, u.psi, u.vn, u.w, u.rho, u.pivbz)
    b = oracle.ustep(mr.edges, mr.node_ptr, mr.node_edges, mr.node_sign, mr.dual_volume, r.psi, r.vn, r.w, r.rho,
                     r.pivbz)
    assert np.max(np.abs(b - a[node_perm])) <= 1e-15 * np.max(np.abs(a))


def test_renumbered_mesh_gives_the_same_step():
    """The same octahedral mesh with nodes and edges numbered at random (the
    unstructured numbering the benchmark compares with the row-by-row one):
    the step gives every node the same value up to the order of its edge
    sum (the oracle sums a node's edges in table order)."""
    u = octa.random_uproblem(6, 5, seed=3, pivbz=0.5)
    r = octa.renumbered_workload(u, 11)
    _, (node_perm, edge_perm) = octa.renumbered(u.mesh, 11)
    assert sorted(node_perm) == list(range(u.mesh.n_nodes)) and sorted(edge_perm) == list(range(u.mesh.n_edges))
    m, mr = u.mesh, r.mesh
    a = oracle.ustep(m.edges, m.node_ptr, m.node_edges, m.node_sign, m.dual_volume, u.psi, u.vn, u.w, u.rho, u.pivbz)
    b = oracle.ustep(mr.edges, mr.node_ptr, mr.node_edges, mr.node_sign, mr.dual_volume, r.psi, r.vn, r.w, r.rho,
                     r.pivbz)
    assert np.max(np.abs(b - a[node_perm])) <= 1e-15 * np.max(np.abs(a))
