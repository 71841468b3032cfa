"""Octahedral reduced grid and its edge-based median dual, generated from the
grid's definition (the inputs of the unstructured MPDATA step).

Grid: 2N latitude rows; row i = 1..N from the north pole has 16 + 4i nodes
(the octahedral "O" rule: 20 nodes next to the pole, 4 more per row, one
more per octant), mirrored in the south.  Latitudes are equally spaced
(a stand-in for Gaussian latitudes); longitudes are 2 pi j / n_i.

Faces: between two rows the nodes are zipped by longitude into triangles;
between the two equator rows (equal counts) the faces are quadrilaterals;
each pole is closed by one polygon of the first row's 20 nodes (no pole
node).  Edges are the faces' sides.  Edge e runs from node ip1 to ip2; its
left face is the face that lists ip1 -> ip2 counter-clockwise seen from
outside the sphere.

Dual: node n's volume is the sum over its faces of (face area) / (face's
node count).  The normal advective flux through edge e's dual face is a
difference of a streamfunction between the edge's two faces,
Vn(e) = Psi(left) - Psi(right), so that at every node the signed sum of its
edges' fluxes telescopes to zero exactly (the Psi samples are rounded to
multiples of 2^-20, which keeps every difference and sum exact).

Layouts: every per-node field is (nodes, levels), every per-edge field
(edges, levels), level fastest.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

QUANTUM = 2.0 ** -20


@dataclass
class OctaMesh:
    N: int
    lat: np.ndarray            # (nodes,) radians
    lon: np.ndarray            # (nodes,)
    row_start: np.ndarray      # (2N + 1,) first node of each row
    edges: np.ndarray          # (edges, 2) int32: ip1, ip2
    edge_faces: np.ndarray     # (edges, 2) int64: left, right face
    faces: list                # node lists, counter-clockwise seen from outside
    face_area: np.ndarray      # (faces,)
    face_centroid: np.ndarray  # (faces, 3) unit vectors
    node_ptr: np.ndarray       # (nodes + 1,) int32 CSR offsets into node_edges
    node_edges: np.ndarray     # (2 * edges,) int32 edge ids, ascending per node
    node_sign: np.ndarray      # (2 * edges,) int8: +1 if the node is the edge's ip1, else -1
    dual_volume: np.ndarray    # (nodes,)

    @property
    def n_nodes(self) -> int:
        return len(self.lat)

    @property
    def n_edges(self) -> int:
        return len(self.edges)


def row_counts(N: int) -> list:
    north = [16 + 4 * i for i in range(1, N + 1)]
    return north + north[::-1]


def _xyz(lat, lon):
    c = np.cos(lat)
    return np.stack([c * np.cos(lon), c * np.sin(lon), np.sin(lat)], axis=-1)


def _zip_rows(a0, na, b0, nb, lon):
    """Faces between row A (nodes a0..a0+na-1, the northern one) and row B.
    Counter-clockwise seen from outside: going east along A, then back along B."""
    faces = []
    if na == nb:
        for j in range(na):
            a, a1 = a0 + j, a0 + (j + 1) % na
            b, b1 = b0 + j, b0 + (j + 1) % nb
            faces.append([a, b, b1, a1])
        return faces
    # merge the two rows by longitude (both start at longitude 0)
    ia = ib = 0
    while ia < na or ib < nb:
        la = 2 * np.pi * (ia + 1) / na     # longitude of A's next node
        lb = 2 * np.pi * (ib + 1) / nb
        a, b = a0 + ia % na, b0 + ib % nb
        if ib >= nb or (ia < na and la <= lb):
            faces.append([a, b, a0 + (ia + 1) % na])          # advance along A
            ia += 1
        else:
            faces.append([a, b, b0 + (ib + 1) % nb])          # advance along B
            ib += 1
    return faces


def _orient_and_measure(faces, xyz):
    """Faces re-ordered counter-clockwise seen from outside (normal pointing
    away from the centre), their flat areas (fan from the node centroid) and
    unit centroids; vectorised over faces of equal size."""
    out = list(faces)
    area = np.empty(len(faces))
    cen = np.empty((len(faces), 3))
    sizes = np.array([len(f) for f in faces])
    for n in np.unique(sizes):
        idx = np.nonzero(sizes == n)[0]
        nodes = np.array([faces[i] for i in idx])                  # (m, n)
        p = xyz[nodes]                                             # (m, n, 3)
        c = p.mean(axis=1, keepdims=True)
        d = p - c
        cr = np.cross(d, np.roll(d, -1, axis=1))                   # (m, n, 3)
        normal = cr.sum(axis=1)
        flip = np.einsum("ij,ij->i", normal, c[:, 0, :]) < 0
        area[idx] = 0.5 * np.linalg.norm(cr, axis=2).sum(axis=1)
        cen[idx] = c[:, 0, :]
        for r, i in enumerate(idx):
            out[i] = list(nodes[r][::-1]) if flip[r] else list(nodes[r])
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    return out, area, cen


def build(N: int) -> OctaMesh:
    counts = row_counts(N)
    nrows = 2 * N
    row_start = np.zeros(nrows + 1, dtype=np.int64)
    row_start[1:] = np.cumsum(counts)
    lat = np.empty(row_start[-1])
    lon = np.empty(row_start[-1])
    for r in range(nrows):
        n = counts[r]
        lat[row_start[r]:row_start[r + 1]] = np.pi / 2 - (r + 0.5) * np.pi / nrows
        lon[row_start[r]:row_start[r + 1]] = 2 * np.pi * np.arange(n) / n
    xyz = _xyz(lat, lon)

    faces = [list(range(row_start[0], row_start[1]))]                      # north cap
    for r in range(nrows - 1):
        faces += _zip_rows(row_start[r], counts[r], row_start[r + 1], counts[r + 1], lon)
    faces.append(list(range(row_start[nrows - 1], row_start[nrows])))      # south cap
    faces, area, centroid = _orient_and_measure(faces, xyz)

    edge_id = {}
    edges, edge_faces = [], []
    for fi, f in enumerate(faces):
        for q in range(len(f)):
            u, v = int(f[q]), int(f[(q + 1) % len(f)])
            key = (min(u, v), max(u, v))
            if key not in edge_id:
                edge_id[key] = len(edges)
                edges.append(key)                  # ip1 < ip2
                edge_faces.append([-1, -1])
            e = edge_id[key]
            # the face lists u -> v counter-clockwise: it is the left face of
            # the edge oriented u -> v
            edge_faces[e][0 if u == edges[e][0] else 1] = fi
    edges = np.array(edges, dtype=np.int32)
    edge_faces = np.array(edge_faces, dtype=np.int64)
    assert (edge_faces >= 0).all(), "every edge has two faces on a closed sphere"

    vol = np.zeros(len(lat))
    for fi, f in enumerate(faces):
        vol[f] += area[fi] / len(f)

    nn = len(lat)
    inc = [[] for _ in range(nn)]
    for e, (a, b) in enumerate(edges):
        inc[a].append((e, 1))
        inc[b].append((e, -1))
    node_ptr = np.zeros(nn + 1, dtype=np.int32)
    node_ptr[1:] = np.cumsum([len(x) for x in inc])
    node_edges = np.array([e for x in inc for e, _ in sorted(x)], dtype=np.int32)
    node_sign = np.array([s for x in inc for _, s in sorted(x)], dtype=np.int8)
    return OctaMesh(N, lat, lon, row_start, edges, edge_faces, faces, area, centroid, node_ptr, node_edges,
                    node_sign, vol)


def streamfunction_flux(mesh: OctaMesh, nz: int, max_courant: float, alpha: float = 0.05,
                        level_factor=None) -> np.ndarray:
    """Vn (edges, levels): solid-body rotation about an axis tilted by alpha,
    Psi = -(sin(lat) cos(alpha) - cos(lon) cos(lat) sin(alpha)) at the face
    centroids, scaled so that max over nodes of (outflow sum / volume) equals
    max_courant (times level_factor[k] <= 1 on level k, default 1), rounded to
    multiples of 2^-20 before differencing."""
    c = mesh.face_centroid
    lat = np.arcsin(np.clip(c[:, 2], -1, 1))
    lon = np.arctan2(c[:, 1], c[:, 0])
    psi = -(np.sin(lat) * np.cos(alpha) - np.cos(lon) * np.cos(lat) * np.sin(alpha))
    raw = psi[mesh.edge_faces[:, 0]] - psi[mesh.edge_faces[:, 1]]
    out = np.zeros(mesh.n_nodes)
    np.add.at(out, mesh.edges[:, 0], np.maximum(raw, 0))
    np.add.at(out, mesh.edges[:, 1], np.maximum(-raw, 0))
    scale = max_courant / np.max(out / mesh.dual_volume)
    fac = np.ones(nz) if level_factor is None else np.asarray(level_factor, dtype=np.float64)
    q = np.round(psi[:, None] * (scale * fac)[None, :] / QUANTUM) * QUANTUM      # (faces, nz)
    vn = q[mesh.edge_faces[:, 0]] - q[mesh.edge_faces[:, 1]]
    return np.ascontiguousarray(vn)


@dataclass
class UWorkload:
    name: str
    mesh: OctaMesh
    nz: int
    psi: np.ndarray    # (nodes, nz)
    vn: np.ndarray     # (edges, nz)
    w: np.ndarray      # (nodes, nz): w[n, k] at the interface between levels k-1 and k (k >= 1)
    rho: np.ndarray    # (nodes, nz)
    pivbz: float

    @property
    def points(self) -> int:
        return self.mesh.n_nodes * self.nz


def octahedral_workload(N: int = 128, nz: int = 80, seed: int = 6, max_courant: float = 0.5) -> UWorkload:
    """The paper's MPDATA upwind benchmark shape (an octahedral grid of about
    70 000 nodes, 80 levels): solid-body winds, no vertical wind, unit
    density, a cosine bell plus U[0, 0.1) noise per point."""
    mesh = build(N)
    rng = np.random.default_rng(seed)
    vn = streamfunction_flux(mesh, nz, max_courant)
    lat, lon = mesh.lat, mesh.lon
    r = np.arccos(np.clip(np.cos(lat) * np.cos(lon - 1.5 * np.pi), -1, 1))   # distance from (3pi/2, 0)
    bell = np.where(r < 1.0 / 3.0, 0.5 * (1 + np.cos(np.pi * r * 3.0)), 0.0)
    psi = np.repeat(bell[:, None], nz, axis=1) + rng.uniform(0, 0.1, size=(mesh.n_nodes, nz))
    return UWorkload(f"octahedral-O{N}-{nz}", mesh, nz, np.ascontiguousarray(psi), vn,
                     np.zeros((mesh.n_nodes, nz)), np.ones((mesh.n_nodes, nz)), 0.0)


def random_uproblem(N: int, nz: int, seed: int, courant: float = 0.4, pivbz: float = 0.0) -> UWorkload:
    """Small random problem for parity tests: random vertical winds and density too."""
    mesh = build(N)
    rng = np.random.default_rng(seed)
    vn = streamfunction_flux(mesh, nz, courant, level_factor=rng.uniform(0.5, 1.0, size=nz))
    w = rng.uniform(-0.2, 0.2, size=(mesh.n_nodes, nz))
    rho = rng.uniform(0.8, 1.2, size=(mesh.n_nodes, nz))
    psi = rng.uniform(0.0, 1.0, size=(mesh.n_nodes, nz))
    return UWorkload(f"random-O{N}-{nz}", mesh, nz, psi, vn, w, rho, pivbz)


def hilbert_index(x: np.ndarray, y: np.ndarray, order: int) -> np.ndarray:
    """Position along the Hilbert curve of the 2^order x 2^order grid of each
    integer point (x, y) (the curve's recursive definition: at each scale the
    quadrant index, with the sub-square rotated or reflected so that the
    curve's pieces join end to end)."""
    x = np.asarray(x, dtype=np.int64).copy()
    y = np.asarray(y, dtype=np.int64).copy()
    d = np.zeros_like(x)
    s = 1 << (order - 1)
    while s > 0:
        rx = (x & s) > 0
        ry = (y & s) > 0
        d += s * s * ((3 * rx) ^ ry)
        # rotate the quadrant so that the curve inside it starts and ends where it must
        flip = ~ry
        swap_x = flip & rx
        x = np.where(swap_x, s - 1 - x, x)
        y = np.where(swap_x, s - 1 - y, y)
        x, y = np.where(flip, y, x), np.where(flip, x, y)
        s >>= 1
    return d


def hilbert_order(mesh: OctaMesh, order: int = 10):
    """Node and edge orders along a Hilbert curve over (longitude, latitude)
    mapped to a 2^order square: the paper's third numbering of its indexing
    study, a space-filling curve.  Returns (node_perm, edge_perm) in the
    convention of `renumbered`; edges follow the curve position of their
    midpoint (the mean of their end nodes' curve coordinates)."""
    n = 1 << order
    gx = np.minimum((mesh.lon / (2 * np.pi) * n).astype(np.int64), n - 1)
    gy = np.minimum(((mesh.lat + np.pi / 2) / np.pi * n).astype(np.int64), n - 1)
    node_perm = np.argsort(hilbert_index(gx, gy, order), kind="stable")
    a, b = mesh.edges[:, 0].astype(np.int64), mesh.edges[:, 1].astype(np.int64)
    edge_perm = np.argsort(hilbert_index((gx[a] + gx[b]) // 2, (gy[a] + gy[b]) // 2, order), kind="stable")
    return node_perm, edge_perm


def renumbered(mesh: OctaMesh, seed: int, perms=None):
    """The same mesh with its nodes and edges numbered in a random order (an
    unstructured numbering, against the row-by-row one of `build`), or in the
    given order perms = (node_perm, edge_perm).  Returns the new mesh and
    (node_perm, edge_perm): new node i is old node node_perm[i], new edge e is
    old edge edge_perm[e].  Each edge keeps its orientation (ip1 -> ip2), so
    fluxes and their signs carry over; a node's edges are listed in ascending
    new edge number."""
    nn, ne = mesh.n_nodes, mesh.n_edges
    if perms is None:
        rng = np.random.default_rng(seed)
        node_perm = rng.permutation(nn)
        edge_perm = rng.permutation(ne)
    else:
        node_perm, edge_perm = (np.asarray(p, dtype=np.int64) for p in perms)
    new_of_node = np.empty(nn, dtype=np.int64)
    new_of_node[node_perm] = np.arange(nn)
    edges = new_of_node[mesh.edges[edge_perm].astype(np.int64)].astype(np.int32)
    inc = [[] for _ in range(nn)]
    for e, (a, b) in enumerate(edges):
        inc[a].append((e, 1))
        inc[b].append((e, -1))
    node_ptr = np.zeros(nn + 1, dtype=np.int32)
    node_ptr[1:] = np.cumsum([len(x) for x in inc])
    node_edges = np.array([e for x in inc for e, _ in sorted(x)], dtype=np.int32)
    node_sign = np.array([s for x in inc for _, s in sorted(x)], dtype=np.int8)
    out = OctaMesh(mesh.N, mesh.lat[node_perm], mesh.lon[node_perm], mesh.row_start, edges,
                   mesh.edge_faces[edge_perm], mesh.faces, mesh.face_area, mesh.face_centroid, node_ptr,
                   node_edges, node_sign, mesh.dual_volume[node_perm])
    return out, (node_perm, edge_perm)


def renumbered_workload(u: UWorkload, seed: int = 7, numbering: str = "random") -> UWorkload:
    """Workload u on its mesh with nodes and edges numbered at random
    (numbering "random") or along a Hilbert curve ("hilbert"), fields
    permuted to match."""
    perms = hilbert_order(u.mesh) if numbering == "hilbert" else None
    mesh, (np_, ep) = renumbered(u.mesh, seed, perms)
    return UWorkload(u.name + "-" + numbering, mesh, u.nz, np.ascontiguousarray(u.psi[np_]),
                     np.ascontiguousarray(u.vn[ep]), np.ascontiguousarray(u.w[np_]),
                     np.ascontiguousarray(u.rho[np_]), u.pivbz)
