"""The unstructured (edge-based) donor-cell step on the GPU against the
oracle (bit for bit: the kernel evaluates the stages' formulas in their
order without contraction), on octahedral meshes with random vertical
winds, densities and both vertical boundary factors."""
import numpy as np
import pytest

import oracle
from workloads import octahedral as octa

pytestmark = pytest.mark.gpu


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("N,nz,pivbz,steps,with_w", [(3, 1, 0.0, 1, True), (4, 7, 0.0, 3, True),
                                                       (6, 80, 1.0, 2, True), (5, 13, 0.5, 4, False),
                                                       (8, 3, 0.0, 5, True)])
@pytest.mark.parametrize("renumber", [None, "random", "hilbert"])
@pytest.mark.parametrize("mapping", ["grouped", "wave"])
def test_ustep_matches_oracle(N, nz, pivbz, steps, with_w, renumber, mapping, monkeypatch):
    """Both kernel mappings (four nodes per wave, and one wave per node),
    on the row-by-row numbered mesh and on a random and a Hilbert-curve
    renumbering of it: bitwise equal to the oracle on the same mesh."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    if mapping == "wave":
        monkeypatch.setenv("MPDATA_USTEP", "wave")
    else:
        monkeypatch.delenv("MPDATA_USTEP", raising=False)
    _say(f"[unstructured] O{N} nz={nz} pivbz={pivbz} steps={steps} w={with_w} renumbered={renumber} {mapping}")
    u = octa.random_uproblem(N, nz, seed=N * 100 + nz, pivbz=pivbz)
    if renumber:
        u = octa.renumbered_workload(u, seed=N, numbering=renumber)
    m = u.mesh
    w = u.w if with_w else np.zeros_like(u.w)
    want = oracle.urun(steps, m.edges, m.node_ptr, m.node_edges, m.node_sign, m.dual_volume, u.psi, u.vn, w,
                       u.rho, pivbz)
    dm = mp.DeviceMesh.from_octa(m, nz, pivbz=pivbz)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    psi = dev(u.psi)
    mp.urun(dm, psi, dev(u.vn), dev(w) if with_w else None, dev(u.rho), steps)
    torch.cuda.synchronize()
    assert np.array_equal(psi.cpu().numpy(), want)


def test_ustep_fp32_close_to_oracle():
    torch = _torch()
    import paper_1908_06094_amd as mp

    _say("[unstructured] O6 nz=9 FP32")
    u = octa.random_uproblem(6, 9, seed=66)
    m = u.mesh
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    psi, vn, w, rho = (f32(a) for a in (u.psi, u.vn, u.w, u.rho))
    vol = f32(m.dual_volume)
    want = oracle.urun(3, m.edges, m.node_ptr, m.node_edges, m.node_sign, vol, psi, vn, w, rho)
    dm = mp.DeviceMesh(m.edges, m.node_ptr, m.node_edges, m.node_sign, vol, 9, dtype="f32")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")
    x = dev(psi)
    mp.urun(dm, x, dev(vn), dev(w), dev(rho), 3)
    torch.cuda.synchronize()
    got = x.double().cpu().numpy()
    assert np.max(np.abs(got - want)) <= 3e-6 * np.max(np.abs(want))


def test_ustep_rejects_bad_calls():
    torch = _torch()
    import paper_1908_06094_amd as mp

    m = octa.build(2)
    dm = mp.DeviceMesh.from_octa(m, 4)
    f = torch.ones(m.n_nodes, 4, dtype=torch.float64, device="cuda")
    vn = torch.zeros(m.n_edges, 4, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        mp.ustep(dm, f, vn, None, f.float())                       # wrong dtype
    with pytest.raises(mp.MpdataError):
        mp.ustep(dm, f, vn, None, f, out=f)                        # aliasing
    bad = m.edges.copy()
    bad[3, 1] = m.n_nodes + 5
    with pytest.raises(ValueError):
        mp.DeviceMesh(bad, m.node_ptr, m.node_edges, m.node_sign, m.dual_volume, 4)


def test_benchmark_mesh_full_size():
    """The benchmark workload itself (O128: 70 144 nodes, 209 864 edges,
    80 levels), 2 steps, bit for bit against the oracle."""
    torch = _torch()
    import paper_1908_06094_amd as mp

    u = octa.octahedral_workload(128, 80)
    m = u.mesh
    _say(f"[unstructured] {u.name} full size, 2 steps")
    want = oracle.urun(2, m.edges, m.node_ptr, m.node_edges, m.node_sign, m.dual_volume, u.psi, u.vn, u.w, u.rho,
                       u.pivbz)
    dm = mp.DeviceMesh.from_octa(m, u.nz, pivbz=u.pivbz)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    psi = dev(u.psi)
    mp.urun(dm, psi, dev(u.vn), dev(u.w), dev(u.rho), 2)
    torch.cuda.synchronize()
    assert np.array_equal(psi.cpu().numpy(), want)
