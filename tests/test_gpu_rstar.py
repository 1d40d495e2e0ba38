"""Entry search through the R*-tree (Section II-E) on the GPU, through the C
ABI: the same entry face as the boundary BVH for every ray (the exact entry
test admits one face per ray of a convex mesh), and the face's owner is the
first tetrahedron of the oracle's traversal."""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _workload(name):
    if name == "cfg0":
        return synth.config(0)
    if name == "cfg1":
        return synth.config(1)
    if name == "cfg2":
        return synth.config(2)
    if name == "delaunay":
        verts, tets = synth.delaunay_mesh(3000, 2)
        cone = synth.Cone(4.0, 8.0, 48, 40, 2.0 / 40, 2.0 / 40, 0.003, -0.002)
        return synth.Workload("delaunay3000", verts, tets, np.zeros(len(tets), np.float32), cone,
                              synth.angles_for(6))
    if name == "graded":
        (verts, tets), _, _ = synth.graded_mesh(24, 8, 1.05, 17)
        du = 2.0 ** -5
        cone = synth.Cone(4.0, 8.0, 64, 64, du, du, du / 2, du / 2)
        return synth.Workload("graded24", verts, tets, np.zeros(len(tets), np.float32), cone, synth.angles_for(12))
    if name == "ragged":
        w = synth.jittered_kuhn(5, 7, 8, 37, 29, 5)
        w.cone = synth.Cone(4.0, 8.0, 37, 29, 0.08, 0.09, 0.013, -0.021)  # wider than the mesh shadow
        return w
    raise KeyError(name)


def _entries(w):
    import paper_1908_06909_amd as tct

    mesh = tct.TetMesh(w.verts, w.tets, device=DEV, rstar=True)
    geom = tct.ConeGeometry(w.cone, w.angles, device=DEV)
    P = tct.Projector(mesh, geom, cache_entry=False)
    eb = P.compute_entry(method="bvh")
    er = P.compute_entry(method="rstar")
    torch.cuda.synchronize()
    st = mesh.stats(reset=True, check=True)
    assert st["failed"] == 0
    return mesh, eb, er


@pytest.mark.parametrize("name", ["cfg0", "delaunay", "graded", "ragged"])
def test_rstar_entry_equals_bvh_and_oracle(name):
    w = _workload(name)
    mesh, eb, er = _entries(w)
    print(f"{name}: {int((er >= 0).sum())} of {er.numel()} rays enter; R*-tree height {mesh.rstar()['height']}")
    assert torch.equal(eb, er)
    # Pin to the oracle: the owner of the entry face is the first tetrahedron
    # the oracle's ray visits (misses: no visit), on a sample of rays.
    orc = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    _, owner = mesh.boundary()
    n = er.numel()
    ids = np.unique(np.concatenate([np.arange(0, n, max(1, n // 3000)), np.arange(n - 64, n)]))
    e = er.cpu().numpy()[ids]
    for rid, ent, (tt, _) in zip(ids, e, orc.trace(ids)):
        if ent < 0:
            assert len(tt) == 0, rid
        else:
            assert len(tt) > 0 and owner[ent] == tt[0], rid
    if name == "ragged":
        assert (e < 0).any() and (e >= 0).any()


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_rstar_entry_full_size(name):
    """Every ray of the benchmark-size geometries, in the launch the entry
    pass uses."""
    mesh, eb, er = _entries(_workload(name))
    assert torch.equal(eb, er)
    assert int((er >= 0).sum()) > 0
