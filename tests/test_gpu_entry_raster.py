"""Entry faces by projecting the boundary onto the detector (tct_entry_raster)
against the boundary-BVH search, through the C ABI: the exact entry test
admits one face per ray of a convex mesh, so the two arrays must be equal
element for element, misses included.  The BVH search itself is pinned to
the oracle's first visited tetrahedron in the R*-tree and parity tests."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _workload(name):
    if name in ("cfg0", "cfg1", "cfg2"):
        return synth.config(int(name[-1]))
    if name == "delaunay":
        verts, tets = synth.delaunay_mesh(3000, 2)
        cone = synth.Cone(4.0, 8.0, 48, 40, 2.0 / 40, 2.0 / 40, 0.003, -0.002)
        return synth.Workload("delaunay3000", verts, tets, np.zeros(len(tets), np.float32), cone,
                              synth.angles_for(6))
    if name == "delaunay_near":
        # Source close to the hull: wide fan of rays, faces seen at steep angles.
        verts, tets = synth.delaunay_mesh(2000, 5)
        cone = synth.Cone(1.1, 2.6, 61, 53, 4.0 / 53, 4.0 / 53, 0.011, 0.007)
        return synth.Workload("delaunay2000_near", verts, tets, np.zeros(len(tets), np.float32), cone,
                              synth.angles_for(7))
    if name == "graded":
        (verts, tets), _, _ = synth.graded_mesh(24, 8, 1.05, 17)
        du = 2.0 ** -5
        cone = synth.Cone(4.0, 8.0, 64, 64, du, du, du / 2, du / 2)
        return synth.Workload("graded24", verts, tets, np.zeros(len(tets), np.float32), cone, synth.angles_for(12))
    if name == "ties":
        # Pixel centres on projected vertices and edges: perturbation decides.
        return synth.plain_kuhn(4, 3, 33, 33, 8, pitch=2.0 ** -4)
    if name == "ragged":
        w = synth.jittered_kuhn(5, 7, 8, 37, 29, 5)
        w.cone = synth.Cone(4.0, 8.0, 37, 29, 0.08, 0.09, 0.013, -0.021)  # wider than the mesh shadow
        return w
    if name == "coplanar":
        # The source lies (to float rounding) in the planes of whole sides of
        # the cube: rays meet those faces edge-on, the projections of the
        # faces collapse to segments, and the perturbed signs decide.
        w = synth.plain_kuhn(8, 4, 64, 64, 4, pitch=2.0 ** -5)
        th = float(np.arcsin(0.5 / 4.0))
        w.angles = np.array([th, np.pi - th, np.pi + th, 0.5 * np.pi - th])
        return w
    if name == "one_pixel":
        w = synth.jittered_kuhn(3, 2, 3, 1, 1, 3)
        w.cone = synth.Cone(4.0, 8.0, 1, 1, 0.05, 0.05, 0.01, 0.02)
        return w
    raise KeyError(name)


def _compare(name):
    import paper_1908_06909_amd as tct

    w = _workload(name)
    mesh = tct.TetMesh(w.verts, w.tets, device=DEV)
    geom = tct.ConeGeometry(w.cone, w.angles, device=DEV)
    P = tct.Projector(mesh, geom, cache_entry=False)
    eb = P.compute_entry(method="bvh")
    er = torch.full_like(eb, 12345)  # every element must be overwritten
    P.compute_entry(er, method="raster")
    torch.cuda.synchronize()
    st = mesh.stats(reset=True, check=True)
    assert st["failed"] == 0
    hits = int((eb >= 0).sum())
    print(f"{name}: {hits} of {eb.numel()} rays enter", flush=True)
    assert torch.equal(eb, er), f"{int((eb != er).sum())} rays differ"
    return hits, eb.numel()


@pytest.mark.parametrize("name", ["cfg0", "delaunay", "delaunay_near", "graded", "ties", "ragged", "one_pixel",
                                  "coplanar"])
def test_raster_entry_equals_bvh(name):
    hits, n = _compare(name)
    assert hits > 0
    if name == "ragged":
        assert hits < n


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_raster_entry_equals_bvh_full_size(name):
    hits, _ = _compare(name)
    assert hits > 0


def test_coplanar_source_entry_and_forward_match_oracle():
    """Source in the planes of boundary faces: the entry face's owner is the
    oracle's first tetrahedron on every ray, and the forward projection
    through the boundary-projection entry cache matches the oracle's."""
    import oracle
    import paper_1908_06909_amd as tct

    w = _workload("coplanar")
    mesh = tct.TetMesh(w.verts, w.tets, device=DEV)
    geom = tct.ConeGeometry(w.cone, w.angles, device=DEV)
    P = tct.Projector(mesh, geom)  # entry cache by boundary projection
    x = mesh.to_internal(torch.as_tensor(w.x, device=DEV))
    got = P.forward(x).reshape(-1).cpu().numpy().astype(np.float64)
    e = P.entry.cpu().numpy()
    torch.cuda.synchronize()
    st = mesh.stats(reset=True, check=True)
    assert st["failed"] == 0
    orc = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    ids = np.arange(orc.nrays)
    _, owner = mesh.boundary()
    trace = orc.trace(ids)
    for rid, (tt, _) in enumerate(trace):
        if e[rid] < 0:
            assert len(tt) == 0, rid
        else:
            assert len(tt) > 0 and owner[e[rid]] == tt[0], rid
    from parity_bars import element_size, forward_reference

    ref, tol = forward_reference(orc, w.x, element_size(w.verts, w.tets, orc.mesh.tables()[1]), ids)
    err = np.abs(got - ref)
    print(f"coplanar: {int((e >= 0).sum())} rays enter; {st['perturbed_ties']} perturbed ties; "
          f"worst err/tol {float(np.max(err / np.maximum(tol, 1e-300))):.3f}")
    assert (err <= tol + 1e-30).all()
