"""The paper's own propagation (Moller-Trumbore with eps escalation,
Algorithms 1-2) on the GPU against the oracle's implementation of the same
algorithms: identical counts (rays, steps, eps escalations, halted and
looping rays) and identical float32 projections, in float32 and float64
arithmetic, on the uniform Kuhn mesh and on a graded sliver mesh with rays
through vertices and along edges.  Also checks that it diverges from the
exact walk where the paper says it does (float32 on slivers) and agrees
with it on the rays where it neither escalates nor loops."""

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(name):
    import paper_1908_06909_amd as tct

    if name == "kuhn8":
        w = synth.config(0)
        verts, tets, x, cone, angles = w.verts, w.tets, w.x, w.cone, w.angles
    elif name == "delaunay":
        verts, tets = synth.delaunay_mesh(3000, 2)
        x = synth.uniform_random(len(tets), 8)
        cone = synth.Cone(4.0, 8.0, 48, 40, 2.0 / 40, 2.0 / 40, 0.003, -0.002)
        angles = synth.angles_for(6)
    else:
        (verts, tets), X, Z = synth.graded_mesh(24, 8, 1.05, 17)
        x = synth.sphere_phantom(verts, tets, 12)
        du = 2.0 ** -5
        cone = synth.Cone(4.0, 8.0, 64, 64, du, du, du / 2, du / 2)
        angles = synth.angles_for(12)
    orc = oracle.Oracle(verts, tets, cone, angles)
    mesh = tct.TetMesh(verts, tets, device=DEV)
    geom = tct.ConeGeometry(cone, angles, device=DEV)
    P = tct.Projector(mesh, geom)
    xi = mesh.to_internal(torch.as_tensor(np.ascontiguousarray(x, np.float32), device=DEV))
    return orc, P, x, xi


@pytest.mark.parametrize("name", ["kuhn8", "graded24", "delaunay"])
@pytest.mark.parametrize("precision", [32, 64])
def test_paper_mode_matches_oracle(name, precision):
    orc, P, x, xi = _case(name)
    got, st = P.forward_paper(xi, precision)
    ref, st_ref = orc.forward_paper(x, precision)
    print(name, precision, st, st_ref)
    assert st == st_ref
    g = got.cpu().numpy().ravel().astype(np.float64)
    diff = np.flatnonzero(g != ref)
    assert len(diff) == 0, (len(diff), diff[:5], g[diff[:5]], ref[diff[:5]])


def test_paper_mode_float32_fails_on_slivers_and_float64_agrees_elsewhere():
    orc, P, x, xi = _case("graded24")
    exact = P.forward(xi).cpu().numpy().ravel().astype(np.float64)
    b32, s32 = P.forward_paper(xi, 32)
    b64, s64 = P.forward_paper(xi, 64)
    b32 = b32.cpu().numpy().ravel()
    b64 = b64.cpu().numpy().ravel()
    tol = 1e-5 * np.maximum(np.abs(exact), 1e-3)
    bad32 = int((np.abs(b32 - exact) > tol).sum())
    bad64 = int((np.abs(b64 - exact) > tol).sum())
    print("float32", s32, "bad", bad32, "float64", s64, "bad", bad64)
    assert s32["escalations"] > 100 * max(1, s64["escalations"])
    assert bad32 > 10 * max(1, bad64)
