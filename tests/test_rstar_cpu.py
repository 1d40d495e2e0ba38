"""The R*-tree over the boundary faces (Section II-E: the paper's entry-search
structure, 4 to 10 entries per node) and the boundary-face export, checked on
the host: the exported faces are the oracle's outward boundary, and the tree
is a valid, balanced R*-tree that covers every face exactly once."""

import numpy as np
import pytest

import oracle
import synth
from paper_1908_06909_amd import TetMesh, _lib

M_MAX, M_MIN = 10, 4


def _meshes():
    X = synth.kuhn_nodes(8)
    yield "kuhn8", synth.kuhn_mesh(X, X, X)
    yield "delaunay2000", synth.delaunay_mesh(2000, 5)
    w = synth.config(0)
    yield "cfg0", (w.verts, w.tets)
    Xg = synth.graded_nodes(12, 1.3, 5)
    yield "graded12", synth.kuhn_mesh(Xg, Xg, synth.kuhn_nodes(4))


@pytest.mark.parametrize("name,mesh", list(_meshes()))
def test_boundary_export_is_the_outward_hull(name, mesh):
    verts, tets = mesh
    m = TetMesh(verts, tets, host_only=True)
    xyz, owner = m.boundary()
    om = oracle.OracleMesh(verts, tets)
    _, _, B, O = om.tables()
    assert len(xyz) == len(B) == m.nboundary
    # Same faces (as sets of vertex coordinates) with the same owners.
    def key(tri):
        return tuple(sorted(tuple(float(c) for c in p) for p in tri))
    ours = sorted((key(xyz[b]), int(owner[b])) for b in range(len(xyz)))
    theirs = sorted((key(verts[B[b]]), int(O[b, 0])) for b in range(len(B)))
    assert ours == theirs
    # Outward orientation: the owner's fourth vertex is strictly behind the face.
    V = np.asarray(verts, np.float64)
    T = np.asarray(tets)
    for b in range(len(xyz)):
        p = xyz[b].astype(np.float64)
        n = np.cross(p[1] - p[0], p[2] - p[0])
        t = T[owner[b]]
        fourth = [v for v in t if not any(np.array_equal(V[v], q) for q in p)]
        assert len(fourth) == 1
        assert np.dot(n, V[fourth[0]] - p[0]) < 0


def _children(link, n, i):
    end = link[i, 0] if link[i, 0] >= 0 else n
    out, j = [], i + 1
    while j < end:
        out.append(j)
        j = link[j, 0] if link[j, 0] >= 0 else n
    return out


@pytest.mark.parametrize("name,mesh", list(_meshes()))
def test_rstar_is_balanced_and_covers_each_face_once(name, mesh):
    verts, tets = mesh
    m = TetMesh(verts, tets, host_only=True, rstar=True)
    R = m.rstar()
    xyz, _ = m.boundary()
    box, link, lst, height = R["box"], R["link"], R["list"], R["height"]
    n = len(box)
    seen = np.zeros(m.nboundary, np.int64)
    leaf_depths = set()

    def visit(i, depth):
        if link[i, 1] >= 0:
            first, cnt = link[i, 1] >> 4, link[i, 1] & 15
            faces = lst[first:first + cnt]
            assert 1 <= cnt <= M_MAX
            if i != 0:
                assert cnt >= M_MIN
            seen[faces] += 1
            leaf_depths.add(depth)
            for f in faces:  # every face inside its leaf's box
                assert np.all(xyz[f].min(0) >= box[i, :3]) and np.all(xyz[f].max(0) <= box[i, 3:])
            return
        ch = _children(link, n, i)
        assert (len(ch) >= 2) if i == 0 else (M_MIN <= len(ch) <= M_MAX)
        for c in ch:  # child boxes nested in the parent's
            assert np.all(box[c, :3] >= box[i, :3]) and np.all(box[c, 3:] <= box[i, 3:])
            visit(c, depth + 1)

    visit(0, 0)
    assert np.all(seen == 1)
    assert leaf_depths == {height - 1}
    # Preorder with skip links: the root's subtree is the whole array.
    assert link[0, 0] == -1
    # Depth is logarithmic in the face count for these fill bounds.
    assert height <= 1 + int(np.ceil(np.log(max(m.nboundary, 2)) / np.log(M_MIN)))


def test_rstar_absent_unless_requested():
    X = synth.kuhn_nodes(2)
    verts, tets = synth.kuhn_mesh(X, X, X)
    m = TetMesh(verts, tets, host_only=True)
    with pytest.raises(_lib.TctError) as e:
        m.rstar()
    assert e.value.status == -1
