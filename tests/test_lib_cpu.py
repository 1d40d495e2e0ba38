"""Library checks that need no GPU: the C ABI loads and exports every symbol
declared in include/tetct.h, and host-side mesh creation (validation,
neighbours, boundary, convexity, reordering) agrees with the oracle."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_1908_06909_amd import TetMesh, _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "tetct.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tct_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = C.CDLL(_lib.LIB_PATH)
    declared = _declared_functions()
    assert len(declared) >= 19
    for name in declared:
        assert hasattr(L, name), f"{name} declared in tetct.h but not exported"
    assert set(declared) == set(_lib.exported_symbols())


def test_version_and_error_text():
    assert b"gfx950" in _lib.lib().tct_version()
    with pytest.raises(_lib.TctError) as e:
        TetMesh(np.zeros((3, 3), np.float32), np.zeros((0, 4), np.int32), host_only=True)
    assert e.value.status == -1


def _kuhn(n):
    X = synth.kuhn_nodes(n)
    return synth.kuhn_mesh(X, X, X)


@pytest.mark.parametrize("n", [1, 2, 5])
def test_host_ingest_matches_oracle(n):
    verts, tets = _kuhn(n)
    m = TetMesh(verts, tets, host_only=True)
    om = oracle.OracleMesh(verts, tets)
    assert m.nboundary == om.nboundary == 12 * n * n
    nb = m.neighbors()
    T, N, _, _ = om.tables()
    for t in range(len(tets)):
        assert set(nb[t]) == set(N[t])
        # neighbour k is across the face opposite the user's vertex k
        for k in range(4):
            if nb[t, k] >= 0:
                face = set(tets[t]) - {tets[t][k]}
                assert face <= set(tets[nb[t, k]])
    # the permutation is a bijection
    assert sorted(m.perm.tolist()) == list(range(len(tets)))


def test_host_ingest_accepts_consistent_neighbours_and_rejects_wrong_ones():
    verts, tets = _kuhn(2)
    m = TetMesh(verts, tets, host_only=True)
    nb = m.neighbors()
    TetMesh(verts, tets, nbrs=nb, host_only=True)
    bad = nb.copy()
    bad[0, 0], bad[0, 1] = bad[0, 1], bad[0, 0]
    if bad[0, 0] == bad[0, 1]:
        bad[0, 0] = 5
    with pytest.raises(_lib.TctError) as e:
        TetMesh(verts, tets, nbrs=bad, host_only=True)
    assert e.value.status == -3


def test_host_ingest_rejections_match_oracle_statuses():
    verts, tets = _kuhn(2)
    cases = []
    bad = tets.copy()
    bad[0, 3] = bad[0, 2]
    cases.append((verts, bad, -2))
    cases.append((verts, np.vstack([tets, tets[:1]]), -3))
    X = synth.kuhn_nodes(2)
    v2, t2 = synth.kuhn_mesh(X, X, synth.kuhn_nodes(1))
    keep = np.array([c // 6 != 3 for c in range(len(t2))])
    cases.append((v2, t2[keep], -4))
    v1, t1 = _kuhn(1)
    cases.append((np.vstack([v1, v1 + np.float32(3)]), np.vstack([t1, t1 + len(v1)]), -5))
    # flat tetrahedron: four coplanar vertices
    flat = verts.copy()
    cases.append((flat, np.array([[0, 1, 2, 3]], np.int32), -2))
    for v, t, status in cases:
        with pytest.raises(_lib.TctError) as e:
            TetMesh(v, t, host_only=True)
        assert e.value.status == status
        with pytest.raises(oracle.oracle.OracleError) as e2:
            oracle.OracleMesh(v, t)
        assert e2.value.status == status


def test_morton_reorder_keeps_neighbours_local():
    """Internal order follows a space-filling curve: face neighbours are close in index."""
    w = synth.jittered_kuhn(12, 1, 2, 16, 16, 2)
    m = TetMesh(w.verts, w.tets, host_only=True)
    inv = np.empty_like(m.perm)
    inv[m.perm] = np.arange(len(m.perm))
    nb = m.neighbors()
    src = np.repeat(np.arange(len(nb)), 4)
    dst = nb.ravel()
    ok = dst >= 0
    gap_internal = np.abs(inv[src[ok]] - inv[dst[ok]])
    gap_user = np.abs(src[ok] - dst[ok])
    # more neighbours within a 64-element window (a few cache lines of records)
    assert (gap_internal < 64).mean() > (gap_user < 64).mean()


@pytest.mark.parametrize("kind", ["self_loop", "out_of_range", "negative_id", "boundary_claimed_interior",
                                  "interior_claimed_boundary", "one_sided"])
def test_neighbour_table_rejections(kind):
    """A caller-given neighbour table (Section II-B's ordered neighbour list)
    that contradicts the connectivity is rejected through the C ABI with
    TCT_E_MESH_NONMANIFOLD: a walk over it could loop or leave the mesh
    through an interior face (the failures Section II-C rules out)."""
    verts, tets = _kuhn(2)
    nb = TetMesh(verts, tets, host_only=True).neighbors()
    bad = nb.copy()
    t_in, k_in = map(int, np.argwhere(nb >= 0)[0])  # an interior face
    t_bd, k_bd = map(int, np.argwhere(nb < 0)[0])  # a boundary face
    if kind == "self_loop":
        bad[t_in, k_in] = t_in
    elif kind == "out_of_range":
        bad[t_in, k_in] = len(tets) + 5
    elif kind == "negative_id":
        bad[t_in, k_in] = -7
    elif kind == "boundary_claimed_interior":
        bad[t_bd, k_bd] = (t_bd + 1) % len(tets)
    elif kind == "interior_claimed_boundary":
        bad[t_in, k_in] = -1
    elif kind == "one_sided":
        # t's neighbour list names u, but u's list does not name t back
        u = int(nb[t_in, k_in])
        back = int(np.flatnonzero(nb[u] == t_in)[0])
        bad[u, back] = -1
    h = C.c_void_p()
    v = np.ascontiguousarray(verts, np.float32)
    t = np.ascontiguousarray(tets, np.int32)
    b = np.ascontiguousarray(bad, np.int32)
    st = _lib.lib().tct_mesh_create(v.ctypes.data, len(v), t.ctypes.data, len(t), b.ctypes.data,
                                    _lib.TCT_MESH_HOST_ONLY, 0, C.byref(h))
    assert st == -3, (kind, st)
    assert not h.value
    assert b"neighbour" in _lib.lib().tct_last_error()


def test_null_arguments_are_rejected():
    L = _lib.lib()
    h = C.c_void_p()
    verts, tets = _kuhn(1)
    v = np.ascontiguousarray(verts, np.float32)
    t = np.ascontiguousarray(tets, np.int32)
    assert L.tct_mesh_create(None, len(v), t.ctypes.data, len(t), None, _lib.TCT_MESH_HOST_ONLY, 0, C.byref(h)) == -1
    assert L.tct_mesh_create(v.ctypes.data, len(v), None, len(t), None, _lib.TCT_MESH_HOST_ONLY, 0, C.byref(h)) == -1
    assert L.tct_mesh_create(v.ctypes.data, len(v), t.ctypes.data, len(t), None, _lib.TCT_MESH_HOST_ONLY, 0,
                             None) == -1
    assert L.tct_mesh_counts(None, None, None, None, None) == -1
    assert L.tct_stats_read(None, None, 0) == -1
    assert L.tct_backproject(None, None, None, None, 0, 0, None, None) == -1


def test_autotune_host_rules():
    """The tuner's choice rules: the default stays unless a candidate beats it
    by more than the margin; timing subsets hold at least min_rays rays."""
    from types import SimpleNamespace

    from paper_1908_06909_amd import autotune

    assert autotune._pick({4: 1.00, 8: 1.02, 16: 1.5}, 8, 0.03) == 8
    assert autotune._pick({4: 0.90, 8: 1.00, 16: 1.5}, 8, 0.03) == 4
    assert autotune._pick({1: 1.0, 2: 0.5}, 8, 0.03) == 2  # default not among the candidates
    P = SimpleNamespace(geom=SimpleNamespace(nu=128, nv=128, na=64))
    assert autotune.subset_angles(P, 4, 0) == 4
    assert autotune.subset_angles(P, 4, 1 << 21) == 64  # capped at all angles
    P.geom.na = 720
    assert autotune.subset_angles(P, 4, 1 << 21) == 128
    P.geom.nu = P.geom.nv = 512
    assert autotune.subset_angles(P, 4, 1 << 21) == 8
