"""Pins of the CPU oracle against exact definitions, closed forms and brute force.

Every test here checks the oracle against something other than itself:
Fraction arithmetic, per-tetrahedron clipping, box chords, the exact
Kuhn-grid traversal generator, hand-derived worked examples, or identities
(adjoint, uniform phantom).  CPU only.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from exact_ref import (F3, KuhnGrid, box_chord, brute_force_lengths, cone_ray, det3, edge_sign, orient3d, sgn, sub)
from golden_io import load_worked_example

f32 = np.float32


# ---------------------------------------------------------------- predicates
def _adversarial_points(rng, n):
    """Float32 point sextuples that stress exact sign evaluation."""
    out = []
    for _ in range(n):
        kind = rng.integers(0, 6)
        if kind == 0:  # generic
            pts = rng.uniform(-2, 2, size=(6, 3))
        elif kind == 1:  # coplanar: all z equal
            pts = rng.uniform(-2, 2, size=(6, 3))
            pts[:, 2] = pts[0, 2]
        elif kind == 2:  # small integers: many exact zeros
            pts = rng.integers(-2, 3, size=(6, 3)).astype(np.float64)
        elif kind == 3:  # wide exponent range
            pts = rng.uniform(-1, 1, size=(6, 3)) * 10.0 ** rng.integers(-30, 30, size=(6, 3))
        elif kind == 4:  # nearly collinear: one ulp off a line
            a = rng.uniform(-1, 1, 3).astype(f32)
            b = rng.uniform(-1, 1, 3).astype(f32)
            pts = np.array([a, b, (a + b) / 2, a, b, (a + b) / 2], dtype=np.float64)
            pts[2] = np.nextafter(pts[2].astype(f32), f32(9)).astype(np.float64)
        else:  # grid points with a dyadic pitch
            pts = rng.integers(-8, 9, size=(6, 3)) * 2.0 ** -5
        out.append(pts.astype(f32))
    return out


def test_det_sign_matches_fractions():
    rng = np.random.default_rng(1234)
    for pts in _adversarial_points(rng, 1500):
        A1, A0, B1, B0, C1, C0 = pts
        ref = sgn(det3(sub(F3(A1), F3(A0)), sub(F3(B1), F3(B0)), sub(F3(C1), F3(C0))))
        assert oracle.det_sign(A1, A0, B1, B0, C1, C0) == ref
        assert oracle.det_sign_exact(A1, A0, B1, B0, C1, C0) == ref


def test_orient3d_matches_fractions():
    rng = np.random.default_rng(7)
    for pts in _adversarial_points(rng, 800):
        a, b, c, d = pts[:4]
        assert oracle.orient3d(a, b, c, d) == orient3d(a, b, c, d)


def test_edge_sign_perturbation_levels():
    """Rays through vertices, inside face planes and parallel to edges."""
    rng = np.random.default_rng(99)
    S = np.array([4, 0, 0], f32)
    P = np.array([-4, 0, 0], f32)
    U = np.array([0, 1, 0], f32)
    V = np.array([0, 0, 1], f32)
    cases = []
    grid = (rng.integers(-4, 5, size=(400, 2, 3)) * 0.125).astype(f32)
    for p, q in grid:
        cases.append((S, P, U, V, p, q))
    # edges parallel to the ray: all three levels vanish
    cases.append((S, P, U, V, np.array([0.25, 0.125, 0], f32), np.array([-0.25, 0.125, 0], f32)))
    # random oblique rays with dyadic grid endpoints (many exact zeros at level 0)
    for _ in range(300):
        S2 = (rng.integers(-16, 17, 3) * 0.25).astype(f32)
        P2 = (-S2 + rng.integers(-2, 3, 3) * 0.125).astype(f32)
        p, q = (rng.integers(-4, 5, size=(2, 3)) * 0.125).astype(f32)
        cases.append((S2, P2, U, V, p, q))
    levels_seen = set()
    for S_, P_, U_, V_, p, q in cases:
        ref = edge_sign(S_, P_, U_, V_, p, q)
        got = oracle.edge_sign(S_, P_, U_, V_, p, q)
        assert got == ref
        # antisymmetry E(p, q) = -E(q, p)
        assert oracle.edge_sign(S_, P_, U_, V_, q, p) == -ref
        levels_seen.add(ref)
    assert levels_seen == {-1, 0, 1}


# ---------------------------------------------------------------- ray frame
@pytest.mark.parametrize("cfg", [0, 2])
def test_frame_matches_restatement(cfg):
    """Ray endpoints are bit-identical to the float32 restatement of the geometry."""
    w = synth.config(cfg) if cfg == 0 else None
    if cfg == 2:
        cone = synth.Cone(4.0, 8.0, 256, 256, 2.0 ** -7, 2.0 ** -7, 2.0 ** -8, 2.0 ** -8)
        angles = synth.angles_for(180)
    else:
        cone, angles = w.cone, w.angles
    rng = np.random.default_rng(5)
    n = len(angles) * cone.nu * cone.nv
    ids = np.concatenate([rng.integers(0, n, 400), np.arange(cone.nu * cone.nv // 2, cone.nu * cone.nv // 2 + 50)])
    S, P, U, V = oracle.rays_of(cone, angles, ids)
    for k, rid in enumerate(ids):
        rs, rp, ru, rv = cone_ray(cone, angles, int(rid))
        assert np.array_equal(S[k], rs) and np.array_equal(P[k], rp)
        assert np.array_equal(U[k], ru) and np.array_equal(V[k], rv)


def test_quarter_turn_frames_are_exact():
    cone = synth.Cone(4.0, 8.0, 4, 4, 0.5, 0.5)
    angles = synth.angles_for(4)
    S, D, U, V, ut, vt = oracle.frame(cone, angles)
    assert np.array_equal(S, np.array([[4, 0, 0], [0, 4, 0], [-4, 0, 0], [0, -4, 0]], f32))
    assert np.array_equal(D, -S)
    assert np.array_equal(ut, np.array([-0.75, -0.25, 0.25, 0.75], f32))


# ---------------------------------------------------------------- ingest
def _kuhn(n):
    X = synth.kuhn_nodes(n)
    return synth.kuhn_mesh(X, X, X)


def test_ingest_orientation_neighbours_boundary():
    verts, tets = _kuhn(3)
    m = oracle.OracleMesh(verts, tets)
    assert m.nboundary == 12 * 3 * 3
    T, N, B, O = m.tables()
    for t in range(len(T)):
        assert orient3d(*verts[T[t]]) == 1
        assert sorted(T[t]) == sorted(tets[t])
        for k in range(4):
            nb = N[t, k]
            face = set(T[t]) - {T[t][k]}
            if nb < 0:
                continue
            assert face <= set(T[nb])
            assert t in N[nb]
    # boundary faces point outward: the owner's fourth vertex is behind them
    for f, (t, k) in zip(B, O):
        assert orient3d(*verts[f], verts[T[t][k]]) == -1
    # exactly half of the Kuhn tetrahedra are built with negative orientation
    assert m.flips == len(tets) // 2


def test_ingest_rejections():
    verts, tets = _kuhn(2)
    # zero-volume tetrahedron
    bad = tets.copy()
    bad[0, 3] = bad[0, 2]
    with pytest.raises(oracle.oracle.OracleError) as e:
        oracle.OracleMesh(verts, bad)
    assert e.value.status in (-2,)
    # a face shared by three tetrahedra
    extra = np.vstack([tets, tets[:1]])
    with pytest.raises(oracle.oracle.OracleError) as e:
        oracle.OracleMesh(verts, extra)
    assert e.value.status == -3
    # non-convex: an L-shaped block of cells (drop the cells of one corner)
    X = synth.kuhn_nodes(2)
    v2, t2 = synth.kuhn_mesh(X, X, synth.kuhn_nodes(1))
    keep = np.array([c // 6 != 3 for c in range(len(t2))])
    with pytest.raises(oracle.oracle.OracleError) as e:
        oracle.OracleMesh(v2, t2[keep])
    assert e.value.status == -4
    # two separate cubes: closed and locally convex but not connected
    v1, t1 = _kuhn(1)
    vv = np.vstack([v1, v1 + f32(3.0)])
    tt = np.vstack([t1, t1 + len(v1)])
    with pytest.raises(oracle.oracle.OracleError) as e:
        oracle.OracleMesh(vv, tt)
    assert e.value.status == -5


def test_rejects_dependent_perturbation_basis():
    verts, tets = _kuhn(1)
    m = oracle.OracleMesh(verts, tets)
    ex, ey, _ = np.eye(3, dtype=f32)
    with pytest.raises(oracle.oracle.OracleError) as e:
        _trace_custom(m, [(np.array([-2, 2, 0], f32), np.array([2, -2, 0], f32), ex, ey)])
    assert e.value.status == -1


# ---------------------------------------------------------------- walk pins
def _random_generic_rays(rng, n, radius=3.0):
    rays = []
    for _ in range(n):
        dirn = rng.normal(size=3)
        dirn /= np.linalg.norm(dirn)
        S = (dirn * radius + rng.uniform(-0.3, 0.3, 3)).astype(f32)
        P = (-dirn * radius + rng.uniform(-0.3, 0.3, 3)).astype(f32)
        U = rng.normal(size=3).astype(f32)
        V = rng.normal(size=3).astype(f32)
        rays.append((S, P, U, V))
    return rays


def test_oracle_vs_brute_force_clipping_jittered():
    verts, tets = _kuhn(3)
    verts, _ = synth.jitter_interior(verts, tets, (3, 3, 3), 1 / 3, 0.2, seed=17)
    m = oracle.OracleMesh(verts, tets)
    rng = np.random.default_rng(2024)
    rays = _random_generic_rays(rng, 60)
    S, P, U, V = (np.array([r[k] for r in rays]) for k in range(4))
    paths = oracle.oracle.trace_rays(m, S, P, U, V)
    for (s, p, _, _), (tt, ll) in zip(rays, paths):
        ref = brute_force_lengths(verts, tets, s, p)
        got = {}
        for t, l in zip(tt, ll):
            assert t not in got, "tetrahedron visited twice"
            got[int(t)] = l
        pos = {t: l for t, l in got.items() if l > 1e-12}
        assert set(pos) == set(ref)
        for t in ref:
            assert abs(pos[t] - ref[t]) <= 1e-12 * max(1.0, sum(ref.values()))


def test_oracle_vs_brute_force_clipping_delaunay():
    """Unstructured mesh (Delaunay of 40 random points, slivers included)."""
    verts, tets = synth.delaunay_mesh(40, 11)
    m = oracle.OracleMesh(verts, tets)
    rng = np.random.default_rng(2025)
    rays = _random_generic_rays(rng, 60)
    S, P, U, V = (np.array([r[k] for r in rays]) for k in range(4))
    paths = oracle.oracle.trace_rays(m, S, P, U, V)
    hits = 0
    for (s, p, _, _), (tt, ll) in zip(rays, paths):
        ref = brute_force_lengths(verts, tets, s, p)
        got = {}
        for t, l in zip(tt, ll):
            assert t not in got, "tetrahedron visited twice"
            got[int(t)] = l
        pos = {t: l for t, l in got.items() if l > 1e-12}
        assert set(pos) == set(ref)
        hits += len(ref) > 0
        for t in ref:
            assert abs(pos[t] - ref[t]) <= 1e-12 * max(1.0, sum(ref.values()))
    assert hits >= 20


def _trace_custom(m, rays):
    S, P, U, V = (np.array([r[k] for r in rays], f32) for k in range(4))
    return oracle.oracle.trace_rays(m, S, P, U, V)


def _compare_kuhn(paths, grid, rays):
    for (s, p, u, v), (tt, ll) in zip(rays, paths):
        ref = grid.trace(s, p, u, v)
        assert [int(t) for t in tt] == [r[0] for r in ref]
        for l, r in zip(ll, ref):
            assert abs(l - r[1]) <= 1e-12


def test_oracle_vs_kuhn_generator_cone_rays():
    """Kuhn 8^3 with the 64^2 x 16 cone geometry: full sequences, zero-length passages included."""
    w = synth.config(0)
    m = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    grid = KuhnGrid(*(synth.kuhn_nodes(8),) * 3)
    rng = np.random.default_rng(3)
    ids = np.concatenate([rng.integers(0, m.nrays, 120), np.arange(32 * 64, 32 * 64 + 64)])
    paths = m.trace(ids)
    S, P, U, V = m.rays(ids)
    _compare_kuhn(paths, grid, list(zip(S, P, U, V)))


def test_oracle_vs_kuhn_generator_degenerate_rays():
    """Axis-aligned rays through vertex lines, diagonals and face planes of Kuhn 4^3."""
    verts, tets = _kuhn(4)
    m = oracle.OracleMesh(verts, tets)
    grid = KuhnGrid(*(synth.kuhn_nodes(4),) * 3)
    ex, ey, ez = np.eye(3, dtype=f32)
    rays = []
    for y in (-0.25, 0.0, 0.125, 0.25):
        for z in (-0.25, 0.0, 0.25, 0.3):
            rays.append((np.array([4, y, z], f32), np.array([-4, y, z], f32), ey, ez))
            rays.append((np.array([y, -4, z], f32), np.array([y, 4, z], f32), ez, ex))
            rays.append((np.array([y, z, 4], f32), np.array([y, z, -4], f32), ex, -ey))
    # main and face diagonals through vertices, with both perturbation orders
    for U, V in ((ex, ey), (ey, ex), (ez, ex), (-ex, ez)):
        rays.append((np.array([-2, -2, -2], f32), np.array([2, 2, 2], f32), U, V))
        rays.append((np.array([-2, -2, 0], f32), np.array([2, 2, 0], f32), U, V))
        rays.append((np.array([-2, 0.25, -2], f32), np.array([2, 0.25, 2], f32), U, V))
        rays.append((np.array([2, -2, 0.25], f32), np.array([-2, 2, 0.25], f32), U, V))
    rays = [r for r in rays if orient3d(np.zeros(3, f32), r[1] - r[0], r[2], r[3]) != 0]
    assert len(rays) >= 58
    paths = _trace_custom(m, rays)
    _compare_kuhn(paths, grid, rays)


def test_oracle_vs_kuhn_generator_graded():
    """Graded product grid (ratio 1.05) with a vertex column on the z axis."""
    X = synth.graded_nodes(12, 1.05, 7)
    Z = synth.kuhn_nodes(4)
    verts, tets = synth.kuhn_mesh(X, X, Z)
    m = oracle.OracleMesh(verts, tets)
    grid = KuhnGrid(X, X, Z)
    cone = synth.Cone(4.0, 8.0, 32, 32, 2.0 ** -4, 2.0 ** -4, 2.0 ** -5, 2.0 ** -5)
    angles = synth.angles_for(8)
    o = oracle.Oracle(verts, tets, cone, angles)
    rng = np.random.default_rng(11)
    n = o.nrays
    central = [a * 1024 + 15 * 32 + i for a in range(8) for i in range(0, 32, 3)]
    column = [a * 1024 + j * 32 + 15 for a in range(8) for j in range(0, 32, 4)]
    ids = np.array(sorted(set(central + column + list(rng.integers(0, n, 60)))), np.int64)
    paths = o.trace(ids)
    S, P, U, V = o.rays(ids)
    _compare_kuhn(paths, grid, list(zip(S, P, U, V)))


@pytest.mark.parametrize("name", ["W1_kuhn1_diagonal.txt", "W2_kuhn4_axis.txt"])
def test_worked_examples(name):
    g = load_worked_example(name)
    verts, tets = _kuhn(g["n"])
    m = oracle.OracleMesh(verts, tets)
    (tt, ll), = _trace_custom(m, [g["ray"]])
    assert list(tt) == list(g["tets"])
    assert np.allclose(ll, g["lengths"], rtol=0, atol=1e-12)


def test_chord_identity_and_uniform_phantom():
    """sum_i a_ij = chord of the ray through the hull box; x = c gives b = c * chord."""
    w = synth.config(0)
    o = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    rng = np.random.default_rng(8)
    ids = rng.integers(0, o.nrays, 3000)
    c = 0.75
    b = o.forward(np.full(o.nt, c, f32), ids)
    S, P, _, _ = o.rays(ids)
    lo, hi = np.full(3, -0.5, f32), np.full(3, 0.5, f32)
    for k in range(len(ids)):
        ch = box_chord(S[k], P[k], lo, hi)
        assert abs(b[k] - c * ch) <= 1e-12 * max(1.0, ch)


def test_adjoint_identity_oracle():
    w = synth.config(0)
    o = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    rng = np.random.default_rng(21)
    x = rng.uniform(-1, 1, o.nt).astype(f32)
    y = rng.uniform(-1, 1, o.nrays).astype(f32)
    Ax = o.forward(x)
    Aty = o.backproject(y)
    lhs = float(np.dot(Ax, y.astype(np.float64)))
    rhs = float(np.dot(x.astype(np.float64), Aty))
    absA_x = o.forward(np.abs(x))
    scale = float(np.dot(absA_x, np.abs(y).astype(np.float64)))
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_walk_invariants_jittered():
    w = synth.jittered_kuhn(6, 5, 6, 32, 32, 6)
    o = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    T, N, _, _ = o.mesh.tables()
    rng = np.random.default_rng(4)
    ids = rng.integers(0, o.nrays, 400)
    for tt, ll in o.trace(ids):
        assert len(set(tt.tolist())) == len(tt)
        assert np.all(ll >= 0)
        for a, b in zip(tt[:-1], tt[1:]):
            assert b in N[a]
        if len(tt):
            assert -1 in N[tt[0]] and -1 in N[tt[-1]]
    st = oracle.oracle.last_stats()
    assert st.failed == 0 and st.multi_entry == 0


def test_check_pass_terms_match_traces():
    """The one-pass bound terms the GPU tests use equal the same quantities
    assembled in numpy from the oracle's traces (a jittered mesh with rays
    that miss and rays that clip the hull; the sums over visits include the
    zero-length passages)."""
    w = synth.jittered_kuhn(3, 5, 13, 13, 11, 3)
    w.cone = synth.Cone(4.0, 8.0, 13, 11, 0.2, 0.23, 0.01, -0.02)  # wider than the mesh's shadow
    o = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    rng = np.random.default_rng(5)
    ids = np.arange(o.nrays)
    y = rng.uniform(-1, 1, o.nrays).astype(np.float32)
    x = rng.uniform(-1, 1, o.nt).astype(np.float32)
    wt = rng.uniform(0.5, 2.0, o.nt)
    r = o.check_pass(x, wt, y, ids)
    b = np.zeros(o.nrays)
    babs = np.zeros(o.nrays)
    chord = np.zeros(o.nrays)
    wx = np.zeros(o.nrays)
    xhat, xabs, supp, suppc, cnt = (np.zeros(o.nt) for _ in range(5))
    for j, (tt, ll) in enumerate(o.trace(ids)):
        b[j] = np.sum(ll * x[tt])
        babs[j] = np.sum(ll * np.abs(x[tt]))
        chord[j] = ll.sum()
        wx[j] = np.max(wt[tt] * np.abs(x[tt])) if len(tt) else 0.0
        np.add.at(xhat, tt, ll * float(y[j]))
        np.add.at(xabs, tt, ll * abs(float(y[j])))
        np.add.at(supp, tt, abs(float(y[j])))
        np.add.at(suppc, tt, chord[j] * abs(float(y[j])))
        np.add.at(cnt, tt, 1)
    assert (chord == 0).sum() > 0 and (chord > 0).sum() > 0
    for k, v in (("b", b), ("babs", babs), ("chord", chord), ("wx", wx), ("xhat", xhat), ("xabs", xabs),
                 ("supp", supp), ("suppc", suppc), ("cnt", cnt)):
        assert np.allclose(r[k], v, rtol=1e-12, atol=1e-13), k
