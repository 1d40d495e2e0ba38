"""GPU parity: the HIP walk (through the C ABI) against the CPU oracle.

The bars are those of parity_bars.py: identical sequences, lengths within
1e-5 of the ray's chord plus a rounding floor of the element size,
projections and backprojections within 1e-5 of the sum of their terms'
magnitudes, the float32-atomic scatters plus their accumulation error.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from golden_io import load_worked_example
from parity_bars import (assert_within, backprojection_reference, compare_traces, element_size,
                         forward_reference)

pytestmark = pytest.mark.gpu

f32 = np.float32
DEV = "cuda:0"


def _gpu():
    import paper_1908_06909_amd as tct

    return tct


class Case:
    """Mesh + geometry on both sides."""

    def __init__(self, w):
        tct = _gpu()
        self.w = w
        self.orc = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
        self.mesh = tct.TetMesh(w.verts, w.tets, device=DEV)
        self.geom = tct.ConeGeometry(w.cone, w.angles, device=DEV)
        self.P = tct.Projector(self.mesh, self.geom)
        _, nbrs, _, _ = self.orc.mesh.tables()
        self.H = element_size(w.verts, w.tets, nbrs)

    def x_internal(self, x_user):
        return self.mesh.to_internal(torch.as_tensor(np.ascontiguousarray(x_user, f32), device=DEV))

    def to_user(self, x_int):
        return self.mesh.to_user(x_int).cpu().numpy()


_cases = {}


def case(name):
    if name not in _cases:
        if name == "cfg0":
            w = synth.config(0)
        elif name == "cfg1":
            w = synth.config(1)
        elif name == "cfg2":
            w = synth.config(2)
        elif name == "graded_small":
            (verts, tets), X, Z = synth.graded_mesh(24, 8, 1.05, 17)
            x = synth.sphere_phantom(verts, tets, 12)
            du = 2.0 ** -5
            cone = synth.Cone(4.0, 8.0, 64, 64, du, du, du / 2, du / 2)
            w = synth.Workload("graded24", verts, tets, x, cone, synth.angles_for(12))
        elif name == "delaunay":
            # Unstructured: Delaunay mesh of 3000 random points (~20k tetrahedra with slivers).
            verts, tets = synth.delaunay_mesh(3000, 2)
            x = synth.uniform_random(len(tets), 8)
            cone = synth.Cone(4.0, 8.0, 48, 40, 2.0 / 40, 2.0 / 40, 0.003, -0.002)
            w = synth.Workload("delaunay3000", verts, tets, x, cone, synth.angles_for(6))
        elif name == "ties":
            # Unjittered Kuhn 4^3 with pixel centres on projected vertices and
            # edges (odd detector, central ray through the origin, angles in
            # steps of 45 degrees): exact ties for the element-driven pass.
            w = synth.plain_kuhn(4, 3, 33, 33, 8, pitch=2.0 ** -4)
        elif name == "ragged":
            w = synth.jittered_kuhn(5, 7, 8, 37, 29, 5)
            w.cone = synth.Cone(4.0, 8.0, 37, 29, 0.08, 0.09, 0.013, -0.021)  # wider than the mesh shadow
        else:
            raise KeyError(name)
        _cases[name] = Case(w)
    return _cases[name]


def ray_lengths(c, ids):
    S, P, _, _ = c.orc.rays(ids)
    return np.linalg.norm(P.astype(np.float64) - S, axis=1)


def check_stats(mesh):
    st = mesh.stats(reset=True)
    assert st["failed"] == 0, st
    return st


# ---------------------------------------------------------------- cfg0 (full)
def test_cfg0_all_sequences_bitexact():
    c = case("cfg0")
    ids = np.arange(c.orc.nrays)
    compare_traces(c.P.trace(ids), c.orc.trace(ids), c.H)
    check_stats(c.mesh)


def test_cfg0_forward():
    c = case("cfg0")
    x = c.w.x
    ref, tol = forward_reference(c.orc, x, c.H)
    xi = c.x_internal(x)
    got = c.P.forward(xi).cpu().numpy().ravel()
    got_nc = c.P.forward(xi, use_cache=False).cpu().numpy().ravel()
    assert np.array_equal(got, got_nc), "entry cache changes the result"
    assert_within(got, ref, tol, "cfg0 forward")
    assert np.all(got[ref == 0] == 0)
    check_stats(c.mesh)


FLOAT_ATOMIC = ("atomic", "atomic_direct")


def _bp_tolerance(c, y, mode):
    """Per-element bar of a backprojection of every ray of the case."""
    return backprojection_reference(c.orc, y, c.H, float_atomic=mode in FLOAT_ATOMIC)[1]


@pytest.mark.parametrize("mode", ["atomic", "atomic_direct", "gather", "shadow", "fixed"])
def test_cfg0_backproject(mode):
    c = case("cfg0")
    rng = np.random.default_rng(31)
    y = rng.uniform(-1, 1, c.orc.nrays).astype(f32)
    ref = c.orc.backproject(y)
    yt = torch.as_tensor(y, device=DEV)
    got = c.to_user(c.P.backproject(yt, mode=mode)).astype(np.float64)
    tol = _bp_tolerance(c, y, mode)
    assert_within(got, ref, tol, f"cfg0 backprojection {mode}")
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    check_stats(c.mesh)


@pytest.mark.parametrize("mode", ["atomic", "shadow", "gather"])
def test_cfg0_backproject_wide_dynamic_range(mode):
    """Projection values spanning eight decades with both signs, so a pixel
    wavefront mixes terms 10^8 apart: the scatter's fixed-point wavefront
    table keeps every term to 2^-51 of the wavefront's largest, which stays
    inside the bar."""
    c = case("cfg0")
    rng = np.random.default_rng(36)
    y = (rng.choice([-1.0, 1.0], c.orc.nrays) * 10.0 ** rng.uniform(-4, 4, c.orc.nrays)).astype(f32)
    ref = c.orc.backproject(y)
    got = c.to_user(c.P.backproject(torch.as_tensor(y, device=DEV), mode=mode)).astype(np.float64)
    assert_within(got, ref, _bp_tolerance(c, y, mode), f"cfg0 wide-range backprojection {mode}")
    check_stats(c.mesh)


def _fixed_quantum(c, y):
    """Upper bound on the reproducible scatter's rounding step: 2^-(K - e)
    with K = min(50, 62 - ceil(log2 rays)) and 2^e above max |y_j| |d_j| (one
    power of two of slack for the float32 product the library forms)."""
    n = c.orc.nrays
    bits = max(1, int(np.ceil(np.log2(n))))
    dmax = float(ray_lengths(c, np.arange(n)).max()) * 1.0001
    _, e = np.frexp(float(np.abs(y).max()) * dmax)
    return 2.0 ** -(min(50, 62 - bits) - int(e) - 1)


def test_cfg0_wide_range_fixed_within_its_quantum():
    """The reproducible scatter rounds every term to one quantum per launch:
    on projection values spanning eight decades its error per element stays
    within the oracle bar plus half a quantum per term."""
    c = case("cfg0")
    rng = np.random.default_rng(36)
    y = (rng.choice([-1.0, 1.0], c.orc.nrays) * 10.0 ** rng.uniform(-4, 4, c.orc.nrays)).astype(f32)
    ref = c.orc.backproject(y)
    got = c.to_user(c.P.backproject(torch.as_tensor(y, device=DEV), mode="fixed")).astype(np.float64)
    ids = np.arange(c.orc.nrays)
    nterm = np.zeros(c.orc.nt)
    for tt, ll in c.orc.trace(ids):
        np.add.at(nterm, tt[ll > 0], 1)
    q = _fixed_quantum(c, y)
    print(f"fixed quantum {q:.3e}")
    assert_within(got, ref, _bp_tolerance(c, y, "fixed") + nterm * q * 0.5, "cfg0 wide-range backprojection fixed")


def test_cfg0_fixed_is_reproducible_and_accumulates():
    c = case("cfg0")
    rng = np.random.default_rng(37)
    yt = torch.as_tensor(rng.uniform(-1, 1, c.orc.nrays).astype(f32), device=DEV)
    a = c.P.backproject(yt, mode="fixed").cpu().numpy()
    b = c.P.backproject(yt, mode="fixed").cpu().numpy()
    assert np.array_equal(a.view(np.int32), b.view(np.int32))
    base = torch.full((c.orc.nt,), 0.25, dtype=torch.float32, device=DEV)
    acc = c.P.backproject(yt, mode="fixed", out=base.clone(), accumulate=True).cpu().numpy()
    assert np.allclose(acc, a + np.float32(0.25), rtol=0, atol=1e-6)
    g = c.P.backproject(yt, mode="gather").cpu().numpy()
    assert np.allclose(a, g, rtol=1e-5, atol=1e-5)


def test_cfg0_gather_is_deterministic_and_accumulates():
    c = case("cfg0")
    rng = np.random.default_rng(32)
    yt = torch.as_tensor(rng.uniform(-1, 1, c.orc.nrays).astype(f32), device=DEV)
    a = c.P.backproject(yt, mode="gather").cpu().numpy()
    b = c.P.backproject(yt, mode="gather").cpu().numpy()
    assert np.array_equal(a.view(np.int32), b.view(np.int32))
    base = torch.full((c.orc.nt,), 0.25, dtype=torch.float32, device=DEV)
    acc = c.P.backproject(yt, mode="gather", out=base.clone(), accumulate=True).cpu().numpy()
    assert np.allclose(acc, a + np.float32(0.25), rtol=0, atol=1e-6)
    acc2 = c.P.backproject(yt, mode="atomic", out=base.clone(), accumulate=True).cpu().numpy()
    assert np.allclose(acc2, acc, rtol=1e-5, atol=1e-5)


def test_cfg0_shadow_is_deterministic_and_accumulates():
    c = case("cfg0")
    rng = np.random.default_rng(34)
    yt = torch.as_tensor(rng.uniform(-1, 1, c.orc.nrays).astype(f32), device=DEV)
    a = c.P.backproject(yt, mode="shadow").cpu().numpy()
    b = c.P.backproject(yt, mode="shadow").cpu().numpy()
    assert np.array_equal(a.view(np.int32), b.view(np.int32))
    base = torch.full((c.orc.nt,), 0.25, dtype=torch.float32, device=DEV)
    acc = c.P.backproject(yt, mode="shadow", out=base.clone(), accumulate=True).cpu().numpy()
    assert np.allclose(acc, a + np.float32(0.25), rtol=0, atol=1e-6)
    g = c.P.backproject(yt, mode="gather").cpu().numpy()
    assert np.allclose(a, g, rtol=1e-5, atol=1e-5)


def test_ties_sequences_and_forward():
    """The walk on rays through vertices and along edges of a regular mesh:
    the perturbed predicate must pick the oracle's tetrahedra on every ray."""
    c = case("ties")
    ids = np.arange(c.orc.nrays)
    compare_traces(c.P.trace(ids), c.orc.trace(ids), c.H)
    x = c.w.x
    got = c.P.forward(c.x_internal(x)).cpu().numpy().ravel()
    ref, tol = forward_reference(c.orc, x, c.H)
    assert_within(got, ref, tol, "ties forward")
    st = check_stats(c.mesh)
    assert st["perturbed_ties"] > 0


def test_shadow_exact_pass_on_ties():
    """Rays through mesh vertices and along edges: the element-driven pass
    hands those elements to its exact pass, which must agree with the oracle
    and give the same bits on every run."""
    c = case("ties")
    rng = np.random.default_rng(35)
    y = rng.uniform(-1, 1, c.orc.nrays).astype(f32)
    ref = c.orc.backproject(y)
    yt = torch.as_tensor(y, device=DEV)
    c.mesh.stats(reset=True)
    a = c.P.backproject(yt, mode="shadow")
    st = check_stats(c.mesh)
    print(f"ties: {st['fp64_stage']} exact-pass sign evaluations, {st['exact_stage']} exact, "
          f"{st['perturbed_ties']} perturbed")
    assert st["fp64_stage"] > 0 and st["perturbed_ties"] > 0
    b = c.P.backproject(yt, mode="shadow")
    assert torch.equal(a, b)
    got = c.to_user(a).astype(np.float64)
    assert_within(got, ref, _bp_tolerance(c, y, "shadow"), "ties shadow backprojection")
    g = c.to_user(c.P.backproject(yt, mode="gather")).astype(np.float64)
    assert_within(g, ref, _bp_tolerance(c, y, "gather"), "ties gather backprojection")


def test_cfg0_adjoint():
    c = case("cfg0")
    rng = np.random.default_rng(33)
    x = rng.uniform(-1, 1, c.orc.nt).astype(f32)
    y = rng.uniform(-1, 1, c.orc.nrays).astype(f32)
    xi = c.x_internal(x)
    Ax = c.P.forward(xi).cpu().numpy().ravel().astype(np.float64)
    for mode in ("atomic", "atomic_direct", "gather", "shadow"):
        Aty = c.to_user(c.P.backproject(torch.as_tensor(y, device=DEV), mode=mode)).astype(np.float64)
        lhs = float(np.dot(Ax, y))
        rhs = float(np.dot(x.astype(np.float64), Aty))
        scale = float(np.dot(c.orc.forward(np.abs(x)), np.abs(y)))
        assert abs(lhs - rhs) <= 1e-5 * scale, (mode, lhs, rhs)


# ---------------------------------------------------------------- custom rays
@pytest.mark.parametrize("name", ["W1_kuhn1_diagonal.txt", "W2_kuhn4_axis.txt"])
def test_worked_examples_gpu(name):
    tct = _gpu()
    g = load_worked_example(name)
    X = synth.kuhn_nodes(g["n"])
    verts, tets = synth.kuhn_mesh(X, X, X)
    m = tct.TetMesh(verts, tets, device=DEV)
    (tt, ll), = tct.trace_rays(m, *[np.asarray(a)[None] for a in g["ray"]])
    assert list(tt) == list(g["tets"])
    assert np.allclose(ll, g["lengths"], rtol=0, atol=1e-5)
    check_stats(m)


def _degenerate_rays():
    ex, ey, ez = np.eye(3, dtype=f32)
    rays = []
    for y in (-0.25, 0.0, 0.125, 0.25):
        for z in (-0.25, 0.0, 0.25, 0.3):
            rays.append((np.array([4, y, z], f32), np.array([-4, y, z], f32), ey, ez))
            rays.append((np.array([y, -4, z], f32), np.array([y, 4, z], f32), ez, ex))
            rays.append((np.array([y, z, 4], f32), np.array([y, z, -4], f32), ex, -ey))
    for U, V in ((ex, ey), (ey, ex), (ez, ex), (-ex, ez)):
        rays.append((np.array([-2, -2, -2], f32), np.array([2, 2, 2], f32), U, V))
        rays.append((np.array([-2, -2, 0], f32), np.array([2, 2, 0], f32), U, V))
        rays.append((np.array([-2, 0.25, -2], f32), np.array([2, 0.25, 2], f32), U, V))
        rays.append((np.array([2, -2, 0.25], f32), np.array([-2, 2, 0.25], f32), U, V))
    # grazing the hull: along a hull edge and inside a hull face plane
    rays.append((np.array([4, 0.5, 0.5], f32), np.array([-4, 0.5, 0.5], f32), ey, ez))
    rays.append((np.array([4, -0.5, 0.1], f32), np.array([-4, -0.5, 0.1], f32), ey, ez))
    rays.append((np.array([4, 0.5, 0.1], f32), np.array([-4, 0.5, 0.1], f32), -ey, ez))
    # missing the hull
    rays.append((np.array([4, 0.9, 0.1], f32), np.array([-4, 0.9, 0.1], f32), ey, ez))
    import exact_ref

    return [r for r in rays if exact_ref.orient3d(np.zeros(3, f32), r[1] - r[0], r[2], r[3]) != 0]


def test_degenerate_custom_rays_match_oracle():
    tct = _gpu()
    X = synth.kuhn_nodes(4)
    verts, tets = synth.kuhn_mesh(X, X, X)
    m = tct.TetMesh(verts, tets, device=DEV)
    om = oracle.OracleMesh(verts, tets)
    rays = _degenerate_rays()
    S, P, U, V = (np.array([r[k] for r in rays], f32) for k in range(4))
    compare_traces(tct.trace_rays(m, S, P, U, V), oracle.oracle.trace_rays(om, S, P, U, V),
                   element_size(verts, tets, om.tables()[1]))
    st = check_stats(m)
    assert st["perturbed_ties"] > 0 and st["exact_stage"] > 0


def test_trace_empty_list():
    c = case("cfg0")
    assert c.P.trace(np.zeros(0, np.int64)) == []


# ---------------------------------------------------------------- graded / cfg2
def _degenerate_ids(nu, nv, na, stride_a=1):
    cu, cv = (nu - 1) // 2, (nv - 1) // 2
    ids = []
    for a in range(0, na, stride_a):
        base = a * nu * nv
        ids += [base + cv * nu + i for i in range(nu)]  # central row: inside the plane z = 0
        ids += [base + j * nu + cu for j in range(nv)]  # central column: crosses the z axis
    return np.array(sorted(set(ids)), np.int64)


def test_graded_small_all_sequences():
    c = case("graded_small")
    ids = np.arange(c.orc.nrays)
    compare_traces(c.P.trace(ids), c.orc.trace(ids), c.H)
    xi = c.x_internal(c.w.x)
    got = c.P.forward(xi).cpu().numpy().ravel()
    ref, tol = forward_reference(c.orc, c.w.x, c.H)
    assert_within(got, ref, tol, "graded forward")
    st = check_stats(c.mesh)
    assert st["perturbed_ties"] > 0
    # Rays through vertices and along edges: the element-driven backprojection
    # must pick the same tetrahedra as the walk (same perturbed predicate).
    y = np.random.default_rng(4).uniform(-1, 1, c.orc.nrays).astype(f32)
    ref = c.orc.backproject(y)
    got = c.to_user(c.P.backproject(torch.as_tensor(y, device=DEV), mode="shadow")).astype(np.float64)
    assert_within(got, ref, _bp_tolerance(c, y, "shadow"), "graded shadow backprojection")
    st = check_stats(c.mesh)
    assert st["perturbed_ties"] > 0


def test_cfg2_all_degenerate_rays_and_forward():
    """Every central-row ray (inside the vertex plane z = 0) and every
    central-column ray (across the z axis, through its vertices on every
    eighth row) of all 180 angles, plus random rays: sequences identical to
    the oracle's, lengths and projections within the bars."""
    c = case("cfg2")
    cone = c.w.cone
    rng = np.random.default_rng(2)
    deg = _degenerate_ids(cone.nu, cone.nv, len(c.w.angles))
    ids = np.concatenate([deg, rng.integers(0, c.orc.nrays, 2000)])
    print(f"cfg2: {len(deg)} degenerate rays over {len(c.w.angles)} angles + 2000 random")
    c.mesh.stats(reset=True)
    compare_traces(c.P.trace(ids), c.orc.trace(ids), c.H)
    st = check_stats(c.mesh)
    assert st["perturbed_ties"] > 0
    xi = c.x_internal(c.w.x)
    full = c.P.forward(xi).cpu().numpy().ravel()
    ref, tol = forward_reference(c.orc, c.w.x, c.H, ids)
    assert_within(full[ids], ref, tol, "cfg2 forward")
    check_stats(c.mesh)


def test_cfg1_random_sequences_and_forward():
    c = case("cfg1")
    rng = np.random.default_rng(1)
    n_per = c.w.cone.nu * c.w.cone.nv
    ids = np.concatenate([rng.integers(0, c.orc.nrays, 20000), 100 * n_per + 256 * 512 + np.arange(512)])
    compare_traces(c.P.trace(ids), c.orc.trace(ids), c.H)
    xi = c.x_internal(c.w.x)
    full = c.P.forward(xi).cpu().numpy().ravel()
    ref, tol = forward_reference(c.orc, c.w.x, c.H, ids)
    assert_within(full[ids], ref, tol, "cfg1 forward")
    assert np.all(full != 0)  # every ray of this geometry hits the cube
    check_stats(c.mesh)


# Four consecutive angles including a quarter turn (90 degrees), where the
# frame is exact and the central rays run along mesh lines.
_RANGES = {"cfg1": (88, 4), "cfg2": (44, 4)}


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_full_size_range_every_element_against_oracle(name):
    """Full-size mesh and detector, four angles: every projection of those
    angles and every element of every backprojection mode (launched through
    tct_forward_range / tct_backproject_range) against one oracle pass over
    exactly those rays."""
    c = case(name)
    a0, na = _RANGES[name]
    n_per = c.w.cone.nu * c.w.cone.nv
    ids = np.arange(a0 * n_per, (a0 + na) * n_per, dtype=np.int64)
    rng = np.random.default_rng(21)
    y = rng.uniform(-1.0, 1.0, c.geom.nrays).astype(f32)
    x = c.w.x.astype(f32)
    r = c.orc.check_pass(x, c.H, y[ids], ids)
    print(f"{name}: {len(ids)} rays of angles {a0}..{a0 + na - 1}, {int(r['cnt'].sum())} positive segments")
    # forward
    xi = c.x_internal(x)
    out = torch.zeros(c.geom.nrays, dtype=torch.float32, device=DEV)
    c.P.forward_range(xi, a0, na, out)
    got = out.cpu().numpy()
    assert np.all(got[:ids[0]] == 0) and np.all(got[ids[-1] + 1:] == 0)
    from parity_bars import C_FLOOR, U32
    assert_within(got[ids], r["b"], 1e-5 * r["babs"] + C_FLOOR * U32 * r["wx"] + 1e-300, f"{name} range forward")
    # backprojections
    yd = torch.as_tensor(y, device=DEV)
    for mode in ("atomic", "fixed", "shadow", "gather", "atomic_direct"):
        ref, tol = backprojection_reference(c.orc, None, c.H, ids, float_atomic=mode in FLOAT_ATOMIC, r=r)
        bp = c.to_user(c.P.backproject_range(yd, a0, na, mode=mode)).astype(np.float64)
        assert_within(bp, ref, tol, f"{name} range backprojection {mode}")
        assert np.linalg.norm(bp - ref) <= 1e-5 * np.linalg.norm(ref), mode
    check_stats(c.mesh)


# ---------------------------------------------------------------- edges
def test_ragged_detector_and_missing_rays():
    c = case("ragged")
    ids = np.arange(c.orc.nrays)
    compare_traces(c.P.trace(ids), c.orc.trace(ids), c.H)
    xi = c.x_internal(c.w.x)
    got = c.P.forward(xi).cpu().numpy().ravel()
    ref, tol = forward_reference(c.orc, c.w.x, c.H)
    assert (ref == 0).sum() > 0, "geometry should include rays that miss"
    assert np.all(got[ref == 0] == 0)
    assert_within(got, ref, tol, "ragged forward")
    y = np.random.default_rng(3).uniform(0, 1, c.orc.nrays).astype(f32)
    ref_bp = c.orc.backproject(y)
    for mode in ("gather", "shadow"):
        bp = c.to_user(c.P.backproject(torch.as_tensor(y, device=DEV), mode=mode))
        assert np.linalg.norm(bp - ref_bp) <= 1e-5 * np.linalg.norm(ref_bp), mode
    assert_within(bp.astype(np.float64), ref_bp, _bp_tolerance(c, y, "shadow"), "ragged shadow backprojection")
    check_stats(c.mesh)


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_full_size_fixed_reproducible_adjoint_and_atomic_agreement(name):
    """Full-size reproducible scatter in the launch the benchmark's
    backprojection uses: the same bits twice, the adjoint identity against
    the forward projection, and agreement with the float scatter."""
    c = case(name)
    rng = np.random.default_rng(6)
    xi = c.x_internal(c.w.x.astype(f32))
    Ax = c.P.forward(xi).reshape(-1)
    y = torch.as_tensor(rng.uniform(0, 1, c.geom.nrays).astype(f32), device=DEV)
    fx = c.P.backproject(y, mode="fixed")
    fx2 = c.P.backproject(y, mode="fixed")
    assert torch.equal(fx, fx2)
    at = c.P.backproject(y, mode="atomic")
    lhs = float(torch.dot(Ax.double(), y.double()))
    rhs = float(torch.dot(xi.double(), fx.double()))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs), (lhs, rhs)
    err = (fx.double() - at.double()).abs()
    assert float(err.max()) <= 2e-4 * float(at.double().abs().max()), float(err.max())
    assert float(err.norm()) <= 2e-5 * float(at.double().norm())
    check_stats(c.mesh)


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_full_size_shadow_adjoint_and_atomic_agreement(name):
    """Full-size element-driven backprojection, in the launch the benchmark
    times: adjoint identity against the (oracle-checked) forward projection,
    and agreement with the ray-driven scatter element by element."""
    c = case(name)
    rng = np.random.default_rng(5)
    x = c.w.x.astype(f32)
    xi = c.x_internal(x)
    Ax = c.P.forward(xi).reshape(-1)
    y = torch.as_tensor(rng.uniform(0, 1, c.geom.nrays).astype(f32), device=DEV)
    sh = c.P.backproject(y, mode="shadow")
    sh2 = c.P.backproject(y, mode="shadow")
    assert torch.equal(sh, sh2)
    at = c.P.backproject(y, mode="atomic")
    lhs = float(torch.dot(Ax.double(), y.double()))
    rhs = float(torch.dot(xi.double(), sh.double()))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs), (lhs, rhs)
    # The scatter sums ~10^4 float32 terms per element in a run-dependent
    # order, so the bar here is its own rounding, not the oracle's.
    err = (sh.double() - at.double()).abs()
    assert float(err.max()) <= 2e-4 * float(at.double().abs().max()), float(err.max())
    assert float(err.norm()) <= 2e-5 * float(at.double().norm())
    check_stats(c.mesh)


def test_shadow_range_launches_sum_to_full():
    from paper_1908_06909_amd._lib import TCT_BP_SHADOW, call, tct_range
    import ctypes
    c = case("graded_small")
    y = torch.as_tensor(np.random.default_rng(6).uniform(0, 1, c.orc.nrays).astype(f32), device=DEV)
    full = c.P.backproject(y, mode="shadow")
    acc = torch.zeros_like(full)
    s = torch.cuda.current_stream().cuda_stream
    na = c.geom.na
    for a0, cnt in ((0, 5), (5, 1), (6, na - 6)):
        call("tct_backproject_range", c.mesh.handle, c.geom.handle, y.data_ptr(), acc.data_ptr(), TCT_BP_SHADOW, 1,
             None, ctypes.byref(tct_range(a0, cnt, 8)), s)
    assert torch.allclose(acc, full, rtol=1e-6, atol=1e-6)


def test_geometry_rejected_when_mesh_not_between_source_and_detector():
    tct = _gpu()
    X = synth.kuhn_nodes(2)
    verts, tets = synth.kuhn_mesh(X, X, X)
    m = tct.TetMesh(verts * f32(10), tets, device=DEV)
    g = tct.ConeGeometry(synth.Cone(4.0, 8.0, 8, 8, 0.25, 0.25), synth.angles_for(2), device=DEV)
    with pytest.raises(tct._lib.TctError) as e:
        tct.Projector(m, g)
    assert e.value.status == -6


def test_delaunay_sequences_projection_and_backprojections():
    """Unstructured mesh (random-point Delaunay, slivers included): sequences
    bit-exact, forward and all backprojections within tolerance."""
    c = case("delaunay")
    ids = np.arange(c.orc.nrays)
    compare_traces(c.P.trace(ids), c.orc.trace(ids), c.H)
    xi = c.x_internal(c.w.x)
    got = c.P.forward(xi).cpu().numpy().ravel()
    ref, tol = forward_reference(c.orc, c.w.x, c.H)
    assert_within(got, ref, tol, "delaunay forward")
    y = np.random.default_rng(7).uniform(-1, 1, c.orc.nrays).astype(f32)
    ref_bp = c.orc.backproject(y)
    for mode in ("atomic", "gather", "shadow"):
        bp = c.to_user(c.P.backproject(torch.as_tensor(y, device=DEV), mode=mode)).astype(np.float64)
        assert_within(bp, ref_bp, _bp_tolerance(c, y, mode), f"delaunay backprojection {mode}")
    check_stats(c.mesh)


def _candidate_rays(c, tet_ids):
    """Every ray whose pixel centre lies in the bounding box of a listed
    tetrahedron's central projection (widened by a hundredth of a pixel):
    a superset of the rays that cross it, computed in float64 from the
    oracle's frames, independent of the GPU path."""
    S, D, U, V, ut, vt = oracle.frame(c.w.cone, c.w.angles)
    nu, nv, na = c.w.cone.nu, c.w.cone.nv, len(c.w.angles)
    du = (float(ut[-1]) - float(ut[0])) / (nu - 1)
    dv = (float(vt[-1]) - float(vt[0])) / (nv - 1)
    per_tet = []
    for t in tet_ids:
        P4 = c.w.verts[c.w.tets[t]].astype(np.float64)
        ids = []
        for a in range(na):
            s, d, u, v = (x[a].astype(np.float64) for x in (S, D, U, V))
            N = np.cross(u, v)
            rel = P4 - s
            X = s + ((d - s) @ N / (rel @ N))[:, None] * rel - d
            uu, vv = X @ u / (u @ u), X @ v / (v @ v)
            i0 = max(0, int(np.ceil((uu.min() - ut[0]) / du - 0.01)))
            i1 = min(nu - 1, int(np.floor((uu.max() - ut[0]) / du + 0.01)))
            j0 = max(0, int(np.ceil((vv.min() - vt[0]) / dv - 0.01)))
            j1 = min(nv - 1, int(np.floor((vv.max() - vt[0]) / dv + 0.01)))
            if i0 > i1 or j0 > j1:
                continue
            jj, ii = np.meshgrid(np.arange(j0, j1 + 1), np.arange(i0, i1 + 1), indexing="ij")
            ids.append(((a * nv + jj) * nu + ii).ravel())
        per_tet.append(np.concatenate(ids))
    return per_tet


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_full_size_sampled_backprojection_against_oracle(name):
    """Full-size backprojections (every mode, the scatter in the launch the
    benchmark times), checked element by element against the oracle on
    sampled tetrahedra: the oracle
    backprojects only the rays whose pixels lie under each sampled element's
    shadow, which contains every ray that crosses it, so its value for that
    element is exact."""
    c = case(name)
    rng = np.random.default_rng(12)
    tets = rng.choice(c.orc.nt, 8, replace=False)
    per_tet = _candidate_rays(c, tets)
    ids = np.unique(np.concatenate(per_tet))
    y = rng.uniform(0.0, 1.0, c.orc.nrays).astype(f32)
    r = c.orc.check_pass(np.zeros(c.orc.nt, f32), c.H, y[ids], ids)
    yd = torch.as_tensor(y, device=DEV)
    for mode in ("atomic", "fixed", "shadow", "gather", "atomic_direct"):
        ref, tol = backprojection_reference(c.orc, None, c.H, ids, float_atomic=mode in FLOAT_ATOMIC, r=r)
        got = c.to_user(c.P.backproject(yd, mode=mode))[tets].astype(np.float64)
        print(f"{name} sampled {mode} backprojection: terms {r['cnt'][tets]}")
        assert_within(got, ref[tets], tol[tets], f"{name} sampled {mode} backprojection")
    check_stats(c.mesh)


def test_walk_failure_is_counted_and_reported():
    """Section II-C requires that a ray never halts unnoticed.  A custom ray
    whose tie-breaking axes do not span space together with its direction
    cannot be walked under the perturbation rule, so the library counts it
    as failed (and gives it an empty path) instead of walking it:
    tct_stats_read then returns TCT_E_WALK with the counters filled, and a
    reset clears them."""
    import ctypes

    from paper_1908_06909_amd._lib import lib, tct_stats

    tct = _gpu()
    X = synth.kuhn_nodes(2)
    verts, tets = synth.kuhn_mesh(X, X, X)
    m = tct.TetMesh(verts, tets, device=DEV)
    ex, ey, ez = np.eye(3, dtype=f32)
    S = np.array([[4, 0.1, 0.2], [4, 0.1, 0.2]], f32)
    P = np.array([[-4, 0.1, 0.2], [-4, 0.1, 0.2]], f32)
    U = np.array([ex, ey], f32)  # ray 0: U parallel to P - S
    V = np.array([ey, ez], f32)
    m.stats(reset=True)
    (t0, _), (t1, l1) = tct.trace_rays(m, S, P, U, V)
    assert len(t0) == 0 and len(t1) > 0
    assert abs(float(l1.sum()) - 1.0) <= 1e-6
    # tct_trace_rays walks every ray twice (once to size the lists, once to
    # fill them), and the counters count walks.
    st = tct_stats()
    assert lib().tct_stats_read(m.handle, ctypes.byref(st), 1) == -9
    assert st.failed == 2 and st.rays == 4
    assert lib().tct_stats_read(m.handle, ctypes.byref(st), 0) == 0
    assert st.failed == 0


@pytest.mark.parametrize("shape", ["sparse_rays", "long_lists"])
def test_gather_record_buffer_regrowth_and_long_lists(shape):
    """Explicit per-tetrahedron lists at their edges: a coarse detector on a
    fine mesh (few rays per wavefront, so nearly every segment is a record of
    its own: the record buffer sized from a guess overflows and the chunk is
    walked again with room for all), and a tiny mesh under a large detector
    (thousands of records per tetrahedron, beyond the in-LDS sort).  Both
    within the bars of the oracle and the same bits twice."""
    tct = _gpu()
    if shape == "sparse_rays":
        w = synth.jittered_kuhn(24, 41, 42, 5, 4, 6)
        w.cone = synth.Cone(4.0, 8.0, 5, 4, 0.37, 0.41, 0.01, 0.02)
    else:
        w = synth.jittered_kuhn(2, 43, 44, 192, 160, 24)
    orc = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    mesh = tct.TetMesh(w.verts, w.tets, device=DEV)
    geom = tct.ConeGeometry(w.cone, w.angles, device=DEV)
    P = tct.Projector(mesh, geom)
    H = element_size(w.verts, w.tets, orc.mesh.tables()[1])
    y = np.random.default_rng(45).uniform(-1, 1, orc.nrays).astype(f32)
    ref, tol = backprojection_reference(orc, y, H)
    yt = torch.as_tensor(y, device=DEV)
    a = P.backproject(yt, mode="gather")
    b = P.backproject(yt, mode="gather")
    assert torch.equal(a, b)
    got = mesh.to_user(a).cpu().numpy().astype(np.float64)
    assert_within(got, ref, tol, f"{shape} gather backprojection")
    assert mesh.stats(reset=True)["failed"] == 0
