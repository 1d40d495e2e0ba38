"""The walk's float32 sign filters, run on the CPU, against exact signs.

The walk decides which face a ray leaves a tetrahedron by from three edge
signs E(v, a) = det[P - S, v - S, a - S] (Section II-C: the sign decisions
that must not fail on rays through vertices and edges).  The kernels take a
float32 estimate whenever a certified error bound says its sign is right and
hand everything else to float64 and exact arithmetic.  The certification
rests on hand-derived constants (walk_filter.h: 72 u and 192 u^2 R per unit
of |e|_inf for the step, 10 u for the entry test, the error of the float64 offset from the
ray).  These tests compile that header for the host (tests/filter_probe.cpp)
and check, over a million adversarial inputs, that every sign it certifies
equals the exact sign the oracle computes:

  * realistic walk states traced by the oracle on uniform Kuhn meshes (rays
    through vertices, along edges, inside face planes), graded slivers,
    jittered and Delaunay meshes, and a source 2^12 away;
  * the same states with one coordinate moved by one ulp (tiny non-zero
    determinants), and scaled by powers of two down to the underflow range;
  * offsets taken from far points of the ray, not only from the entry point.

A copy of the filter built with its bounds divided by 2^12 must fail the
same check: the inputs do reach the certified band's edge.
"""

import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
f32 = np.float32
u = 2.0 ** -24


def _build_probe(tag, extra):
    import ctypes as C

    os.makedirs(BUILD, exist_ok=True)
    out = os.path.join(BUILD, f"libfilter_probe{tag}.so")
    src = os.path.join(HERE, "filter_probe.cpp")
    hdrs = [os.path.join(ROOT, "paper_1908_06909_amd", "csrc", h) for h in ("walk_filter.h", "common.h")]
    if not os.path.exists(out) or os.path.getmtime(out) < max(os.path.getmtime(f) for f in [src, *hdrs]):
        cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-x", "hip", "--offload-arch=gfx950", "-O2",
               "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-rdc",
               "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "paper_1908_06909_amd", "csrc"),
               "-I", os.path.join(ROOT, "include"), *extra, src, "-o", out + ".tmp"]
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(out + ".tmp", out)
    L = C.CDLL(out)
    P = np.ctypeslib.ndpointer
    f3 = P(np.float32, flags="C_CONTIGUOUS")
    f8 = P(np.float64, flags="C_CONTIGUOUS")
    i4 = P(np.int32, flags="C_CONTIGUOUS")
    L.probe_step.argtypes = [C.c_longlong, f3, f3, f3, f8, f3, f3, f3, f3, i4, i4, i4]
    L.probe_step.restype = None
    L.probe_entry.argtypes = [C.c_longlong, f3, f3, f3, f3, f3, i4]
    L.probe_entry.restype = None
    L.probe_offset.argtypes = [C.c_longlong, f3, f3, f3, f8, f3, f3, f3, f3]
    L.probe_offset.restype = None
    L.probe_exit_table.argtypes = [C.c_int]
    L.probe_xcd_block.argtypes = [C.c_longlong, C.c_longlong]
    L.probe_xcd_block.restype = C.c_longlong
    L.probe_loc_remap.argtypes = [C.c_uint]
    L.probe_loc_remap.restype = C.c_uint
    return L


@pytest.fixture(scope="module")
def probe():
    return _build_probe("", [])


@pytest.fixture(scope="module")
def weak_probe():
    return _build_probe("_weak", ["-DTCT_FILTER_BOUND_SCALE=0x1p-12f"])


# ---------------------------------------------------------------- inputs
class Steps:
    """Walk states: ray S -> P, mesh extent, vertex v, entry-face slots a0..a2, parameter s."""

    def __init__(self, S, P, ext, v, a0, a1, a2, s):
        self.S, self.P, self.ext = S, P, ext
        self.v, self.a = v, (a0, a1, a2)
        self.s = s

    def __len__(self):
        return len(self.v)

    @staticmethod
    def cat(parts):
        return Steps(*[np.concatenate([getattr(p, k) for p in parts]) for k in ("S", "P", "ext", "v")],
                     *[np.concatenate([p.a[i] for p in parts]) for i in range(3)],
                     np.concatenate([p.s for p in parts]))


def _closest_s(S, P, v):
    d = P.astype(np.float64) - S
    t = np.einsum("ij,ij->i", v.astype(np.float64) - S, d) / np.einsum("ij,ij->i", d, d)
    return np.clip(t - 0.5, -0.5, 0.5)


def _steps_from_paths(verts, tets, paths, S, P, rng, far_fraction=0.1):
    """Every step after the first of every traced ray: the new vertex v of
    the tetrahedron and the three vertices of the face the ray came in by."""
    prev, cur, ray = [], [], []
    for j, (tt, _) in enumerate(paths):
        if len(tt) > 1:
            prev.append(tt[:-1])
            cur.append(tt[1:])
            ray.append(np.full(len(tt) - 1, j))
    prev, cur, ray = (np.concatenate(x) for x in (prev, cur, ray))
    P4, C4 = tets[prev], tets[cur]
    shared = (C4[:, :, None] == P4[:, None, :]).any(axis=2)
    assert np.all(shared.sum(axis=1) == 3)
    vi = np.argmin(shared, axis=1)
    order = np.argsort(~shared, axis=1, kind="stable")[:, :3]  # the three shared vertices, in order
    face = np.take_along_axis(C4, order, axis=1)
    v = verts[C4[np.arange(len(C4)), vi]]
    a0, a1, a2 = (verts[face[:, k]] for k in range(3))
    Sr, Pr = S[ray], P[ray]
    s = _closest_s(Sr, Pr, v)
    far = rng.random(len(s)) < far_fraction
    s[far] = rng.uniform(-0.5, 0.5, far.sum())
    ext = np.full(len(v), float(np.abs(verts).max()), f32)
    return Steps(Sr, Pr, ext, v, a0, a1, a2, s)


def _pixel_steps(w, stride, rng):
    orc = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    ids = np.arange(0, orc.nrays, stride)
    S, P, _, _ = orc.rays(ids)
    return _steps_from_paths(w.verts, w.tets, orc.trace(ids), S, P, rng)


def _axis_rays():
    """Rays along vertex lines, inside face planes and through the cube
    diagonal of a uniform Kuhn mesh (every kind of exact tie)."""
    ex, ey, ez = np.eye(3, dtype=f32)
    rays = []
    for y in (-0.25, 0.0, 0.125, 0.25):
        for z in (-0.25, 0.0, 0.25, 0.3):
            rays.append((np.array([4, y, z], f32), np.array([-4, y, z], f32), ey, ez))
            rays.append((np.array([y, -4, z], f32), np.array([y, 4, z], f32), ez, ex))
            rays.append((np.array([y, z, 4], f32), np.array([y, z, -4], f32), ex, -ey))
    for U, V in ((ex, ey), (ey, ex), (ez, ex)):
        rays.append((np.array([-2, -2, -2], f32), np.array([2, 2, 2], f32), U, V))
        rays.append((np.array([-2, -2, 0], f32), np.array([2, 2, 0], f32), U, V))
        rays.append((np.array([-2, 0.25, -2], f32), np.array([2, 0.25, 2], f32), U, V))
    rays = [r for r in rays if np.linalg.det(np.array([r[1] - r[0], r[2], r[3]], np.float64)) != 0]
    return [np.array([r[k] for r in rays], f32) for k in range(4)]


_cache = {}


def base_steps():
    if "base" in _cache:
        return _cache["base"]
    rng = np.random.default_rng(2024)
    parts = []
    # uniform Kuhn meshes: pixel rays through projected vertices and edges
    parts.append(_pixel_steps(synth.plain_kuhn(4, 3, 33, 33, 8, pitch=2.0 ** -4), 1, rng))
    parts.append(_pixel_steps(synth.config(0), 3, rng))
    # custom rays along vertex lines and face planes
    X = synth.kuhn_nodes(4)
    verts, tets = synth.kuhn_mesh(X, X, X)
    S, P, U, V = _axis_rays()
    om = oracle.OracleMesh(verts, tets)
    parts.append(_steps_from_paths(verts, tets, oracle.oracle.trace_rays(om, S, P, U, V), S, P, rng))
    # graded slivers (aspect ratios ~1e3 at full size), z axis a vertex column
    (gv, gt), _, _ = synth.graded_mesh(24, 8, 1.05, 17)
    du = 2.0 ** -5
    parts.append(_pixel_steps(synth.Workload("graded24", gv, gt, synth.uniform_random(len(gt), 1),
                                             synth.Cone(4.0, 8.0, 64, 64, du, du, du / 2, du / 2),
                                             synth.angles_for(12)), 2, rng))
    # jittered and Delaunay meshes
    parts.append(_pixel_steps(synth.jittered_kuhn(6, 5, 6, 48, 48, 6), 1, rng))
    dv, dt = synth.delaunay_mesh(2000, 3)
    parts.append(_pixel_steps(synth.Workload("delaunay", dv, dt, synth.uniform_random(len(dt), 2),
                                             synth.Cone(4.0, 8.0, 40, 40, 0.05, 0.05, 0.003, -0.002),
                                             synth.angles_for(5)), 1, rng))
    # a source 2^12 away: the 192 u^2 R term of the walk bound
    far = synth.plain_kuhn(8, 0, 48, 48, 6, pitch=2.0 ** -5)
    far.cone = synth.Cone(4096.0, 8192.0, 48, 48, 2.0 ** -5, 2.0 ** -5, 0.0, 0.0)
    parts.append(_pixel_steps(far, 1, rng))
    _cache["base"] = Steps.cat(parts)
    return _cache["base"]


def _nudge(x, rng):
    """One coordinate of each point moved by one ulp up or down."""
    x = x.copy()
    k = rng.integers(0, 3, len(x))
    up = rng.random(len(x)) < 0.5
    rows = np.arange(len(x))
    x[rows, k] = np.where(up, np.nextafter(x[rows, k], f32(np.inf)), np.nextafter(x[rows, k], f32(-np.inf)))
    return x


def adversarial_steps():
    if "adv" in _cache:
        return _cache["adv"]
    rng = np.random.default_rng(7)
    b = base_steps()
    ex = _exact_step(b)
    ties = np.any(ex == 0, axis=1)
    parts = [b]
    # tiny non-zero determinants: one-ulp moves of v, or of one slot, on every tie and a sample of the rest
    pick = ties | (rng.random(len(b)) < 0.1)
    for which in ("v", 0, 1, 2):
        a = [x[pick] for x in b.a]
        v = b.v[pick]
        if which == "v":
            v = _nudge(v, rng)
        else:
            a[which] = _nudge(a[which], rng)
        parts.append(Steps(b.S[pick], b.P[pick], b.ext[pick], v, *a, b.s[pick]))
    # exact power-of-two scalings, down to where the products underflow
    sel = np.flatnonzero(rng.random(len(b)) < 0.04)
    for e in (-44, -40, -30, -12, 12, 30):
        f = f32(2.0 ** e)
        parts.append(Steps(b.S[sel] * f, b.P[sel] * f, b.ext[sel] * f, b.v[sel] * f, *[x[sel] * f for x in b.a],
                           b.s[sel]))
    _cache["adv"] = Steps.cat(parts)
    return _cache["adv"]


def _exact_step(st):
    """Exact signs of E(v, a_k) = det[P - S, v - S, a_k - S], [n, 3]."""
    return np.stack([oracle.oracle.det_sign_batch(st.P, st.S, st.v, st.S, a, st.S) for a in st.a], axis=1)


def _run_step(probe, st):
    n = len(st)
    edge = np.zeros(3 * n, np.int32)
    common = np.zeros(n, np.int32)
    fsign = np.zeros(3 * n, np.int32)
    c = np.ascontiguousarray
    probe.probe_step(n, c(st.S), c(st.P), c(st.ext), c(st.s), c(st.v), *[c(a) for a in st.a], edge, common, fsign)
    return edge.reshape(n, 3), common, fsign.reshape(n, 3)


def _step_violations(probe, st):
    ex = _exact_step(st)
    edge, common, fsign = _run_step(probe, st)
    wrong_edge = (edge != 0) & (edge != ex)
    settled = common >= 0
    wrong_common = settled & np.any(fsign != ex, axis=1)
    return ex, edge, common, wrong_edge, wrong_common


# ---------------------------------------------------------------- tests
def test_exit_table_encodes_the_exit_rule(probe):
    for n in range(8):
        assert probe.probe_exit_table(n) >= 0, n


def test_walk_step_filter_certifies_only_exact_signs(probe):
    st = adversarial_steps()
    ex, edge, common, wrong_edge, wrong_common = _step_violations(probe, st)
    n_signs = ex.size
    zeros = int((ex == 0).sum())
    certified = int((edge != 0).sum())
    print(f"step filter: {len(st)} walk states, {n_signs} signs, {zeros} exact zeros, "
          f"{certified / n_signs:.4f} certified per edge, {(common >= 0).mean():.4f} settled by the shared bound")
    assert n_signs >= 1_000_000
    assert zeros > 1000  # the inputs do contain exact ties
    assert not wrong_edge.any(), np.flatnonzero(wrong_edge.any(axis=1))[:10]
    assert not wrong_common.any(), np.flatnonzero(wrong_common)[:10]
    # exact zeros are never certified, by either path
    assert not np.any((ex == 0) & (edge != 0))
    assert not np.any(np.any(ex == 0, axis=1) & (common >= 0))
    # the filter is not vacuous: most signs of ordinary steps are settled in float32
    assert (common[: len(base_steps())] >= 0).mean() > 0.9


def test_entry_filter_certifies_only_exact_signs(probe):
    st = adversarial_steps()
    c = np.ascontiguousarray
    bad = 0
    total = 0
    zeros = 0
    cert = 0
    for p, q in ((st.a[0], st.a[1]), (st.a[1], st.a[2]), (st.a[2], st.a[0]), (st.v, st.a[0])):
        n = len(p)
        out = np.zeros(n, np.int32)
        probe.probe_entry(n, c(st.S), c(st.P), c(st.ext), c(p), c(q), out)
        ex = oracle.oracle.det_sign_batch(st.P, st.S, p, st.S, q, st.S)
        certified = out != 2
        bad += int((certified & (out != ex)).sum())
        total += n
        zeros += int((ex == 0).sum())
        cert += int(certified.sum())
    print(f"entry filter: {total} signs, {zeros} exact zeros, {cert / total:.4f} certified")
    assert total >= 1_000_000 and zeros > 1000
    assert bad == 0
    assert cert / total > 0.5


def test_offset_from_ray_error_bound(probe):
    """|D - (v - Q)| <= u |D| + 2^-51 R per component, Q = S + (1/2 + s)(P - S)
    exactly, R bounding the coordinates of S, P and the mesh plus |P - S|_inf."""
    st = adversarial_steps()
    rng = np.random.default_rng(3)
    sel = rng.choice(len(st), 4000, replace=False)
    n = len(sel)
    c = np.ascontiguousarray
    S, P, ext, v, s = (c(x[sel]) for x in (st.S, st.P, st.ext, st.v, st.s))
    D = np.zeros((n, 3), np.float32)
    kA = np.zeros(n, np.float32)
    kB = np.zeros(n, np.float32)
    probe.probe_offset(n, S, P, ext, s, v, D, kA, kB)
    worst = 0.0
    for k in range(n):
        R = max(float(np.abs(S[k]).max()), float(np.abs(P[k]).max()), float(ext[k])) + \
            float(np.abs(P[k].astype(np.float64) - S[k]).max())
        t = Fraction(0.5) + Fraction(float(s[k]))
        for i in range(3):
            exact = Fraction(float(v[k, i])) - Fraction(float(S[k, i])) - t * (
                Fraction(float(P[k, i])) - Fraction(float(S[k, i])))
            err = abs(Fraction(float(D[k, i])) - exact)
            bound = Fraction(u) * abs(Fraction(float(D[k, i]))) + Fraction(2.0 ** -51) * Fraction(R)
            assert err <= bound, (k, i, float(err), float(bound))
            worst = max(worst, float(err / bound))
    print(f"offset error: worst {worst:.3f} of its bound over {3 * n} components")


def test_weakened_filter_is_caught(weak_probe):
    """The same inputs against the filter with its bounds divided by 2^12:
    the check must find wrong certified signs, so it does reach the edge of
    the certified band."""
    st = adversarial_steps()
    _, _, _, wrong_edge, wrong_common = _step_violations(weak_probe, st)
    print(f"weakened filter: {int(wrong_edge.sum())} wrong per-edge signs, {int(wrong_common.sum())} wrong settled steps")
    assert wrong_edge.any() and wrong_common.any()


@pytest.mark.parametrize("n", [1, 7, 8, 9, 63, 1000, 1024 * 45 + 5])
def test_xcd_block_order_is_a_bijection_with_one_run_per_die(probe, n):
    """The walks' XCD-aware block order (common.h): a permutation of the
    launch's blocks in which the blocks dispatched to each die (b mod 8)
    form one contiguous run of the logical order, in dispatch order."""
    L = np.array([probe.probe_xcd_block(b, n) for b in range(n)], np.int64)
    assert np.array_equal(np.sort(L), np.arange(n))
    for x in range(8):
        run = L[x::8]
        if len(run):
            assert np.array_equal(run, np.arange(run[0], run[0] + len(run)))


def test_local_index_remap_table_follows_sorted_ranks(probe):
    """The library numbers an element's vertices by ascending node id (mesh
    ingest), so a vertex's local index is its rank among the element's four
    node ids, and face neighbours share three of them (Section II-B, Fig. 1).
    Every entry of the remap table the walks read, for every slot order, exit
    slot k and rank of the new vertex, must give the ranks of the slots in the
    neighbour across the face opposite slot k: slot k takes the old v, v the
    neighbour's new vertex."""
    rng = np.random.default_rng(5)
    import itertools

    n = 0
    for perm in itertools.permutations(range(4)):
        for k in range(3):
            for back in range(4):
                # Four ids of the current element, sorted; slot s holds rank perm[s].
                ids = np.sort(rng.choice(1000, 4, replace=False)) * 4 + 4
                slots = [int(ids[p]) for p in perm]  # a0, a1, a2, v
                gone = slots[k]
                shared = sorted(x for x in ids.tolist() if x != gone)
                # A new vertex whose rank among the neighbour's ids is `back`.
                lo = shared[back - 1] if back > 0 else 0
                hi = shared[back] if back < 3 else 10 ** 6
                w = (lo + hi) // 2
                assert lo < w < hi
                nb = sorted(shared + [w])
                new_slots = slots[:3] + [w]
                new_slots[k] = slots[3]
                want = sum(nb.index(x) << (2 * s) for s, x in enumerate(new_slots))
                loc = sum(p << (2 * s) for s, p in enumerate(perm))
                assert probe.probe_loc_remap((loc * 3 + k) * 4 + back) == want
                n += 1
    assert n == 288
