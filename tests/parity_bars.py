"""Parity bars of the GPU tests (float32 library against the float64 oracle).

chord_j is ray j's length inside the mesh (the sum of its oracle lengths)
and H_t the element size of tetrahedron t: the longest edge of t and of its
face neighbours.  "Visits" are the oracle's sequence entries, zero-length
passages included.

  * sequences, zero-length passages included: identical;
  * segment lengths: |dL| <= 1e-5 chord_j + C u H_t;
  * projections: |db_j| <= 1e-5 sum_i a_ij |x_i| + C u max_i (H_i |x_i|)
    over the tetrahedra the ray visits; misses exactly 0;
  * backprojections, per element: |dxhat_i| <= 1e-5 sum_j chord_j |y_j|
    + C u H_i sum_j |y_j| over the rays j that visit i; the float32-atomic
    modes add n_i 2^-24 (A^T |y|)_i for their float32 accumulation of the
    n_i terms in arrival order; and l2-relative <= 1e-5;
  * adjoint: |<Ax, y> - <x, A^T y>| <= 1e-5 <|A||x|, |y|>.

Why the C u H term (u = 2^-24, C = 256).  The walk keeps the ray parameter
in float64 and forms, per step, the offset D = v - Q of the element's fourth
vertex from the entry point Q in float64, rounded once to float32 (an error
of u |D| + 2^-51 R, |D| <= H).  The exit crossing is D.n / d.n with the face
normal n a float32 cross product of two edges: the crossing point moves
along the ray by about 5 u |D| / (cos phi sin alpha), phi the angle between
the ray and n, alpha the face's smallest angle (the normal's relative
rounding); the walk recomputes it in float64 when cos phi < 1/128.  A
segment's length is the difference of two crossings, each computed in the
element or its neighbour, and a zero-length passage can come out as a
length of that size.  Such errors are a multiple of u times the element
size, not of the chord: on a ray that clips the hull with a chord shorter
than an element, 1e-5 chord_j alone is below the rounding of one crossing.
C = 256 covers both crossings of a segment down to cos phi sin alpha = 1/25;
the tests print the largest |dL| / (u H) they see (145 at most over the
twenty million segments of the full-size and small workloads).  Crossing
errors enter a projection telescoped, sum_k delta_k (x_k - x_{k+1}), which
the 1e-5 term covers for rays of several elements; the max term covers one
crossing pair on short chords.
"""

from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24
C_FLOOR = 256.0


def element_size(verts, tets, nbrs) -> np.ndarray:
    """H_t: the longest edge of tetrahedron t and of its face neighbours (float64)."""
    P = np.asarray(verts, np.float64)[np.asarray(tets)]
    h = np.zeros(len(P))
    for a in range(4):
        for b in range(a + 1, 4):
            h = np.maximum(h, np.linalg.norm(P[:, a] - P[:, b], axis=1))
    H = h.copy()
    nb = np.asarray(nbrs)
    for k in range(4):
        m = nb[:, k] >= 0
        H[m] = np.maximum(H[m], h[nb[m, k]])
    return H


def length_tolerance(tets_seq, lens_ref, H):
    """Per-segment bar of one ray."""
    return 1e-5 * float(np.sum(lens_ref)) + C_FLOOR * U32 * H[tets_seq]


def compare_traces(gpu, ref, H, what="segment lengths"):
    """Sequences identical and every length within the bar; prints the worst
    ratio to the bar and the largest |dL| / (u H) seen."""
    assert len(gpu) == len(ref)
    worst = 0.0
    worst_uh = 0.0
    for k, ((gt, gl), (rt, rl)) in enumerate(zip(gpu, ref)):
        assert np.array_equal(gt, rt), f"ray {k}: sequences differ\n gpu {gt[:40]}\n ref {rt[:40]}"
        if not len(rl):
            continue
        err = np.abs(gl.astype(np.float64) - rl)
        tol = length_tolerance(rt, rl, H)
        i = int(np.argmax(err / tol))
        assert np.all(err <= tol), (
            f"ray {k}: lengths; chord {rl.sum():.6e} n {len(rl)} worst seg {i} gpu {gl[i]:.9e} ref {rl[i]:.9e} "
            f"err {err[i]:.3e} tol {tol[i]:.3e}; all gpu {gl[:8]} ref {rl[:8]}")
        worst = max(worst, float(np.max(err / tol)))
        worst_uh = max(worst_uh, float(np.max(err / (U32 * H[rt]))))
    print(f"{what}: worst err/tol {worst:.3f}, worst err/(u H) {worst_uh:.2f} over {len(gpu)} rays")


def forward_reference(orc, x, H, ids=None):
    """(oracle projection, its bar) for the listed rays (all when None)."""
    ids = np.arange(orc.nrays) if ids is None else np.asarray(ids)
    r = orc.check_pass(x, H, np.zeros(len(ids), np.float32), ids)
    return r["b"], 1e-5 * r["babs"] + C_FLOOR * U32 * r["wx"] + 1e-300


def backprojection_reference(orc, y, H, ids=None, float_atomic=False, r=None):
    """(oracle backprojection, its per-element bar) over the listed rays, y per
    listed ray (or the check pass r already run on them)."""
    ids = np.arange(orc.nrays) if ids is None else np.asarray(ids)
    if r is None:
        r = orc.check_pass(np.zeros(orc.nt, np.float32), H, y, ids)
    tol = 1e-5 * r["suppc"] + C_FLOOR * U32 * H * r["supp"] + 1e-300
    if float_atomic:
        tol = tol + r["cnt"] * U32 * r["xabs"]
    return r["xhat"], tol


def assert_within(got, ref, tol, what):
    got = np.asarray(got, np.float64)
    err = np.abs(got - ref)
    bad = err > tol
    if bad.any():
        k = int(np.argmax(err / np.maximum(tol, 1e-300)))
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} out of tolerance; worst index {k}: "
                             f"got {got[k]!r} ref {ref[k]!r} err {err[k]:.3e} tol {tol[k]:.3e}")
    print(f"{what}: worst err/tol {float(np.max(err / np.maximum(tol, 1e-300))) if err.size else 0.0:.3f}")
