"""Pins of the oracle's implementation of the paper's own propagation
(Moller-Trumbore with the safety parameter, Algorithms 1-2):

* on a jittered mesh at generic angles its float64 result is the exact walk's
  projection, with no eps escalation, halt or loop;
* its float32 result agrees to the accuracy of float32 Moller-Trumbore there;
* the printed parallel test |a| < 1e-8 is absolute: on a mesh scaled down to
  1e-5 every face is rejected whatever eps, so every ray that enters halts
  after ten escalations (eps = 1e-9 ... 1 tried, then 10 > 1);
* on the uniform Kuhn mesh (rays through its vertices and along its edges)
  float32 escalates while float64 does not."""

import numpy as np

import oracle
import synth


def _jittered():
    # Boundary nodes are not jittered, so at the equispaced angles some rays
    # run inside boundary-cell face planes, where both algorithms are right
    # and pick different sides; a generic angle offset avoids such ties.
    w = synth.jittered_kuhn(4, 21, 22, 24, 24, 6)
    w.angles = np.asarray(w.angles, np.float64) + 0.1234
    return w, oracle.Oracle(w.verts, w.tets, w.cone, w.angles)


def test_float64_equals_exact_walk_on_generic_rays():
    w, o = _jittered()
    b = o.forward(w.x)
    bp, c = o.forward_paper(w.x, 64)
    assert c["escalations"] == 0 and c["halted"] == 0 and c["looped"] == 0
    assert c["rays"] == int((b != 0).sum())
    assert np.allclose(bp, b.astype(np.float32).astype(np.float64), rtol=1e-6, atol=1e-7)


def test_float32_agrees_to_float32_accuracy_on_generic_rays():
    w, o = _jittered()
    b = o.forward(w.x)
    bp, c = o.forward_paper(w.x, 32)
    assert c["halted"] == 0 and c["looped"] == 0
    # Float32 Moller-Trumbore measures t from the source: its error is a few
    # ulps of |S - P1| / |E1 x E2| relative, ~1e-4 of the projection here.
    assert np.max(np.abs(bp - b)) <= 2.0 ** -13 * np.max(np.abs(b))
    assert np.median(np.abs(bp - b)) <= 1e-6 * np.max(np.abs(b))


def test_absolute_parallel_threshold_halts_every_ray_on_a_tiny_mesh():
    X = synth.kuhn_nodes(2) * 1e-5
    verts, tets = synth.kuhn_mesh(X, X, X)
    cone = synth.Cone(4.0, 8.0, 8, 8, 2.5e-6, 2.5e-6)
    o = oracle.Oracle(verts, tets, cone, synth.angles_for(2))
    x = np.ones(len(tets), np.float32)
    b = o.forward(x)
    assert (b != 0).sum() > 0
    for prec in (32, 64):
        bp, c = o.forward_paper(x, prec)
        assert c["rays"] == int((b != 0).sum())
        # eps = 1e-9, 1e-8, ..., 1 (the product of nine x10 steps rounds to at
        # most 1 in both precisions) are all tried; the tenth step passes 1.
        assert c["halted"] == c["rays"] and c["escalations"] == 10 * c["rays"], c
        assert np.all(bp == 0)


def test_float32_escalates_on_the_uniform_kuhn_mesh_and_float64_does_not():
    w = synth.config(0)
    o = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    _, c64 = o.forward_paper(w.x, 64)
    _, c32 = o.forward_paper(w.x, 32)
    assert c64["escalations"] == 0
    assert c32["escalations"] > 0
