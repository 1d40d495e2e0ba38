"""Pins of the float64 reference solvers: the explicit matrix reproduces the
oracle's walks, the gradient matches central differences (exact for a
quadratic up to rounding), CGLS is monotone and reaches the least-squares
solution of the dense normal equations, SIRT decreases its weighted residual."""

import numpy as np
import pytest

import oracle
import synth
from oracle import solvers


@pytest.fixture(scope="module")
def small():
    w = synth.plain_kuhn(4, seed=5, nu=24, nv=24, na=8, pitch=2.0 / 24)
    w.x = synth.uniform_random(w.nt, 6)
    o = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    A = solvers.system_matrix(o)
    return w, o, A


def test_matrix_reproduces_walks(small):
    w, o, A = small
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, o.nt).astype(np.float32)
    y = rng.uniform(-1, 1, o.nrays).astype(np.float32)
    assert np.allclose(A @ x.astype(np.float64), o.forward(x), rtol=1e-12, atol=1e-13)
    assert np.allclose(A.T @ y.astype(np.float64), o.backproject(y), rtol=1e-12, atol=1e-12)
    # every stored entry is a non-negative length; row sums are chords
    assert A.data.min() >= 0


def test_gradient_matches_central_differences(small):
    w, o, A = small
    rng = np.random.default_rng(2)
    b = A @ rng.uniform(0, 1, o.nt)
    x = w.x.astype(np.float64)
    g = solvers.gradient(A, x, b)
    for _ in range(3):
        v = rng.normal(size=o.nt)
        h = 1e-3
        fd = (solvers.loss(A, x + h * v, b) - solvers.loss(A, x - h * v, b)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-8 * (abs(g @ v) + np.abs(g) @ np.abs(v))


def test_cgls_monotone_and_converges_to_least_squares(small):
    w, o, A = small
    rng = np.random.default_rng(3)
    b = A @ rng.uniform(0, 1, o.nt) + 0.01 * rng.normal(size=o.nrays)
    Ad = A.toarray()
    x_ls = np.linalg.lstsq(Ad, b, rcond=None)[0]
    x, rr, xs = solvers.cgls(A, b, 400)
    assert np.all(np.diff(rr) <= 1e-12 * rr[0])
    err = [np.linalg.norm(xk - x_ls) for xk in xs]
    assert np.all(np.diff(err) <= 1e-9 * err[0])
    assert np.linalg.norm(x - x_ls) <= 1e-6 * np.linalg.norm(x_ls)


def test_sirt_decreases_weighted_residual(small):
    w, o, A = small
    rng = np.random.default_rng(4)
    b = A @ rng.uniform(0, 1, o.nt)
    x, rr = solvers.sirt(A, b, 30)
    assert rr[-1] < 0.1 * rr[0]
    row = np.asarray(A.sum(axis=1)).ravel()
    R = np.where(row > 0, 1 / np.where(row > 0, row, 1), 0)
    # the R-weighted residual is non-increasing for lam in (0, 2)
    x = np.zeros(o.nt)
    prev = np.inf
    col = np.asarray(A.sum(axis=0)).ravel()
    C = np.where(col > 0, 1 / np.where(col > 0, col, 1), 0)
    for _ in range(20):
        r = b - A @ x
        cur = float(r @ (R * r))
        assert cur <= prev * (1 + 1e-12)
        prev = cur
        x = x + C * (A.T @ (R * r))
