"""Pins of the float64 reference solvers: the explicit matrix reproduces the
oracle's walks, the gradient matches central differences (exact for a
quadratic up to rounding), CGLS is monotone and reaches the least-squares
solution of the dense normal equations, SIRT decreases its weighted residual,
OS-SART reproduces a hand-worked iteration and converges on a consistent system."""

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


def test_os_sart_hand_worked_iteration():
    # A = [[1, 2], [3, 1]], b = (5, 5), subsets {row 0}, {row 1}, x0 = 0, lam = 1.
    # Row 0: R = 1/3, C = (1/1, 1/2): x = (1, 1/2) * (1, 2) * 5/3 = (5/3, 5/3).
    # Row 1: A_1 x = 20/3, residual -5/3, R = 1/4, C = (1/3, 1/1):
    #   x += (1/3, 1) * (3, 1) * (-5/12) = (-5/12, -5/12)  ->  x = (5/4, 5/4).
    import scipy.sparse as sp

    A = sp.csr_matrix(np.array([[1.0, 2.0], [3.0, 1.0]]))
    b = np.array([5.0, 5.0])
    x, rr = solvers.os_sart(A, b, 1, [[0], [1]])
    assert np.allclose(x, [1.25, 1.25], rtol=0, atol=1e-15)
    assert rr[0] == 50.0
    # second iteration, row 0: A_0 x = 15/4, r = 5/4, R = 1/3 -> x += (1, 1/2)(1, 2) 5/12 = 5/12 each
    x2, _ = solvers.os_sart(A, b, 2, [[0], [1]])
    # then row 1: A_1 x = 3 * 5/3 + 5/3 = 20/3 again -> the same correction -5/12 each
    assert np.allclose(x2, [1.25, 1.25], rtol=0, atol=1e-15)


def test_os_sart_converges_on_consistent_system(small):
    w, o, A = small
    rng = np.random.default_rng(4)
    xt = rng.uniform(0, 1, o.nt)
    b = A @ xt
    per_angle = w.cone.nu * w.cone.nv
    subsets = [np.arange(a * per_angle, (a + 2) * per_angle) for a in range(0, len(w.angles), 2)]
    x, rr = solvers.os_sart(A, b, 200, subsets)
    assert rr[-1] <= 1e-6 * rr[0]
    # with one subset holding every row it is SIRT
    xs, rrs = solvers.sirt(A, b, 5)
    x1, rr1 = solvers.os_sart(A, b, 5, [np.arange(o.nrays)])
    assert np.allclose(x1, xs, rtol=1e-12, atol=1e-14) and np.allclose(rr1, rrs, rtol=1e-12)


@pytest.fixture(scope="module")
def cfg0_system():
    w = synth.config(3)
    o = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    A = solvers.system_matrix(o)
    b = A @ synth.uniform_random(o.nt, w.meta["target_seed"]).astype(np.float64)
    return A, b


def test_cgls_float32_departs_from_float64(cfg0_system):
    """The CGLS recurrence with float32 vectors (the precision of the GPU
    solver) follows float64 CGLS to 1e-6 for ten iterations on the Kuhn 8^3 /
    64^2 x 16 system, then departs by tens of percent and more: rounding
    erodes the conjugacy of the search directions.  The departure is a
    property of float32 arithmetic, not of one rounding order: the same
    recurrence on the rows in another order departs the same way, while
    float64 CGLS is order-independent over the same early span."""
    A, b = cfg0_system
    iters = 50
    _, rr64, _ = solvers.cgls(A, b, iters)
    _, rr32, _ = solvers.cgls(A, b, iters, precision=32)
    ratio = rr32 / rr64
    print("float32 / float64 residuals every 5 iterations:", np.round(ratio[::5], 3))
    assert np.all(np.abs(ratio[:11] - 1) <= 1e-6), ratio[:11]
    assert np.max(np.abs(ratio[15:] - 1)) > 0.2
    assert np.all(np.diff(rr32) <= 0)  # still a descent method
    perm = np.random.default_rng(8).permutation(A.shape[0])
    _, rr32p, _ = solvers.cgls(A[perm], b[perm], iters, precision=32)
    spread = np.abs(rr32p / rr32 - 1)
    print(f"float32, rows permuted: largest relative change {spread.max():.3f}")
    assert np.all(spread <= 0.25)
    _, rr64p, _ = solvers.cgls(A[perm], b[perm], iters)
    assert np.all(np.abs(rr64p[:16] / rr64[:16] - 1) <= 1e-6)
