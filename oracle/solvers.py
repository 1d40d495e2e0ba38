"""Float64 reference solvers on the oracle's explicit system matrix.

TEST INFRASTRUCTURE ONLY.  The paper's operator A (Section II-A, Eq. 1:
a_ij = length of ray j inside tetrahedron i) is assembled explicitly from the
oracle's traced walks as a scipy sparse matrix, and the textbook algorithms
the paper names as consumers of A and A^T (CGLS, SART-family SIRT, and the
ordered-subset SART of its reconstructions, Section III-A) are written out
plainly in float64.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def system_matrix(orc, ids=None) -> sp.csr_matrix:
    """A restricted to the listed rays (all when None): rows = rays, columns = user tetrahedra."""
    ids = np.arange(orc.nrays) if ids is None else np.asarray(ids, np.int64)
    rows, cols, vals = [], [], []
    for k, (tt, ll) in enumerate(orc.trace(ids)):
        rows.append(np.full(len(tt), k, np.int64))
        cols.append(tt.astype(np.int64))
        vals.append(ll)
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    vals = np.concatenate(vals) if vals else np.zeros(0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(ids), orc.nt))


def loss(A, x, b) -> float:
    r = A @ x - b
    return 0.5 * float(r @ r)


def gradient(A, x, b) -> np.ndarray:
    """Gradient of 0.5 ||A x - b||^2: A^T (A x - b)."""
    return A.T @ (A @ x - b)


def cgls(A, b, iters: int, x0=None, precision: int = 64):
    """Conjugate gradients on A^T A x = A^T b (Hestenes-Stiefel form for least squares).

    precision=32 runs the same recurrence with float32 vectors: the matrix
    entries, b and every vector are float32, each product with A or A^T is
    accumulated in float64 and rounded to float32 (as a float32 projector
    returns it), and the inner products are float64 scalars.

    Returns (x, rr, xs) with rr[k] = ||b - A x_k||^2 (float64) for k = 0..iters
    and xs the iterates.
    """
    if precision == 64:
        vec = np.float64
        Am = A
    elif precision == 32:
        vec = np.float32
        Am = sp.csr_matrix(A, dtype=np.float32).astype(np.float64)
    else:
        raise ValueError("precision must be 32 or 64")

    def mv(M, v):
        return (M @ v.astype(np.float64)).astype(vec)

    def dot(a, c):
        return float(np.dot(a.astype(np.float64), c.astype(np.float64)))

    b = np.asarray(b).astype(vec)
    x = np.zeros(A.shape[1], vec) if x0 is None else np.array(x0, vec)
    r = (b - mv(Am, x)).astype(vec)
    s = mv(Am.T, r)
    p = s.copy()
    gamma = dot(s, s)
    rr = [dot(r, r)]
    xs = [x.copy()]
    for _ in range(iters):
        q = mv(Am, p)
        delta = dot(q, q)
        alpha = gamma / delta if delta != 0 else 0.0
        x = (x + vec(alpha) * p).astype(vec)
        r = (r - vec(alpha) * q).astype(vec)
        s = mv(Am.T, r)
        gamma_new = dot(s, s)
        beta = gamma_new / gamma if gamma != 0 else 0.0
        p = (s + vec(beta) * p).astype(vec)
        gamma = gamma_new
        rr.append(dot(r, r))
        xs.append(x.copy())
    return x, np.array(rr), xs


def sirt(A, b, iters: int, lam: float = 1.0, x0=None):
    """x += lam * C A^T R (b - A x), R = diag(1 / row sums), C = diag(1 / column sums).

    Returns (x, rr) with rr[k] = ||b - A x_k||^2 before iteration k.
    """
    row = np.asarray(A.sum(axis=1)).ravel()
    col = np.asarray(A.sum(axis=0)).ravel()
    R = np.where(row > 0, 1.0 / np.where(row > 0, row, 1.0), 0.0)
    Cw = np.where(col > 0, 1.0 / np.where(col > 0, col, 1.0), 0.0)
    x = np.zeros(A.shape[1]) if x0 is None else np.array(x0, np.float64)
    rr = []
    for _ in range(iters):
        r = b - A @ x
        rr.append(float(r @ r))
        x = x + lam * Cw * (A.T @ (R * r))
    return x, np.array(rr)


def os_sart(A, b, iters: int, subsets, lam: float = 1.0, x0=None):
    """Ordered-subset SART (the reconstructions of Section III-A: blocks of
    projections).  One iteration visits the row subsets in the given order;
    for subset k with rows A_k:

        x += lam * C_k A_k^T R_k (b_k - A_k x),
        R_k = diag(1 / row sums of A_k),  C_k = diag(1 / column sums of A_k),

    zero where a sum is zero.  Returns (x, rr) with rr[k] = ||b - A x_k||^2
    before iteration k.
    """
    A = sp.csr_matrix(A)
    parts = []
    for rows in subsets:
        rows = np.asarray(rows, np.int64)
        Ak = A[rows]
        row = np.asarray(Ak.sum(axis=1)).ravel()
        col = np.asarray(Ak.sum(axis=0)).ravel()
        R = np.where(row > 0, 1.0 / np.where(row > 0, row, 1.0), 0.0)
        Cw = np.where(col > 0, 1.0 / np.where(col > 0, col, 1.0), 0.0)
        parts.append((Ak, b[rows], R, Cw))
    x = np.zeros(A.shape[1]) if x0 is None else np.array(x0, np.float64)
    rr = []
    for _ in range(iters):
        r = b - A @ x
        rr.append(float(r @ r))
        for Ak, bk, R, Cw in parts:
            x = x + lam * Cw * (Ak.T @ (R * (bk - Ak @ x)))
    return x, np.array(rr)
