"""Independent exact checkers written with Python Fractions.

These share nothing with the oracle's C++ code: they restate the definitions
(system-matrix entry a_ij = length of ray j inside tetrahedron i, paper
Section II-A, Eq. 1) in exact rational arithmetic so the oracle can be pinned
to something other than itself.

* det / perturbed edge signs by plain Fraction arithmetic;
* per-tetrahedron clipping of a segment by the four face half-spaces
  (brute force over every tetrahedron);
* slab clipping of a segment by an axis-aligned box (chord lengths);
* an exact traversal generator for Kuhn-subdivided product grids that steps
  through cells by axis-plane crossings and through the six Kuhn tetrahedra
  of a cell by diagonal-plane crossings, breaking ties by translating the ray
  by eps*U + eps^2*V (eps -> 0+), with every event time a polynomial in eps
  compared lexicographically.
* the cone-beam ray construction restated with numpy float32 scalars.
"""

from __future__ import annotations

import math
from fractions import Fraction as Fr
from itertools import permutations

import numpy as np

KUHN_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def F3(v):
    return [Fr(float(c)) for c in np.asarray(v, dtype=np.float32).reshape(3)]


def det3(a, b, c):
    return (a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0])
            + a[2] * (b[0] * c[1] - b[1] * c[0]))


def sub(a, b):
    return [x - y for x, y in zip(a, b)]


def sgn(v):
    return (v > 0) - (v < 0)


def orient3d(a, b, c, d):
    a, b, c, d = map(F3, (a, b, c, d))
    return sgn(det3(sub(b, a), sub(c, a), sub(d, a)))


def edge_sign(S, P, U, V, p, q):
    """Sign of the edge (p, q) seen by the ray S->P translated by eps U + eps^2 V."""
    S, P, U, V, p, q = map(F3, (S, P, U, V, p, q))
    d = sub(P, S)
    e0 = det3(d, sub(p, S), sub(q, S))
    if e0:
        return sgn(e0)
    pq = sub(p, q)
    e1 = det3(d, U, pq)
    if e1:
        return sgn(e1)
    return sgn(det3(d, V, pq))


# ---------------------------------------------------------------------------
# Cone-beam rays restated with numpy float32 scalars (one rounding per op).
# ---------------------------------------------------------------------------
def snapped_cos_sin(th):
    k = round(th / (math.pi / 2))
    if abs(th - k * (math.pi / 2)) < 1e-12:
        return [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)][k % 4]
    return math.cos(th), math.sin(th)


def cone_ray(cone, angles, rid):
    nu, nv = cone.nu, cone.nv
    i = rid % nu
    j = (rid // nu) % nv
    a = rid // (nu * nv)
    c, s = snapped_cos_sin(float(angles[a]))
    f = np.float32
    S = [f(cone.dso * c), f(cone.dso * s), f(0.0)]
    D = [f(-(cone.dsd - cone.dso) * c), f(-(cone.dsd - cone.dso) * s), f(0.0)]
    U = [f(-s), f(c), f(0.0)]
    V = [f(0.0), f(0.0), f(1.0)]
    u = f((i - (nu - 1) / 2.0) * cone.du + cone.off_u)
    v = f((j - (nv - 1) / 2.0) * cone.dv + cone.off_v)
    P = [f(f(D[k] + f(u * U[k])) + f(v * V[k])) for k in range(3)]
    return (np.array(S, np.float32), np.array(P, np.float32), np.array(U, np.float32), np.array(V, np.float32))


# ---------------------------------------------------------------------------
# Brute-force clipping.
# ---------------------------------------------------------------------------
def clip_tet(S, P, tv):
    """Exact parameter interval [t0, t1] of segment S->P inside the tetrahedron
    with vertices tv (4 x 3), or None.  Each face plane contributes the linear
    constraint that the point stays on the side of the opposite vertex."""
    S, P = F3(S), F3(P)
    V = [F3(v) for v in tv]
    d = sub(P, S)
    lo, hi = Fr(0), Fr(1)
    for k in range(4):
        f = [V[j] for j in range(4) if j != k]
        n = [(f[1][1] - f[0][1]) * (f[2][2] - f[0][2]) - (f[1][2] - f[0][2]) * (f[2][1] - f[0][1]),
             (f[1][2] - f[0][2]) * (f[2][0] - f[0][0]) - (f[1][0] - f[0][0]) * (f[2][2] - f[0][2]),
             (f[1][0] - f[0][0]) * (f[2][1] - f[0][1]) - (f[1][1] - f[0][1]) * (f[2][0] - f[0][0])]
        side = sum(n[i] * (V[k][i] - f[0][i]) for i in range(3))
        if side < 0:
            n = [-x for x in n]
        # n . (S + t d - f0) >= 0
        c0 = sum(n[i] * (S[i] - f[0][i]) for i in range(3))
        c1 = sum(n[i] * d[i] for i in range(3))
        if c1 == 0:
            if c0 < 0:
                return None
            continue
        t = -c0 / c1
        if c1 > 0:
            lo = max(lo, t)
        else:
            hi = min(hi, t)
        if lo > hi:
            return None
    return lo, hi


def brute_force_lengths(verts, tets, S, P):
    """{tet: length} for every tetrahedron the segment crosses with positive length."""
    dn = math.sqrt(float(sum(x * x for x in sub(F3(P), F3(S)))))
    out = {}
    for t, tv in enumerate(tets):
        iv = clip_tet(S, P, verts[tv])
        if iv is not None and iv[1] > iv[0]:
            out[t] = dn * float(iv[1] - iv[0])
    return out


def box_chord(S, P, lo, hi):
    """Exact length of segment S->P inside the box [lo, hi] (slab method)."""
    S, P = F3(S), F3(P)
    lo, hi = F3(lo), F3(hi)
    d = sub(P, S)
    t0, t1 = Fr(0), Fr(1)
    for a in range(3):
        if d[a] == 0:
            if not (lo[a] <= S[a] <= hi[a]):
                return 0.0
            continue
        ta, tb = (lo[a] - S[a]) / d[a], (hi[a] - S[a]) / d[a]
        if ta > tb:
            ta, tb = tb, ta
        t0, t1 = max(t0, ta), min(t1, tb)
    if t1 <= t0:
        return 0.0
    return math.sqrt(float(sum(x * x for x in d))) * float(t1 - t0)


# ---------------------------------------------------------------------------
# Exact Kuhn-grid traversal with the eps-translated ray.
# Polynomials in eps are tuples (c0, c1, c2); tuple comparison is the
# lexicographic order, i.e. the order for all small enough eps > 0.
# ---------------------------------------------------------------------------
def _padd(a, b):
    return tuple(x + y for x, y in zip(a, b))


def _pscale(a, s):
    return tuple(x * s for x in a)


class KuhnGrid:
    def __init__(self, X, Y, Z):
        self.N = [[Fr(float(v)) for v in np.asarray(A, np.float32)] for A in (X, Y, Z)]
        self.n = [len(a) - 1 for a in self.N]

    def tet_id(self, cell, order):
        nx, ny, _ = self.n
        c = cell[0] + nx * (cell[1] + ny * cell[2])
        return 6 * c + KUHN_PERMS.index(tuple(order))

    def trace(self, S, P, U, V):
        """List of (tet id, length) for the eps-translated ray; [] for a miss."""
        S, P, U, V = map(F3, (S, P, U, V))
        d = sub(P, S)
        dn = math.sqrt(float(sum(x * x for x in d)))
        base = [(S[a], U[a], V[a]) for a in range(3)]  # coordinate a at t = 0 as a poly in eps

        def cross_time(a, c):  # time the coordinate a reaches value c
            return tuple(x / d[a] for x in ((c - base[a][0]), -base[a][1], -base[a][2]))

        # Hull entry/exit (slab method on the eps-translated ray).
        t_in = t_out = None
        for a in range(3):
            lo, hi = self.N[a][0], self.N[a][-1]
            if d[a] == 0:
                if not ((lo, 0, 0) < base[a] < (hi, 0, 0)):
                    return []
                continue
            ta, tb = cross_time(a, lo), cross_time(a, hi)
            if d[a] < 0:
                ta, tb = tb, ta
            t_in = ta if t_in is None or ta > t_in else t_in
            t_out = tb if t_out is None or tb < t_out else t_out
        if t_in >= t_out:
            return []

        def pos(a, t):  # coordinate a at poly time t (degree <= 2 kept: t has degree <= 2)
            return _padd(base[a], _pscale(t, d[a]))

        def locate(a, p):
            nodes = self.N[a]
            for i in range(len(nodes) - 1):
                lo, hi = (nodes[i], 0, 0), (nodes[i + 1], 0, 0)
                if p == lo:
                    return i if d[a] > 0 else i - 1
                if p == hi:
                    if d[a] > 0:
                        continue
                    return i
                if lo < p < hi:
                    return i
            raise AssertionError("point outside the grid")

        cell = [locate(a, pos(a, t_in)) for a in range(3)]

        def xi(a, t):
            lo = self.N[a][cell[a]]
            h = self.N[a][cell[a] + 1] - lo
            p = pos(a, t)
            return tuple(x / h for x in ((p[0] - lo), p[1], p[2])), d[a] / h

        def order_at(t):
            keys = []
            for a in range(3):
                v, rate = xi(a, t)
                keys.append((v, rate, a))
            keys.sort(reverse=True)
            return [k[2] for k in keys]

        order = order_at(t_in)
        out = []
        t_cur = t_in
        t_enter = t_in
        cap = 10 * sum(self.n) + 10
        for _ in range(cap):
            best = None
            # Cell faces.
            for a in range(3):
                if d[a] == 0:
                    continue
                bound = self.N[a][cell[a] + 1] if d[a] > 0 else self.N[a][cell[a]]
                t = cross_time(a, bound)
                if t > t_cur and (best is None or t < best[0]):
                    best = (t, "axis", a)
            # Diagonal planes xi_a = xi_b.
            for a, b in ((0, 1), (0, 2), (1, 2)):
                ha = self.N[a][cell[a] + 1] - self.N[a][cell[a]]
                hb = self.N[b][cell[b] + 1] - self.N[b][cell[b]]
                k = d[a] / ha - d[b] / hb
                if k == 0:
                    continue
                la, lb = self.N[a][cell[a]], self.N[b][cell[b]]
                c = ((base[a][0] - la) / ha - (base[b][0] - lb) / hb,
                     base[a][1] / ha - base[b][1] / hb,
                     base[a][2] / ha - base[b][2] / hb)
                t = tuple(-x / k for x in c)
                if t > t_cur and (best is None or t < best[0]):
                    best = (t, "diag", (a, b))
            t_ev, kind, what = best
            out.append((self.tet_id(cell, order), dn * float(t_ev[0] - t_enter[0])))
            if kind == "diag":
                a, b = what
                ia, ib = order.index(a), order.index(b)
                assert abs(ia - ib) == 1, "non-adjacent diagonal crossing"
                order[ia], order[ib] = order[ib], order[ia]
            else:
                a = what
                if d[a] > 0:
                    assert order[0] == a, "leaving through a face not of the current tetrahedron"
                    cell[a] += 1
                    if cell[a] >= self.n[a]:
                        return out
                    order = order[1:] + [a]
                else:
                    assert order[2] == a, "leaving through a face not of the current tetrahedron"
                    cell[a] -= 1
                    if cell[a] < 0:
                        return out
                    order = [a] + order[:2]
            t_cur = t_ev
            t_enter = t_ev
        raise AssertionError("Kuhn traversal did not terminate")


def all_perms():
    return list(permutations(range(3)))
