"""Kuhn-subdivided product-grid meshes, interior jitter and geometric grading;
unstructured Delaunay meshes of random points.

A product grid with node arrays X (nx+1), Y (ny+1), Z (nz+1) is cut into
cells; every cell is split into the six Kuhn tetrahedra

    T_pi = { xi_pi0 >= xi_pi1 >= xi_pi2 }    (xi = local coordinates in [0,1]^3)

for the six permutations pi of the axes, which makes a conforming mesh
(neighbouring cells split their shared square along the same diagonal).
The vertices of T_pi are the cell's minimum corner c, c + e_pi0,
c + e_pi0 + e_pi1 and the maximum corner.  Orientation is left as the
construction gives it (half of the tetrahedra are negatively oriented);
consumers normalise it.

Vertex id of grid node (i, j, k) is i + (nx+1) * (j + (ny+1) * k).
Tetrahedra are listed cell by cell (i fastest, then j, then k) and, within a
cell, by permutation in lexicographic order.
"""

from __future__ import annotations

import numpy as np

# Lexicographic order of the axis permutations; row p gives (pi0, pi1, pi2).
KUHN_PERMS = np.array(
    [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)], dtype=np.int64
)


def kuhn_nodes(n: int, lo: float = -0.5, hi: float = 0.5) -> np.ndarray:
    """Uniform node coordinates lo + (hi-lo) * i / n, i = 0..n, in float64."""
    i = np.arange(n + 1, dtype=np.float64)
    return lo + (hi - lo) * i / n


def graded_nodes(n: int, ratio: float, zero_index: int) -> np.ndarray:
    """Geometrically graded nodes: cell k has width proportional to ratio**k.

    The widths sum to 1.  The whole node array is shifted so that node
    ``zero_index`` is exactly 0.0 (the subtraction of a value from itself).
    Computed in float64.
    """
    w = ratio ** np.arange(n, dtype=np.float64)
    w /= w.sum()
    nodes = np.concatenate([[0.0], np.cumsum(w)])
    return nodes - nodes[zero_index]


def kuhn_mesh(X, Y, Z):
    """Kuhn mesh of the product grid X x Y x Z.

    Returns (verts float32 [nv, 3], tets int32 [nt, 4]).  Coordinates are the
    node values rounded once to float32.
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    nx, ny, nz = len(X) - 1, len(Y) - 1, len(Z) - 1
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    verts = np.stack([X[ii.ravel()], Y[jj.ravel()], Z[kk.ravel()]], axis=1).astype(np.float32)

    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cell = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)  # [ncell, 3] (i, j, k)
    sx, sy = 1, nx + 1
    sz = (nx + 1) * (ny + 1)
    stride = np.array([sx, sy, sz], dtype=np.int64)
    base = cell @ stride  # vertex id of the min corner
    ncell = cell.shape[0]
    tets = np.empty((ncell, 6, 4), dtype=np.int64)
    for p, perm in enumerate(KUHN_PERMS):
        v0 = base
        v1 = v0 + stride[perm[0]]
        v2 = v1 + stride[perm[1]]
        v3 = v2 + stride[perm[2]]
        tets[:, p, 0] = v0
        tets[:, p, 1] = v1
        tets[:, p, 2] = v2
        tets[:, p, 3] = v3
    return verts, tets.reshape(-1, 4).astype(np.int32)


def _signed_volumes6(verts64: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Six times the signed volume of each tetrahedron, float64 (a mesh-quality
    check of the generator only, with a wide margin; not an exact predicate)."""
    p = verts64[tets]
    a = p[:, 1] - p[:, 0]
    b = p[:, 2] - p[:, 0]
    c = p[:, 3] - p[:, 0]
    return np.einsum("ij,ij->i", a, np.cross(b, c))


def interior_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    m = (ii > 0) & (ii < nx) & (jj > 0) & (jj < ny) & (kk > 0) & (kk < nz)
    return m.ravel()


def jitter_interior(verts, tets, dims, h, amplitude: float, seed: int, max_rounds: int = 100):
    """Move every interior vertex by U(-amplitude*h, amplitude*h) per coordinate.

    Boundary vertices stay fixed, so the hull is unchanged.  Offsets are drawn
    in float64 from numpy's PCG64 generator (``default_rng(seed)``), three per
    interior vertex in ascending vertex order, added to the float64 node value
    and rounded once to float32.  Any tetrahedron whose orientation flips or
    collapses below 1e-3 of its unjittered volume has its interior vertices
    redrawn, in ascending vertex order, from the same stream; repeated until
    none remain.  Returns (new_verts float32, redraw_count).
    """
    nx, ny, nz = dims
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), (3,))
    rng = np.random.default_rng(seed)
    base64 = verts.astype(np.float64)
    vol0 = _signed_volumes6(base64, tets)
    interior = np.nonzero(interior_mask(nx, ny, nz))[0]
    out = base64.copy()
    off = rng.uniform(-amplitude, amplitude, size=(interior.size, 3)) * h
    out[interior] = base64[interior] + off
    out32 = out.astype(np.float32)
    is_int = np.zeros(len(verts), dtype=bool)
    is_int[interior] = True
    redraws = 0
    for _ in range(max_rounds):
        vol = _signed_volumes6(out32.astype(np.float64), tets)
        bad = (np.sign(vol) != np.sign(vol0)) | (np.abs(vol) < 1e-3 * np.abs(vol0))
        if not bad.any():
            return out32, redraws
        vids = np.unique(tets[bad].ravel())
        vids = vids[is_int[vids]]
        redraws += len(vids)
        off = rng.uniform(-amplitude, amplitude, size=(len(vids), 3)) * h
        fixed = base64[vids] + off
        out32[vids] = fixed.astype(np.float32)
    raise RuntimeError("jitter_interior: could not produce a valid mesh")


def tet_centroids(verts, tets) -> np.ndarray:
    """Mean of the four vertices of each tetrahedron, float64."""
    return verts.astype(np.float64)[tets].mean(axis=1)


def delaunay_mesh(n_points: int, seed: int, lo: float = -0.5, hi: float = 0.5):
    """Delaunay tetrahedralisation of n_points uniform random points in the
    cube [lo, hi]^3 (PCG64 seed), coordinates rounded to float32 first so the
    triangulation is of the float32 points.  Unstructured, with the slivers a
    Delaunay mesh of random points has; its boundary is the (convex) hull of
    the points.  Returns (verts float32 [n][3], tets int32 [nt][4])."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    pts = rng.uniform(lo, hi, size=(n_points, 3)).astype(np.float32)
    tri = Delaunay(pts.astype(np.float64))
    tets = np.ascontiguousarray(tri.simplices, dtype=np.int32)
    vol = _signed_volumes6(pts.astype(np.float64), tets)
    if np.any(vol == 0.0):
        raise ValueError("degenerate Delaunay tetrahedron; choose another seed")
    return pts, tets
