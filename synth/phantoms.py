"""Per-tetrahedron attenuation values (piecewise-constant images on the mesh)."""

from __future__ import annotations

import numpy as np

from .meshes import tet_centroids


def uniform_random(nt: int, seed: int) -> np.ndarray:
    """x_i ~ U[0, 1) drawn in float64 from default_rng(seed), rounded to float32."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=nt).astype(np.float32)


def sphere_phantom(verts, tets, seed: int, radius: float = 0.3, inside: float = 0.5,
                   outside: float = 0.1, sigma: float = 0.01) -> np.ndarray:
    """Centred-sphere phantom.

    A tetrahedron is inside when the float64 norm of its centroid is below
    ``radius``; it gets ``inside``, otherwise ``outside``, plus Gaussian noise
    N(0, sigma^2) from default_rng(seed), summed in float64 and rounded to
    float32.  No clamping.
    """
    c = tet_centroids(verts, tets)
    r = np.sqrt((c * c).sum(axis=1))
    base = np.where(r < radius, inside, outside)
    noise = np.random.default_rng(seed).normal(0.0, sigma, size=len(tets))
    return (base + noise).astype(np.float32)
