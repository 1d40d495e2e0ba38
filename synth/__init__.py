"""Seeded synthetic inputs for the tetrahedral cone-beam projector.

This package produces the *inputs* every consumer shares: mesh node
coordinates and tetrahedron connectivity (Kuhn-subdivided product grids,
interior jitter, geometric grading), per-tetrahedron attenuation phantoms,
cone-beam geometry parameters and projection angles, and unstructured
Delaunay meshes of random points.  It contains none of
the projector's arithmetic (no ray construction, no intersection, no
traversal): the CPU oracle and the GPU library each derive everything else
from these arrays on their own.
"""

from .meshes import (
    kuhn_nodes,
    graded_nodes,
    kuhn_mesh,
    jitter_interior,
    tet_centroids,
    delaunay_mesh,
)
from .phantoms import uniform_random, sphere_phantom
from .configs import Cone, Workload, config, batch_problem, batch_problems, angles_for, jittered_kuhn, plain_kuhn, graded_mesh

__all__ = [
    "kuhn_nodes",
    "graded_nodes",
    "kuhn_mesh",
    "jitter_interior",
    "tet_centroids",
    "uniform_random",
    "sphere_phantom",
    "Cone",
    "Workload",
    "config",
    "batch_problem",
    "batch_problems",
    "angles_for",
    "jittered_kuhn",
    "plain_kuhn",
    "graded_mesh",
]
