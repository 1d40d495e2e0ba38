"""CPU reference oracle for the tetrahedral cone-beam projector.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports it.
"""

from .oracle import Oracle, OracleMesh, frame, rays_of, edge_sign, orient3d, det_sign, det_sign_exact, build

__all__ = ["Oracle", "OracleMesh", "frame", "rays_of", "edge_sign", "orient3d", "det_sign", "det_sign_exact", "build"]
