"""MI355X-native tetrahedral-mesh cone-beam CT projector (HIP / gfx950).

The operator A of the linear CT model A x = b with a_ij = length of ray j in
tetrahedron i (Biguri et al., Section II-A), computed on the fly by walking
every ray through the mesh.  The compute path is libtetct.so (include/tetct.h);
this package only marshals arguments.
"""

from .projector import ConeGeometry, Projector, TetMesh, trace_rays

__all__ = ["TetMesh", "ConeGeometry", "Projector", "trace_rays"]

from .solvers import CGLS, OSSART, TetProject, cgls, os_sart, project, sirt  # noqa: E402

__all__ += ["TetProject", "project", "CGLS", "cgls", "sirt", "OSSART", "os_sart"]

from .batch import BatchCGLS, BatchProjector, BatchTetProject, PlainCGLS, SetOps, VecSet, project_batch  # noqa: E402
from . import autotune  # noqa: E402

__all__ += ["VecSet", "SetOps", "BatchProjector", "BatchTetProject", "project_batch", "BatchCGLS", "PlainCGLS",
            "autotune"]
