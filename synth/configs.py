"""The five benchmark workloads and the batched-problem ladder.

Every number here is an input choice (mesh resolution, jitter, seeds,
detector size and pitch, source distances, angle count).  Geometry follows a
circular cone-beam orbit with equispaced angles (the paper's experiments,
Section III-A): source-to-rotation-centre distance ``dso``, source-to-detector
distance ``dsd``, ``nu`` x ``nv`` pixels of pitch ``du`` x ``dv`` with centre
offsets ``off_u`` / ``off_v``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .meshes import graded_nodes, jitter_interior, kuhn_mesh, kuhn_nodes
from .phantoms import sphere_phantom, uniform_random


@dataclass(frozen=True)
class Cone:
    dso: float
    dsd: float
    nu: int
    nv: int
    du: float
    dv: float
    off_u: float = 0.0
    off_v: float = 0.0

    @property
    def rays_per_angle(self) -> int:
        return self.nu * self.nv


def angles_for(na: int) -> np.ndarray:
    """theta_k = 2*pi*k/na, k = 0..na-1 (endpoint excluded), float64."""
    return 2.0 * math.pi * np.arange(na, dtype=np.float64) / na


@dataclass
class Workload:
    name: str
    verts: np.ndarray  # float32 [nv, 3]
    tets: np.ndarray  # int32 [nt, 4]
    x: np.ndarray  # float32 [nt]
    cone: Cone
    angles: np.ndarray  # float64 [na]
    dims: tuple = ()
    meta: dict = field(default_factory=dict)

    @property
    def nt(self) -> int:
        return int(self.tets.shape[0])

    @property
    def nrays(self) -> int:
        return int(len(self.angles) * self.cone.nu * self.cone.nv)


def _uniform_kuhn(n: int):
    X = kuhn_nodes(n)
    return kuhn_mesh(X, X, X)


def plain_kuhn(n: int, seed: int = 0, nu: int = 64, nv: int = 64, na: int = 16,
               pitch: Optional[float] = None) -> Workload:
    """Unjittered Kuhn n^3 cube [-0.5,0.5]^3 with U[0,1) attenuation."""
    verts, tets = _uniform_kuhn(n)
    pitch = 2.0 / nu if pitch is None else pitch
    cone = Cone(4.0, 8.0, nu, nv, pitch, pitch)
    return Workload(f"kuhn{n}", verts, tets, uniform_random(len(tets), seed), cone,
                    angles_for(na), (n, n, n), {"seed": seed})


def jittered_kuhn(n: int, jitter_seed: int, noise_seed: int, nu: int, nv: int, na: int,
                  amplitude: float = 0.2) -> Workload:
    verts, tets = _uniform_kuhn(n)
    verts, redraws = jitter_interior(verts, tets, (n, n, n), 1.0 / n, amplitude, jitter_seed)
    x = sphere_phantom(verts, tets, noise_seed)
    cone = Cone(4.0, 8.0, nu, nv, 2.0 / nu, 2.0 / nv)
    return Workload(f"kuhn{n}_jit", verts, tets, x, cone, angles_for(na), (n, n, n),
                    {"jitter_seed": jitter_seed, "noise_seed": noise_seed, "redraws": redraws})


def graded_mesh(nxy: int = 128, nz: int = 32, ratio: float = 1.05, zero_index: int = 114):
    X = graded_nodes(nxy, ratio, zero_index)
    Z = kuhn_nodes(nz)
    return kuhn_mesh(X, X, Z), X, Z


def config(idx: int) -> Workload:
    """Workload ``idx`` (0..3); index 4 is :func:`batch_problems`."""
    if idx == 0 or idx == 3:
        w = plain_kuhn(8, seed=0, nu=64, nv=64, na=16, pitch=2.0 ** -5)
        w.name = "kuhn8_64x64x16" if idx == 0 else "grad_kuhn8_64x64x16"
        if idx == 3:
            w.meta["target_seed"] = 3
            w.meta["fd_seed"] = 33
        return w
    if idx == 1:
        w = jittered_kuhn(64, 1, 11, 512, 512, 360)
        w.name = "kuhn64_jit_512x512x360"
        return w
    if idx == 2:
        (verts, tets), X, Z = graded_mesh()
        x = sphere_phantom(verts, tets, 12)
        du = 2.0 ** -7
        cone = Cone(4.0, 8.0, 256, 256, du, du, du / 2, du / 2)
        return Workload("graded128x128x32_256x256x180", verts, tets, x, cone, angles_for(180),
                        (128, 128, 32), {"noise_seed": 12})
    raise ValueError(f"unknown workload {idx}")


def batch_problem(b: int) -> Workload:
    """Problem b (0..31) of the batched ladder.

    n_b = 16 + floor(80 b / 31) cells per edge; detector 128 (1 + b mod 4)
    square with pitch 2 / det; 64 + floor(656 ((7 b) mod 32) / 31) angles;
    jitter seed 400 + b, phantom noise seed 500 + b.
    """
    n = 16 + (80 * b) // 31
    det = 128 * (1 + b % 4)
    na = 64 + (656 * ((7 * b) % 32)) // 31
    w = jittered_kuhn(n, 400 + b, 500 + b, det, det, na)
    w.name = f"batch{b:02d}_kuhn{n}_{det}x{det}x{na}"
    return w


def batch_problems(count: int = 32):
    return [batch_problem(b) for b in range(count)]
