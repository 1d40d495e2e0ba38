"""Python front end of the tetrahedral projector (libtetct.so).

Tensors live on a HIP device and are handed to the library as raw pointers
together with torch's current stream; every computation runs in the
library's kernels.
"""

from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import (TCT_BP_ATOMIC, TCT_BP_ATOMIC_DIRECT, TCT_BP_FIXED, TCT_BP_GATHER, TCT_BP_SHADOW, call, lib,
                   tct_cone, tct_paper_stats, tct_range, tct_stats)


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev_index(device) -> int:
    d = torch.device(device if device is not None else "cuda")
    return d.index if d.index is not None else torch.cuda.current_device()


def _ptr(t: torch.Tensor, dtype, device_index: int, numel: Optional[int] = None, name: str = "tensor") -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda or t.device.index != device_index:
        raise ValueError(f"{name} must be on cuda:{device_index}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


class TetMesh:
    """A validated, reordered tetrahedral mesh resident on one device."""

    def __init__(self, verts, tets, nbrs=None, device=None, reorder: bool = True, host_only: bool = False,
                 rstar: bool = False):
        self.verts = np.ascontiguousarray(verts, dtype=np.float32).reshape(-1, 3)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
        nb = None if nbrs is None else np.ascontiguousarray(nbrs, dtype=np.int32).reshape(-1, 4)
        self.device_index = 0 if host_only else _dev_index(device)
        flags = ((0 if reorder else _lib.TCT_MESH_NO_REORDER) | (_lib.TCT_MESH_HOST_ONLY if host_only else 0)
                 | (_lib.TCT_MESH_RSTAR if rstar else 0))
        h = C.c_void_p()
        call("tct_mesh_create", self.verts.ctypes.data, len(self.verts), self.tets.ctypes.data, len(self.tets),
             None if nb is None else nb.ctypes.data, flags, self.device_index, C.byref(h))
        self._h = h
        nv, nt, nbd = C.c_int32(), C.c_int32(), C.c_int32()
        nbytes = C.c_int64()
        call("tct_mesh_counts", h, C.byref(nv), C.byref(nt), C.byref(nbd), C.byref(nbytes))
        self.nv, self.nt, self.nboundary, self.device_bytes = nv.value, nt.value, nbd.value, nbytes.value
        self.perm = np.zeros(self.nt, np.int32)
        call("tct_mesh_permutation", h, self.perm.ctypes.data)
        self.host_only = host_only

    @property
    def handle(self):
        return self._h

    @property
    def device(self):
        return torch.device("cuda", self.device_index)

    def boundary(self):
        """Boundary faces in entry-id order: vertices [nb][3][3] (outward
        orientation) and the user id of each face's tetrahedron."""
        xyz = np.zeros((self.nboundary, 3, 3), np.float32)
        owner = np.zeros(self.nboundary, np.int32)
        call("tct_mesh_boundary", self._h, xyz.ctypes.data, owner.ctypes.data)
        return xyz, owner

    def rstar(self) -> dict:
        """The R*-tree (mesh created with rstar=True) in its preorder layout:
        boxes [n][6], skip and leaf fields [n][2], leaf face list, height."""
        n, nl, h = C.c_int32(), C.c_int32(), C.c_int32()
        call("tct_mesh_rstar", self._h, C.byref(n), C.byref(nl), C.byref(h), None, None, None)
        box = np.zeros((n.value, 6), np.float32)
        link = np.zeros((n.value, 2), np.int32)
        lst = np.zeros(nl.value, np.int32)
        call("tct_mesh_rstar", self._h, C.byref(n), C.byref(nl), C.byref(h), box.ctypes.data, link.ctypes.data,
             lst.ctypes.data)
        return {"box": box, "link": link, "list": lst, "height": h.value}

    def neighbors(self) -> np.ndarray:
        out = np.zeros((self.nt, 4), np.int32)
        call("tct_mesh_neighbors", self._h, out.ctypes.data)
        return out

    def to_internal(self, x_user: torch.Tensor) -> torch.Tensor:
        out = torch.empty(self.nt, dtype=torch.float32, device=self.device)
        call("tct_mesh_to_internal", self._h, _ptr(x_user, torch.float32, self.device_index, self.nt, "x_user"),
             out.data_ptr(), _stream(self.device))
        return out

    def to_user(self, x_internal: torch.Tensor) -> torch.Tensor:
        out = torch.empty(self.nt, dtype=torch.float32, device=self.device)
        call("tct_mesh_to_user", self._h, _ptr(x_internal, torch.float32, self.device_index, self.nt, "x_internal"),
             out.data_ptr(), _stream(self.device))
        return out

    def stats(self, reset: bool = False, check: bool = False) -> dict:
        st = tct_stats()
        status = lib().tct_stats_read(self._h, C.byref(st), 1 if reset else 0)
        if check:
            _lib.check(status)
        elif status not in (0, -9):
            _lib.check(status)
        return st.as_dict()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib._lib is not None:
            _lib._lib.tct_mesh_destroy(h)
            self._h = None


class ConeGeometry:
    """Circular cone-beam geometry: cone parameters plus projection angles (radians)."""

    def __init__(self, cone, angles, device=None):
        self.cone = cone
        self.angles = np.ascontiguousarray(angles, dtype=np.float64)
        self.na = len(self.angles)
        self.nu, self.nv = int(cone.nu), int(cone.nv)
        self.device_index = _dev_index(device)
        c = tct_cone(float(cone.dso), float(cone.dsd), self.nu, self.nv, float(cone.du), float(cone.dv),
                     float(getattr(cone, "off_u", 0.0)), float(getattr(cone, "off_v", 0.0)))
        h = C.c_void_p()
        call("tct_geom_create", C.byref(c), self.angles.ctypes.data, self.na, self.device_index, C.byref(h))
        self._h = h
        self.nrays = int(lib().tct_geom_nrays(h))

    @property
    def handle(self):
        return self._h

    @property
    def shape(self):
        return (self.na, self.nv, self.nu)

    def frame(self):
        """(S, D, U, V [na,3], u [nu], v [nv]) float32 as used by the kernels."""
        S, D, U, V = (np.zeros((self.na, 3), np.float32) for _ in range(4))
        u = np.zeros(self.nu, np.float32)
        v = np.zeros(self.nv, np.float32)
        call("tct_geom_frame", self._h, S.ctypes.data, D.ctypes.data, U.ctypes.data, V.ctypes.data, u.ctypes.data,
             v.ctypes.data)
        return S, D, U, V, u, v

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib._lib is not None:
            _lib._lib.tct_geom_destroy(h)
            self._h = None


class Projector:
    """A = system matrix of (mesh, geometry): forward A x, backprojection A^T y, traces.

    x-like tensors are float32 [nt] in the mesh's internal order; projections
    are float32 [na, nv, nu].
    """

    def __init__(self, mesh: TetMesh, geom: ConeGeometry, cache_entry: bool = True):
        if mesh.device_index != geom.device_index:
            raise ValueError("mesh and geometry on different devices")
        self.mesh, self.geom = mesh, geom
        self.device = mesh.device
        self.entry = None
        if cache_entry:
            self.entry = torch.empty(geom.nrays, dtype=torch.int32, device=self.device)
            call("tct_entry_raster", mesh.handle, geom.handle, self.entry.data_ptr(), _stream(self.device))

    @property
    def nt(self):
        return self.mesh.nt

    @property
    def proj_shape(self):
        return self.geom.shape

    def _entry_ptr(self, use_cache: bool):
        return self.entry.data_ptr() if (use_cache and self.entry is not None) else None

    def forward(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, use_cache: bool = True) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.geom.shape, dtype=torch.float32, device=self.device)
        call("tct_forward", self.mesh.handle, self.geom.handle,
             _ptr(x, torch.float32, self.mesh.device_index, self.nt, "x"),
             _ptr(out, torch.float32, self.mesh.device_index, self.geom.nrays, "proj"),
             self._entry_ptr(use_cache), _stream(self.device))
        return out

    def backproject(self, y: torch.Tensor, mode: str = "atomic", out: Optional[torch.Tensor] = None,
                    accumulate: bool = False, use_cache: bool = True) -> torch.Tensor:
        m = {"atomic": TCT_BP_ATOMIC, "atomic_direct": TCT_BP_ATOMIC_DIRECT, "gather": TCT_BP_GATHER,
             "shadow": TCT_BP_SHADOW, "fixed": TCT_BP_FIXED}[mode]
        if out is None:
            out = torch.empty(self.nt, dtype=torch.float32, device=self.device)
            accumulate = False
        call("tct_backproject", self.mesh.handle, self.geom.handle,
             _ptr(y, torch.float32, self.mesh.device_index, self.geom.nrays, "proj"),
             _ptr(out, torch.float32, self.mesh.device_index, self.nt, "xhat"), m, 1 if accumulate else 0,
             self._entry_ptr(use_cache), _stream(self.device))
        return out

    def forward_paper(self, x: torch.Tensor, precision: int = 64, out: Optional[torch.Tensor] = None):
        """The paper's own propagation (Moller-Trumbore with eps escalation,
        Algorithms 1-2) in float32 or float64; returns (proj, stats dict).
        Needs the entry cache.  Synchronises the stream."""
        if self.entry is None:
            raise ValueError("the paper-faithful walk needs the entry cache (Projector(cache_entry=True))")
        if out is None:
            out = torch.empty(self.geom.shape, dtype=torch.float32, device=self.device)
        st = tct_paper_stats()
        call("tct_forward_paper", self.mesh.handle, self.geom.handle,
             _ptr(x, torch.float32, self.mesh.device_index, self.nt, "x"),
             _ptr(out, torch.float32, self.mesh.device_index, self.geom.nrays, "proj"), self.entry.data_ptr(),
             int(precision), C.byref(st), _stream(self.device))
        return out, st.as_dict()

    _BP_MODES = {"atomic": TCT_BP_ATOMIC, "atomic_direct": TCT_BP_ATOMIC_DIRECT, "gather": TCT_BP_GATHER,
                 "shadow": TCT_BP_SHADOW, "fixed": TCT_BP_FIXED}

    def forward_range(self, x: torch.Tensor, a0: int, na: int, out: torch.Tensor, tile_u: int = 8,
                      use_cache: bool = True) -> torch.Tensor:
        """A x for the angles [a0, a0 + na) only, into their slab of the full
        [na_total, nv, nu] array ``out`` (other angles untouched)."""
        call("tct_forward_range", self.mesh.handle, self.geom.handle,
             _ptr(x, torch.float32, self.mesh.device_index, self.nt, "x"),
             _ptr(out, torch.float32, self.mesh.device_index, self.geom.nrays, "proj"),
             self._entry_ptr(use_cache), C.byref(tct_range(int(a0), int(na), int(tile_u))), _stream(self.device))
        return out

    def backproject_range(self, y: torch.Tensor, a0: int, na: int, mode: str = "atomic",
                          out: Optional[torch.Tensor] = None, accumulate: bool = False, tile_u: int = 8,
                          use_cache: bool = True) -> torch.Tensor:
        """A^T y restricted to the rays of the angles [a0, a0 + na) (y keeps
        the full [na_total, nv, nu] layout)."""
        if out is None:
            out = torch.empty(self.nt, dtype=torch.float32, device=self.device)
            accumulate = False
        call("tct_backproject_range", self.mesh.handle, self.geom.handle,
             _ptr(y, torch.float32, self.mesh.device_index, self.geom.nrays, "proj"),
             _ptr(out, torch.float32, self.mesh.device_index, self.nt, "xhat"), self._BP_MODES[mode],
             1 if accumulate else 0, self._entry_ptr(use_cache), C.byref(tct_range(int(a0), int(na), int(tile_u))),
             _stream(self.device))
        return out

    def compute_entry(self, out: Optional[torch.Tensor] = None, method: str = "raster") -> torch.Tensor:
        """Entry face of every ray (-1: miss) by projecting the boundary faces
        onto the detector (the default), through the boundary BVH
        (method="bvh") or the R*-tree (method="rstar", mesh built with
        rstar=True); all three give the same faces."""
        fn = {"bvh": "tct_entry", "rstar": "tct_entry_rstar", "raster": "tct_entry_raster"}.get(method)
        if fn is None:
            raise ValueError(f"unknown entry search {method!r}")
        if out is None:
            out = torch.empty(self.geom.nrays, dtype=torch.int32, device=self.device)
        call(fn, self.mesh.handle, self.geom.handle,
             _ptr(out, torch.int32, self.mesh.device_index, self.geom.nrays, "entry"), _stream(self.device))
        return out

    def trace(self, ray_ids) -> list:
        """Visited tetrahedra (user ids) and lengths per listed ray, zero-length passages included."""
        ids = torch.as_tensor(np.ascontiguousarray(ray_ids, dtype=np.int64), device=self.device)
        return _trace(self.mesh, lambda off, tt, ll, cap, need: lib().tct_trace(
            self.mesh.handle, self.geom.handle, ids.data_ptr(), len(ids), off, tt, ll, cap, need,
            _stream(self.device)), len(ids), self.device)


def trace_rays(mesh: TetMesh, S, P, U, V) -> list:
    """Trace caller-given rays (float32 [n, 3] each) through the mesh."""
    dev = mesh.device
    arrs = [torch.as_tensor(np.ascontiguousarray(np.asarray(a, np.float32).reshape(-1, 3)), device=dev)
            for a in (S, P, U, V)]
    n = arrs[0].shape[0]
    return _trace(mesh, lambda off, tt, ll, cap, need: lib().tct_trace_rays(
        mesh.handle, arrs[0].data_ptr(), arrs[1].data_ptr(), arrs[2].data_ptr(), arrs[3].data_ptr(), n, off, tt, ll,
        cap, need, _stream(dev)), n, dev)


def _trace(mesh, fn, n, dev):
    off = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    cap = max(1024, 64 * n)
    while True:
        tt = torch.empty(cap, dtype=torch.int32, device=dev)
        ll = torch.empty(cap, dtype=torch.float32, device=dev)
        need = C.c_int64(0)
        st = fn(off.data_ptr(), tt.data_ptr(), ll.data_ptr(), cap, C.byref(need))
        if st == -10:
            cap = int(need.value)
            continue
        _lib.check(st)
        o = off.cpu().numpy()
        t = tt.cpu().numpy()
        l = ll.cpu().numpy()
        return [(t[o[i]:o[i + 1]].copy(), l[o[i]:o[i + 1]].copy()) for i in range(n)]
