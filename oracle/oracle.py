"""ctypes front end of the C++ oracle (oracle.cpp) plus float64 solvers.

TEST INFRASTRUCTURE ONLY.  Everything here runs on the CPU in float64 with
exact sign decisions; see oracle.cpp for the definitions it follows.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")


def build(verbose: bool = False) -> str:
    """Compile oracle.cpp into liboracle.so (g++, OpenMP, no FP contraction)."""
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           _SRC, "-o", _LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    override = os.environ.get("TCT_ORACLE_LIB")  # an instrumented build (sanitizer tests)
    if override:
        L = C.CDLL(override)
    else:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
    L.orc_last_error.restype = C.c_char_p
    L.orc_exact_calls.restype = C.c_longlong
    L.orc_last_stats.argtypes = [_i64p]
    for name in ("orc_orient3d",):
        getattr(L, name).argtypes = [_f32p] * 4
        getattr(L, name).restype = C.c_int
    for name in ("orc_det_sign", "orc_det_sign_exact", "orc_edge_sign"):
        getattr(L, name).argtypes = [_f32p] * 6
        getattr(L, name).restype = C.c_int
    L.orc_det_sign_batch.argtypes = [C.c_longlong] + [_f32p] * 6 + [_i32p]
    L.orc_det_sign_batch.restype = None
    L.orc_mesh_create.argtypes = [_f32p, C.c_int, _i32p, C.c_int, C.POINTER(C.c_void_p)]
    L.orc_mesh_destroy.argtypes = [C.c_void_p]
    L.orc_mesh_nboundary.argtypes = [C.c_void_p]
    L.orc_mesh_flips.argtypes = [C.c_void_p]
    L.orc_mesh_tables.argtypes = [C.c_void_p, _i32p, _i32p, _i32p, _i32p]
    L.orc_frame.argtypes = [_f64p, _f64p, C.c_int, _f32p, _f32p, _f32p, _f32p, _f32p, _f32p]
    L.orc_rays.argtypes = [_f64p, _f64p, C.c_int, _i64p, C.c_longlong, _f32p, _f32p, _f32p, _f32p]
    L.orc_forward.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int, _f32p, C.c_void_p, C.c_longlong, _f64p,
                              C.c_void_p, C.c_int]
    L.orc_forward_paper.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int, _f32p, C.c_void_p, C.c_longlong, C.c_int,
                                    _f64p, _i64p, C.c_int]
    L.orc_backproject.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int, _f32p, C.c_void_p, C.c_longlong, _f64p,
                                  C.c_int]
    L.orc_backproject_ext.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int, _f32p, C.c_void_p, C.c_longlong,
                                      _f64p, _f64p, _f64p, C.c_int]
    L.orc_check_pass.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int, _f32p, _f64p, _f32p, _i64p, C.c_longlong] + \
        [_f64p] * 9 + [C.c_int]
    L.orc_trace.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int, _i64p, C.c_longlong, _i64p, _i32p, _f64p,
                            C.c_longlong]
    L.orc_trace_rays.argtypes = [C.c_void_p, _f32p, _f32p, _f32p, _f32p, C.c_longlong, _i64p, _i32p, _f64p,
                                 C.c_longlong]
    _lib = L
    return L


def max_threads() -> int:
    """Threads the oracle's parallel loops use by default."""
    return int(lib().orc_max_threads())


def _f3(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float32).reshape(3))


def orient3d(a, b, c, d) -> int:
    """Exact sign of det[b-a, c-a, d-a] for float32 points."""
    return lib().orc_orient3d(_f3(a), _f3(b), _f3(c), _f3(d))


def det_sign(A1, A0, B1, B0, C1, C0) -> int:
    """Exact sign of det[A1-A0, B1-B0, C1-C0] (float64 filter, then exact)."""
    return lib().orc_det_sign(*(map(_f3, (A1, A0, B1, B0, C1, C0))))


def det_sign_exact(A1, A0, B1, B0, C1, C0) -> int:
    """Same determinant sign, always through the big-integer path."""
    return lib().orc_det_sign_exact(*(map(_f3, (A1, A0, B1, B0, C1, C0))))


def det_sign_batch(A1, A0, B1, B0, C1, C0) -> np.ndarray:
    """Exact signs of det[A1-A0, B1-B0, C1-C0] for [n, 3] float32 arrays."""
    arrs = [np.ascontiguousarray(np.asarray(a, np.float32).reshape(-1, 3)) for a in (A1, A0, B1, B0, C1, C0)]
    n = len(arrs[0])
    assert all(len(a) == n for a in arrs)
    out = np.zeros(n, np.int32)
    lib().orc_det_sign_batch(n, *arrs, out)
    return out


def edge_sign(S, P, U, V, p, q) -> int:
    """Perturbed sign of det[P-S, p-S, q-S] (levels: U, then V)."""
    return lib().orc_edge_sign(*(map(_f3, (S, P, U, V, p, q))))


def _cone_arr(cone) -> np.ndarray:
    return np.array([cone.dso, cone.dsd, cone.nu, cone.nv, cone.du, cone.dv, cone.off_u, cone.off_v],
                    dtype=np.float64)


def frame(cone, angles):
    """(S, D, U, V per angle [na,3] float32, u table [nu], v table [nv])."""
    angles = np.ascontiguousarray(angles, dtype=np.float64)
    na = len(angles)
    S, D, U, V = (np.zeros((na, 3), np.float32) for _ in range(4))
    ut = np.zeros(cone.nu, np.float32)
    vt = np.zeros(cone.nv, np.float32)
    lib().orc_frame(_cone_arr(cone), angles, na, S, D, U, V, ut, vt)
    return S, D, U, V, ut, vt


def rays_of(cone, angles, ids):
    """Float32 endpoints S, P and detector axes U, V of the listed ray ids."""
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    n = len(ids)
    S, P, U, V = (np.zeros((n, 3), np.float32) for _ in range(4))
    angles = np.ascontiguousarray(angles, dtype=np.float64)
    lib().orc_rays(_cone_arr(cone), angles, len(angles), ids, n, S, P, U, V)
    return S, P, U, V


class OracleError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"oracle status {status}: {msg}")
        self.status = status


@dataclass
class Stats:
    rays: int
    hits: int
    segments: int
    zero_len: int
    failed: int
    multi_entry: int
    perturbed: int
    parallel: int


def last_stats() -> Stats:
    v = np.zeros(8, np.int64)
    lib().orc_last_stats(v)
    return Stats(*[int(x) for x in v])


class OracleMesh:
    """An oriented, neighbour-linked, convexity-checked mesh held by the oracle."""

    def __init__(self, verts, tets):
        self.verts = np.ascontiguousarray(verts, dtype=np.float32)
        self.tets_in = np.ascontiguousarray(tets, dtype=np.int32)
        h = C.c_void_p()
        st = lib().orc_mesh_create(self.verts, len(self.verts), self.tets_in, len(self.tets_in), C.byref(h))
        if st != 0:
            raise OracleError(st, lib().orc_last_error().decode())
        self._h = h
        self.nt = len(self.tets_in)
        self.nboundary = lib().orc_mesh_nboundary(h)
        self.flips = lib().orc_mesh_flips(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_mesh_destroy(h)
            self._h = None

    def tables(self):
        """(oriented tets [nt,4], neighbours [nt,4], outward boundary faces [nb,3], owners [nb,2])."""
        t = np.zeros((self.nt, 4), np.int32)
        n = np.zeros((self.nt, 4), np.int32)
        b = np.zeros((self.nboundary, 3), np.int32)
        o = np.zeros((self.nboundary, 2), np.int32)
        lib().orc_mesh_tables(self._h, t, n, b, o)
        return t, n, b, o


class Oracle:
    """Float64 projector on one mesh and one cone-beam geometry."""

    def __init__(self, verts, tets, cone, angles, nthreads: int = 0):
        self.mesh = OracleMesh(verts, tets)
        self.cone = cone
        self.angles = np.ascontiguousarray(angles, dtype=np.float64)
        self.na = len(self.angles)
        self.nrays = self.na * cone.nu * cone.nv
        self.nthreads = nthreads
        self._cone = _cone_arr(cone)

    @property
    def nt(self):
        return self.mesh.nt

    def _ids(self, ids):
        if ids is None:
            return None, self.nrays
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        return ids, len(ids)

    def _check(self, st):
        if st != 0:
            raise OracleError(st, lib().orc_last_error().decode())

    def forward(self, x, ids=None, return_counts=False):
        """b_j = sum_i a_ij x_i for the listed rays (all when ids is None), float64."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        ids_a, n = self._ids(ids)
        out = np.zeros(n, np.float64)
        cnt = np.zeros(n, np.int64)
        st = lib().orc_forward(self.mesh._h, self._cone, self.angles, self.na, x,
                               None if ids_a is None else ids_a.ctypes.data, n, out, cnt.ctypes.data,
                               self.nthreads)
        self._check(st)
        return (out, cnt) if return_counts else out

    def forward_paper(self, x, precision=64, ids=None):
        """The paper's Moller-Trumbore / eps-escalation propagation (Algorithms
        1-2) in float32 or float64 for the listed rays; returns (b rounded to
        float32, counts {rays, steps, escalations, halted, looped})."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        ids_a, n = self._ids(ids)
        out = np.zeros(n, np.float64)
        cnt = np.zeros(5, np.int64)
        st = lib().orc_forward_paper(self.mesh._h, self._cone, self.angles, self.na, x,
                                     None if ids_a is None else ids_a.ctypes.data, n, int(precision), out, cnt,
                                     self.nthreads)
        self._check(st)
        return out, dict(zip(("rays", "steps", "escalations", "halted", "looped"), (int(c) for c in cnt)))

    def backproject(self, y, ids=None):
        """xhat_i = sum_j a_ij y_j over the listed rays (y given per listed ray), float64."""
        y = np.ascontiguousarray(y, dtype=np.float32).ravel()
        ids_a, n = self._ids(ids)
        assert len(y) == n
        out = np.zeros(self.nt, np.float64)
        st = lib().orc_backproject(self.mesh._h, self._cone, self.angles, self.na, y,
                                   None if ids_a is None else ids_a.ctypes.data, n, out, self.nthreads)
        self._check(st)
        return out

    def backproject_ext(self, y, ids=None):
        """(xhat, support, count) over the listed rays: xhat_i = sum_j a_ij y_j,
        support_i = sum of y_j over the rays j with a_ij > 0, count_i = their
        number (the last two size error bounds in tests)."""
        y = np.ascontiguousarray(y, dtype=np.float32).ravel()
        ids_a, n = self._ids(ids)
        assert len(y) == n
        out = [np.zeros(self.nt, np.float64) for _ in range(3)]
        st = lib().orc_backproject_ext(self.mesh._h, self._cone, self.angles, self.na, y,
                                       None if ids_a is None else ids_a.ctypes.data, n, *out, self.nthreads)
        self._check(st)
        return tuple(out)

    def check_pass(self, x, w, y, ids):
        """One walk of the listed rays giving values and error-bound terms:
        per ray b (Eq. 2), babs = sum a|x|, chord, wx = max of w_t |x_t| over
        the visited tetrahedra; per tetrahedron xhat (Eq. 3), xabs = sum a|y|,
        supp = sum of |y_j| over the rays that visit it (zero-length passages
        included), suppc = the same weighted by chord_j, cnt = the number of
        visits.  y is given per listed ray."""
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        n = len(ids)
        x = np.ascontiguousarray(x, dtype=np.float32)
        w = np.ascontiguousarray(w, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float32).ravel()
        assert len(x) == self.nt and len(w) == self.nt and len(y) == n
        per_ray = [np.zeros(n, np.float64) for _ in range(4)]
        per_tet = [np.zeros(self.nt, np.float64) for _ in range(5)]
        st = lib().orc_check_pass(self.mesh._h, self._cone, self.angles, self.na, x, w, y, ids, n, *per_ray,
                                  *per_tet, self.nthreads)
        self._check(st)
        names = ("b", "babs", "chord", "wx", "xhat", "xabs", "supp", "suppc", "cnt")
        return dict(zip(names, per_ray + per_tet))

    def trace(self, ids):
        """List of (tets int32, lengths float64) per listed ray."""
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        n = len(ids)
        off = np.zeros(n + 1, np.int64)
        cap = max(1024, 64 * n)
        while True:
            tets = np.zeros(cap, np.int32)
            lens = np.zeros(cap, np.float64)
            st = lib().orc_trace(self.mesh._h, self._cone, self.angles, self.na, ids, n, off, tets, lens, cap)
            if st == -10:
                cap = int(off[-1])
                continue
            self._check(st)
            return [(tets[off[i]:off[i + 1]].copy(), lens[off[i]:off[i + 1]].copy()) for i in range(n)]

    def trace_rays(self, S, P, U, V):
        return trace_rays(self.mesh, S, P, U, V)

    def rays(self, ids):
        return rays_of(self.cone, self.angles, ids)


def trace_rays(mesh: OracleMesh, S, P, U, V):
    """Trace caller-given rays (float32 [n,3] arrays) through an OracleMesh."""
    S, P, U, V = (np.ascontiguousarray(np.asarray(a, np.float32).reshape(-1, 3)) for a in (S, P, U, V))
    n = len(S)
    off = np.zeros(n + 1, np.int64)
    cap = max(1024, 64 * n)
    while True:
        tets = np.zeros(cap, np.int32)
        lens = np.zeros(cap, np.float64)
        st = lib().orc_trace_rays(mesh._h, S, P, U, V, n, off, tets, lens, cap)
        if st == -10:
            cap = int(off[-1])
            continue
        if st != 0:
            raise OracleError(st, lib().orc_last_error().decode())
        return [(tets[off[i]:off[i + 1]].copy(), lens[off[i]:off[i + 1]].copy()) for i in range(n)]
