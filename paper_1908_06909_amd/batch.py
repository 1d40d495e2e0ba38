"""Batched projection and reconstruction over many independent problems.

One persistent launch walks the pixel blocks of every problem (each with its
own mesh and cone-beam geometry) from device work lists (one per die of the
chip, each a contiguous run of every problem's blocks); vector arguments
are device-resident pointer tables ("vector sets"), so one CGLS iteration over
all problems is a fixed sequence of library launches with no host data and
can be captured once and replayed as a HIP graph.
"""

from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import TCT_VECSET_DOT_WORKSPACE, call, lib
from .projector import Projector, _stream
from .solvers import Vec


class VecSet:
    """Device table of pointers to float32 tensors (kept alive by this object)."""

    def __init__(self, tensors: Sequence[torch.Tensor]):
        self.tensors = list(tensors)
        dev = self.tensors[0].device
        for t in self.tensors:
            if t.dtype != torch.float32 or not t.is_contiguous() or t.device != dev:
                raise ValueError("vector sets need contiguous float32 tensors on one device")
        n = len(self.tensors)
        ptrs = (C.c_void_p * n)(*[t.data_ptr() for t in self.tensors])
        lens = (C.c_int64 * n)(*[t.numel() for t in self.tensors])
        h = C.c_void_p()
        call("tct_vecset_create", n, ptrs, lens, dev.index, C.byref(h))
        self._h = h
        self.n = n
        self.device = dev

    @property
    def handle(self):
        return self._h

    def __getitem__(self, k):
        return self.tensors[k]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib._lib is not None:
            _lib._lib.tct_vecset_destroy(h)
            self._h = None


class SetOps:
    """Batched vector kernels over vector sets (one launch for all problems)."""

    def __init__(self, device, n):
        self.device = device
        self.ws = torch.empty(n * TCT_VECSET_DOT_WORKSPACE, dtype=torch.float64, device=device)

    def dot(self, a: VecSet, b: VecSet, out: torch.Tensor):
        call("tct_vecset_dot", a.handle, b.handle, out.data_ptr(), self.ws.data_ptr(), _stream(self.device))

    def axpy_ratio(self, y: VecSet, x: VecSet, num, den, sign):
        call("tct_vecset_axpy_ratio", y.handle, x.handle, num.data_ptr(), den.data_ptr(), float(sign),
             _stream(self.device))

    def xpay_ratio(self, p: VecSet, x: VecSet, num, den):
        call("tct_vecset_xpay_ratio", p.handle, x.handle, num.data_ptr(), den.data_ptr(), _stream(self.device))

    def fill(self, y: VecSet, value: float):
        call("tct_vecset_fill", y.handle, float(value), _stream(self.device))


class BatchProjector:
    """A_k for k = 0..n-1 behind one persistent launch per direction."""

    def __init__(self, projectors: Sequence[Projector], tile_u: Optional[Sequence[int]] = None):
        self.projectors = list(projectors)
        n = len(self.projectors)
        self.n = n
        self.device = self.projectors[0].device
        meshes = (C.c_void_p * n)(*[P.mesh.handle.value for P in self.projectors])
        geoms = (C.c_void_p * n)(*[P.geom.handle.value for P in self.projectors])
        tiles = None if tile_u is None else (C.c_int32 * n)(*[int(t) for t in tile_u])
        entries = (C.c_void_p * n)(*[(P.entry.data_ptr() if P.entry is not None else None) for P in self.projectors])
        h = C.c_void_p()
        call("tct_batch_create", meshes, geoms, n, tiles, entries, C.byref(h))
        self._h = h
        self.items = int(lib().tct_batch_items(h))
        self.tile_u = list(tile_u) if tile_u is not None else [8] * n
        self.queue_chunk = 1

    def set_queue_chunk(self, blocks_per_fetch: int):
        """Pixel blocks a workgroup takes from a work list per fetch (1..64)."""
        call("tct_batch_set_queue_chunk", self._h, int(blocks_per_fetch))
        self.queue_chunk = int(blocks_per_fetch)

    def forward(self, x: VecSet, proj: VecSet):
        call("tct_batch_forward", self._h, x.handle, proj.handle, _stream(self.device))

    def backproject(self, proj: VecSet, xhat: VecSet, accumulate: bool = False):
        call("tct_batch_backproject", self._h, proj.handle, xhat.handle, 1 if accumulate else 0, _stream(self.device))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib._lib is not None:
            _lib._lib.tct_batch_destroy(h)
            self._h = None


class BatchTetProject(torch.autograd.Function):
    """(b_0, ..., b_{n-1}) = (A_0 x_0, ..., A_{n-1} x_{n-1}) for every problem of
    a BatchProjector in one launch, with dL/dx_k = A_k^T dL/db_k for all k in
    one batched backprojection launch (the batched form of TetProject)."""

    @staticmethod
    def forward(ctx, batch: "BatchProjector", *xs: torch.Tensor):
        ctx.batch = batch
        dev = batch.device
        xs = [x.detach().contiguous() for x in xs]
        outs = [torch.empty(P.geom.shape, dtype=torch.float32, device=dev) for P in batch.projectors]
        batch.forward(VecSet(xs), VecSet(outs))
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads: torch.Tensor):
        batch = ctx.batch
        dev = batch.device
        gs = [torch.zeros(P.geom.shape, dtype=torch.float32, device=dev) if g is None
              else g.detach().contiguous().to(torch.float32) for g, P in zip(grads, batch.projectors)]
        xh = [torch.empty(P.nt, dtype=torch.float32, device=dev) for P in batch.projectors]
        batch.backproject(VecSet(gs), VecSet(xh))
        return (None, *xh)


def project_batch(batch: "BatchProjector", xs: Sequence[torch.Tensor]) -> List[torch.Tensor]:
    """Differentiable forward projections of every problem of `batch` (x_k
    float32 [nt_k], internal order; each result shaped like the problem's
    projections, as `project` returns them), one launch per direction."""
    if len(xs) != batch.n:
        raise ValueError(f"expected {batch.n} tensors, got {len(xs)}")
    return list(BatchTetProject.apply(batch, *xs))


class BatchCGLS:
    """CGLS on every problem of a batch at once; one iteration is nine launches.

    ``step()`` runs one iteration eagerly; ``capture()`` records one iteration
    as a graph and ``run(k, graph=True)`` replays it k times.
    """

    def __init__(self, batch: BatchProjector, b: Sequence[torch.Tensor]):
        self.B = batch
        dev = batch.device
        n = batch.n
        self.ops = SetOps(dev, n)
        nts = [P.nt for P in batch.projectors]
        nrs = [P.geom.nrays for P in batch.projectors]
        f = lambda m: torch.zeros(m, dtype=torch.float32, device=dev)  # noqa: E731
        self.x = [f(m) for m in nts]
        self.s = [f(m) for m in nts]
        self.p = [f(m) for m in nts]
        self.r = [bk.reshape(-1).to(torch.float32).clone() for bk in b]
        self.q = [f(m) for m in nrs]
        for k in range(n):
            if self.r[k].numel() != nrs[k]:
                raise ValueError(f"b[{k}] has {self.r[k].numel()} elements, expected {nrs[k]}")
        self.X, self.S, self.P, self.R, self.Q = (VecSet(v) for v in (self.x, self.s, self.p, self.r, self.q))
        self.gamma = torch.zeros(n, dtype=torch.float64, device=dev)
        self.gamma_new = torch.zeros(n, dtype=torch.float64, device=dev)
        self.delta = torch.zeros(n, dtype=torch.float64, device=dev)
        self.rr = torch.zeros(n, dtype=torch.float64, device=dev)
        self.vec = Vec(dev)
        # r = b (x0 = 0); s = A^T r; p = s; gamma = |s|^2
        batch.backproject(self.R, self.S)
        for k in range(n):
            self.p[k].copy_(self.s[k])
        self.ops.dot(self.S, self.S, self.gamma)
        self.ops.dot(self.R, self.R, self.rr)
        self.rr0 = self.rr.clone()
        self.graph = None
        self.k = 0

    def step(self):
        B, o = self.B, self.ops
        B.forward(self.P, self.Q)
        o.dot(self.Q, self.Q, self.delta)
        o.axpy_ratio(self.X, self.P, self.gamma, self.delta, +1.0)
        o.axpy_ratio(self.R, self.Q, self.gamma, self.delta, -1.0)
        B.backproject(self.R, self.S)
        o.dot(self.S, self.S, self.gamma_new)
        o.xpay_ratio(self.P, self.S, self.gamma_new, self.gamma)
        self.vec.copy_f64(self.gamma, self.gamma_new, self.B.n)
        o.dot(self.R, self.R, self.rr)

    def capture(self):
        """Record one iteration as a graph (recording runs nothing; replays do)."""
        s = torch.cuda.Stream(device=self.B.device)
        s.wait_stream(torch.cuda.current_stream(self.B.device))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.step()
        torch.cuda.current_stream(self.B.device).wait_stream(s)
        self.graph = g
        return g

    def run(self, iters: int, graph: bool = False):
        if graph and self.graph is None:
            self.capture()
        for _ in range(iters):
            if graph:
                self.graph.replay()
            else:
                self.step()
            self.k += 1
        return self.x


class PlainCGLS:
    """The same iterations with one solver object per problem (per-problem launches)."""

    def __init__(self, projectors: Sequence[Projector], b: Sequence[torch.Tensor]):
        from .solvers import CGLS

        self.solvers = [CGLS(P, bk.reshape(-1)) for P, bk in zip(projectors, b)]

    def run(self, iters: int):
        for _ in range(iters):
            for s in self.solvers:
                s.step()

    @property
    def x(self):
        return [s.x for s in self.solvers]
