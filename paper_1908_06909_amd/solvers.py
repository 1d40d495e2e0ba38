"""Differentiable projector and iterative reconstruction on top of A and A^T.

The paper's operator is the linear model A x = b (Section II-A, Eq. 1); the
solvers it names (SART, CGLS) need only A x and A^T y computed on the fly
(matrix-free).  Here:

* ``TetProject`` is a ``torch.autograd.Function`` whose forward is the
  projection and whose backward is the backprojection (A^T is the adjoint of
  A, so the gradient of any loss L(A x) is A^T dL/d(Ax)).
* ``cgls`` runs conjugate gradients on the normal equations
  (A^T A x = A^T b) with the textbook recurrence.
* ``sirt`` runs x += lam * C A^T R (b - A x), R = 1 / (A 1), C = 1 / (A^T 1).
* ``os_sart`` is the ordered-subset form the paper reconstructs with
  (Section III-A: 50 iterations, blocks of 20 projections): the same update
  per block of consecutive angles, with the block's own R and C, through
  angle-range launches.

Every vector operation is a library kernel (tct_dot, tct_axpy_ratio, ...);
step-size scalars stay on the device.  Vectors are float32 in the mesh's
internal order.
"""

from __future__ import annotations

from typing import Callable, Optional

import torch

from ._lib import TCT_DOT_WORKSPACE, call
from .projector import Projector, _stream


class TetProject(torch.autograd.Function):
    """b = A x with dL/dx = A^T dL/db."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, projector: Projector, bp_mode: str = "atomic"):
        ctx.projector = projector
        ctx.bp_mode = bp_mode
        return projector.forward(x.detach().contiguous())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        g = ctx.projector.backproject(grad_out.detach().contiguous().to(torch.float32), mode=ctx.bp_mode)
        return g, None, None


def project(x: torch.Tensor, projector: Projector, bp_mode: str = "atomic") -> torch.Tensor:
    """Differentiable forward projection of x (float32 [nt], internal order)."""
    return TetProject.apply(x, projector, bp_mode)


class Vec:
    """Device vector kernels on one stream with a reusable dot workspace."""

    def __init__(self, device):
        self.device = device
        self.ws = torch.empty(TCT_DOT_WORKSPACE, dtype=torch.float64, device=device)

    def s(self):
        return _stream(self.device)

    def dot(self, a, b, out):
        call("tct_dot", a.data_ptr(), b.data_ptr(), a.numel(), out.data_ptr(), self.ws.data_ptr(), self.s())

    def axpy_ratio(self, y, x, num, den, sign):
        call("tct_axpy_ratio", y.data_ptr(), x.data_ptr(), y.numel(), num.data_ptr(), den.data_ptr(), float(sign),
             self.s())

    def xpay_ratio(self, p, x, num, den):
        call("tct_xpay_ratio", p.data_ptr(), x.data_ptr(), p.numel(), num.data_ptr(), den.data_ptr(), self.s())

    def axpby(self, y, x, a, b):
        call("tct_axpby", y.data_ptr(), x.data_ptr(), y.numel(), float(a), float(b), self.s())

    def mul(self, y, a, b):
        call("tct_mul", y.data_ptr(), a.data_ptr(), b.data_ptr(), y.numel(), self.s())

    def recip(self, y, a, eps=0.0):
        call("tct_recip", y.data_ptr(), a.data_ptr(), y.numel(), float(eps), self.s())

    def copy_f64(self, dst, src, n=1):
        call("tct_copy_f64", dst.data_ptr(), src.data_ptr(), int(n), self.s())


def _f32(t, n, device):
    t = t.reshape(-1)
    if t.dtype != torch.float32 or t.device != device or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"expected a contiguous float32 tensor of {n} elements on {device}")
    return t


class CGLS:
    """Conjugate gradients for least squares on one projector.

    State (x, r, p, s, q) lives on the device; ``residuals`` holds ||r_k||^2
    (float64, device) for k = 0..iterations done.
    """

    def __init__(self, P: Projector, b: torch.Tensor, x0: Optional[torch.Tensor] = None, bp_mode: str = "atomic"):
        self.P = P
        self.bp_mode = bp_mode
        dev = P.device
        nt, nr = P.nt, P.geom.nrays
        self.vec = Vec(dev)
        self.b = _f32(b, nr, dev)
        self.x = torch.zeros(nt, dtype=torch.float32, device=dev) if x0 is None else _f32(x0, nt, dev).clone()
        self.r = self.b.clone()
        self.q = torch.empty(nr, dtype=torch.float32, device=dev)
        if x0 is not None:
            P.forward(self.x, out=self.q.view(P.proj_shape))
            self.vec.axpby(self.r, self.q, -1.0, 1.0)
        self.s = P.backproject(self.r, mode=bp_mode)
        self.p = self.s.clone()
        # scalars: [0] gamma = ||s||^2, [1] gamma_new, [2] delta = ||A p||^2
        self.sc = torch.zeros(4, dtype=torch.float64, device=dev)
        self.vec.dot(self.s, self.s, self.sc[0:1])
        self.hist = [torch.zeros(1, dtype=torch.float64, device=dev)]
        self.vec.dot(self.r, self.r, self.hist[0])
        self.k = 0

    def step(self):
        P, v, sc = self.P, self.vec, self.sc
        P.forward(self.p, out=self.q.view(P.proj_shape))
        v.dot(self.q, self.q, sc[2:3])
        v.axpy_ratio(self.x, self.p, sc[0:1], sc[2:3], +1.0)
        v.axpy_ratio(self.r, self.q, sc[0:1], sc[2:3], -1.0)
        P.backproject(self.r, mode=self.bp_mode, out=self.s)
        v.dot(self.s, self.s, sc[1:2])
        v.xpay_ratio(self.p, self.s, sc[1:2], sc[0:1])
        v.copy_f64(sc[0:1], sc[1:2])
        h = torch.empty(1, dtype=torch.float64, device=P.device)
        v.dot(self.r, self.r, h)
        self.hist.append(h)
        self.k += 1

    def run(self, iters: int, callback: Optional[Callable] = None):
        for _ in range(iters):
            self.step()
            if callback is not None:
                callback(self)
        return self.x

    @property
    def residuals(self):
        """||r_k||^2 for every iteration so far (host float64)."""
        return torch.cat(self.hist).cpu().numpy()


def cgls(P: Projector, b: torch.Tensor, iters: int, x0=None, bp_mode: str = "atomic", callback=None):
    """Run ``iters`` CGLS iterations; returns (x, ||r_k||^2 history)."""
    c = CGLS(P, b, x0, bp_mode)
    c.run(iters, callback)
    return c.x, c.residuals


def sirt(P: Projector, b: torch.Tensor, iters: int, lam: float = 1.0, x0=None, bp_mode: str = "atomic",
         eps: float = 1e-12):
    """SIRT: x += lam * C A^T (R (b - A x)) with R = 1/(A 1), C = 1/(A^T 1)."""
    dev = P.device
    nt, nr = P.nt, P.geom.nrays
    v = Vec(dev)
    b = _f32(b, nr, dev)
    x = torch.zeros(nt, dtype=torch.float32, device=dev) if x0 is None else _f32(x0, nt, dev).clone()
    Rw = P.forward(torch.ones(nt, dtype=torch.float32, device=dev)).reshape(-1)
    v.recip(Rw, Rw, eps)
    Cw = P.backproject(torch.ones(nr, dtype=torch.float32, device=dev), mode=bp_mode)
    v.recip(Cw, Cw, eps)
    r = torch.empty(nr, dtype=torch.float32, device=dev)
    s = torch.empty(nt, dtype=torch.float32, device=dev)
    hist = []
    for _ in range(iters):
        P.forward(x, out=r.view(P.proj_shape))
        v.axpby(r, b, 1.0, -1.0)  # r = b - A x
        h = torch.empty(1, dtype=torch.float64, device=dev)
        v.dot(r, r, h)
        hist.append(h)
        v.mul(r, r, Rw)
        P.backproject(r, mode=bp_mode, out=s)
        v.mul(s, s, Cw)
        v.axpby(x, s, lam, 1.0)
    return x, torch.cat(hist).cpu().numpy() if hist else None


class OSSART:
    """Ordered-subset SART on blocks of ``block`` consecutive angles.

    Per block k (angles [a_k, a_k + n_k)):
        x += lam * C_k A_k^T R_k (b_k - A_k x),
    R_k = 1 / (A_k 1) on the block's rays, C_k = 1 / (A_k^T 1) per element.
    A_k and A_k^T are range launches on the full geometry, so the projection
    arrays keep their [na, nv, nu] layout and the entry cache is shared.
    """

    def __init__(self, P: Projector, b: torch.Tensor, block: int = 20, lam: float = 1.0, x0=None,
                 bp_mode: str = "atomic", eps: float = 1e-12):
        dev = P.device
        nt, na = P.nt, P.geom.na
        self.P, self.lam, self.bp_mode = P, float(lam), bp_mode
        self.v = Vec(dev)
        self.b = _f32(b, P.geom.nrays, dev).reshape(P.proj_shape)
        self.x = torch.zeros(nt, dtype=torch.float32, device=dev) if x0 is None else _f32(x0, nt, dev).clone()
        self.blocks = [(a, min(block, na - a)) for a in range(0, na, block)]
        ones_x = torch.ones(nt, dtype=torch.float32, device=dev)
        ones_y = torch.ones(P.proj_shape, dtype=torch.float32, device=dev)
        # R: every block's slab of A 1 (disjoint slabs make one array).
        self.R = torch.empty(P.proj_shape, dtype=torch.float32, device=dev)
        self.C = []
        for a0, n in self.blocks:
            P.forward_range(ones_x, a0, n, self.R)
            c = P.backproject_range(ones_y, a0, n, mode=bp_mode)
            self.v.recip(c, c, eps)
            self.C.append(c)
        self.v.recip(self.R.view(-1), self.R.view(-1), eps)
        self.r = torch.empty(P.proj_shape, dtype=torch.float32, device=dev)
        self.s = torch.empty(nt, dtype=torch.float32, device=dev)
        self.hist = []

    def residual(self):
        """||b - A x||^2 (float64 device scalar)."""
        self.P.forward(self.x, out=self.r)
        self.v.axpby(self.r.view(-1), self.b.view(-1), 1.0, -1.0)
        h = torch.empty(1, dtype=torch.float64, device=self.P.device)
        self.v.dot(self.r.view(-1), self.r.view(-1), h)
        return h

    def step(self):
        P, v = self.P, self.v
        for (a0, n), c in zip(self.blocks, self.C):
            P.forward_range(self.x, a0, n, self.r)
            rk, bk, Rk = self.r[a0:a0 + n].reshape(-1), self.b[a0:a0 + n].reshape(-1), self.R[a0:a0 + n].reshape(-1)
            v.axpby(rk, bk, 1.0, -1.0)  # r_k = b_k - A_k x
            v.mul(rk, rk, Rk)
            P.backproject_range(self.r, a0, n, mode=self.bp_mode, out=self.s)
            v.mul(self.s, self.s, c)
            v.axpby(self.x, self.s, self.lam, 1.0)

    def run(self, iters: int, track: bool = True):
        for _ in range(iters):
            if track:
                self.hist.append(self.residual())
            self.step()
        return self.x


def os_sart(P: Projector, b: torch.Tensor, iters: int, block: int = 20, lam: float = 1.0, x0=None,
            bp_mode: str = "atomic", track: bool = True):
    """Run ``iters`` OS-SART sweeps; returns (x, ||b - A x_k||^2 before each sweep)."""
    s = OSSART(P, b, block, lam, x0, bp_mode)
    s.run(iters, track)
    return s.x, (torch.cat(s.hist).cpu().numpy() if s.hist else None)
