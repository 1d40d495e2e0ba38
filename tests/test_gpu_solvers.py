"""GPU autograd and iterative reconstruction against the float64 oracle.

* gradient of 0.5 ||A x - b||^2 through TetProject (backward = backprojection)
  vs the oracle's A^T (A x - b), on the Kuhn 8^3 / 64^2 x 16 workload with
  b = A x_tilde, x_tilde ~ U[0,1] (seed 3);
* float32 directional central differences of the same loss on the GPU;
* CGLS residual history vs float64 CGLS on the oracle's matrix;
* SIRT residual history vs float64 SIRT;
* OS-SART (blocks of consecutive angles through range launches) residual
  history and iterate vs float64 OS-SART on the oracle's matrix, with the
  scatter and the element-driven backprojection;
* 50 CGLS iterations on the 64^3 jittered mesh / 512^2 x 360 geometry
  reconstructing the sphere phantom from its own projections: residual and
  error norms non-increasing.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import solvers as osolv

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
f32 = np.float32


class Setup:
    def __init__(self):
        import paper_1908_06909_amd as tct

        self.tct = tct
        self.w = synth.config(3)
        self.orc = oracle.Oracle(self.w.verts, self.w.tets, self.w.cone, self.w.angles)
        self.A = osolv.system_matrix(self.orc)
        self.xt = synth.uniform_random(self.orc.nt, self.w.meta["target_seed"]).astype(np.float64)
        self.b = self.A @ self.xt
        self.mesh = tct.TetMesh(self.w.verts, self.w.tets, device=DEV)
        self.geom = tct.ConeGeometry(self.w.cone, self.w.angles, device=DEV)
        self.P = tct.Projector(self.mesh, self.geom)
        self.b_t = torch.as_tensor(self.b.astype(f32), device=DEV)

    def internal(self, x_user):
        return self.mesh.to_internal(torch.as_tensor(np.ascontiguousarray(x_user, f32), device=DEV))

    def user(self, x_int):
        return self.mesh.to_user(x_int.detach().contiguous()).cpu().numpy().astype(np.float64)


_S = None


def setup():
    global _S
    if _S is None:
        _S = Setup()
    return _S


@pytest.mark.parametrize("bp_mode", ["atomic", "gather"])
def test_gradient_matches_oracle(bp_mode):
    S = setup()
    x = S.w.x.astype(np.float64)
    xi = S.internal(S.w.x).requires_grad_(True)
    proj = S.tct.project(xi, S.P, bp_mode)
    loss = 0.5 * ((proj.reshape(-1).double() - S.b_t.double()) ** 2).sum()
    loss.backward()
    g = S.user(xi.grad)
    r = S.A @ x - S.b
    g_ref = S.A.T @ r
    # error sources: lengths/projections (1e-5 relative), residual cancellation,
    # float32 accumulation of n_i terms into each element
    nterm = np.diff(S.A.tocsc().indptr)
    scale = S.A.T @ (np.abs(r) + S.A @ np.abs(x) + np.abs(S.b))
    tol = 3e-5 * scale + nterm * 2.0 ** -24 * (S.A.T @ np.abs(r)) + 1e-30
    err = np.abs(g - g_ref)
    assert np.all(err <= tol), f"worst {np.max(err / tol):.3f} x tolerance"
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    # loss value itself
    assert abs(loss.item() - osolv.loss(S.A, x, S.b)) <= 1e-4 * osolv.loss(S.A, x, S.b)


def test_gradient_matches_fp32_central_differences():
    S = setup()
    xi = S.internal(S.w.x).requires_grad_(True)
    proj = S.tct.project(xi, S.P)
    loss = 0.5 * ((proj.reshape(-1).double() - S.b_t.double()) ** 2).sum()
    loss.backward()
    g = xi.grad.detach().double()
    rng = np.random.default_rng(S.w.meta["fd_seed"])
    with torch.no_grad():
        for _ in range(3):
            v = torch.as_tensor(rng.normal(size=S.orc.nt).astype(f32), device=DEV)
            h = 1e-2 * float(xi.norm()) / np.sqrt(S.orc.nt)
            lp = 0.5 * ((S.P.forward(xi + h * v).reshape(-1).double() - S.b_t.double()) ** 2).sum()
            lm = 0.5 * ((S.P.forward(xi - h * v).reshape(-1).double() - S.b_t.double()) ** 2).sum()
            fd = float((lp - lm) / (2 * h))
            gv = float((g * v.double()).sum())
            tol = 1e-3 * abs(gv) + 1e-5 * float((g.abs() * v.double().abs()).sum())
            assert abs(fd - gv) <= tol, (fd, gv, tol)


def test_cgls_history_matches_oracle():
    S = setup()
    iters = 50
    x, rr = S.tct.cgls(S.P, S.b_t, iters)
    _, rr_ref, _ = osolv.cgls(S.A, S.b, iters)
    _, rr32, _ = osolv.cgls(S.A, S.b, iters, precision=32)
    rel = np.abs(rr - rr_ref) / rr_ref
    # Identical recurrences agree closely until float32 rounding erodes the
    # conjugacy of the search directions; after that the float64 history is
    # no longer the reference: the same recurrence with float32 vectors on
    # the CPU departs from it by up to a factor ~4 on this system (pinned in
    # test_oracle_solvers.py), and the GPU, another float32 evaluation of
    # it, must follow that float32 history within a factor 1.5.
    print("GPU / float64:", np.round((rr / rr_ref)[::5], 3))
    print("GPU / float32 CPU:", np.round((rr / rr32)[::5], 3))
    assert np.all(rel[:11] <= 1e-4), rel[:11]
    ratio32 = rr / rr32
    assert np.all((ratio32 > 1 / 1.5) & (ratio32 < 1.5)), ratio32
    assert np.all(np.diff(rr) <= 1e-6 * rr[0])
    assert rr[-1] <= 1e-5 * rr[0]


def test_sirt_history_matches_oracle():
    S = setup()
    iters = 10
    x, rr = S.tct.sirt(S.P, S.b_t, iters)
    _, rr_ref = osolv.sirt(S.A, S.b, iters)
    rel = np.abs(rr - rr_ref) / rr_ref
    assert np.all(rel <= 1e-4), rel


@pytest.mark.parametrize("bp_mode", ["atomic", "shadow"])
def test_os_sart_history_matches_oracle(bp_mode):
    S = setup()
    iters, block = 8, 5  # 16 angles: blocks of 5, 5, 5, 1
    per_angle = S.w.cone.nu * S.w.cone.nv
    na = len(S.w.angles)
    subsets = [np.arange(a * per_angle, min(a + block, na) * per_angle) for a in range(0, na, block)]
    x, rr = S.tct.os_sart(S.P, S.b_t, iters, block=block, bp_mode=bp_mode)
    x_ref, rr_ref = osolv.os_sart(S.A, S.b, iters, subsets)
    rel = np.abs(rr - rr_ref) / rr_ref
    assert np.all(rel <= 1e-4), rel
    xu = S.user(x)
    assert np.linalg.norm(xu - x_ref) <= 1e-4 * np.linalg.norm(x_ref)
    assert rr[-1] < 0.05 * rr[0]


def test_cgls_50_iterations_on_jittered_64():
    import paper_1908_06909_amd as tct

    w = synth.config(1)
    mesh = tct.TetMesh(w.verts, w.tets, device=DEV)
    geom = tct.ConeGeometry(w.cone, w.angles, device=DEV)
    P = tct.Projector(mesh, geom)
    xs = mesh.to_internal(torch.as_tensor(w.x, device=DEV))
    b = P.forward(xs).reshape(-1).clone()
    errs = []
    solver = tct.CGLS(P, b)
    errs.append(float((solver.x - xs).double().norm()))
    solver.run(50, callback=lambda c: errs.append(float((c.x - xs).double().norm())))
    rr = solver.residuals
    assert len(rr) == 51
    assert np.all(np.diff(rr) <= 1e-3 * rr[0]), "residual must not grow"
    assert np.all(np.diff(errs) <= 1e-3 * errs[0]), "error must not grow"
    assert rr[-1] < 1e-2 * rr[0]
    assert errs[-1] < 0.5 * errs[0]
    st = mesh.stats(reset=True)
    assert st["failed"] == 0
