"""The allocation-free reproducible scatter (tct_backproject_fixed_noalloc)
against tct_backproject(mode = TCT_BP_FIXED), through the C ABI.

Both compute the same exact integer sums with the same per-launch scale, so
the results must be the same bits.  Two calls in a row share the device's
static scratch, the second on a smaller mesh and detector, so a stale sum
left by the first call would show.
"""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _problem(n, nu, nv, na, seed):
    import paper_1908_06909_amd as tct

    w = synth.jittered_kuhn(n, seed, seed + 10, nu, nv, na)
    mesh = tct.TetMesh(w.verts, w.tets, device=DEV)
    geom = tct.ConeGeometry(w.cone, w.angles, device=DEV)
    P = tct.Projector(mesh, geom)
    y = torch.as_tensor(np.random.default_rng(seed).uniform(-1, 1, geom.nrays).astype(np.float32), device=DEV)
    return mesh, geom, P, y


def _noalloc(mesh, geom, P, y, out, accumulate):
    from paper_1908_06909_amd._lib import lib

    s = torch.cuda.current_stream().cuda_stream
    return lib().tct_backproject_fixed_noalloc(mesh.handle, geom.handle, y.data_ptr(), out.data_ptr(),
                                               1 if accumulate else 0, P.entry.data_ptr(), s)


def test_noalloc_fixed_scatter_equals_fixed_mode_two_calls():
    for n, nu, nv, na, seed in ((12, 96, 80, 24, 3), (5, 40, 36, 7, 4)):  # second call: smaller input
        mesh, geom, P, y = _problem(n, nu, nv, na, seed)
        ref = P.backproject(y, mode="fixed")
        out = torch.full((mesh.nt,), float("nan"), dtype=torch.float32, device=DEV)
        assert _noalloc(mesh, geom, P, y, out, False) == 0
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"n={n}: {float((out - ref).abs().max())}"
        base = torch.full((mesh.nt,), 0.25, dtype=torch.float32, device=DEV)
        ref_acc = P.backproject(y, mode="fixed", out=base.clone(), accumulate=True)
        acc = base.clone()
        assert _noalloc(mesh, geom, P, y, acc, True) == 0
        torch.cuda.synchronize()
        assert torch.equal(acc, ref_acc)
        print(f"kuhn {n}^3, {geom.nrays} rays: allocation-free scatter equals the fixed mode bit for bit")


def test_noalloc_rejects_meshes_beyond_its_scratch():
    import paper_1908_06909_amd as tct
    from paper_1908_06909_amd._lib import TCT_NOALLOC_MAX_TETS, lib

    X = synth.kuhn_nodes(89)  # 6 * 89^3 = 4,229,814 tetrahedra > 4,194,304
    verts, tets = synth.kuhn_mesh(X, X, X)
    assert len(tets) > TCT_NOALLOC_MAX_TETS
    mesh = tct.TetMesh(verts, tets, device=DEV)
    geom = tct.ConeGeometry(synth.Cone(4.0, 8.0, 8, 8, 0.25, 0.25), synth.angles_for(1), device=DEV)
    y = torch.zeros(geom.nrays, dtype=torch.float32, device=DEV)
    out = torch.zeros(mesh.nt, dtype=torch.float32, device=DEV)
    s = torch.cuda.current_stream().cuda_stream
    st = lib().tct_backproject_fixed_noalloc(mesh.handle, geom.handle, y.data_ptr(), out.data_ptr(), 0, None, s)
    assert st == -1
    assert b"TCT_NOALLOC_MAX_TETS" in lib().tct_last_error()
