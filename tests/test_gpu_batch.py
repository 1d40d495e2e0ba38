"""Batched persistent launches, vector sets, angle ranges, graph replay and the tile autotuner."""

import ctypes
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from parity_bars import assert_within, backprojection_reference, element_size

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
f32 = np.float32


def _tct():
    import paper_1908_06909_amd as tct

    return tct


_problems = None


def problems():
    """Six problems of uneven size: Kuhn n^3 with jitter, own detectors and angle counts."""
    global _problems
    if _problems is None:
        tct = _tct()
        out = []
        for k, (n, det, na) in enumerate([(3, 16, 5), (6, 24, 9), (4, 40, 3), (9, 32, 12), (5, 20, 17), (7, 48, 6)]):
            w = synth.jittered_kuhn(n, 600 + k, 700 + k, det, det, na)
            mesh = tct.TetMesh(w.verts, w.tets, device=DEV)
            geom = tct.ConeGeometry(w.cone, w.angles, device=DEV)
            P = tct.Projector(mesh, geom)
            out.append((w, P))
        _problems = out
    return _problems


def test_batch_forward_is_bitwise_the_plain_forward_with_any_tiles():
    tct = _tct()
    probs = problems()
    Ps = [P for _, P in probs]
    xs = [P.mesh.to_internal(torch.as_tensor(w.x, device=DEV)) for w, P in probs]
    plain = [P.forward(x).reshape(-1).clone() for P, x in zip(Ps, xs)]
    for tiles in (None, [4, 8, 16, 32, 64, 8]):
        B = tct.BatchProjector(Ps, tiles)
        assert B.items > 0
        outs = [torch.full((P.geom.nrays,), -7.0, device=DEV) for P in Ps]
        B.forward(tct.VecSet(xs), tct.VecSet(outs))
        for k in range(len(Ps)):
            assert torch.equal(outs[k], plain[k]), (tiles, k)
    for P in Ps:
        assert P.mesh.stats(reset=True)["failed"] == 0


def test_batch_backprojection_matches_plain_and_oracle():
    tct = _tct()
    probs = problems()
    Ps = [P for _, P in probs]
    rng = np.random.default_rng(5)
    ys = [torch.as_tensor(rng.uniform(0, 1, P.geom.nrays).astype(f32), device=DEV) for P in Ps]
    B = tct.BatchProjector(Ps)
    outs = [torch.full((P.nt,), 3.0, device=DEV) for P in Ps]
    B.backproject(tct.VecSet(ys), tct.VecSet(outs))
    for k, ((w, P), y, o) in enumerate(zip(probs, ys, outs)):
        ref_plain = P.backproject(y)
        assert torch.allclose(o, ref_plain, rtol=1e-5, atol=1e-6)
        # Every element against the oracle at the float-atomic scatter's bar.
        orc = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
        H = element_size(w.verts, w.tets, orc.mesh.tables()[1])
        ref, tol = backprojection_reference(orc, y.cpu().numpy(), H, float_atomic=True)
        got = P.mesh.to_user(o).cpu().numpy()
        assert_within(got, ref, tol, f"batched backprojection, problem {k}")
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


def test_range_launches_assemble_the_full_projection():
    from paper_1908_06909_amd._lib import call, tct_range

    w, P = problems()[3]
    x = P.mesh.to_internal(torch.as_tensor(w.x, device=DEV))
    full = P.forward(x).reshape(-1)
    part = torch.full_like(full, -1.0)
    s = torch.cuda.current_stream().cuda_stream
    na = P.geom.na
    for a0, cnt, tile in ((0, 5, 16), (5, 4, 4), (9, na - 9, 64)):
        call("tct_forward_range", P.mesh.handle, P.geom.handle, x.data_ptr(), part.data_ptr(), P.entry.data_ptr(),
             ctypes.byref(tct_range(a0, cnt, tile)), s)
    assert torch.equal(part, full)
    y = torch.rand(P.geom.nrays, device=DEV)
    acc = torch.zeros(P.nt, device=DEV)
    for a0, cnt in ((0, 7), (7, na - 7)):
        call("tct_backproject_range", P.mesh.handle, P.geom.handle, y.data_ptr(), acc.data_ptr(), 1, 1,
             P.entry.data_ptr(), ctypes.byref(tct_range(a0, cnt, 8)), s)
    whole = P.backproject(y, mode="gather")
    assert torch.allclose(acc, whole, rtol=1e-6, atol=1e-6)


def test_vector_set_kernels():
    tct = _tct()
    rng = np.random.default_rng(9)
    lens = [1, 300, 70000, 5]
    a = [torch.as_tensor(rng.normal(size=n).astype(f32), device=DEV) for n in lens]
    b = [torch.as_tensor(rng.normal(size=n).astype(f32), device=DEV) for n in lens]
    A, Bv = tct.VecSet(a), tct.VecSet(b)
    ops = tct.SetOps(torch.device(DEV), len(lens))
    out = torch.zeros(len(lens), dtype=torch.float64, device=DEV)
    ops.dot(A, Bv, out)
    ref = [float((x.double() * y.double()).sum()) for x, y in zip(a, b)]
    assert np.allclose(out.cpu().numpy(), ref, rtol=1e-12, atol=1e-12)
    num = torch.tensor([1.0, 2.0, 3.0, 4.0], dtype=torch.float64, device=DEV)
    den = torch.tensor([2.0, 0.0, 3.0, 8.0], dtype=torch.float64, device=DEV)
    y0 = [t.clone() for t in a]
    ops.axpy_ratio(A, Bv, num, den, -1.0)
    for k in range(len(lens)):
        ratio = 0.0 if den[k] == 0 else float(num[k] / den[k])
        assert torch.allclose(a[k], y0[k] - np.float32(ratio) * b[k], rtol=1e-6, atol=1e-6)
    ops.xpay_ratio(A, Bv, num, den)
    ops.fill(Bv, 2.5)
    assert all(torch.all(t == 2.5) for t in b)


def test_batch_cgls_graph_replays_match_eager_and_plain():
    tct = _tct()
    probs = problems()
    Ps = [P for _, P in probs]
    bs = [P.forward(P.mesh.to_internal(torch.as_tensor(w.x, device=DEV))).reshape(-1).clone() for w, P in probs]
    B = tct.BatchProjector(Ps)
    eager = tct.BatchCGLS(B, bs)
    graphed = tct.BatchCGLS(B, bs)
    plain = tct.PlainCGLS(Ps, bs)
    graphed.capture()
    for it in range(5):
        eager.step()
        graphed.graph.replay()
        plain.run(1)
        torch.cuda.synchronize()
        _ = Ps[0].forward(Ps[0].mesh.to_internal(torch.as_tensor(probs[0][0].x, device=DEV)))  # eager work between replays
        torch.cuda.synchronize()
        for k in range(len(Ps)):
            xe, xg, xp = eager.x[k], graphed.x[k], plain.x[k]
            scale = float(xe.norm()) + 1e-30
            assert float((xg - xe).norm()) <= 1e-4 * scale, (it, k)
            assert float((xp - xe).norm()) <= 1e-4 * scale, (it, k)
        rre, rrg = eager.rr.cpu().numpy(), graphed.rr.cpu().numpy()
        assert np.allclose(rrg, rre, rtol=1e-4, atol=0), (it, rre, rrg)
    # residuals decreased for every problem
    assert np.all(eager.rr.cpu().numpy() < eager.rr0.cpu().numpy())


def test_autotune_picks_a_candidate_and_caches(tmp_path):
    tct = _tct()
    w, P = problems()[5]
    path = os.path.join(str(tmp_path), "tune.json")
    res = tct.autotune.tune(P, n_angles=2, reps=1, cache_path=path, min_rays=0)
    assert res["tile_u"] in (4, 8, 16, 32, 64)
    assert set(res["ms"]) == {"4", "8", "16", "32", "64"}
    with open(path) as f:
        cached = json.load(f)
    assert len(cached) == 1
    assert tct.autotune.tune(P, cache_path=path) == res


def test_batch_autotune_tiles_and_queue_chunk_then_same_results():
    """The batch tuner times tiles per problem and the queue chunk on the
    persistent batched kernel itself; whatever it picks, the batched forward
    equals the plain one bit for bit and the batched backprojection matches
    the plain scatter."""
    tct = _tct()
    probs = problems()
    Ps = [P for _, P in probs]
    tuned = tct.autotune.tune_batch(Ps, n_angles=2, reps=1, min_rays=0)
    assert len(tuned["tile_u"]) == len(Ps) and all(t in (4, 8, 16, 32, 64) for t in tuned["tile_u"])
    assert tuned["queue_chunk"] in (1, 2, 4, 8)
    assert set(tuned["queue_ms"]) == {"1", "2", "4", "8"}
    B = tct.BatchProjector(Ps, tuned["tile_u"])
    B.set_queue_chunk(tuned["queue_chunk"])
    xs = [P.mesh.to_internal(torch.as_tensor(w.x, device=DEV)) for w, P in probs]
    outs = [torch.empty(P.geom.nrays, device=DEV) for P in Ps]
    B.forward(tct.VecSet(xs), tct.VecSet(outs))
    for P, x, o in zip(Ps, xs, outs):
        assert torch.equal(o, P.forward(x).reshape(-1))
    ys = [torch.rand(P.geom.nrays, device=DEV) for P in Ps]
    xh = [torch.empty(P.nt, device=DEV) for P in Ps]
    for c in (1, 3, 64):
        B.set_queue_chunk(c)
        B.backproject(tct.VecSet(ys), tct.VecSet(xh))
        for P, y, got in zip(Ps, ys, xh):
            ref = P.backproject(y)
            assert torch.allclose(got, ref, rtol=1e-5, atol=1e-6 * float(ref.abs().max())), c
    with pytest.raises(tct._lib.TctError):
        B.set_queue_chunk(0)
    for P in Ps:
        assert P.mesh.stats(reset=True)["failed"] == 0


def test_batched_autograd_matches_per_problem_autograd():
    """The batched autograd Function (one launch per direction for all
    problems): projections equal the per-problem TetProject ones bit for
    bit, the gradients of sum_k 0.5 |A_k x_k - b_k|^2 match the per-problem
    gradients (the two backprojections add the same terms in different
    float orders), and steepest-descent steps with exact line search driven
    by those gradients follow the same losses."""
    tct = _tct()
    probs = problems()
    Ps = [P for _, P in probs]
    B = tct.BatchProjector(Ps)
    rng = np.random.default_rng(11)
    bs = [torch.as_tensor(rng.uniform(0, 1, P.geom.nrays).astype(f32), device=DEV).reshape(P.geom.shape)
          for P in Ps]
    xb = [torch.as_tensor(rng.uniform(0, 1, P.nt).astype(f32), device=DEV) for P in Ps]
    xp = [x.clone() for x in xb]
    losses_b, losses_p = [], []
    for it in range(3):
        vb = [x.clone().requires_grad_() for x in xb]
        vp = [x.clone().requires_grad_() for x in xp]
        pb = tct.project_batch(B, vb)
        pp = [tct.project(v, P) for v, P in zip(vp, Ps)]
        if it == 0:
            for a, c in zip(pb, pp):
                assert torch.equal(a.detach(), c.detach())
        lb = [0.5 * ((p - b) ** 2).sum() for p, b in zip(pb, bs)]
        lp = [0.5 * ((p - b) ** 2).sum() for p, b in zip(pp, bs)]
        sum(lb).backward()
        sum(lp).backward()
        for v1, v2 in zip(vb, vp):
            scale = float(v2.grad.abs().max())
            assert torch.allclose(v1.grad, v2.grad, rtol=1e-5, atol=1e-6 * scale), it
        losses_b.append([float(l.detach()) for l in lb])
        losses_p.append([float(l.detach()) for l in lp])
        # x <- x - alpha g with alpha = |g|^2 / |A g|^2 (exact for least squares)
        gb = [v.grad.detach() for v in vb]
        gp = [v.grad.detach() for v in vp]
        agb = tct.project_batch(B, gb)
        agp = [P.forward(g) for g, P in zip(gp, Ps)]
        xb = [x - (g.square().sum() / a.square().sum()) * g for x, g, a in zip(xb, gb, agb)]
        xp = [x - (g.square().sum() / a.square().sum()) * g for x, g, a in zip(xp, gp, agp)]
    lb, lp = np.array(losses_b), np.array(losses_p)
    assert np.all(lb[1:] < lb[:-1])
    assert np.allclose(lb, lp, rtol=1e-4, atol=0), (lb, lp)
