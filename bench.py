#!/usr/bin/env python3
"""Throughput of the tetrahedral projector's hot path on one MI355X.

Workload: jittered Kuhn 64^3 mesh of the unit cube (1,572,864 tetrahedra),
sphere phantom, cone beam DSO 4 / DSD 8, 512 x 512 detector, 360 angles
(94,371,840 rays).  One step = entry face of every ray (boundary faces
projected onto the detector and tested exactly, cached for the step) +
forward projection A x + atomic backprojection A^T b of that projection.  The value is tet-segments (walk steps, zero-length
passages included) per second over both walks.

Prints one JSON line.  Main options: --steps K (timed, default 5; kernel
times are medians over the steps), --warmup W (default 2), --gpus N (1
only), --bp MODE (backprojection of the step: atomic, fixed, shadow,
atomic_direct or gather), --gather (also time the gather backprojection as
a variant), --angles N (first N angles only, for profiling passes),
--no-cpu-baseline, --json-extra FILE (per-kernel details), --cgls-problems N
(default 32; 0 skips the batched-vs-plain CGLS leg).  Other modes replace
the line: --batch-cgls N, --os-sart BLOCK, --paper-mode, --init-sweep
SIZES, --copy-calibration BYTES (see --help).
The line's `batched_cgls` object is the metric's second half: CGLS
iterations over the 32-problem ladder in one graph-replayed persistent
launch per direction (autotuned tiles and queue chunk) against one solver
per problem on the plain operators, with both residual histories.  The roofline
object gives the dominant kernel's algorithmic bandwidth against the 8 TB/s
peak and against this box's measured copy bandwidth (`stream_gbs`).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
ROOT = os.path.dirname(os.path.abspath(__file__))
# Measured HBM traffic of the walk kernels (rocprofv3 FETCH_SIZE / WRITE_SIZE
# on this workload, scaled by a copy-kernel calibration), valid only for the
# kernel sources it was measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_walk_kernels_kuhn64_jit_512x512x360.txt")
KERNEL_SOURCES = ["walk.hip", "walk_filter.h", "ray.h", "exact.h", "common.h", "kernels.h"]


def kernel_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1908_06909_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic_bytes(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when it is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(("#", " ")))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_source_sha256") != kernel_digest():
        return None
    try:
        fetch = float(kv[kernel + ".fetch_kib"]) * float(kv["fetch_factor"])
        write = float(kv[kernel + ".write_kib"]) * float(kv["write_factor"])
    except (KeyError, ValueError):
        return None
    return (fetch + write) * 1024.0
FWD_BYTES_PER_SEG = 24  # neighbour id + new vertex id + its xyz + x_i
BWD_BYTES_PER_SEG = 28  # walk geometry (20) + read-modify-write of xhat_i (8)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=1, help="workload index (1 = the benchmark configuration)")
    ap.add_argument("--angles", type=int, default=0,
                    help="use only the first N angles of the workload (profiling passes); 0 = all")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--gather", action="store_true")
    ap.add_argument("--os-sart", type=int, default=0, metavar="BLOCK",
                    help="time OS-SART sweeps with blocks of BLOCK consecutive angles instead")
    ap.add_argument("--paper-mode", action="store_true",
                    help="compare the paper's Moller-Trumbore propagation (float32, float64) with the exact walk")
    ap.add_argument("--init-mesh", default="delaunay", choices=["delaunay", "kuhn"],
                    help="with --init-sweep: mesh family (sizes are points, or n for Kuhn n^3)")
    ap.add_argument("--init-sweep", default="",
                    help="comma-separated mesh sizes (see --init-mesh): entry search (BVH and R*-tree) vs walk "
                         "time, one 1024x1024 projection each")
    ap.add_argument("--bp", default="atomic", choices=["atomic", "fixed", "shadow", "atomic_direct", "gather"],
                    help="backprojection of the timed step")
    ap.add_argument("--json-extra", default=None)
    ap.add_argument("--batch-cgls", type=int, default=0, metavar="NPROB",
                    help="instead of the default line: only batched (one persistent launch per direction, "
                         "graph-replayed) vs plain per-problem CGLS on the first NPROB problems of the 32-problem ladder")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched CGLS with 8-wide tiles and one pixel block per queue fetch instead of autotuned ones")
    ap.add_argument("--cgls-problems", type=int, default=32,
                    help="problems of the ladder in the default line's batched-vs-plain CGLS leg (0 = skip it)")
    ap.add_argument("--cgls-iters", type=int, default=2, help="timed CGLS iterations of that leg")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a device-to-device copy of this many bytes (3 times) to calibrate HBM counters")
    return ap.parse_args()


def cpu_baseline(w, budget_s):
    """The oracle (float64, exact signs) on every k-th ray of the workload,
    forward + backprojection, on all host threads; extrapolated to seg/s."""
    import oracle

    t0 = time.time()
    o = oracle.Oracle(w.verts, w.tets, w.cone, w.angles)
    build_s = time.time() - t0
    n = o.nrays
    # First a small probe to size the sample for the time budget.
    probe = np.arange(0, n, max(1, n // 2000), dtype=np.int64)
    t0 = time.time()
    _, cnt = o.forward(w.x, probe, return_counts=True)
    dt = max(time.time() - t0, 1e-3)
    rate = cnt.sum() / dt
    seg_per_ray = max(cnt.mean(), 1.0)
    want = int(budget_s * 0.5 * rate / seg_per_ray)
    k = max(1, n // max(want, 1))
    ids = np.arange(0, n, k, dtype=np.int64)
    t0 = time.time()
    b, cnt = o.forward(w.x, ids, return_counts=True)
    t1 = time.time()
    o.backproject(b.astype(np.float32), ids)
    t2 = time.time()
    segs = 2 * int(cnt.sum())
    threads = oracle.oracle.max_threads() if o.nthreads == 0 else o.nthreads
    # The same on one thread, on a sample sized for about a sixth of the budget.
    o.nthreads = 1
    rate_all = segs / (t2 - t0)
    k1 = max(1, n // max(1, int(budget_s / 6.0 * rate_all / threads / (2 * seg_per_ray))))
    ids1 = np.arange(0, n, k1, dtype=np.int64)
    t3 = time.time()
    b1, cnt1 = o.forward(w.x, ids1, return_counts=True)
    o.backproject(b1.astype(np.float32), ids1)
    t4 = time.time()
    o.nthreads = 0
    return {
        "value": rate_all,
        "unit": "tet-segments/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"every {k}-th ray ({len(ids)} rays, {segs} segments fwd+back) of the same workload; "
                  f"forward {t1 - t0:.1f}s, backprojection {t2 - t1:.1f}s; mesh build {build_s:.1f}s untimed",
        "single_thread_value": 2 * int(cnt1.sum()) / (t4 - t3),
        "single_thread_sample": f"every {k1}-th ray ({len(ids1)} rays), forward + backprojection {t4 - t3:.1f}s",
        "cpu_model": cpu_model(),
    }


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo) and logical CPU count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name} ({os.cpu_count()} logical CPUs visible, {len(os.sched_getaffinity(0))} usable)"


def init_sweep_bench(args):
    """Initialisation (boundary entry search) against propagation (the walk)
    as the mesh grows, one 1024 x 1024 projection each (the shape of the
    paper's Section III-D study).  Meshes: Delaunay tetrahedralisations of
    random points in the unit cube (few boundary faces), or triangulated
    regular grids (Kuhn n^3, 12 n^2 boundary faces, the paper's benchmark
    meshes).  The entry search is timed through the boundary BVH, through
    the R*-tree of Section II-E and by projecting the boundary onto the
    detector; all three must return the same faces."""
    import torch

    import paper_1908_06909_amd as tct
    import synth

    dev = torch.device("cuda:0")
    cone = synth.Cone(4.0, 8.0, 1024, 1024, 2.0 / 1024, 2.0 / 1024)
    rows = []
    for n in [int(float(v)) for v in args.init_sweep.split(",")]:
        t0 = time.time()
        if args.init_mesh == "kuhn":
            X = synth.kuhn_nodes(n)
            verts, tets = synth.kuhn_mesh(X, X, X)
        else:
            verts, tets = synth.delaunay_mesh(n, 1000 + n % 997)
        t_gen = time.time() - t0
        t0 = time.time()
        mesh = tct.TetMesh(verts, tets, device=dev, rstar=True)
        geom = tct.ConeGeometry(cone, np.array([0.3]), device=dev)
        t_ingest = time.time() - t0
        P = tct.Projector(mesh, geom, cache_entry=False)
        x = torch.ones(mesh.nt, dtype=torch.float32, device=dev)
        entry = torch.empty(geom.nrays, dtype=torch.int32, device=dev)
        entry_r = torch.empty(geom.nrays, dtype=torch.int32, device=dev)
        entry_p = torch.empty(geom.nrays, dtype=torch.int32, device=dev)
        proj = torch.empty(geom.shape, dtype=torch.float32, device=dev)
        P.compute_entry(entry, method="bvh")
        P.compute_entry(entry_r, method="rstar")
        P.compute_entry(entry_p, method="raster")
        P.entry = entry
        P.forward(x, out=proj)
        torch.cuda.synchronize()
        agree = bool(torch.equal(entry, entry_r)) and bool(torch.equal(entry, entry_p))
        mesh.stats(reset=True)
        reps = max(1, args.steps)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        e[0].record()
        for _ in range(reps):
            P.compute_entry(entry, method="bvh")
        e[1].record()
        for _ in range(reps):
            P.compute_entry(entry_r, method="rstar")
        e[2].record()
        for _ in range(reps):
            P.forward(x, out=proj)
        e[3].record()
        for _ in range(reps):
            P.compute_entry(entry_p, method="raster")
        e[4].record()
        torch.cuda.synchronize()
        st = mesh.stats(reset=True)
        walk_rays = st["rays"] - 2 * reps * geom.nrays  # the entry passes count their rays too
        rows.append({"mesh": args.init_mesh, "size": n, "tets": mesh.nt, "boundary_faces": mesh.nboundary,
                     "rstar_height": mesh.rstar()["height"],
                     "entry_bvh_ms": e[0].elapsed_time(e[1]) / reps, "entry_rstar_ms": e[1].elapsed_time(e[2]) / reps,
                     "entry_raster_ms": e[3].elapsed_time(e[4]) / reps,
                     "walk_ms": e[2].elapsed_time(e[3]) / reps, "entries_agree": agree,
                     "segments_per_ray": st["segments"] / max(1, walk_rays),
                     "host_generate_s": t_gen, "host_ingest_s": t_ingest})
        print(json.dumps(rows[-1]), flush=True)
        del P, mesh, geom, entry, entry_r, entry_p, proj, x
    print(json.dumps({"metric": "entry search (BVH, R*-tree, boundary projection) vs walk, one 1024x1024 projection",
                      "data": "synthetic", "rows": rows}))
    if not all(r["entries_agree"] for r in rows):
        sys.exit(1)


def paper_mode_bench(args):
    """The paper's propagation in float32 and float64 against the exact walk
    (the single versus double precision experiment, on a synthetic stand-in)."""
    import torch

    import paper_1908_06909_amd as tct
    import synth

    dev = torch.device("cuda:0")
    w = synth.config(args.workload)
    mesh = tct.TetMesh(w.verts, w.tets, device=dev)
    geom = tct.ConeGeometry(w.cone, w.angles, device=dev)
    P = tct.Projector(mesh, geom)
    x = mesh.to_internal(torch.as_tensor(w.x, device=dev))

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t) * 1e3

    exact, t_exact = timed(lambda: P.forward(x))
    mesh.stats(reset=True)
    exact = exact.reshape(-1).double()
    hit = int((exact != 0).sum())
    out = {"metric": "paper-faithful propagation vs exact walk", "config": {"workload": w.name, "rays": geom.nrays,
           "rays_hitting": hit}, "exact_ms": t_exact, "data": "synthetic"}
    for prec in (32, 64):
        (b, st), ms = timed(lambda: P.forward_paper(x, prec))
        b = b.reshape(-1).double()
        err = (b - exact).abs()
        tol = 1e-5 * torch.clamp(exact.abs(), min=1e-3)
        out[f"float{prec}"] = dict(st, ms=ms, rays_off_by_more_than_1e_5=int((err > tol).sum()),
                                   rays_off_by_more_than_1e_2=int((err > 1e-2 * torch.clamp(exact.abs(), min=1e-3))
                                                                  .sum()),
                                   escalations_per_million_rays=st["escalations"] / max(1, st["rays"]) * 1e6,
                                   max_abs_error=float(err.max()))
    print(json.dumps(out))


def os_sart_bench(args):
    """OS-SART sweeps (blocks of consecutive angles, range launches) on the benchmark workload."""
    import torch

    import paper_1908_06909_amd as tct
    import synth

    dev = torch.device("cuda:0")
    w = synth.config(args.workload)
    mesh = tct.TetMesh(w.verts, w.tets, device=dev)
    geom = tct.ConeGeometry(w.cone, w.angles, device=dev)
    P = tct.Projector(mesh, geom)
    xt = mesh.to_internal(torch.as_tensor(w.x, device=dev))
    b = P.forward(xt).reshape(-1).clone()
    solver = tct.OSSART(P, b, block=args.os_sart, bp_mode=args.bp)
    r0 = float(solver.residual().item())
    solver.run(args.warmup, track=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    solver.run(args.steps, track=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    r = float(solver.residual().item())
    err = float((solver.x - xt).double().norm() / xt.double().norm())
    out = {
        "metric": "OS-SART sweeps/s", "value": args.steps / el, "unit": "sweeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_sweep": el * 1e3 / args.steps,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "block": args.os_sart, "blocks": len(solver.blocks), "bp": args.bp},
        "residual_ratio_after": r / r0, "relative_error_after": err, "sweeps_done": args.steps + args.warmup,
    }
    print(json.dumps(out))


def batched_cgls_leg(n_problems, iters, warmup, tune=True, cache_path=None):
    """Batched against per-problem CGLS on the first n_problems problems of the
    32-problem ladder (independent meshes and geometries).  The batched
    solver runs one persistent launch per direction with autotuned tiles and
    queue chunk, one iteration replayed as a HIP graph; the per-problem
    solvers call the library's plain operators (default tiles).  Both start
    from x = 0 with b = A x_sphere, so their residual histories must agree."""
    import torch

    import paper_1908_06909_amd as tct
    import synth

    dev = torch.device("cuda:0")
    t0 = time.time()
    Ps, bs = [], []
    for b in range(n_problems):
        w = synth.batch_problem(b)
        mesh = tct.TetMesh(w.verts, w.tets, device=dev)
        geom = tct.ConeGeometry(w.cone, w.angles, device=dev)
        P = tct.Projector(mesh, geom)
        x = mesh.to_internal(torch.as_tensor(w.x, device=dev))
        bs.append(P.forward(x).reshape(-1).clone())
        Ps.append(P)
        del w, x
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    t0 = time.time()
    tuned = tct.autotune.tune_batch(Ps, cache_path=cache_path) if tune else {"tile_u": [8] * len(Ps),
                                                                             "queue_chunk": 1}
    tune_s = time.time() - t0
    B = tct.BatchProjector(Ps, tuned["tile_u"])
    B.set_queue_chunk(tuned["queue_chunk"])

    def timed(fn, k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn(k)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    bat = tct.BatchCGLS(B, bs)
    bat.capture()
    bat.run(warmup, graph=True)
    t_bat = timed(lambda k: bat.run(k, graph=True), iters)
    rr_bat = (bat.rr / bat.rr0).cpu().numpy()
    del bat
    pl = tct.PlainCGLS(Ps, bs)
    pl.run(warmup)
    t_pl = timed(pl.run, iters)
    rr_pl = np.array([float(s.hist[-1].item() / s.hist[0].item()) for s in pl.solvers])
    del pl
    for P in Ps:
        P.mesh.stats(reset=True)
    agree = float(np.max(np.abs(rr_bat - rr_pl) / np.maximum(rr_pl, 1e-300)))
    return {
        "problems": len(Ps),
        "tets": int(sum(P.nt for P in Ps)),
        "rays": int(sum(P.geom.nrays for P in Ps)),
        "iterations_timed": iters,
        "warmup": warmup,
        "ms_per_iteration_batched": t_bat * 1e3 / iters,
        "ms_per_iteration_plain": t_pl * 1e3 / iters,
        "speedup": t_pl / t_bat,
        "tile_u": tuned["tile_u"],
        "queue_chunk": tuned["queue_chunk"],
        "residual_ratio_batched_max": float(np.max(rr_bat)),
        "residual_ratio_plain_max": float(np.max(rr_pl)),
        "residual_relative_difference_max": agree,
        # Both are float32 CGLS on the same operators; only the order of the
        # scatter's float atomics differs between them.
        "residual_agreement_bar": 1e-3,
        "residuals_agree": bool(agree <= 1e-3),
        "setup_s": setup_s,
        "tune_s": tune_s,
    }


def batch_cgls_bench(args):
    """Only the batched against per-problem CGLS comparison, as its own line."""
    leg = batched_cgls_leg(args.batch_cgls, max(1, args.steps), args.warmup, tune=not args.no_tune)
    out = {"metric": "batched vs plain CGLS iterations/s", "value": 1e3 / leg["ms_per_iteration_batched"],
           "unit": "CGLS iterations/s (all problems)", "plain_value": 1e3 / leg["ms_per_iteration_plain"],
           "higher_is_better": True, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"batch ladder, first {leg['problems']} problems"}, **leg}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this projector runs on one GPU only: sharding over several GPUs "
                                   "(by angle, one all-reduce for the backprojection) is not launched",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 4 * n, "copies": 3}))
        return

    import synth
    from paper_1908_06909_amd import ConeGeometry, Projector, TetMesh

    if args.batch_cgls:
        batch_cgls_bench(args)
        return
    if args.os_sart:
        os_sart_bench(args)
        return
    if args.paper_mode:
        paper_mode_bench(args)
        return
    if args.init_sweep:
        init_sweep_bench(args)
        return

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.config(args.workload)
    if args.angles:
        w.angles = w.angles[: args.angles]
        w.name += f"_first{args.angles}angles"
    t0 = time.time()
    mesh = TetMesh(w.verts, w.tets, device=dev)
    geom = ConeGeometry(w.cone, w.angles, device=dev)
    ingest_s = time.time() - t0
    P = Projector(mesh, geom, cache_entry=False)
    x = mesh.to_internal(torch.as_tensor(w.x, device=dev))
    entry = torch.empty(geom.nrays, dtype=torch.int32, device=dev)
    proj = torch.empty(geom.shape, dtype=torch.float32, device=dev)
    xhat = torch.empty(mesh.nt, dtype=torch.float32, device=dev)

    ev = {k: [] for k in ("entry", "forward", "backproject")}

    def step(record):
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e3 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        P.compute_entry(entry)
        e1.record(s)
        P.entry = entry
        P.forward(x, out=proj)
        e2.record(s)
        P.backproject(proj, mode=args.bp, out=xhat)
        e3.record(s)
        if record:
            ev["entry"].append((e0, e1))
            ev["forward"].append((e1, e2))
            ev["backproject"].append((e2, e3))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    mesh.stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = mesh.stats(reset=True)
    ms = {k: float(np.median([a.elapsed_time(b) for a, b in v])) for k, v in ev.items()}
    # Segments per walk: the counters hold forward + backprojection walks of
    # every timed step (the entry pass walks nothing).
    segs_total = st["segments"]
    segs_per_walk = segs_total / (2 * args.steps)
    value = segs_total / elapsed
    fwd_gbs = FWD_BYTES_PER_SEG * segs_per_walk / (ms["forward"] * 1e-3) / 1e9
    bwd_gbs = BWD_BYTES_PER_SEG * segs_per_walk / (ms["backproject"] * 1e-3) / 1e9
    bp_kernel = {"atomic": "atomic backprojection walk (pixel_walk_kernel<2>)",
                 "atomic_direct": "direct-atomic backprojection walk (pixel_walk_kernel<7>)",
                 "gather": "gather backprojection (walk fill + records into lists + exact sums)",
                 "fixed": "reproducible fixed-point scatter (pixel_walk_kernel<9>)",
                 "shadow": "element-driven backprojection (shadow_fast_kernel + shadow_exact_kernel)"}[args.bp]
    if ms["forward"] >= ms["backproject"]:
        dom, ach, bps, dom_ms, key = "forward walk (pixel_walk_kernel<1>)", fwd_gbs, FWD_BYTES_PER_SEG, ms["forward"], \
            "pixel_walk_kernel<1>"
    else:
        dom, ach, bps, dom_ms = bp_kernel, bwd_gbs, BWD_BYTES_PER_SEG, ms["backproject"]
        key = {"atomic": "pixel_walk_kernel<2>", "atomic_direct": "pixel_walk_kernel<7>",
               "fixed": "pixel_walk_kernel<9>"}.get(args.bp, "")
    traffic_bytes = measured_traffic_bytes(key) if (key and args.workload == 1 and not args.angles) else None
    traffic = traffic_bytes / (dom_ms * 1e-3) / 1e9 if traffic_bytes else None
    out = {
        "metric": "tet-segments/s fwd+back at 1 GPU",
        "value": value,
        "unit": "tet-segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "tets": mesh.nt,
            "rays": geom.nrays,
            "detector": [w.cone.nv, w.cone.nu],
            "angles": len(w.angles),
            "segments_per_walk": segs_per_walk,
            "step": f"entry faces (boundary projection) + forward + {args.bp} backprojection",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": ach,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_bytes_per_launch": traffic_bytes,
            "bytes_per_segment": bps,
        },
        "kernels_ms": ms,
        "walk_stats": st,
        "ingest_s": ingest_s,
    }
    # The other backprojection variants, one timed call each (not part of the step).
    others = [m for m in ("atomic", "fixed", "shadow", "atomic_direct") if m != args.bp]
    if args.gather and args.bp != "gather":
        others.append("gather")
    for mode in others:
        torch.cuda.synchronize()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record()
        P.backproject(proj, mode=mode, out=xhat)
        g1.record()
        torch.cuda.synchronize()
        t_ms = g0.elapsed_time(g1)
        out.setdefault("variants", {})[mode] = {"ms": t_ms, "seg_per_s": segs_per_walk / (t_ms * 1e-3),
                                                "hbm_frac": BWD_BYTES_PER_SEG * segs_per_walk / (t_ms * 1e-3)
                                                / 1e9 / HBM_PEAK_GBS}
    mesh.stats(reset=True)
    # The box's own streaming bandwidth (device-to-device copy of 1 GiB: one
    # read and one write per byte), for the roofline against what the memory
    # delivers in practice.
    n_copy = 1 << 28
    src = torch.ones(n_copy, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    stream_gbs = 5 * 2 * 4 * n_copy / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst
    out["roofline"]["stream_gbs"] = stream_gbs
    out["roofline"]["frac_of_stream"] = ach / stream_gbs
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    if args.cgls_problems > 0 and args.workload == 1 and not args.angles:
        del P, x, entry, proj, xhat, mesh, geom
        torch.cuda.empty_cache()
        out["batched_cgls"] = batched_cgls_leg(args.cgls_problems, args.cgls_iters, 1, tune=not args.no_tune)
    if args.json_extra:
        with open(args.json_extra, "w") as f:
            json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
