"""Pixel-tile and work-queue autotuner for batched launches.

The paper found 8 x 8 thread blocks fastest on its GPUs and recommends
re-tuning the block shape on other hardware (Section II-F).  Two knobs are
tuned here, both on the persistent batched kernel itself:

* per problem, the wavefront's pixel tile (tile_u x 64/tile_u, four tiles
  per 256-thread block): each candidate width is timed on a one-problem
  batch over a few evenly spaced angles of the problem (forward and
  backprojection), and the fastest is kept;
* for the whole batch, the number of pixel blocks a workgroup takes from the
  work queue per fetch: each candidate is timed on the batch of all problems
  restricted to the same few angles, with the tiles just chosen.

Results are cached in a JSON file keyed by device, mesh size and
detector/angle shape (tiles) and by the batch's problem keys (queue).
"""

from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from .projector import ConeGeometry, Projector

TILES = (4, 8, 16, 32, 64)
CHUNKS = (1, 2, 4, 8)


def _key(P: Projector) -> str:
    name = torch.cuda.get_device_name(P.device)
    c = P.geom.cone
    return (f"{name}|nt={P.nt}|nb={P.mesh.nboundary}|det={P.geom.nu}x{P.geom.nv}|na={P.geom.na}|"
            f"dso={float(c.dso)}|dsd={float(c.dsd)}|du={float(c.du)}")


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store(path, cache):
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, path)


def subset_projector(P: Projector, n_angles: int) -> Projector:
    """P restricted to n_angles evenly spaced angles of its geometry (own entry cache)."""
    na = P.geom.na
    sel = sorted(set(int(round(k * na / n_angles)) % na for k in range(n_angles)))
    geom = ConeGeometry(P.geom.cone, np.asarray(P.geom.angles)[sel], device=P.device)
    return Projector(P.mesh, geom)


def _time_batch(B, xs, ys, xh, pr, reps: int) -> float:
    from .batch import VecSet

    X, Y, XH, PR = VecSet(xs), VecSet(ys), VecSet(xh), VecSet(pr)
    s = torch.cuda.current_stream(B.device)

    def once():
        B.forward(X, PR)
        B.backproject(Y, XH)

    once()  # warm-up
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        once()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def _vectors(Ps):
    dev = Ps[0].device
    xs = [torch.rand(P.nt, device=dev) for P in Ps]
    ys = [torch.rand(P.geom.nrays, device=dev) for P in Ps]
    xh = [torch.zeros(P.nt, device=dev) for P in Ps]
    pr = [torch.empty(P.geom.nrays, device=dev) for P in Ps]
    return xs, ys, xh, pr


def tune_tile(P: Projector, n_angles: int = 4, reps: int = 2, candidates=TILES,
              cache_path: Optional[str] = None, sub: Optional[Projector] = None) -> Dict:
    """Best tile width for P, timed on one-problem batches; {"tile_u": t, "ms": {t: ms}}."""
    from .batch import BatchProjector

    cache = _load(cache_path)
    key = _key(P)
    if key in cache:
        return cache[key]
    sub = sub or subset_projector(P, n_angles)
    vec = _vectors([sub])
    ms = {t: _time_batch(BatchProjector([sub], [t]), *vec, reps) for t in candidates}
    best = min(ms, key=ms.get)
    res = {"tile_u": int(best), "ms": {str(k): v for k, v in ms.items()}}
    cache = _load(cache_path)
    cache[key] = res
    _store(cache_path, cache)
    return res


def tune_batch(projectors: Sequence[Projector], n_angles: int = 4, reps: int = 2, tiles=TILES, chunks=CHUNKS,
               cache_path: Optional[str] = None) -> Dict:
    """Tile width per problem and queue chunk for the batch of `projectors`:
    {"tile_u": [..], "queue_chunk": c, "queue_ms": {c: ms}}."""
    from .batch import BatchProjector

    subs = [subset_projector(P, n_angles) for P in projectors]
    tile_u: List[int] = [tune_tile(P, n_angles, reps, tiles, cache_path, sub=S)["tile_u"]
                         for P, S in zip(projectors, subs)]
    cache = _load(cache_path)
    bkey = "batch|" + hashlib.sha256("\n".join(_key(P) for P in projectors).encode()).hexdigest()[:16]
    if bkey in cache:
        return {"tile_u": tile_u, **cache[bkey]}
    vec = _vectors(subs)
    B = BatchProjector(subs, tile_u)
    ms = {}
    for c in chunks:
        B.set_queue_chunk(c)
        ms[c] = _time_batch(B, *vec, reps)
    best = min(ms, key=ms.get)
    res = {"queue_chunk": int(best), "queue_ms": {str(k): v for k, v in ms.items()}}
    cache = _load(cache_path)
    cache[bkey] = res
    _store(cache_path, cache)
    return {"tile_u": tile_u, **res}


def tune(P: Projector, n_angles: int = 4, reps: int = 2, candidates=TILES, cache_path: Optional[str] = None) -> Dict:
    """Best tile width for one projector (see tune_tile)."""
    return tune_tile(P, n_angles, reps, candidates, cache_path)


def tune_all(projectors: Sequence[Projector], cache_path: Optional[str] = None, **kw):
    """Tile width per projector (list), tuning each one."""
    return [tune_tile(P, cache_path=cache_path, **kw)["tile_u"] for P in projectors]
