"""Pixel-tile and work-queue autotuner for batched launches.

The paper found 8 x 8 thread blocks fastest on its GPUs and recommends
re-tuning the block shape on other hardware (Section II-F).  Two knobs are
tuned here, both on the persistent batched kernel itself:

* per problem, the wavefront's pixel tile (tile_u x 64/tile_u, four tiles
  per 256-thread block): each candidate width is timed on a one-problem
  batch over evenly spaced angles of the problem (forward and
  backprojection), at least `min_rays` rays of them so that launch overhead
  does not decide;
* for the whole batch, the number of pixel blocks a workgroup takes from the
  work lists per fetch: each candidate is timed on the batch of all problems
  restricted to the same angles, with the tiles just chosen.

Each candidate is run `reps` times after a warm-up and scored by its fastest
run.  The default (8-wide tiles, one block per fetch) is kept unless another
candidate is faster by more than `margin` (a fraction), so timing noise does
not move the choice.  Results are cached in a JSON file keyed by device,
mesh size and detector/angle shape (tiles) and by the batch's problem keys
(queue).
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
DEFAULT_TILE = 8
DEFAULT_CHUNK = 1
MIN_RAYS = 1 << 21
REPS = 3
MARGIN = 0.03


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


def subset_angles(P: Projector, n_angles: int, min_rays: int = 0) -> int:
    """Angles to time P on: n_angles, raised until they hold min_rays rays (at most all)."""
    per_angle = max(1, P.geom.nu * P.geom.nv)
    return int(min(P.geom.na, max(n_angles, -(-min_rays // per_angle))))


def subset_projector(P: Projector, n_angles: int) -> Projector:
    """P restricted to n_angles evenly spaced angles of its geometry (own entry cache)."""
    na = P.geom.na
    if n_angles >= na:
        return P
    sel = sorted(set(int(round(k * na / n_angles)) % na for k in range(n_angles)))
    geom = ConeGeometry(P.geom.cone, np.asarray(P.geom.angles)[sel], device=P.device)
    return Projector(P.mesh, geom)


def _time_batch(B, xs, ys, xh, pr, reps: int) -> float:
    """Fastest of `reps` runs (after one warm-up) of forward + backprojection, ms."""
    from .batch import VecSet

    X, Y, XH, PR = VecSet(xs), VecSet(ys), VecSet(xh), VecSet(pr)
    s = torch.cuda.current_stream(B.device)

    def once():
        B.forward(X, PR)
        B.backproject(Y, XH)

    once()  # warm-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(s)
    for k in range(reps):
        once()
        ev[k + 1].record(s)
    ev[-1].synchronize()
    return min(ev[k].elapsed_time(ev[k + 1]) for k in range(reps))


def _pick(ms: Dict, default, margin: float):
    """The fastest candidate, unless the default is within `margin` of it."""
    best = min(ms, key=ms.get)
    if default in ms and ms[best] >= (1.0 - margin) * ms[default]:
        return default
    return best


def _vectors(Ps):
    dev = Ps[0].device
    g = torch.Generator(device=dev).manual_seed(0)
    xs = [torch.rand(P.nt, device=dev, generator=g) for P in Ps]
    ys = [torch.rand(P.geom.nrays, device=dev, generator=g) for P in Ps]
    xh = [torch.zeros(P.nt, device=dev) for P in Ps]
    pr = [torch.empty(P.geom.nrays, device=dev) for P in Ps]
    return xs, ys, xh, pr


def tune_tile(P: Projector, n_angles: int = 4, reps: int = REPS, candidates=TILES,
              cache_path: Optional[str] = None, sub: Optional[Projector] = None, min_rays: int = MIN_RAYS,
              margin: float = MARGIN) -> Dict:
    """Tile width for P, timed on one-problem batches; {"tile_u": t, "ms": {t: ms}}."""
    from .batch import BatchProjector

    cache = _load(cache_path)
    key = _key(P)
    if key in cache:
        return cache[key]
    sub = sub or subset_projector(P, subset_angles(P, n_angles, min_rays))
    vec = _vectors([sub])
    ms = {t: _time_batch(BatchProjector([sub], [t]), *vec, reps) for t in candidates}
    res = {"tile_u": int(_pick(ms, DEFAULT_TILE, margin)), "ms": {str(k): v for k, v in ms.items()},
           "angles": sub.geom.na}
    cache = _load(cache_path)
    cache[key] = res
    _store(cache_path, cache)
    return res


def tune_batch(projectors: Sequence[Projector], n_angles: int = 4, reps: int = REPS, tiles=TILES, chunks=CHUNKS,
               cache_path: Optional[str] = None, min_rays: int = MIN_RAYS, margin: float = MARGIN) -> Dict:
    """Tile width per problem and queue chunk for the batch of `projectors`:
    {"tile_u": [..], "queue_chunk": c, "queue_ms": {c: ms}}."""
    from .batch import BatchProjector

    subs = [subset_projector(P, subset_angles(P, n_angles, min_rays)) for P in projectors]
    tile_u: List[int] = [tune_tile(P, n_angles, reps, tiles, cache_path, sub=S, min_rays=min_rays,
                                   margin=margin)["tile_u"]
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
    res = {"queue_chunk": int(_pick(ms, DEFAULT_CHUNK, margin)), "queue_ms": {str(k): v for k, v in ms.items()}}
    cache = _load(cache_path)
    cache[bkey] = res
    _store(cache_path, cache)
    return {"tile_u": tile_u, **res}


def tune(P: Projector, n_angles: int = 4, reps: int = REPS, candidates=TILES, cache_path: Optional[str] = None,
         **kw) -> Dict:
    """Tile width for one projector (see tune_tile)."""
    return tune_tile(P, n_angles, reps, candidates, cache_path, **kw)


def tune_all(projectors: Sequence[Projector], cache_path: Optional[str] = None, **kw):
    """Tile width per projector (list), tuning each one."""
    return [tune_tile(P, cache_path=cache_path, **kw)["tile_u"] for P in projectors]
