"""Pixel-tile autotuner.

The paper found 8 x 8 thread blocks fastest on its GPUs and recommends
re-tuning the block shape on other hardware (Section II-F).  Here the tuned
knob is the wavefront's pixel tile (tile_u x 64/tile_u, four tiles per
256-thread block): for each (mesh, geometry) the forward and backprojection
walks over a few evenly spaced angles are timed with HIP events for every
candidate width, and the fastest is kept.  Results can be cached in a JSON
file keyed by device, mesh size and detector/angle shape.
"""

from __future__ import annotations

import ctypes as C
import json
import os
from typing import Dict, Optional, Sequence

import torch

from ._lib import TCT_BP_ATOMIC, call, tct_range
from .projector import Projector, _stream

CANDIDATES = (4, 8, 16, 32, 64)


def _key(P: Projector) -> str:
    name = torch.cuda.get_device_name(P.device)
    c = P.geom.cone
    return (f"{name}|nt={P.nt}|nb={P.mesh.nboundary}|det={P.geom.nu}x{P.geom.nv}|na={P.geom.na}|"
            f"dso={float(c.dso)}|dsd={float(c.dsd)}|du={float(c.du)}")


def _time_tile(P: Projector, tile_u: int, angles: Sequence[int], x, y, xhat, proj, reps: int) -> float:
    s = torch.cuda.current_stream(P.device)
    entry = P.entry.data_ptr() if P.entry is not None else None
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def once():
        for a in angles:
            r = C.byref(tct_range(a, 1, tile_u))
            call("tct_forward_range", P.mesh.handle, P.geom.handle, x.data_ptr(), proj.data_ptr(), entry, r,
                 _stream(P.device))
            call("tct_backproject_range", P.mesh.handle, P.geom.handle, y.data_ptr(), xhat.data_ptr(), TCT_BP_ATOMIC,
                 1, entry, r, _stream(P.device))

    once()  # warm-up
    e0.record(s)
    for _ in range(reps):
        once()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(P: Projector, n_angles: int = 4, reps: int = 2, candidates=CANDIDATES,
         cache_path: Optional[str] = None) -> Dict:
    """Best tile width for P; returns {"tile_u": t, "ms": {t: ms, ...}}."""
    cache = {}
    key = _key(P)
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]
    na = P.geom.na
    angles = sorted(set(int(round(k * na / n_angles)) % na for k in range(n_angles)))
    dev = P.device
    x = torch.rand(P.nt, device=dev)
    y = torch.rand(P.geom.nrays, device=dev)
    proj = torch.empty(P.geom.nrays, device=dev)
    xhat = torch.zeros(P.nt, device=dev)
    ms = {t: _time_tile(P, t, angles, x, y, xhat, proj, reps) for t in candidates}
    best = min(ms, key=ms.get)
    res = {"tile_u": int(best), "ms": {str(k): v for k, v in ms.items()}, "angles": angles}
    if cache_path:
        cache[key] = res
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return res


def tune_all(projectors: Sequence[Projector], cache_path: Optional[str] = None, **kw):
    """Tile width per projector (list), tuning each one."""
    return [tune(P, cache_path=cache_path, **kw)["tile_u"] for P in projectors]
