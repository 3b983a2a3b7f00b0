"""Launch-shape autotuner.

For a box class (box edge, density, colloid count, precision, n_md) it times
a few intervals of a seeded system for each point of a small grid of launch
parameters -- Verlet-list entries per thread of the MD chain (which sets the
number of chain workgroups), cells per collision tile, particles per
streaming thread -- and caches the fastest in a JSON file keyed by the box
class.  Tuning never changes results: every launch shape evaluates the same
operations (the FP64 parity tests run several shapes against the oracle).
"""
from __future__ import annotations

import itertools
import json
import os
import time

# collide_cells 0: sized from the density (the library's default)
GRID = dict(chain_k=(1, 2), collide_cells=(0, 32, 40), stream_ppt=(1, 2))
DEFAULT = dict(chain_k=1, collide_cells=0, stream_block=256, stream_ppt=2)


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "rmpmd", "autotune.json")


def box_class(params: dict) -> str:
    L = params["L"]
    vol = L[0] * L[1] * L[2]
    rho = round(params["n_solvent"] / vol) if vol else 0
    return (f"L{L[0]}x{L[1]}x{L[2]}_rho{rho}_nc{len(params['colloids'])}"
            f"_p{int(params.get('precision', 64))}_nmd{int(params['n_md'])}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(params: dict, cache_path: str | None = None) -> dict:
    """Cached best launch parameters for this box class (defaults if none)."""
    d = _load(cache_path or default_cache_path()).get(box_class(params))
    return dict(d["best"]) if d else dict(DEFAULT)


def time_config(params: dict, cfg: dict, seed: int, intervals: int, timer=None) -> float:
    """Mean milliseconds per interval of a seeded system with `cfg`."""
    import torch
    import paper_1608_04904_amd as rm
    s = rm.System(params, seed)
    s.set_tuning(use_graph=1, **cfg)
    n_md = int(params["n_md"])
    s.step(n_md, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(n_md, intervals)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / intervals
    s.close()
    return ms


def tune(params: dict, seed: int = 1, intervals: int = 6, grid: dict | None = None,
         cache_path: str | None = None, timer=None, force: bool = False) -> dict:
    """Grid search for the box class of `params`; returns the best launch
    parameters and records every point in the cache."""
    path = cache_path or default_cache_path()
    key = box_class(params)
    data = _load(path)
    if key in data and not force:
        return dict(data[key]["best"])
    grid = grid or GRID
    timer = timer or time_config
    names = sorted(grid)
    points = []
    for values in itertools.product(*(grid[n] for n in names)):
        cfg = dict(zip(names, values))
        points.append(dict(cfg=cfg, ms=float(timer(params, cfg, seed, intervals))))
    best = min(points, key=lambda q: q["ms"])
    data[key] = dict(best=best["cfg"], ms=best["ms"], points=points)
    _store(path, data)
    return dict(best["cfg"])
