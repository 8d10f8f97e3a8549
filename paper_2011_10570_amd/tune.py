"""Launch-shape autotuner of the fused stage kernels.

The shape of a fused launch (tile side t of the LDS tiles, workgroup size, cap on
the persistent grid) changes which workgroup computes which grid point but not
the arithmetic: every candidate gives bitwise the same state, which `tune`
checks.  Each candidate advances a private copy of the initial state by
`n_coarse` coarse steps (graph-captured, as lts_advance runs in production) and
is timed with device events; the fastest is applied and cached per mesh shape.
"""
from __future__ import annotations

import itertools
from typing import Dict, Iterable, Optional, Tuple

from . import MODE_LTS, Sim, get_launch, set_launch

_CACHE: Dict[tuple, tuple] = {}


def _key(mesh, equation, precision, tableau, mode):
    i = mesh.info()
    return (i["n_oct"], i["lmin"], i["lmax"], tuple(i["level_count"]), equation, int(precision), tableau, int(mode))


def tune(mesh, U0, equation: str = "wave", precision: int = 0, tableau: str = "rk4", mode: int = MODE_LTS,
         tiles: Iterable[int] = (1, 2), threads: Iterable[int] = (256, 512),
         max_workgroups: Iterable[int] = (1024, 2048, 4096), n_coarse: int = 1, reps: int = 2,
         check: bool = True, ko_sigma: float = 0.1, device: str = "cuda", use_cache: bool = True) -> dict:
    """Time every (tile, threads, max_workgroups) candidate on (mesh, U0) and apply
    the fastest (mesh.set_tile + set_launch).  Returns {"best", "ms", "table"}."""
    import torch
    key = _key(mesh, equation, precision, tableau, mode)
    if use_cache and key in _CACHE:
        best, ms = _CACHE[key]
        mesh.set_tile(best[0])
        set_launch(best[1], best[2])
        return {"best": best, "ms": ms, "table": None}
    if equation == "maxwell":
        tiles = [t for t in tiles if t == 1]
    old_tile = mesh.info()["tile"]
    old_shape = get_launch()
    table = []
    ref = None
    try:
        for t, nt, wg in itertools.product(tiles, threads, max_workgroups):
            mesh.set_tile(t)
            set_launch(nt, wg)
            sim = Sim(mesh, equation, precision, tableau, ko_sigma=ko_sigma, device=device)
            times = []
            for r in range(reps + 1):        # first pass captures the graph and warms up
                sim.set_state(U0)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                sim.advance(n_coarse, mode, graph=True)
                e1.record()
                e1.synchronize()
                if r > 0:
                    times.append(e0.elapsed_time(e1))
            if check:
                out = sim.current()
                if ref is None:
                    ref = out
                elif not torch.equal(out, ref):
                    raise RuntimeError(f"launch shape {(t, nt, wg)} changed the result")
            table.append(((t, nt, wg), min(times)))
            del sim
    except Exception:
        mesh.set_tile(old_tile)
        set_launch(*old_shape)
        raise
    best, ms = min(table, key=lambda r: r[1])
    mesh.set_tile(best[0])
    set_launch(best[1], best[2])
    _CACHE[key] = (best, ms)
    return {"best": best, "ms": ms, "table": table}


def clear_cache():
    _CACHE.clear()
