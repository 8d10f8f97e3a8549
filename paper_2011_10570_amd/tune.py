"""Launch-shape autotuner of the fused stage kernels (one mesh, and batches).

The shape of a fused launch (tile side t: 1 or 2 for LDS-resident tiles, 4 for
streamed whole blocks; workgroup sizes of the tile and streaming kernels; cap on
the grid) changes which workgroup computes which grid point but not
the FP64 arithmetic: every candidate gives bitwise the same state, which `tune`
checks (FP32-RHS results depend on the tile side at FP32 rounding, so there the
check compares candidates of one tile side only).  Each candidate advances a
private copy of the initial state by reps + 1 times `n_coarse` coarse steps
(graph-captured, as lts_advance runs in production; the first pass captures and
warms up), and the later passes are timed with device events; the fastest is applied and cached per mesh shape.
"""
from __future__ import annotations

import itertools
from typing import Dict, Iterable, Optional, Tuple

from . import MODE_LTS, Batch, Sim, get_batch_launch, get_launch, set_batch_launch, set_launch

_CACHE: Dict[tuple, tuple] = {}


def _key(mesh, equation, precision, tableau, mode):
    i = mesh.info()
    return (i["n_oct"], i["lmin"], i["lmax"], tuple(i["level_count"]), equation, int(precision), tableau, int(mode))


def _candidates(tiles, threads, max_workgroups, stream_threads):
    # side-1 tiles run 256-thread workgroups whatever the thread count asked for
    for t in tiles:
        for nt, wg in itertools.product(threads if t != 1 else threads[:1], max_workgroups):
            for st in (stream_threads if t == 4 else stream_threads[:1]):
                yield (t, nt, wg, st)


def tune(mesh, U0, equation: str = "wave", precision: int = 0, tableau: str = "rk4", mode: int = MODE_LTS,
         tiles: Iterable[int] = (1, 2, 4), threads: Iterable[int] = (256, 512),
         max_workgroups: Iterable[int] = (4096, 16384, 65536), stream_threads: Iterable[int] = (512, 256),
         n_coarse: int = 1, reps: int = 2, check: bool = True, ko_sigma: float = 0.1, device: str = "cuda",
         use_cache: bool = True) -> dict:
    """Time every (tile, threads, max_workgroups, stream_threads) candidate on
    (mesh, U0) and apply the fastest (mesh.set_tile + set_launch).  Returns
    {"best", "ms", "table"}."""
    import torch
    key = _key(mesh, equation, precision, tableau, mode)
    if use_cache and key in _CACHE:
        best, ms = _CACHE[key]
        mesh.set_tile(best[0])
        set_launch(best[1], best[2], best[3])
        return {"best": best, "ms": ms, "table": None}
    if equation == "maxwell":   # side-1 and side-2 tiles (no streamed side-4 blocks)
        tiles = [t for t in tiles if t in (1, 2)]
    stream_threads = list(stream_threads)
    old_tile = mesh.info()["tile"]
    old_shape = get_launch()
    table = []
    ref = {}
    try:
        for t, nt, wg, st in _candidates(list(tiles), list(threads), list(max_workgroups), stream_threads):
            mesh.set_tile(t)
            set_launch(nt, wg, st)
            sim = Sim(mesh, equation, precision, tableau, ko_sigma=ko_sigma, device=device)
            # the state is set once: setting it again rebinds the sim, which drops
            # the captured graph; every candidate advances (reps + 1) n_coarse
            # steps from U0, so the final states stay comparable
            sim.set_state(U0)
            times = []
            for r in range(reps + 1):        # first pass captures the graph and warms up
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                sim.advance(n_coarse, mode, graph=True)
                e1.record()
                e1.synchronize()
                if r > 0:
                    times.append(e0.elapsed_time(e1))
            if check:
                out = sim.current()
                k = t if precision != 0 else 0
                if k not in ref:
                    ref[k] = out
                elif not torch.equal(out, ref[k]):
                    raise RuntimeError(f"launch shape {(t, nt, wg, st)} changed the result")
            table.append(((t, nt, wg, st), min(times)))
            del sim
    except Exception:
        mesh.set_tile(old_tile)
        set_launch(*old_shape)
        raise
    best, ms = min(table, key=lambda r: r[1])
    mesh.set_tile(best[0])
    set_launch(best[1], best[2], best[3])
    _CACHE[key] = (best, ms)
    return {"best": best, "ms": ms, "table": table}


def tune_batch(meshes, states, equation: str = "wave", precision: int = 0, tableau: str = "rk4",
               mode: int = MODE_LTS, tiles: Iterable[int] = (1, 2), threads: Iterable[int] = (256, 512),
               max_workgroups: Iterable[int] = (1024, 2048, 4096, 8192, 16384), n_coarse: int = 1,
               reps: int = 1, check: bool = True, ko_sigma: float = 0.1, device: str = "cuda",
               use_cache: bool = True) -> dict:
    """Batched launches: time every (tile side of all meshes, threads, grid cap)
    candidate on the batch of (meshes[i], states[i]) advanced n_coarse coarse steps
    together (graph-captured rounds, after one untimed warm-up drain), check that
    every candidate gives bitwise the same states, and apply the fastest
    (mesh.set_tile on every mesh + set_batch_launch).  Cached per batch
    composition.  Returns {"best", "ms", "table"}."""
    import torch
    key = ("batch",) + tuple(_key(m, equation, precision, tableau, mode) for m in meshes)
    if use_cache and key in _CACHE:
        best, ms = _CACHE[key]
        for m in meshes:
            m.set_tile(best[0])
        set_batch_launch(best[1], best[2])
        return {"best": best, "ms": ms, "table": None}
    old_tiles = [m.info()["tile"] for m in meshes]
    old_shape = get_batch_launch()
    table = []
    ref = {}
    try:
        threads, wgs = list(threads), list(max_workgroups)
        cands = [(t, nt, wg) for t in tiles for nt in (threads if t != 1 else threads[:1]) for wg in wgs]
        for t, nt, wg in cands:
            for m in meshes:
                m.set_tile(t)
            set_batch_launch(nt, wg)
            times = []
            outs = None
            for r in range(reps + 1):       # the first pass captures the round graph and warms up
                sims = []
                for m, st in zip(meshes, states):
                    sim = Sim(m, equation, precision, tableau, ko_sigma=ko_sigma, device=device)
                    sim.set_state(st)
                    sims.append(sim)
                b = Batch(equation, precision, tableau, mode, capacity=max(1, len(sims)))
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for sim in sims:
                    b.attach(sim, n_coarse)
                b.drain()
                e1.record()
                e1.synchronize()
                if r > 0:
                    times.append(e0.elapsed_time(e1))
                outs = [sim.current() for sim in sims]
                del b, sims
            if check:
                k = t if precision != 0 else 0
                if k not in ref:
                    ref[k] = outs
                elif not all(torch.equal(a, c) for a, c in zip(outs, ref[k])):
                    raise RuntimeError(f"batch launch shape {(t, nt, wg)} changed the result")
            table.append(((t, nt, wg), min(times)))
    except Exception:
        for m, t in zip(meshes, old_tiles):
            m.set_tile(t)
        set_batch_launch(*old_shape)
        raise
    best, ms = min(table, key=lambda r: r[1])
    for m in meshes:
        m.set_tile(best[0])
    set_batch_launch(best[1], best[2])
    _CACHE[key] = (best, ms)
    return {"best": best, "ms": ms, "table": table}


def clear_cache():
    _CACHE.clear()
