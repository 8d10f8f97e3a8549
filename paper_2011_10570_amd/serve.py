"""Serving loop: independent LTS simulations arriving over time, admitted by their
device-memory footprint and advanced by continuous batching.

Each request is one problem (mesh specification, equation, initial pulse, T as a
number of coarse steps).  A request's mesh is built on the host (thread pool, the
C++ builder releases the GIL) when it arrives; it is admitted, first come first
served, once its footprint fits the device-memory budget:

    footprint = N * 125 * F * (2 * 8 + p * sizeof(K)) + device tables
                + ghost entries * F * 729 * 8

(two U buffers in float64, p stage arrays, the mesh's tile and slot tables and
its region of the batch's ghost-table scratch).  A request whose footprint
exceeds the whole budget is refused (status "rejected"), not queued.  Admitted sims are attached to the
batch of their equation (wave or Maxwell: one fused kernel each) at the next
round boundary; each round advances every attached sim by one of its own
substeps; sims leave when they reach T and their memory returns to the budget.
Time-to-T of a request = completion - arrival (host clock, taken when the round
that finished it has completed on the device).

    python -m paper_2011_10570_amd.serve [--requests N] [--budget-gib G]
"""
from __future__ import annotations

import argparse
import collections
import concurrent.futures as cf
import json
import threading
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import FP32_RHS, FP64, MODE_LTS, NFIELDS, NSTAGES, EQUATIONS, TABLEAUS, Batch, Mesh, Sim


@dataclass
class Request:
    rid: int
    equation: str
    mesh_spec: dict
    centre: list
    n_coarse: int
    arrival: float = 0.0          # seconds after the start
    sigma: float = 0.1
    cancel_after: Optional[float] = None   # cancel this many seconds after arrival
    # filled by the server
    mesh: Optional[Mesh] = None
    sim: Optional[Sim] = None
    footprint: int = 0
    node_updates: int = 0
    admitted: float = float("nan")
    finished: float = float("nan")
    status: str = "pending"       # pending | done | rejected | cancelled
    state: Optional[object] = None  # final state [F][N][125] when kept

    @property
    def time_to_t(self) -> float:
        return self.finished - self.arrival


def footprint_bytes(info: dict, equation: str, precision: int, tableau: str = "rk4") -> int:
    F = NFIELDS[EQUATIONS[equation]]
    p = NSTAGES[TABLEAUS[tableau]]
    kb = 4 if precision == FP32_RHS else 8
    return (int(info["n_oct"]) * 125 * F * (2 * 8 + p * kb) + int(info["table_bytes"])
            + int(info["ghost_entries"]) * F * 729 * 8)


def initial_state(mesh: Mesh, equation: str, centre, sigma: float, device):
    """Gaussian pulse data of the request on `device`: [F][N][125]."""
    from workloads import maxwell_gaussian_torch, wave_gaussian_torch
    gen = wave_gaussian_torch if equation == "wave" else maxwell_gaussian_torch
    return gen(mesh.leaves(), mesh.info()["L"], [centre], sigma=sigma, device=device)


class Server:
    """Admission by footprint, continuous batching per equation.  The wave and
    Maxwell batches run on two streams (default priority), so their rounds
    overlap on the device; a tick enqueues a few rounds of both and then waits
    for both."""

    def __init__(self, budget_bytes: int, precision: int = FP64, tableau: str = "rk4", mode: int = MODE_LTS,
                 capacity: int = 64, tick_rounds: int = 4, keep_state: bool = False, device: str = "cuda",
                 builders: int = 4, ko_sigma: float = 0.1, verbose: bool = False):
        import torch
        self.verbose = verbose
        self.budget = int(budget_bytes)
        self.prec = precision
        self.tab = tableau
        self.mode = mode
        self.tick_rounds = max(1, int(tick_rounds))
        self.keep_state = keep_state
        self.device = device
        self.ko_sigma = ko_sigma
        self.batches = {eq: Batch(eq, precision, tableau, mode, capacity) for eq in ("wave", "maxwell")}
        self.streams = {"wave": torch.cuda.current_stream(), "maxwell": torch.cuda.Stream()}
        self.capacity = capacity
        self.pool = cf.ThreadPoolExecutor(max_workers=builders)
        self._cancel = set()
        self._lock = threading.Lock()

    def cancel(self, rid: int):
        """Cancel request rid (thread-safe): dropped if not yet admitted, else
        released at its next coarse-step boundary."""
        with self._lock:
            self._cancel.add(rid)

    def _cancelled(self, r: Request, now: float) -> bool:
        if r.cancel_after is not None and now >= r.arrival + r.cancel_after:
            return True
        with self._lock:
            return r.rid in self._cancel

    def _prepare(self, req: Request):
        m = Mesh(req.mesh_spec)
        m.set_tile(2)
        return m

    def _admit(self, req: Request, now: float):
        req.sim = Sim(req.mesh, req.equation, self.prec, self.tab, ko_sigma=self.ko_sigma, device=self.device)
        req.sim.set_state(initial_state(req.mesh, req.equation, req.centre, req.sigma, self.device))
        self.batches[req.equation].attach(req.sim, req.n_coarse)
        req.admitted = now

    def run(self, requests: List[Request]) -> dict:
        import torch
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = collections.deque(reqs)
        building = collections.deque()     # (req, future) in arrival order
        resident: List[Request] = []
        used = 0
        peak = 0
        nb_att = {eq: 0 for eq in self.batches}
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        main = torch.cuda.current_stream()

        def release(r: Request, status: str, now: float):
            nonlocal used
            r.status = status
            r.finished = now
            used -= r.footprint
            nb_att[r.equation] -= 1
            if self.verbose:
                print(f"[serve] request {r.rid} ({r.equation}, {r.node_updates} node-updates) {status}: "
                      f"queued {r.admitted - r.arrival:.3f} s, time-to-T {r.time_to_t:.3f} s", flush=True)
            if self.keep_state and status == "done":
                r.state = r.sim.current()
            r.sim = None
            r.mesh = None

        while pending or building or resident:
            now = clock()
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                building.append((r, self.pool.submit(self._prepare, r)))
            # first come, first served: the head of the queue blocks later requests
            while building and building[0][1].done():
                r, fut = building[0]
                if self._cancelled(r, clock()):
                    building.popleft()
                    r.status, r.finished = "cancelled", clock()
                    continue
                if r.mesh is None:
                    r.mesh = fut.result()
                    info = r.mesh.info()
                    r.footprint = footprint_bytes(info, r.equation, self.prec, self.tab)
                    r.node_updates = int(info["node_updates_lts" if self.mode == MODE_LTS
                                              else "node_updates_gts"]) * r.n_coarse
                    if r.footprint > self.budget:
                        # can never fit: refused, not queued
                        building.popleft()
                        r.status, r.finished, r.mesh = "rejected", clock(), None
                        if self.verbose:
                            print(f"[serve] request {r.rid} rejected: {r.footprint} B > budget {self.budget} B",
                                  flush=True)
                        continue
                if used + r.footprint > self.budget or nb_att[r.equation] >= self.capacity:
                    break
                building.popleft()
                self._admit(r, clock())
                nb_att[r.equation] += 1
                used += r.footprint
                peak = max(peak, used)
                resident.append(r)
            if not resident:
                wait = (pending[0].arrival - clock()) if pending else 0.0
                time.sleep(min(max(wait, 0.0), 0.01) if pending else 0.001)
                continue
            # cancelled residents leave at their next coarse-step boundary
            now = clock()
            keep = []
            bound = []
            for r in resident:
                if self._cancelled(r, now):
                    nsub = int(r.mesh.info()["n_substeps"])
                    to_b = r.sim.rounds_left % nsub
                    if to_b == 0:
                        self.batches[r.equation].detach(r.sim, stream=self.streams[r.equation])
                        self.streams[r.equation].synchronize()
                        release(r, "cancelled", now)
                        continue
                    bound.append(to_b)
                keep.append(r)
            resident = keep
            if not resident:
                continue
            k = min([self.tick_rounds, min(r.sim.rounds_left for r in resident)] + bound)
            done = []
            for eq, b in self.batches.items():
                if nb_att[eq]:
                    st = self.streams[eq]
                    if st is not main:
                        st.wait_stream(main)      # initial states were written on the main stream
                    done += b.run(k, stream=st)
            for eq, st in self.streams.items():
                if nb_att[eq]:
                    st.synchronize()
            now = clock()
            fin = {id(s) for s in done}
            keep = []
            for r in resident:
                if id(r.sim) in fin:
                    release(r, "done", now)
                else:
                    keep.append(r)
            resident = keep
        wall = clock()
        ok = [r for r in reqs if r.status == "done"]
        tt = np.array([r.time_to_t for r in ok]) if ok else np.array([float("nan")])
        total = sum(r.node_updates for r in ok)
        return {"requests": len(reqs), "done": len(ok), "rejected": sum(r.status == "rejected" for r in reqs),
                "cancelled": sum(r.status == "cancelled" for r in reqs), "wall_s": wall, "node_updates": total,
                "node_updates_per_s": total / wall if wall > 0 else float("nan"),
                "p50_time_to_t_s": float(np.percentile(tt, 50)), "p99_time_to_t_s": float(np.percentile(tt, 99)),
                "mean_queue_s": float(np.mean([r.admitted - r.arrival for r in ok])) if ok else float("nan"),
                "peak_resident_bytes": peak, "budget_bytes": self.budget,
                "wave": sum(r.equation == "wave" for r in ok), "maxwell": sum(r.equation == "maxwell" for r in ok)}

    def close(self):
        self.pool.shutdown(wait=True)


def requests_from_config(n: Optional[int] = None, rate: Optional[float] = None) -> List[Request]:
    """The stored serving workload; arrival gaps (unit-rate exponential draws)
    divided by `rate` requests/s (None: everything arrives at t = 0)."""
    from workloads import config
    cfg = config("serve")
    out = []
    t = 0.0
    for i, q in enumerate(cfg["requests"][:n]):
        if rate:
            t += q["gap"] / rate
        out.append(Request(i, q["equation"], q["mesh"], q["centre"], cfg["n_coarse"], arrival=t, sigma=cfg["sigma"]))
    return out


def batch_throughput(problems: list, n_coarse: int = 1, precision: int = FP64, device: str = "cuda",
                     mode: int = MODE_LTS, alone: bool = False) -> dict:
    """Wave problems advanced together in one batch from a Gaussian pulse: raw
    node-updates per second over the wall time until all reach T (setup excluded).
    With alone, the same problems are also advanced one after another, each with
    its own graph-captured lts_advance (one untimed coarse step captures the
    graph; the timed n_coarse steps follow it), and the two rates are compared."""
    import torch
    from workloads import wave_gaussian_torch
    meshes, states, sims = [], [], []
    work = 0
    for p in problems:
        m = Mesh(p["mesh"])
        c = p["mesh"]["criteria"][0]["center"]
        U0 = wave_gaussian_torch(m.leaves(), m.info()["L"], [c], sigma=0.1, device=device)
        s = Sim(m, "wave", precision, "rk4", ko_sigma=0.1, device=device)
        s.set_state(U0)
        info = m.info()
        work += info["node_updates_lts" if mode == MODE_LTS else "node_updates_gts"] * n_coarse
        meshes.append(m)
        states.append(U0)
        sims.append(s)
    b = Batch("wave", precision, "rk4", mode, capacity=max(1, len(sims)))
    torch.cuda.synchronize()
    t = time.perf_counter()
    for s in sims:
        b.attach(s, n_coarse)
    b.drain()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    out = {"problems": len(sims), "node_updates": work, "wall_s": wall, "node_updates_per_s": work / wall}
    del b, sims
    if alone:
        solo = []
        for m, U0 in zip(meshes, states):
            s = Sim(m, "wave", precision, "rk4", ko_sigma=0.1, device=device)
            s.set_state(U0)
            s.advance(1, mode, graph=True)       # captures the coarse-step graph (untimed);
            solo.append(s)                       # every coarse step does the same work
        torch.cuda.synchronize()
        t = time.perf_counter()
        for s in solo:
            s.advance(n_coarse, mode, graph=True)
        torch.cuda.synchronize()
        wall1 = time.perf_counter() - t
        out["alone_wall_s"] = wall1
        out["alone_node_updates_per_s"] = work / wall1
        out["batch_over_alone"] = wall1 / wall
    return out


def run_config(capacity: Optional[float] = None, n: Optional[int] = None, budget: Optional[int] = None,
               tick_rounds: int = 4, verbose: bool = False) -> dict:
    """The stored serving workload end to end.  Arrival rate = rho * capacity /
    mean work per request, capacity in node-updates/s (default: measured on the
    batched-problems workload)."""
    import torch
    from workloads import config
    if budget is None:
        budget = int(torch.cuda.mem_get_info()[0] * 0.5)
    if capacity is None:
        capacity = batch_throughput(config("batch")["problems"], 1)["node_updates_per_s"]
    cfg = config("serve")
    work = [Mesh(r.mesh_spec).info()["node_updates_lts"] * r.n_coarse for r in requests_from_config(n)]
    rate = cfg["rho"] * capacity / float(np.mean(work))
    reqs = requests_from_config(n, rate)
    srv = Server(budget, tick_rounds=tick_rounds, verbose=verbose)
    try:
        stats = srv.run(reqs)
    finally:
        srv.close()
    stats.update({"rho": cfg["rho"], "capacity_node_updates_per_s": capacity, "arrival_rate_per_s": rate})
    return stats


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=None, help="first N stored requests (default all)")
    ap.add_argument("--budget-gib", type=float, default=None, help="device memory budget (default half free)")
    ap.add_argument("--capacity", type=float, default=None,
                    help="node-updates/s used to set the arrival rate (default: measured on the batch workload)")
    ap.add_argument("--tick-rounds", type=int, default=4)
    args = ap.parse_args(argv)
    budget = int(args.budget_gib * 2 ** 30) if args.budget_gib else None
    stats = run_config(args.capacity, args.requests, budget, args.tick_rounds, verbose=True)
    print(json.dumps(stats))


if __name__ == "__main__":
    main()
