"""Benchmark of the octree LTS hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Workload (the metric's configuration): the 3D scalar wave equation on the
periodic octree "wave_c2" -- levels 3-8, refined by a gradient criterion around
four seeded Gaussian pulses, 201,216 octants of 5^3 nodes (25.2M nodes), RK4,
sixth-order FD + Kreiss-Oliger, dt_l = 0.25 h_l.  A step is one coarsest step:
2^5 = 32 substeps x 4 stages of the fused stage kernel over the active tiles
(Alg. 2 with the schedule of fig. blk_loop), i.e. the whole hot path once.

Reported (one JSON line):
  value          raw LTS FP64 node-updates/s (a node-update = one DG node advanced
                 one RK step at its own level's dt), inputs resident in HBM;
  lts_vs_gts     GTS node-updates/s on the same mesh and final time, the measured
                 LTS-over-GTS wall-time speedup and the speedup model of eq. invS;
  fp32_rhs       the same LTS run with FP32 stencils (FP64 state/RK/time interp.);
  accuracy       L2 / max error against the analytic solution at T = 8 dt_lmin
                 for LTS, GTS and FP32-RHS, and FP32-RHS vs FP64;
  roofline       the fused stage (ghost-table pre-passes + fused tile launches of
                 one RK stage): algorithmic HBM bytes (224 B per FP64 LTS
                 node-update) / event-timed stage duration, against 8 TB/s;
  cpu_baseline   the FP64 oracle on a bounded sample of the same workload
                 (value), the host's CPU model and core count, and the oracle
                 run in full on the C1 configuration (LTS and GTS to T, one
                 process each, beside the GPU legs): wall times, node-updates/s
                 and the oracle's own LTS-over-GTS speedup;
  c3             the C1 configuration to T with FP32 stencils on the GPU against
                 that FP64 oracle result: l2 / max error per field;
  maxwell        6-field Maxwell on the same mesh (tile side 2), FP64 LTS:
                 node-updates/s and its roofline fraction (672 B per update);
  batch          64 independent wave problems (1k-50k leaves, levels 2..4-8)
                 advanced to T together by continuous batching, FP64 and
                 FP32-RHS: raw node-updates/s until all reach T (--no-batch);
  serve          the Poisson-arrival wave/Maxwell serving loop over the stored
                 requests: throughput, p50/p99 time-to-T (--no-serve skips it).

    python bench.py --copy-probe-mib N   only times the device copy probe (the
                                         known-size kernel that scales counters)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("dev_common.h", "dev_fused.h", "k_fused.hip", "k_fused_batch.hip", "k_ghost.hip", "k_stream.hip",
                  "k_phase.hip", "api.cpp", "mesh.cpp")   # mesh.cpp: tile order and XCD ranges
WORKLOAD = "wave_c2"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="fused tile side (0: the mesh default, 2)")
    ap.add_argument("--tune", action="store_true", help="autotune tile side and launch shape first")
    ap.add_argument("--only", default="", help="comma list of legs: lts,gts,fp32")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-problems leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving loop")
    ap.add_argument("--serve-requests", type=int, default=None, help="first N stored requests (default all)")
    ap.add_argument("--no-maxwell", action="store_true", help="skip the Maxwell leg")
    ap.add_argument("--no-nl", action="store_true", help="skip the non-linear wave leg")
    ap.add_argument("--no-n7", action="store_true", help="skip the 7^3-node leg")
    ap.add_argument("--unfused", action="store_true", help="also time one coarse step of the phase-by-phase path")
    ap.add_argument("--jsonl", default="", help="also append the result line to this JSONL file")
    ap.add_argument("--copy-probe-mib", type=int, default=0, help="only time a copy of this many MiB")
    return ap.parse_args()


def copy_probe_gbs(P, torch, mib: int = 2048, reps: int = 5) -> float:
    """Device-to-device copy through the library's copy kernel: (read + write) GB/s."""
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    P.copy_probe(a, b, n)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        P.copy_probe(a, b, n)
    e1.record()
    torch.cuda.synchronize()
    return 2 * n * reps / (e0.elapsed_time(e1) / 1e3) / 1e9


def source_digest() -> str:
    """sha256 over the kernel and launch sources (device headers, kernels, api.cpp, and mesh.cpp for
    the tile order and XCD ranges)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2011_10570_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def stored_traffic(path=None):
    """Measured HBM bytes per fused stage from the committed counter summary, or
    None when the kernel or launch sources have changed since it was taken."""
    import re
    path = path or os.path.join(ROOT, "profiles", "fused_stage_wave_c2_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"sources_sha256:\s*([0-9a-f]{64})", txt)
    t = re.search(r"traffic_bytes_per_stage:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != source_digest():
        return None
    return float(t.group(1))


# algorithmic passes over the DG arrays per stage (per field): read U0 and the
# stages the stage state needs, write K_s; the last stage also writes U_new.
def passes_rk4(stage: int) -> int:
    return {0: 2, 1: 3, 2: 3, 3: 6}[stage]


def stage_accounting(info: dict, tiles: np.ndarray, nfields: int = 2) -> dict:
    """Algorithmic bytes of one LTS coarse step of RK4 (FP64), counted per fused
    stage: substep j runs the tiles of levels >= its lowest active level (all
    levels at j = 0, lmax - ctz(j) otherwise; Alg. 2 with the schedule B_j), and
    each of its 4 stages moves passes_rk4(s) x 8 B per node and field.  Also the
    launches of the step: one per tile side present per stage, the ghost
    pre-pass of every stage while receivers above the lowest active level exist
    (lo < lmax), and the multi-stage pre-pass at the first stage of a substep
    whose lowest active level has coarser neighbours (lo > lmin)."""
    nsub = int(info["n_substeps"])
    lev = tiles[:, 2]
    nodes_t = 125 * tiles[:, 4].astype(np.int64) ** 3
    alg = stages = launches = 0
    for j in range(nsub):
        lo = info["lmin"] if j == 0 else info["lmax"] - ((j & -j).bit_length() - 1)
        act = lev >= lo
        nodes = int(nodes_t[act].sum())
        sides = len(set(tiles[act, 4].tolist()))
        for s in range(4):
            alg += nodes * passes_rk4(s) * 8 * nfields
            stages += 1
            launches += sides + (1 if lo < info["lmax"] else 0) + (1 if s == 0 and lo > info["lmin"] else 0)
    return {"alg_bytes": alg, "stages": stages, "launches": launches}


def analytic_fields(leaves, L, pulses, sigma, T, device, nodes: int = 5):
    """(u, v) [2, N, n^3] of the periodic Gaussian spherical wave at time T on every
    DG node: u = (phi(r+T) + phi(r-T)) / (2r), v = (phi'(r+T) - phi'(r-T)) / (2r),
    phi(xi) = xi g(xi), summed over the pulses and their 27 nearest images; below
    r = 1e-4 the limits u = phi'(T) + r^2 phi'''(T) / 6, v = phi''(T)."""
    import torch
    ni = nodes - 1
    lv = torch.as_tensor(np.asarray(leaves), dtype=torch.int64, device=device)
    s = torch.bitwise_left_shift(torch.ones_like(lv[:, 3]), L - lv[:, 3]).to(torch.float64)
    i = torch.arange(nodes, dtype=torch.float64, device=device)
    k_, j_, i_ = torch.meshgrid(i, i, i, indexing="ij")
    loc = torch.stack([i_, j_, k_], -1).reshape(nodes ** 3, 3)
    X = float(ni) * lv[:, None, :3].to(torch.float64) + loc[None] * s[:, None, None]
    x = -1.0 + 2.0 * X / float(ni * (1 << L))
    u = torch.zeros(x.shape[:2], dtype=torch.float64, device=device)
    v = torch.zeros_like(u)
    s2 = sigma * sigma

    def g(xi):
        return torch.exp(-xi * xi / (2 * s2))

    def phi(xi):
        return xi * g(xi)

    def d1(xi):
        return g(xi) * (1 - xi * xi / s2)

    def d2(xi):
        return g(xi) * (xi ** 3 / s2 ** 2 - 3 * xi / s2)

    def d3(xi):
        return g(xi) * (-xi ** 4 / s2 ** 3 + 6 * xi * xi / s2 ** 2 - 3 / s2)

    Tt = torch.full((), float(T), dtype=torch.float64, device=device)
    for cc in pulses:
        c = -1.0 + 2.0 * torch.tensor(cc, dtype=torch.float64, device=device) / float(ni * (1 << L))
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                for d in (-1, 0, 1):
                    dd = x - (c + 2.0 * torch.tensor([d, b, a], dtype=torch.float64, device=device))
                    r = torch.sqrt((dd * dd).sum(-1))
                    small = r < 1e-4
                    rs = torch.where(small, torch.ones_like(r), r)
                    u += torch.where(small, d1(Tt) + r * r * d3(Tt) / 6, (phi(rs + T) + phi(rs - T)) / (2 * rs))
                    v += torch.where(small, d2(Tt).expand_as(r), (d1(rs + T) - d1(rs - T)) / (2 * rs))
    return torch.stack([u, v])


def analytic_error(sim_out, leaves, L, pulses, sigma, T, nodes: int = 5):
    """Per field (u, v): volume-weighted L2 and max error against the periodic
    Gaussian spherical wave at T, and the L2 of the exact field itself."""
    import torch
    dev = sim_out.device
    ex = analytic_fields(leaves, L, pulses, sigma, T, dev, nodes)
    nn = float(nodes ** 3)
    lv = torch.as_tensor(np.asarray(leaves), dtype=torch.int64, device=dev)
    w = (2.0 ** (L - lv[:, 3].to(torch.float64))) ** 3
    out = {}
    for f, name in enumerate(("u", "v")):
        e = sim_out[f] - ex[f]
        out[f"l2_{name}"] = torch.sqrt((w * (e * e).sum(1)).sum() / (nn * w.sum())).item()
        out[f"linf_{name}"] = e.abs().max().item()
        out[f"l2_exact_{name}"] = torch.sqrt((w * (ex[f] * ex[f]).sum(1)).sum() / (nn * w.sum())).item()
    return out


def time_leg(P, gm, U0, mode, prec, steps, warmup, torch, equation="wave"):
    """Warmup + timed coarse steps; HIP events on the launch stream bracket the
    timed region, torch.cuda.synchronize() on both sides."""
    sim = P.Sim(gm, equation, prec, "rk4", ko_sigma=0.1, device="cuda:0")
    sim.set_state(U0)
    stream = torch.cuda.current_stream()
    sim.advance(warmup, mode, graph=True, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.advance(steps, mode, graph=True, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = e0.elapsed_time(e1) / 1e3
    del sim
    return wall, ev


def unfused_leg(P, torch, gm, U0) -> dict:
    """One LTS coarse step of the phase-by-phase path (unzip, rhs and zip per
    stage through HBM, then the RK update; the structure of the paper's
    per-phase bars), event-timed after one warm-up step, beside the fused
    stage's step.  The split between the phases is in the kernel trace of the
    same path (profiles/)."""
    sim = P.Sim(gm, "wave", P.FP64, "rk4", ko_sigma=0.1, device="cuda:0")
    sim.set_state(U0)
    stream = torch.cuda.current_stream()
    sim.advance_unfused(1, P.MODE_LTS, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.advance_unfused(1, P.MODE_LTS, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del sim
    return {"ms_per_step": ms, "rate": gm.info()["node_updates_lts"] / (ms / 1e3)}


def nl_leg(P, torch, steps, warmup) -> dict:
    """The non-linear wave with the radiative outer boundary (Sec. 4.2) on the
    bounded shell mesh nl_c2: LTS and GTS throughput, the fused stage against
    the same 224 / 208 B per node-update as the linear wave (the boundary
    geometry comes from one leaf coordinate per tile)."""
    from workloads import config, mesh_spec, nlwave_shell
    cfg = config("nl_c2")
    gm = P.build_mesh(mesh_spec("nl_c2"))
    gm.set_tile(2)
    info = gm.info()
    lv = gm.leaves()
    U0 = torch.as_tensor(nlwave_shell(lv[:, :3], lv[:, 3], info["L"], cfg["shell_radius"], cfg["sigma"],
                                      cfg["amp"]).reshape(2, -1, 125), device="cuda:0")
    out = {"config": f"nl_c2: chi_tt = lap chi - sin(2 chi) / r^2 (Sec. 4.2, c = {cfg['nl_coeff']}) on [-1,1]^3 "
                     f"with the radiative outer "
                     f"boundary, levels {info['lmin']}-{info['lmax']} around the shell r = {cfg['shell_radius']}, "
                     f"{info['n_oct']} octants, RK4, tile side 2",
           "n_octants": info["n_oct"], "steps": steps}
    for leg in ("lts", "gts"):
        mode = P.MODE_GTS if leg == "gts" else P.MODE_LTS
        sim = P.Sim(gm, "nlwave", P.FP64, "rk4", ko_sigma=cfg["ko_sigma"], device="cuda:0",
                    nl_coeff=cfg["nl_coeff"])
        sim.set_state(U0)
        stream = torch.cuda.current_stream()
        sim.advance(warmup, mode, graph=True, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        sim.advance(steps, mode, graph=True, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ev = e0.elapsed_time(e1) / 1e3
        nu = info["node_updates_gts" if leg == "gts" else "node_updates_lts"] * steps
        out[leg] = {"rate": nu / wall, "ms_per_step": 1e3 * wall / steps, "event_s": ev}
        del sim
    a = 224 * info["node_updates_lts"] * steps / out["lts"]["event_s"] / 1e9
    out["roofline"] = {"achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(a / HBM_PEAK_GBS, 4),
                       "bytes_per_node_update": 224}
    out["measured_speedup"] = out["gts"]["ms_per_step"] / out["lts"]["ms_per_step"]
    out["model_speedup_eq_invS"] = info["s_est"]
    return out


def nodes7_leg(P, torch, steps, warmup) -> dict:
    """7^3 nodes per octant with 2:1 balance and SSP-RK3 (the paper's
    discretisation) on wave7_c2, fused side-1 tiles: LTS and GTS
    throughput, the error against the analytic solution after the timed steps,
    and the rate against the algorithmic minimum of SSP-RK3 (stage s reads U and
    the K's its stage value needs and writes K_s; the last stage also writes the
    new U): (2 + 3 + 5) x 16 B = 160 B per node-update in LTS."""
    from workloads import config, mesh_spec, wave_gaussian_torch
    cfg = config("wave7_c2")
    gm = P.build_mesh(mesh_spec("wave7_c2"))
    info = gm.info()
    lv = gm.leaves()
    U0 = wave_gaussian_torch(lv, info["L"], cfg["pulses"], sigma=cfg["sigma"], device="cuda:0", nodes=7)
    out = {"config": f"wave7_c2: 3D scalar wave, periodic [-1,1]^3, 7^3 nodes per octant, 2:1 balance, levels "
                     f"{info['lmin']}-{info['lmax']}, 4 Gaussian pulses, {info['n_oct']} octants x 343 nodes, "
                     f"SSP-RK3, fused side-1 tiles with a 13^3-point ghost table",
           "n_octants": info["n_oct"], "nodes": 343 * info["n_oct"], "steps": steps}
    for leg in ("lts", "gts"):
        mode = P.MODE_GTS if leg == "gts" else P.MODE_LTS
        sim = P.Sim(gm, "wave", P.FP64, cfg["tableau"], ko_sigma=cfg["ko_sigma"], device="cuda:0")
        sim.set_state(U0)
        stream = torch.cuda.current_stream()
        sim.advance(warmup, mode, graph=True, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        sim.advance(steps, mode, graph=True, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        nu = info["node_updates_gts" if leg == "gts" else "node_updates_lts"] * steps
        out[leg] = {"rate": nu / wall, "ms_per_step": 1e3 * wall / steps, "event_s": e0.elapsed_time(e1) / 1e3}
        T = (warmup + steps) * 0.25 * (2.0 ** (1 - info["lmin"]) / 6.0)
        out[leg]["accuracy"] = analytic_error(sim.current(), lv, info["L"], cfg["pulses"], cfg["sigma"], T, nodes=7)
        out[leg]["accuracy"]["T"] = T
        del sim
    a = 160 * info["node_updates_lts"] * steps / out["lts"]["event_s"] / 1e9
    out["roofline"] = {"achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(a / HBM_PEAK_GBS, 4),
                       "bytes_per_node_update": 160}
    out["measured_speedup"] = out["gts"]["ms_per_step"] / out["lts"]["ms_per_step"]
    out["model_speedup_eq_invS"] = info["s_est"]
    return out


def cpu_baseline(spec, cfg, target_s=15.0):
    """The oracle (FP64 NumPy, single process) on a bounded sample of the workload:
    stage-by-stage RK steps (unzip, rhs, zip, update) of the first blocks of B_0 of
    the first coarse step, until ~target_s of CPU time."""
    from oracle import fd
    from oracle import octree as ot
    from oracle import solver as so
    from workloads import wave_gaussian_torch
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except Exception:  # pragma: no cover
        lim = None
    om = ot.build_mesh(ot.MeshSpec.from_dict(spec))
    st = so.State(om, 2, "rk4", "lts")
    act = st.open_records(0)
    leaves = np.concatenate([om.anchors, om.levels[:, None]], axis=1)
    U0 = wave_gaussian_torch(leaves, om.L, cfg["pulses"], sigma=cfg["sigma"], device="cpu").numpy()
    st.U[0] = U0.reshape(st.U[0].shape)
    done_nodes = 0
    nblk = 0
    t0 = time.process_time()
    w0 = time.perf_counter()
    batch = 16
    while time.process_time() - t0 < target_s and nblk < len(act):
        blk = act[nblk:nblk + batch]
        for s in range(4):
            st.stage(blk, s, fd.rhs_wave, cfg["ko_sigma"])
        st.rk_update(blk)
        done_nodes += int((125 * om.blocks[blk, 1] ** 3).sum())
        nblk += len(blk)
    cpu = time.process_time() - t0
    wall = time.perf_counter() - w0
    if lim is not None:
        lim.unregister() if hasattr(lim, "unregister") else None
    return {"value": done_nodes / wall, "unit": "node-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{nblk} blocks of B_0 (first coarse step) of {WORKLOAD}, one full RK4 step each "
                      f"(4 x unzip+rhs+zip, update): {done_nodes} node-updates in {wall:.1f} s wall "
                      f"({cpu:.1f} s CPU), single thread"}


def host_cpu() -> dict:
    """CPU model and core count of the host the oracle runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc_online": os.cpu_count(), "cores_available": avail}


def oracle_c1_run(mode: str) -> dict:
    """The oracle in full on the C1 configuration (one Gaussian pulse, levels 2-4,
    8 coarse steps to T), single thread: wall time and the state at T."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    from oracle import octree as ot
    from oracle import solver as so
    from workloads import config, mesh_spec, wave_gaussian
    cfg = config("wave_c1")
    om = ot.build_mesh(ot.MeshSpec.from_dict(mesh_spec("wave_c1")))
    U0 = wave_gaussian(om.anchors, om.levels, om.L, cfg["pulses"], sigma=cfg["sigma"])
    t = time.perf_counter()
    out = so.run(om, U0, cfg["n_coarse"], mode, sigma=cfg["ko_sigma"])
    wall = time.perf_counter() - t
    return {"wall_s": wall, "state": out.reshape(2, om.n_oct, 125)}


def start_oracle_c1():
    """The two C1 oracle runs (LTS, GTS) in background processes (spawned: the
    parent holds a GPU context)."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    ex = ProcessPoolExecutor(2, mp_context=mp.get_context("spawn"))
    return ex, {m: ex.submit(oracle_c1_run, m) for m in ("lts", "gts")}


def field_errors(got, want, levels, L) -> dict:
    """Per field: volume-weighted l2 and max error relative to the field's max."""
    w = (2.0 ** (L - np.asarray(levels, dtype=np.float64))) ** 3
    out = {}
    for f, name in enumerate(("u", "v")):
        e = got[f] - want[f]
        scale = np.abs(want[f]).max()
        out[f"rel_l2_{name}"] = float(np.sqrt((w * (e ** 2).sum(1)).sum() / (125 * w.sum())) / scale)
        out[f"rel_linf_{name}"] = float(np.abs(e).max() / scale)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding "
              "of the path is a design, not built here.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2011_10570_amd as P
    from workloads import config, mesh_spec, wave_gaussian_torch

    # the oracle's C1 runs start before this process touches the GPU
    oracle_pool = start_oracle_c1() if not (args.no_cpu or args.copy_probe_mib) else None
    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        print(json.dumps({"copy_probe_mib": args.copy_probe_mib,
                          "gbs": copy_probe_gbs(P, torch, args.copy_probe_mib)}))
        return
    cfg = config(WORKLOAD)
    spec = mesh_spec(WORKLOAD)
    gm = P.build_mesh(spec)
    if args.tile:
        gm.set_tile(args.tile)
    info = gm.info()
    leaves = gm.leaves()
    U0 = wave_gaussian_torch(leaves, info["L"], cfg["pulses"], sigma=cfg["sigma"], device="cuda:0")
    legs = set(args.only.split(",")) if args.only else {"lts", "gts", "fp32"}
    tuned = None
    if args.tune:
        from paper_2011_10570_amd import tune
        tuned = tune.tune(gm, U0, reps=1)
        print(f"[bench] tuned: {tuned['best']} {tuned['ms']:.2f} ms", file=sys.stderr, flush=True)
        info = gm.info()

    w_lts = info["node_updates_lts"]       # DG node-updates per coarse step (eq. w_nuts)
    w_gts = info["node_updates_gts"]       # (eq. w_uts)
    res = {}
    for leg in ("lts", "gts", "fp32"):
        if leg not in legs:
            continue
        mode = P.MODE_GTS if leg == "gts" else P.MODE_LTS
        prec = P.FP32_RHS if leg == "fp32" else P.FP64
        wall, ev = time_leg(P, gm, U0, mode, prec, args.steps, args.warmup, torch)
        nu = (w_gts if leg == "gts" else w_lts) * args.steps
        res[leg] = {"wall_s": wall, "event_s": ev, "node_updates": nu, "rate": nu / wall,
                    "ms_per_step": 1e3 * wall / args.steps}
        print(f"[bench] {leg}: {res[leg]['rate']:.4e} node-updates/s, {res[leg]['ms_per_step']:.3f} ms/step",
              file=sys.stderr, flush=True)

    # accuracy at the configuration's final time T = n_coarse dt_lmin
    acc = {}
    if not args.no_accuracy:
        nco = cfg["n_coarse"]
        T = nco * 2.0 ** (-info["lmin"] - 3)
        outs = {}
        for leg in ("lts", "gts", "fp32"):
            if leg not in legs:
                continue
            mode = P.MODE_GTS if leg == "gts" else P.MODE_LTS
            prec = P.FP32_RHS if leg == "fp32" else P.FP64
            sim = P.Sim(gm, "wave", prec, "rk4", ko_sigma=0.1, device="cuda:0")
            sim.set_state(U0)
            sim.advance(nco, mode, graph=True)
            outs[leg] = sim.current()
            acc[leg] = analytic_error(outs[leg], leaves, info["L"], cfg["pulses"], cfg["sigma"], T)
            del sim
        if "lts" in outs and "gts" in outs:
            d = (outs["lts"] - outs["gts"])[0].abs().max().item()
            acc["lts_minus_gts_linf"] = d
        if "lts" in outs and "fp32" in outs:
            for f in range(2):
                den = outs["lts"][f].abs().max().item()
                acc[f"fp32_vs_fp64_rel_linf_field{f}"] = (outs["fp32"][f] - outs["lts"][f]).abs().max().item() / den
        acc["T"] = T

    # roofline of the fused stage: one RK stage of every active tile is one
    # ghost-table pre-pass plus one fused launch per tile side; the timed region
    # holds these and one 1-thread counter increment per coarse step.
    lts = res.get("lts")
    roof = None
    if lts:
        tiles = gm.tiles()
        acc_ = stage_accounting(info, tiles)
        alg, stages, launches = acc_["alg_bytes"], acc_["stages"], acc_["launches"]
        assert alg == 224 * w_lts
        t_step = lts["event_s"] / args.steps
        achieved = alg / t_step / 1e9
        cp = copy_probe_gbs(P, torch)
        side_names = {1: "k_fused<1>", 2: "k_fused<2>", 4: "k_stream"}
        kern = " + ".join(["k_ghost_pre", "k_ghost_multi"] + [side_names[t] for t in sorted(set(tiles[:, 4].tolist()), reverse=True)])
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": stored_traffic(),
                "kernel": f"fused stage ({kern}), FP64 wave",
                "algorithmic_bytes_per_stage": round(alg / stages), "stages_per_step": stages,
                "launches_per_step": launches, "avg_stage_us": round(1e6 * t_step / stages, 2),
                "copy_probe_gbs": round(cp, 1), "frac_of_copy": round(achieved / cp, 4),
                "sources_sha256": source_digest()}

    # GTS moves 208 B per node-update (its last stage stores no K): the same
    # fused stage kernels against the same peak
    gts_roof = None
    if res.get("gts"):
        t_step = res["gts"]["event_s"] / args.steps
        n_stages = 4 * int(info["n_substeps"])
        a_g = 208 * w_gts / t_step / 1e9
        gts_roof = {"achieved": round(a_g, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(a_g / HBM_PEAK_GBS, 4),
                    "bytes_per_node_update": 208, "avg_stage_us": round(1e6 * t_step / n_stages, 2)}

    maxwell = None
    if not args.no_maxwell and "lts" in legs:
        # 6 fields (E, B) from divergence-free Gaussian data, side-2 tiles (one
        # workgroup per CU; 1.4x the side-1 tiles' rate)
        from workloads import maxwell_gaussian_torch
        gm.set_tile(2)
        Um = maxwell_gaussian_torch(leaves, info["L"], cfg["pulses"], sigma=cfg["sigma"], device="cuda:0")
        steps_m = max(1, min(args.steps, 4))
        wall, ev = time_leg(P, gm, Um, P.MODE_LTS, P.FP64, steps_m, 1, torch, equation="maxwell")
        del Um
        gm.set_tile(args.tile or 2)
        rate = w_lts * steps_m / wall
        a_m = 672 * w_lts * steps_m / ev / 1e9
        maxwell = {"rate": rate, "ms_per_step": 1e3 * wall / steps_m, "steps": steps_m, "tile": 2,
                   "roofline": {"achieved": round(a_m, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(a_m / HBM_PEAK_GBS, 4), "bytes_per_node_update": 672}}
        print(f"[bench] maxwell: {rate:.4e} node-updates/s, frac {a_m / HBM_PEAK_GBS:.3f}", file=sys.stderr,
              flush=True)

    unf = None
    if args.unfused and "lts" in legs:
        unf = unfused_leg(P, torch, gm, U0)
        print(f"[bench] unfused: {unf['ms_per_step']:.1f} ms per coarse step", file=sys.stderr, flush=True)

    nl = None
    if not args.no_nl and "lts" in legs:
        nl = nl_leg(P, torch, max(1, min(args.steps, 8)), args.warmup)
        print(f"[bench] nlwave: lts {nl['lts']['rate']:.4e}, gts {nl['gts']['rate']:.4e} node-updates/s, "
              f"frac {nl['roofline']['frac']:.3f}", file=sys.stderr, flush=True)

    n7 = None
    if not args.no_n7 and "lts" in legs:
        n7 = nodes7_leg(P, torch, max(1, min(args.steps, 4)), 1)
        print(f"[bench] nodes7: lts {n7['lts']['rate']:.4e}, gts {n7['gts']['rate']:.4e} node-updates/s, "
              f"frac {n7['roofline']['frac']:.3f}", file=sys.stderr, flush=True)

    batch = None
    if not args.no_batch:
        from paper_2011_10570_amd import serve
        bc = config("batch")
        # the batch launch shape, tuned on one coarse step of the same problems
        # (every candidate's states bitwise equal); then every problem to T
        from paper_2011_10570_amd import tune
        from workloads import wave_gaussian_torch
        tms, tst = [], []
        for p in bc["problems"]:
            m = P.Mesh(p["mesh"])
            tms.append(m)
            tst.append(wave_gaussian_torch(m.leaves(), m.info()["L"], [p["mesh"]["criteria"][0]["center"]],
                                           sigma=0.1, device="cuda:0"))
        tb = tune.tune_batch(tms, tst, tiles=(2,), threads=(256, 512), max_workgroups=(2048, 4096, 16384))
        batch = {"tuned_shape": {"tile": tb["best"][0], "threads": tb["best"][1], "max_workgroups": tb["best"][2],
                                 "candidates_ms": {str(k): round(v, 3) for k, v in tb["table"]}}}
        del tms, tst
        for name, prec in (("fp64", P.FP64), ("fp32_rhs", P.FP32_RHS)):
            print(f"[bench] batch {name}: 64 problems to T...", file=sys.stderr, flush=True)
            batch[name] = serve.batch_throughput(bc["problems"], bc["n_coarse"], precision=prec,
                                                 alone=(prec == P.FP64))
            print(f"[bench] batch {name}: {batch[name]['node_updates_per_s']:.4e} node-updates/s", file=sys.stderr,
                  flush=True)
    served = None
    if not args.no_serve:
        from paper_2011_10570_amd import serve
        print("[bench] serving loop...", file=sys.stderr, flush=True)
        cap = batch["fp64"]["node_updates_per_s"] if batch else None
        served = serve.run_config(capacity=cap, n=args.serve_requests)
        print(f"[bench] serve: p50 {served['p50_time_to_t_s']:.3f} s, p99 {served['p99_time_to_t_s']:.3f} s",
              file=sys.stderr, flush=True)

    cpu = None
    c3 = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle sample)...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(spec, cfg)
        cpu.update(host_cpu())
        ex, futs = oracle_pool
        full = {m: f.result() for m, f in futs.items()}
        ex.shutdown()
        c1cfg = config("wave_c1")
        gc1 = P.build_mesh(mesh_spec("wave_c1"))
        ic1 = gc1.info()
        c1 = {"config": "wave_c1: levels 2-4, 596 octants, one Gaussian pulse, RK4, 8 coarse steps to T = 0.25",
              "threads": 1, "processes": 2}
        for m in ("lts", "gts"):
            nu = ic1["node_updates_lts" if m == "lts" else "node_updates_gts"] * c1cfg["n_coarse"]
            c1[m] = {"wall_s": full[m]["wall_s"], "node_updates": nu, "rate": nu / full[m]["wall_s"]}
        c1["oracle_lts_over_gts_speedup"] = full["gts"]["wall_s"] / full["lts"]["wall_s"]
        c1["model_speedup_eq_invS"] = ic1["s_est"]
        cpu["c1_full_run"] = c1
        # C3: the C1 configuration with FP32 stencils on the GPU vs the FP64 oracle at T
        lv1 = gc1.leaves()
        U1 = wave_gaussian_torch(lv1, ic1["L"], c1cfg["pulses"], sigma=c1cfg["sigma"], device="cuda:0")
        c3 = {"config": "C1 mesh and data to T, FP32 stencils, FP64 state / RK / time interpolation"}
        for name, prec in (("fp32_rhs", P.FP32_RHS), ("fp64", P.FP64)):
            sim = P.Sim(gc1, "wave", prec, "rk4", ko_sigma=c1cfg["ko_sigma"], device="cuda:0")
            sim.set_state(U1)
            sim.advance(c1cfg["n_coarse"], P.MODE_LTS, graph=True)
            c3[f"{name}_vs_oracle"] = field_errors(sim.current().cpu().numpy(), full["lts"]["state"], lv1[:, 3],
                                                   ic1["L"])
            del sim

    value = lts["rate"] if lts else None
    out = {
        "metric": "node-updates/s (LTS vs GTS, FP64 vs FP32-RHS) at fixed L2 error; p99 latency",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": lts["ms_per_step"] if lts else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}: 3D scalar wave (u, v), periodic [-1,1]^3 octree, levels "
                               f"{info['lmin']}-{info['lmax']}, 4 seeded Gaussian pulses (sigma 0.1), "
                               f"{info['n_oct']} octants x 125 nodes, RK4, 6th-order FD + KO, LTS, "
                               f"dt_l = 0.25 h_l; step = one coarsest step ({info['n_substeps']} substeps)",
                   "n_octants": info["n_oct"], "nodes": 125 * info["n_oct"],
                   "level_count": {str(l): int(c) for l, c in enumerate(info["level_count"]) if c},
                   "node_updates_per_step_lts": w_lts, "node_updates_per_step_gts": w_gts,
                   "tile": info["tile"]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if "gts" in res and lts:
        out["lts_vs_gts"] = {"gts_rate": res["gts"]["rate"], "gts_ms_per_step": res["gts"]["ms_per_step"],
                             "measured_speedup": res["gts"]["wall_s"] / lts["wall_s"],
                             "model_speedup_eq_invS": info["s_est"], "model_s_max": info["s_max"],
                             "effective_gts_equivalent_rate": w_gts * args.steps / lts["wall_s"]}
    if "fp32" in res and lts:
        out["fp32_rhs"] = {"rate": res["fp32"]["rate"], "speedup_over_fp64": lts["wall_s"] / res["fp32"]["wall_s"]}
    if acc:
        out["accuracy"] = acc
    if gts_roof:
        out["gts_roofline"] = gts_roof
    if maxwell:
        out["maxwell"] = maxwell
    if unf:
        out["unfused"] = unf
    if nl:
        out["nlwave"] = nl
    if n7:
        out["nodes7"] = n7
    if c3:
        out["c3"] = c3
    if batch:
        out["batch"] = batch
    if served:
        out["serve"] = served
        out["p99_time_to_t_s"] = served["p99_time_to_t_s"]
    if tuned:
        out["tuned"] = {"best": tuned["best"], "ms": tuned["ms"]}
    line = json.dumps(out)
    print(line)
    if args.jsonl:
        with open(args.jsonl, "a") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
