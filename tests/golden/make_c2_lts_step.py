"""Writes tests/golden/c2_lts_step.txt: the oracle's wave_c2 state (201,216
octants, levels 3-8, 4 Gaussian pulses, RK4, FP64) after one LTS coarse step
(Alg. 2: 32 substeps), at a seeded sample of nodes, with the per-field maximum
and sum of squares of the whole state and the run's wall time and cores; with
--config wave7_c2 the same for the 7^3-node workload (75,230 octants, SSP-RK3)
into tests/golden/wave7_c2_lts_step.txt.

Test infrastructure: it calls oracle/ (and the input generator of workloads/)
only.  The blocks of one stage are independent (each reads the step records and
earlier stages of its neighbours and writes K_s of its own octants; Alg. 2,
eqs. fc_1/fc_2), so persistent worker processes, each owning the blocks
b = w mod P, run them over state arrays in shared memory; the parent opens and
closes the step records and orders the stages.  Every block's arithmetic is the
oracle's own (State.unzip, fd.rhs_wave, State.zip_into, the RK update).

usage: python tests/golden/make_c2_lts_step.py [--config wave_c2|wave7_c2] [--procs 8] [--samples 4096]
       python tests/golden/make_c2_lts_step.py --config wave_c1 --check   (the parallel driver
       against oracle.solver.run, bitwise; no file written)
"""
import argparse
import os
import sys
import time
from multiprocessing import get_context, shared_memory

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fd  # noqa: E402
from oracle import octree as ot  # noqa: E402
from oracle import solver as so  # noqa: E402
from workloads import config, mesh_spec, wave_gaussian  # noqa: E402

OUT = {"wave_c2": os.path.join(ROOT, "tests", "golden", "c2_lts_step.txt"),
       "wave7_c2": os.path.join(ROOT, "tests", "golden", "wave7_c2_lts_step.txt")}
SEED = 2011


def to_shared(st, name, shms):
    a = getattr(st, name)
    shm = shared_memory.SharedMemory(create=True, size=max(1, a.nbytes))
    b = np.ndarray(a.shape, a.dtype, buffer=shm.buf)
    b[...] = a
    setattr(st, name, b)
    shms.append(shm)


def worker(st, w, nproc, sigma, conn):
    """Blocks b with b mod nproc == w: stage s (unzip, rhs, zip into K_s) or the
    RK update of substep j, on command."""
    try:
        while True:
            cmd = conn.recv()
            if cmd[0] == "quit":
                break
            j = cmd[1]
            act = [b for b in ot.active_blocks(st.mesh, j, "lts") if b % nproc == w]
            if cmd[0] == "stage":
                st.stage(act, cmd[2], fd.rhs_wave, sigma)
            else:
                st.rk_update(act)
            conn.send("ok")
    except BaseException as e:  # report, then stop
        conn.send(f"error: {e!r}")
    conn.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--samples", type=int, default=4096)
    ap.add_argument("--config", default="wave_c2")
    ap.add_argument("--check", action="store_true",
                    help="compare with oracle.solver.run bitwise instead of writing a fixture")
    a = ap.parse_args()
    cfg, spec = config(a.config), mesh_spec(a.config)
    tableau = cfg.get("tableau", "rk4")
    t0 = time.time()
    om = ot.build_mesh(ot.MeshSpec.from_dict(spec))
    nn = om.nodes ** 3
    U0 = wave_gaussian(om.anchors, om.levels, om.L, cfg["pulses"], sigma=cfg["sigma"], nodes=om.nodes)
    st = so.State(om, 2, tableau, "lts")
    st.set_initial(U0)
    shms = []
    for name in ("U", "K", "cur_par", "cur_t", "rec_par", "rec_t0"):
        to_shared(st, name, shms)
    print(f"[c2-oracle] mesh {om.n_oct} octants, {len(om.blocks)} blocks ({time.time() - t0:.1f} s)", flush=True)
    ctx = get_context("fork")
    conns, procs = [], []
    for w in range(a.procs):
        parent, child = ctx.Pipe()
        p = ctx.Process(target=worker, args=(st, w, a.procs, cfg["ko_sigma"], child))
        p.start()
        conns.append(parent)
        procs.append(p)

    def run(cmd):
        for c in conns:
            c.send(cmd)
        for c in conns:
            r = c.recv()
            if r != "ok":
                raise RuntimeError(r)

    try:
        t1 = time.time()
        for j in range(ot.substeps(om)):
            act = st.open_records(j)
            for s in range(st.p):
                run(("stage", j, s))
            run(("rk", j))
            st.close_records(act)
            print(f"[c2-oracle] substep {j}: {len(act)} blocks, {time.time() - t1:.0f} s", flush=True)
        wall = time.time() - t1
    finally:
        for c in conns:
            c.send(("quit", 0))
        for p in procs:
            p.join(timeout=10)
    assert (st.cur_t == st.cur_t[0]).all()
    out = st.current().reshape(2, om.n_oct, -1)
    for shm in shms:
        shm.close()
        shm.unlink()
    if a.check:
        want = so.run(om, U0, 1, "lts", "wave", tableau, cfg["ko_sigma"]).reshape(2, om.n_oct, -1)
        assert np.array_equal(out, want), np.abs(out - want).max()
        print(f"[c2-oracle] {a.config}: the parallel driver equals oracle.solver.run bitwise", flush=True)
        return
    nu = sum(len(ot.active_blocks(om, j, "lts")) for j in range(ot.substeps(om)))
    node_updates = int(sum(nn * int(om.blocks[b, 1]) ** 3 for j in range(ot.substeps(om))
                           for b in ot.active_blocks(om, j, "lts")))
    rng = np.random.default_rng(SEED)
    octs = rng.integers(0, om.n_oct, a.samples)
    nodes = rng.integers(0, nn, a.samples)
    out_path = OUT[a.config]
    with open(out_path, "w") as f:
        f.write(f"# {a.config}, one LTS coarse step ({ot.substeps(om)} substeps), {tableau.upper()}, FP64, KO sigma "
                f"{cfg['ko_sigma']}: oracle state at seeded nodes (seed {SEED})\n")
        f.write("# written by tests/golden/make_c2_lts_step.py (calls oracle/ only)\n")
        f.write(f"# wall_s {wall:.1f} procs {a.procs} block_steps {nu} node_updates {node_updates}\n")
        for k in range(2):
            f.write(f"max_abs {k} {float(np.abs(out[k]).max())!r}\n")
            f.write(f"sum_sq {k} {float(np.sum(out[k] * out[k]))!r}\n")
        for o, n in zip(octs, nodes):
            f.write(f"{int(o)} {int(n)} {float(out[0, o, n])!r} {float(out[1, o, n])!r}\n")
    print(f"[c2-oracle] wrote {out_path}: {wall:.0f} s on {a.procs} processes, "
          f"{node_updates / wall:.3e} node-updates/s", flush=True)


if __name__ == "__main__":
    main()
