"""GPU parity at the benchmark's full size: wave_c2 (201,216 octants, levels
3-8, 4 Gaussian pulses), in the launch configuration bench.py times (default
launch shape, side-2 tiles).

* The first fused stage of a coarse step from seeded random DG data: every stage
  state is U0 there (stage 1 of Alg. 2, all time cases start together), so the
  oracle computes K_1 of any block on its own.  A seeded sample of blocks of
  every level is compared, element by element, at the FP64 tolerance.
* Later stages at positions inside a coarse step (seeded random U and K, step
  records positioned at substep j of coarse step n): every time case of the
  stage conversion (same level, finer source, coarser source at a common start
  and one fine step later) occurs; a sample of 8 active blocks per level is
  compared element by element with the oracle's stage (and RK update at the
  last stage).
* One whole coarse step, graph-captured as in the benchmark: properties that
  hold at any size -- LTS and GTS agree to the scheme's error, and both are
  close to the analytic spherical wave (image sums over the periodic box).
* One whole LTS coarse step against the oracle's own full run of it (a stored
  fixture: 4096 seeded nodes, the whole state's maximum and sum of squares)."""
import os
import sys

import numpy as np
import pytest
import torch

import paper_2011_10570_amd as P
from oracle import fd
from oracle import octree as ot
from oracle import solver as so
from workloads import config, mesh_spec, random_dg, wave_gaussian, wave_gaussian_torch

from gpu_common import TOL, positioned_state, rel_err

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def c2():
    cfg, spec = config("wave_c2"), mesh_spec("wave_c2")
    print("[c2] building meshes", flush=True)
    gm = P.build_mesh(spec)
    gm.set_tile(2)
    om = ot.build_mesh(ot.MeshSpec.from_dict(spec))
    return cfg, gm, om


def test_c2_first_stage_sampled_blocks(c2):
    cfg, gm, om = c2
    U0 = random_dg((2, om.n_oct, 125), 2011)
    assert P.get_launch() == (512, 65536, 512)
    sim = P.Sim(gm, "wave", P.FP64, "rk4", ko_sigma=cfg["ko_sigma"], device=DEV)
    sim.set_state(U0)
    print("[c2] fused stage 1 of substep 0", flush=True)
    P.fused_stage(gm, sim.U, sim.K, P.EQ_WAVE, cfg["ko_sigma"], 0, 0, P.MODE_LTS, 0)
    got = sim.K[0].cpu().numpy()                                   # [F][N][125]
    st = so.State(om, 2, "rk4", "lts")
    st.set_initial(U0.reshape(st.U[0].shape))
    act = np.asarray(st.open_records(0))
    lev = om.blocks[act, 2]
    rng = np.random.default_rng(2011)
    sample = np.concatenate([rng.choice(act[lev == l], size=min(8, int((lev == l).sum())), replace=False)
                             for l in np.unique(lev)])
    assert len(np.unique(om.blocks[sample, 2])) == len(np.unique(om.levels))
    st.stage(sample, 0, fd.rhs_wave, cfg["ko_sigma"])
    octs = np.concatenate([np.arange(om.blocks[b, 0], om.blocks[b, 0] + om.blocks[b, 1] ** 3) for b in sample])
    want = st.K[0].reshape(2, om.n_oct, 125)[:, octs]
    assert rel_err(got[:, octs], want) < TOL


def _sample_active(om, act, seed, per_level=8):
    lev = om.blocks[act, 2]
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.choice(act[lev == l], size=min(per_level, int((lev == l).sum())), replace=False)
                           for l in np.unique(lev)])


@pytest.mark.parametrize("mode,n,j,stage", [("lts", 1, 16, 3), ("lts", 3, 1, 1), ("lts", 0, 31, 2),
                                            ("lts", 2, 2, 3), ("gts", 1, 7, 2), ("gts", 0, 3, 3)])
def test_c2_positioned_stage_sampled_blocks(c2, mode, n, j, stage):
    """Fused stage `stage` of substep j of coarse step n on the full C2 mesh vs the
    oracle's unzip + rhs + zip (+ RK update) of a sample of the active blocks."""
    cfg, gm, om = c2
    print(f"[c2] positioned {mode} n={n} j={j} stage={stage}", flush=True)
    st, act = positioned_state(om, 2, mode, n, j, seed=7000 + 100 * n + j)
    act = np.asarray(act)
    U = torch.from_numpy(st.U.reshape(2, 2, om.n_oct, 125)).to(DEV)
    K = torch.from_numpy(st.K.reshape(4, 2, om.n_oct, 125)).to(DEV)
    md = P.MODE_GTS if mode == "gts" else P.MODE_LTS
    P.fused_stage(gm, U, K, P.EQ_WAVE, cfg["ko_sigma"], stage, j, md, n)
    sample = _sample_active(om, act, 11 * n + j)
    if mode == "lts":   # every active level is sampled
        assert len(np.unique(om.blocks[sample, 2])) == len(np.unique(om.blocks[act, 2]))
    st.stage(sample, stage, fd.rhs_wave, cfg["ko_sigma"])
    octs = np.concatenate([np.arange(om.blocks[b, 0], om.blocks[b, 0] + om.blocks[b, 1] ** 3) for b in sample])
    if not (mode == "gts" and stage == 3):   # GTS does not store the last stage
        got = K[stage][:, torch.from_numpy(octs).to(DEV)].cpu().numpy()
        want = st.K[stage].reshape(2, om.n_oct, 125)[:, octs]
        assert rel_err(got, want) < TOL
    if stage == 3:
        st.rk_update(sample)
        par = st.rec_par[sample]
        for b, pb in zip(sample, par):
            o = np.arange(om.blocks[b, 0], om.blocks[b, 0] + om.blocks[b, 1] ** 3)
            got = U[1 - pb][:, torch.from_numpy(o).to(DEV)].cpu().numpy()
            want = st.U[1 - pb].reshape(2, om.n_oct, 125)[:, o]
            assert rel_err(got, want) < TOL, b


def test_c2_coarse_step_properties(c2):
    cfg, gm, om = c2
    info = gm.info()
    U0 = wave_gaussian_torch(gm.leaves(), info["L"], cfg["pulses"], sigma=cfg["sigma"], device=DEV)
    out = {}
    for name, mode in (("lts", P.MODE_LTS), ("gts", P.MODE_GTS)):
        print(f"[c2] one coarse step {name}", flush=True)
        sim = P.Sim(gm, "wave", P.FP64, "rk4", ko_sigma=cfg["ko_sigma"], device=DEV)
        sim.set_state(U0)
        sim.advance(1, mode, graph=True)
        out[name] = sim.current()
        assert torch.isfinite(out[name]).all()
        del sim
    T = 2.0 ** (-info["lmin"] - 3)
    lv = gm.leaves()
    for name in out:
        e = bench.analytic_error(out[name], lv, info["L"], cfg["pulses"], cfg["sigma"], T)
        assert e["l2_u"] < 1e-6 and e["linf_u"] < 2e-5, (name, e)
        assert e["l2_v"] < 1e-4 and e["linf_v"] < 1e-3, (name, e)
    # LTS and GTS differ by the time discretisation error only: per field, far
    # below the field's scale
    for f in range(2):
        d = (out["lts"][f] - out["gts"][f]).abs().max().item()
        scale = out["gts"][f].abs().max().item()
        assert d < 1e-6 * scale, (f, d, scale)


def _golden_c2_step():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_lts_step.txt")
    stats, rows = {}, []
    for line in open(path):
        if line.startswith("#"):
            continue
        p = line.split()
        if p[0] in ("max_abs", "sum_sq"):
            stats[(p[0], int(p[1]))] = float(p[2])
        else:
            rows.append((int(p[0]), int(p[1]), float(p[2]), float(p[3])))
    return stats, np.array(rows)


def test_c2_lts_coarse_step_vs_oracle(c2):
    """One whole LTS coarse step of the benchmark workload (graph-captured, the
    launch configuration bench.py times) against the oracle's full C2 run
    (tests/golden/c2_lts_step.txt, written by make_c2_lts_step.py from oracle/
    only): element by element at 4096 seeded nodes, and the whole state's
    per-field maximum and sum of squares."""
    cfg, gm, om = c2
    stats, rows = _golden_c2_step()
    assert len(rows) == 4096
    lv = gm.leaves()
    U0 = wave_gaussian(lv[:, :3], lv[:, 3], gm.info()["L"], cfg["pulses"], sigma=cfg["sigma"])
    print("[c2] one LTS coarse step vs the oracle's full run", flush=True)
    sim = P.Sim(gm, "wave", P.FP64, "rk4", ko_sigma=cfg["ko_sigma"], device=DEV)
    sim.set_state(U0)
    sim.advance(1, P.MODE_LTS, graph=True)
    out = sim.current().reshape(2, om.n_oct, 125)
    o = torch.from_numpy(rows[:, 0].astype(np.int64)).to(DEV)
    n = torch.from_numpy(rows[:, 1].astype(np.int64)).to(DEV)
    for f in range(2):
        got = out[f][o, n].cpu().numpy()
        scale = stats[("max_abs", f)]
        assert np.abs(got - rows[:, 2 + f]).max() <= TOL * scale, f
        assert abs(out[f].abs().max().item() - scale) <= TOL * scale, f
        ss = (out[f] * out[f]).sum().item()
        assert abs(ss - stats[("sum_sq", f)]) <= 1e-11 * stats[("sum_sq", f)], f
