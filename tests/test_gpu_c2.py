"""GPU parity at the benchmark's full size: wave_c2 (201,216 octants, levels
3-8, 4 Gaussian pulses), in the launch configuration bench.py times (default
launch shape, side-2 tiles).

* The first fused stage of a coarse step from seeded random DG data: every stage
  state is U0 there (stage 1 of Alg. 2, all time cases start together), so the
  oracle computes K_1 of any block on its own.  A seeded sample of blocks of
  every level is compared, element by element, at the FP64 tolerance.
* One whole coarse step, graph-captured as in the benchmark: properties that
  hold at any size -- LTS and GTS agree to the scheme's error, and both are
  close to the analytic spherical wave (image sums over the periodic box)."""
import os
import sys

import numpy as np
import pytest
import torch

import paper_2011_10570_amd as P
from oracle import fd
from oracle import octree as ot
from oracle import solver as so
from workloads import config, mesh_spec, random_dg, wave_gaussian_torch

from gpu_common import TOL, rel_err

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
