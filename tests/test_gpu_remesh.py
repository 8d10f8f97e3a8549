"""GPU parity of remeshing at coarse-step boundaries (Sec. 3.2.2 wavelet
criterion, Sec. 5) through the C ABI against the oracle: wavelet indicators,
the new octree (bit-exact), the intergrid transfer, and an LTS run on C1 that
remeshes after every coarse step so the octree follows the pulse."""
import numpy as np
import pytest
import torch

import paper_2011_10570_amd as P
from oracle import octree as ot
from oracle import remesh as rm
from oracle import solver as so
from workloads import config, mesh_spec, wave_gaussian

from gpu_common import TOL, oracle_mesh, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
EPS = 1e-3


def _c1():
    om = oracle_mesh("wave_c1")
    gm = P.build_mesh(mesh_spec("wave_c1"))
    cfg = config("wave_c1")
    U0 = wave_gaussian(om.anchors, om.levels, om.L, cfg["pulses"], sigma=cfg["sigma"])
    return om, gm, U0


def _dev(a, N):
    return torch.from_numpy(np.ascontiguousarray(a).reshape(2, N, 125)).to(DEV)


def _clear_of_thresholds(leaf, fam, eps):
    """No indicator close to a decision threshold (the two sides round the
    indicator sums in different orders)."""
    for v, t in ((leaf, eps), (fam[fam >= 0], eps / 4)):
        if len(v) and (np.abs(v - t) <= 1e-9 * t).any():
            return False
    return True


def test_indicators_match_oracle():
    om, gm, U0 = _c1()
    lw, fw = P.remesh_indicators(gm, _dev(U0, om.n_oct))
    leaf, fam, fwo = rm.indicators(om, U0)
    assert np.abs(lw - leaf).max() <= 1e-12 * leaf.max()
    assert np.array_equal(np.nonzero(fw >= 0)[0], fam)
    assert np.abs(fw[fam] - fwo).max() <= 1e-12 * max(leaf.max(), 1e-300)


def test_remesh_and_transfer_match_oracle():
    om, gm, U0 = _c1()
    U = _dev(U0, om.n_oct)
    lw, fw = P.remesh_indicators(gm, U)
    assert _clear_of_thresholds(lw, fw, EPS)
    new = P.remesh(gm, U, EPS, 2, 4)
    onew = rm.remesh(om, U0, EPS, 2, 4)
    lv = new.leaves()
    assert np.array_equal(lv[:, :3], onew.anchors) and np.array_equal(lv[:, 3], onew.levels)
    assert np.array_equal(new.blocks(), onew.blocks)
    got = P.transfer(gm, new, U).cpu().numpy()
    want = rm.transfer(om, onew, U0).reshape(2, onew.n_oct, 125)
    assert rel_err(got, want) < TOL
    # identity transfer is a copy
    assert torch.equal(P.transfer(gm, gm, U), U)


def test_lts_with_remeshing_follows_oracle():
    """C1 pulse: 3 rounds of (one LTS coarse step, remesh, transfer) on the GPU and
    in the oracle; the octrees agree bit for bit and the states to 1e-12."""
    om, gm, U0 = _c1()
    cfg = config("wave_c1")
    ostate = U0
    gstate = _dev(U0, om.n_oct)
    for rnd in range(3):
        print(f"[remesh] round {rnd}: {om.n_oct} octants", flush=True)
        sim = P.Sim(gm, "wave", P.FP64, "rk4", ko_sigma=cfg["ko_sigma"], device=DEV)
        sim.set_state(gstate)
        sim.advance(1, P.MODE_LTS)
        gcur = sim.current()
        ostate = so.run(om, ostate, 1, "lts", sigma=cfg["ko_sigma"])
        assert rel_err(gcur.cpu().numpy(), ostate.reshape(2, om.n_oct, 125)) < TOL
        lw, fw = P.remesh_indicators(gm, gcur)
        assert _clear_of_thresholds(lw, fw, EPS)
        gnew = P.remesh(gm, gcur, EPS, 2, 4)
        onew = rm.remesh(om, ostate, EPS, 2, 4)
        lv = gnew.leaves()
        assert np.array_equal(lv[:, :3], onew.anchors) and np.array_equal(lv[:, 3], onew.levels)
        gstate = P.transfer(gm, gnew, gcur)
        ostate = rm.transfer(om, onew, ostate)
        assert rel_err(gstate.cpu().numpy(), ostate.reshape(2, onew.n_oct, 125)) < TOL
        gm, om = gnew, onew
        del sim
