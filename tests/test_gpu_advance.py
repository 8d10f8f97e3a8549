"""End-to-end GPU parity of lts_advance (fused, graph-captured) and
lts_advance_unfused with the oracle's LTS / GTS drivers."""
import numpy as np
import pytest
import torch

import paper_2011_10570_amd as P
from oracle import octree as ot
from oracle import solver as so
from workloads import (config, consistent_random_dg, mesh_spec, wave_gaussian, wave_plane, maxwell_gaussian,
                       random_dg)

from gpu_common import TOL, oracle_c1_at_T, oracle_mesh, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _run_gpu(gm, U0, n, mode, eq="wave", prec=P.FP64, graph=True, unfused=False, tile=2, tableau="rk4"):
    gm.set_tile(tile)
    sim = P.Sim(gm, eq, prec, tableau, ko_sigma=0.1, device=DEV)
    sim.set_state(U0)
    if unfused:
        sim.advance_unfused(n, mode)
    else:
        sim.advance(n, mode, graph=graph)
    out = sim.current().cpu().numpy()
    gm.set_tile(2)
    return out


@pytest.fixture(scope="module")
def c1():
    om = oracle_mesh("wave_c1")
    gm = P.build_mesh(mesh_spec("wave_c1"))
    cfg = config("wave_c1")
    U0 = wave_gaussian(om.anchors, om.levels, om.L, cfg["pulses"], sigma=0.1)
    return om, gm, U0


N_C1 = config("wave_c1")["n_coarse"]


@pytest.fixture(scope="module")
def c1_oracle(c1):
    """LTS and GTS of the oracle on the whole C1 configuration, to its final time
    T = 8 dt_lmin (8 coarse steps), computed in two processes."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    print(f"[oracle] wave_c1 lts+gts {N_C1} coarse steps", flush=True)
    with ProcessPoolExecutor(2, mp_context=mp.get_context("spawn")) as ex:
        res = dict(zip(("lts", "gts"), ex.map(oracle_c1_at_T, ("lts", "gts"))))
    return res


@pytest.mark.parametrize("mode", ["lts", "gts"])
def test_advance_fused_graph(c1, c1_oracle, mode):
    """C1 to T: LTS / GTS with the graph-captured fused path vs the oracle."""
    om, gm, U0 = c1
    md = P.MODE_LTS if mode == "lts" else P.MODE_GTS
    got = _run_gpu(gm, U0, N_C1, md)
    assert rel_err(got, c1_oracle[mode]) < TOL


@pytest.mark.parametrize("mode", ["lts", "gts"])
def test_advance_unfused(c1, c1_oracle, mode):
    om, gm, U0 = c1
    md = P.MODE_LTS if mode == "lts" else P.MODE_GTS
    got = _run_gpu(gm, U0, N_C1, md, unfused=True)
    assert rel_err(got, c1_oracle[mode]) < TOL


def test_fused_equals_unfused_and_tiles_and_graph(c1):
    """Tile shape, graph capture and fusion change nothing: bitwise equal runs."""
    om, gm, U0 = c1
    a = _run_gpu(gm, U0, 3, P.MODE_LTS, graph=True, tile=2)
    b = _run_gpu(gm, U0, 3, P.MODE_LTS, graph=False, tile=1)
    c = _run_gpu(gm, U0, 3, P.MODE_LTS, unfused=True)
    d = _run_gpu(gm, U0, 3, P.MODE_LTS, graph=True, tile=4)
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)
    assert np.array_equal(a, d)


@pytest.mark.parametrize("mode", [P.MODE_LTS, P.MODE_GTS])
def test_streamed_blocks_equal_tiles(mode):
    """A mesh with several 4^3 blocks next to coarser and finer leaves: streamed
    whole blocks (tile side 4) give bitwise the side-2 tile result."""
    p = config("batch")["problems"][6]
    gm = P.build_mesh(p["mesh"])
    lv = gm.leaves()
    U0 = wave_gaussian(lv[:, :3], lv[:, 3], gm.info()["L"], [p["mesh"]["criteria"][0]["center"]], sigma=0.1)
    a = _run_gpu(gm, U0, 2, mode, tile=2)
    b = _run_gpu(gm, U0, 2, mode, tile=4)
    assert np.array_equal(a, b)


def _blocky_mesh():
    """A batch problem with several 4^3 blocks next to coarser and finer leaves."""
    p = config("batch")["problems"][6]
    gm = P.build_mesh(p["mesh"])
    lv = gm.leaves()
    U0 = wave_gaussian(lv[:, :3], lv[:, 3], gm.info()["L"], [p["mesh"]["criteria"][0]["center"]], sigma=0.1)
    return gm, U0


def test_streamed_blocks_ssprk3():
    """Streamed blocks with SSP-RK3 (stage masks with two same-level stages)."""
    gm, U0 = _blocky_mesh()
    a = _run_gpu(gm, U0, 2, P.MODE_LTS, tile=2, tableau="ssprk3")
    b = _run_gpu(gm, U0, 2, P.MODE_LTS, tile=4, tableau="ssprk3")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", [P.FP64, P.FP32_RHS])
@pytest.mark.parametrize("tile", [1, 2, 4])
def test_walked_tiles_equal_one_per_workgroup(tile, prec):
    """Under a small grid cap every workgroup walks many tiles, loading the next
    tile's tables while the current one runs: results equal one workgroup per
    tile, bitwise."""
    gm, U0 = _blocky_mesh()
    old = P.get_launch()
    try:
        P.set_launch(512, 65536, 512)
        a = _run_gpu(gm, U0, 1, P.MODE_LTS, prec=prec, tile=tile)
        for shape in ((512, 16, 512), (256, 64, 256)):
            print(f"[walk] tile {tile} prec {prec} shape {shape}", flush=True)
            P.set_launch(*shape)
            b = _run_gpu(gm, U0, 1, P.MODE_LTS, prec=prec, tile=tile)
            assert np.array_equal(a, b), shape
    finally:
        P.set_launch(*old)


def test_graph_replays_repeatable(c1):
    """Several graph replays with eager work and syncs between them."""
    om, gm, U0 = c1
    sim = P.Sim(gm, "wave", P.FP64, "rk4", ko_sigma=0.1, device=DEV)
    sim.set_state(U0)
    ref = P.Sim(gm, "wave", P.FP64, "rk4", ko_sigma=0.1, device=DEV)
    ref.set_state(U0)
    for k in range(3):
        sim.advance(1, P.MODE_LTS, graph=True)
        ref.advance(1, P.MODE_LTS, graph=False)
        torch.cuda.synchronize()
        _ = (ref.U * 2).sum().item()          # unrelated eager work between replays
        assert torch.equal(sim.current(), ref.current()), k
    assert sim.coarse_step == 3


def test_small_mesh_four_coarse_steps():
    om = oracle_mesh("small")
    gm = P.build_mesh(mesh_spec("small"))
    U0 = wave_plane(om.anchors, om.levels, om.L, (1, 1, 0))
    want = so.run(om, U0, 4, "lts", sigma=0.1).reshape(2, om.n_oct, 125)
    got = _run_gpu(gm, U0, 4, P.MODE_LTS)
    assert rel_err(got, want) < TOL


def test_uniform_mesh_lts_equals_gts_bitwise():
    a, l = ot.uniform_leaves(2, 3)
    gm = P.build_mesh(leaves=np.concatenate([a, l[:, None]], 1), L=3)
    om = ot.mesh_from_leaves(a, l, 3)
    U0 = wave_plane(om.anchors, om.levels, om.L, (1, 2, 0))
    x = _run_gpu(gm, U0, 2, P.MODE_LTS)
    y = _run_gpu(gm, U0, 2, P.MODE_GTS)
    assert np.array_equal(x, y)
    want = so.run(om, U0, 2, "lts", sigma=0.1).reshape(2, om.n_oct, 125)
    assert rel_err(x, want) < TOL


def test_ssprk3(c1):
    om, gm, U0 = c1
    want = so.run(om, U0, 1, "lts", sigma=0.1, tableau="ssprk3").reshape(2, om.n_oct, 125)
    got = _run_gpu(gm, U0, 1, P.MODE_LTS, tableau="ssprk3")
    assert rel_err(got, want) < TOL


@pytest.fixture(scope="module")
def maxwell_small():
    om = oracle_mesh("small")
    gm = P.build_mesh(mesh_spec("small"))
    cfg = config("small")
    U0 = maxwell_gaussian(om.anchors, om.levels, om.L, cfg["pulses"], sigma=0.1)
    return om, gm, U0


@pytest.mark.parametrize("mode", ["lts", "gts"])
def test_maxwell_tiles(maxwell_small, mode):
    """Maxwell on side-1 and side-2 tiles against the oracle; the two tile sides
    agree bitwise (FP64); a mesh with streamed side-4 blocks is refused (the
    small mesh has none: its tile side 4 is side-1 and side-2 tiles)."""
    om, gm, U0 = maxwell_small
    md = P.MODE_LTS if mode == "lts" else P.MODE_GTS
    want = so.run(om, U0, 1, mode, equation="maxwell", sigma=0.1).reshape(6, om.n_oct, 125)
    got = _run_gpu(gm, U0, 1, md, eq="maxwell", tile=1)
    assert rel_err(got, want) < TOL
    got2 = _run_gpu(gm, U0, 1, md, eq="maxwell", tile=2)
    assert np.array_equal(got2, got)
    assert 4 not in set(gm.blocks()[:, 1].tolist())
    assert np.array_equal(_run_gpu(gm, U0, 1, md, eq="maxwell", tile=4), got)
    g4 = P.build_mesh(mesh_spec("wave_c1"))
    assert 4 in set(g4.blocks()[:, 1].tolist())
    lv = g4.leaves()
    U4 = maxwell_gaussian(lv[:, :3], lv[:, 3], g4.info()["L"], config("wave_c1")["pulses"], sigma=0.1)
    with pytest.raises(P.LTSError):
        _run_gpu(g4, U4, 1, md, eq="maxwell", tile=4)


def _field_errors(got, want, om):
    """Per field: volume-weighted l2 and max error, relative to the field's max."""
    w = (2.0 ** (om.L - om.levels)) ** 3
    out = []
    for f in range(want.shape[0]):
        e = got[f] - want[f]
        scale = np.abs(want[f]).max()
        l2 = np.sqrt((w * (e ** 2).sum(1)).sum() / (125 * w.sum()))
        out.append((l2 / scale, np.abs(e).max() / scale))
    return out


def test_maxwell_fp32_rhs_error_stated(maxwell_small):
    """Maxwell with FP32 stencils (FP64 state, RK and time interpolation) vs the
    FP64 oracle, one coarse step: error stated per field."""
    om, gm, U0 = maxwell_small
    want = so.run(om, U0, 1, "lts", equation="maxwell", sigma=0.1).reshape(6, om.n_oct, 125)
    got = _run_gpu(gm, U0, 1, P.MODE_LTS, eq="maxwell", prec=P.FP32_RHS, tile=1)
    for f, (l2, linf) in enumerate(_field_errors(got, want, om)):
        print(f"maxwell fp32-rhs field {'EB'[f // 3]}{'xyz'[f % 3]}: rel l2 {l2:.3e}  rel max {linf:.3e}")
        assert linf < 1e-4


def test_fp32_rhs_error_stated(c1, c1_oracle):
    """C3: the C1 mesh and data to T with FP32 stencils and FP64 state, RK and
    time interpolation, against the FP64 oracle at T; per field l2 and max error
    relative to the field's scale.  The bound follows from the stencil's
    cancellation error, about eps32 |u| / h^2 relative per RHS evaluation
    (6e-5 at h = 2^-5), not growing over the 8 coarse steps."""
    om, gm, U0 = c1
    want = c1_oracle["lts"]
    for tile in (2, 4):
        got = _run_gpu(gm, U0, N_C1, P.MODE_LTS, prec=P.FP32_RHS, tile=tile)
        for f, (l2, linf) in enumerate(_field_errors(got, want, om)):
            print(f"C3 fp32-rhs tile {tile} field {'uv'[f]} at T: rel l2 {l2:.3e}  rel max {linf:.3e}")
            assert linf < 2e-4


def test_graph_recaptured_after_table_and_shape_changes(c1):
    """A captured coarse step bakes in device table addresses and the launch
    shape: rebuilding the tile tables (set_tile away and back) or changing the
    launch shape between replays must not replay a stale graph."""
    om, gm, U0 = c1
    gm.set_tile(2)
    sim = P.Sim(gm, "wave", P.FP64, "rk4", ko_sigma=0.1, device=DEV)
    sim.set_state(U0)
    sim.advance(1, P.MODE_LTS, graph=True)
    gm.set_tile(1)
    gm.set_tile(2)
    sim.advance(1, P.MODE_LTS, graph=True)
    old = P.get_launch()
    try:
        P.set_launch(512, 1024)
        sim.advance(1, P.MODE_LTS, graph=True)
    finally:
        P.set_launch(*old)
    want = _run_gpu(gm, U0, 3, P.MODE_LTS, graph=False)
    assert np.array_equal(sim.current().cpu().numpy(), want)


def test_finiteness_flag_reports_nan(c1):
    """A NaN forced into the initial state from the host: lts_advance with the
    finiteness check returns LTS_ENONFINITE; clean data passes the check."""
    om, gm, U0 = c1
    sim = P.Sim(gm, "wave", P.FP64, "rk4", ko_sigma=0.1, device=DEV)
    sim.set_state(U0)
    sim.advance(1, P.MODE_LTS, check_finite=True)
    bad = np.array(U0, copy=True).reshape(2, om.n_oct, 125)
    bad[0, 17, 62] = np.nan
    sim.set_state(bad)
    with pytest.raises(P.LTSError) as e:
        sim.advance(1, P.MODE_LTS, check_finite=True)
    assert e.value.status == 5


@pytest.mark.parametrize("mode", [P.MODE_LTS, P.MODE_GTS])
def test_checkpoint_resume_bitwise(c1, tmp_path, mode):
    """Checkpoint after 2 coarse steps, save and load it (npz, no pickling),
    resume in a new sim for 2 more: bitwise the uninterrupted 4-step run."""
    om, gm, U0 = c1
    ref = P.Sim(gm, "wave", P.FP64, "rk4", ko_sigma=0.1, device=DEV)
    ref.set_state(U0)
    ref.advance(2, mode)
    ck = ref.checkpoint()
    path = str(tmp_path / "ck.npz")
    P.Sim.save_checkpoint(ck, path)
    ref.advance(2, mode)
    a = ref.current().cpu().numpy()
    sim = P.Sim(gm, "wave", P.FP64, "rk4", ko_sigma=0.1, device=DEV)
    sim.restore(P.Sim.load_checkpoint(path))
    assert sim.coarse_step == 2
    sim.advance(2, mode)
    assert sim.coarse_step == 4
    assert np.array_equal(sim.current().cpu().numpy(), a)


@pytest.mark.parametrize("name,mode,eq", [("wave_c1", P.MODE_LTS, "wave"), ("wave_c1", P.MODE_GTS, "wave"),
                                          ("wave7_small", P.MODE_LTS, "wave"), ("wave7_small", P.MODE_GTS, "maxwell")])
def test_poison_race_check(name, mode, eq):
    """Race check: with every stage's K entries of its active octants set to NaN
    before the stage, two coarse steps report no non-finite update and give
    bitwise the state of the plain run, so no stage reads a K it has not yet
    written (fused tiles; Maxwell on 7-node octants takes the phase kernels).
    In GTS on the fused tiles the unstored last K stays NaN: the poison covered
    every octant and nothing read it."""
    gm = P.build_mesh(mesh_spec(name))
    info = gm.info()
    lv = gm.leaves()
    n = info["nodes"]
    F = 2 if eq == "wave" else 6
    U0 = consistent_random_dg(lv[:, :3], lv[:, 3], info["L"], F, seed=3, nodes=n)
    outs = []
    for poison in (False, True):
        s = P.Sim(gm, eq, P.FP64, "rk4", ko_sigma=0.1, device=DEV)
        s.set_state(U0)
        s.advance(2, mode, graph=True, check_finite=True, poison=poison)
        outs.append((s.current(), s.K.clone()))
    assert torch.equal(outs[0][0], outs[1][0])
    if mode == P.MODE_GTS and eq == "wave":
        assert torch.isnan(outs[1][1][3]).all() and not torch.isnan(outs[1][1][:3]).any()
