"""GPU parity of the 7^3-node path (the paper's octants, 2:1 balance; phase and
fused kernels templated on the node count) with the oracle, through the C ABI:
unzip at positioned LTS/GTS states, block RHS, zip, RK update, the fused stage
(side-1 tiles, ghost table of 13^3 points), whole runs with classic RK4 and
SSP-RK3, the graph-captured fused lts_advance against the eager phase calls
(bitwise), FP32 stencils, norms, checkpoint/restore, the refusals, and one
whole coarse step of the full-size wave7_c2 workload against the oracle's own
run of it (a stored fixture)."""
import numpy as np
import pytest
import torch

import paper_2011_10570_amd as P
from oracle import fd
from oracle import octree as ot
from oracle import solver as so
from workloads import config, mesh_spec, random_dg, wave_gaussian

from gpu_common import TOL, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NAME = "wave7_small"
N7 = 7


@pytest.fixture(scope="module")
def mesh7():
    om = ot.build_mesh(ot.MeshSpec.from_dict(mesh_spec(NAME)))
    gm = P.build_mesh(mesh_spec(NAME))
    assert gm.info()["nodes"] == 7 and om.nodes == 7
    return om, gm


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _positioned(om, nfields, mode, n, j, seed, tableau="rk4"):
    st = so.State(om, nfields, tableau, mode)
    nsub = ot.substeps(om)
    for _ in range(n):
        for jj in range(nsub):
            st.close_records(st.open_records(jj))
    for jj in range(j):
        st.close_records(st.open_records(jj))
    act = st.open_records(j)
    st.U[:] = random_dg(st.U.shape, seed)
    st.K[:] = random_dg(st.K.shape, seed + 1, 0.5)
    return st, act


CASES = [("lts", 0, 0), ("lts", 0, 1), ("lts", 1, 2), ("lts", 1, 3), ("gts", 1, 2)]


@pytest.mark.parametrize("mode,n,j", CASES)
@pytest.mark.parametrize("stage", [0, 1, 2, 3])
def test_unzip7(mesh7, mode, n, j, stage):
    om, gm = mesh7
    print(f"[unzip7] {mode} n={n} j={j} s={stage}", flush=True)
    st, act = _positioned(om, 2, mode, n, j, seed=10 * n + j + stage)
    S = 6 * om.blocks[act, 1] + 7
    out = torch.full((2, int((S ** 3).sum())), np.nan, dtype=torch.float64, device=DEV)
    md = P.MODE_GTS if mode == "gts" else P.MODE_LTS
    P.unzip(gm, _dev(st.U), _dev(st.K), stage, j, md, n, None, out)
    want = np.concatenate([st.unzip(int(b), stage).reshape(2, -1) for b in act], axis=1)
    assert rel_err(out.cpu().numpy(), want) < TOL


@pytest.mark.parametrize("eq,prec", [("wave", P.FP64), ("maxwell", P.FP64), ("wave", P.FP32_RHS)])
def test_rhs7(mesh7, eq, prec):
    om, gm = mesh7
    F = 2 if eq == "wave" else 6
    ids = np.arange(len(om.blocks))
    S = 6 * om.blocks[ids, 1] + 7
    G = 6 * om.blocks[ids, 1] + 1
    pad = random_dg((F, int((S ** 3).sum())), 5)
    kdt = torch.float32 if prec == P.FP32_RHS else torch.float64
    out = torch.zeros((F, int((G ** 3).sum())), dtype=kdt, device=DEV)
    P.rhs(gm, P.EQ_WAVE if eq == "wave" else P.EQ_MAXWELL, 0.1, _dev(pad), prec, ids, out)
    rfun = fd.rhs_wave if eq == "wave" else fd.rhs_maxwell
    po, want = 0, []
    for b, s in zip(ids, S):
        h = ot.h_level(int(om.blocks[b, 2]), N7)
        want.append(rfun(pad[:, po:po + s ** 3].reshape(F, s, s, s), h, 0.1).reshape(F, -1))
        po += s ** 3
    tol = 2e-5 if prec == P.FP32_RHS else TOL
    assert rel_err(out.double().cpu().numpy(), np.concatenate(want, axis=1)) < tol


def test_zip7(mesh7):
    om, gm = mesh7
    ids = np.arange(0, len(om.blocks), 2)
    G = 6 * om.blocks[ids, 1] + 1
    kb = random_dg((2, int((G ** 3).sum())), 8)
    N = om.n_oct
    out = torch.full((2, N, 343), 7.0, dtype=torch.float64, device=DEV)
    P.zip(gm, 2, P.FP64, _dev(kb), ids, out)
    st, _ = _positioned(om, 2, "lts", 0, 0, seed=1)
    want = np.full((2, N, 7, 7, 7), 7.0)
    go = 0
    for b, g in zip(ids, G):
        st.zip_into(int(b), kb[:, go:go + g ** 3].reshape(2, g, g, g), want)
        go += g ** 3
    assert np.array_equal(out.cpu().numpy(), want.reshape(2, N, 343))


@pytest.mark.parametrize("mode,n,j", [("lts", 0, 0), ("lts", 1, 3), ("gts", 0, 2)])
def test_rk_update7(mesh7, mode, n, j):
    om, gm = mesh7
    st, act = _positioned(om, 2, mode, n, j, seed=21, tableau="ssprk3")
    U, K = _dev(st.U), _dev(st.K)
    md = P.MODE_GTS if mode == "gts" else P.MODE_LTS
    P.rk_stage(gm, U, K, list(st.b), j, md, n, None, None, tableau=P.SSPRK3)
    st.rk_update(act)
    assert rel_err(U.cpu().numpy().reshape(2, 2, -1), st.U.reshape(2, 2, -1)) < TOL


@pytest.mark.parametrize("mode,n,j", [("lts", 0, 0), ("lts", 0, 1), ("lts", 1, 2), ("lts", 1, 3), ("gts", 1, 1)])
@pytest.mark.parametrize("stage", [0, 1, 2, 3])
def test_fused_stage7(mesh7, mode, n, j, stage):
    """One fused launch (ghost pre-pass + side-1 tiles) == oracle unzip + rhs +
    zip (+ the RK update at the last stage)."""
    om, gm = mesh7
    assert gm.info()["tile"] == 1
    print(f"[fused7] {mode} n={n} j={j} s={stage}", flush=True)
    st, act = _positioned(om, 2, mode, n, j, seed=100 + 10 * j + stage)
    U, K = _dev(st.U), _dev(st.K)
    k_in = K.clone()
    md = P.MODE_GTS if mode == "gts" else P.MODE_LTS
    P.fused_stage(gm, U, K, P.EQ_WAVE, 0.1, stage, j, md, n)
    st.stage(act, stage, fd.rhs_wave, 0.1)
    if stage == 3:
        st.rk_update(act)
    if mode == "gts" and stage == 3:
        assert torch.equal(K.reshape(4, -1)[stage], k_in.reshape(4, -1)[stage])
    else:
        assert rel_err(K.cpu().numpy().reshape(4, 2, -1)[stage], st.K[stage].reshape(2, -1)) < TOL
    assert rel_err(U.cpu().numpy().reshape(2, 2, -1).transpose(1, 0, 2),
                   st.U.reshape(2, 2, -1).transpose(1, 0, 2)) < TOL


@pytest.mark.parametrize("threads,cap", [(256, 16), (512, 65536)])
def test_fused_walk7(mesh7, threads, cap):
    """Workgroups walking many tiles (small grid cap) equal one workgroup per
    tile, bitwise, for the 7-node tiles."""
    om, gm = mesh7
    old = P.get_launch()
    try:
        outs = []
        for shape in ((512, 65536, 512), (threads, cap, 512)):
            P.set_launch(*shape)
            st, act = _positioned(om, 2, "lts", 1, 0, seed=5)
            U, K = _dev(st.U), _dev(st.K)
            for stage in range(4):
                P.fused_stage(gm, U, K, P.EQ_WAVE, 0.1, stage, 0, P.MODE_LTS, 1)
            outs.append((U, K))
        assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    finally:
        P.set_launch(*old)


@pytest.fixture(scope="module")
def initial7(mesh7):
    om, _ = mesh7
    cfg = config(NAME)
    return wave_gaussian(om.anchors, om.levels, om.L, cfg["pulses"], sigma=cfg["sigma"], nodes=N7)


@pytest.mark.parametrize("mode,tableau", [("lts", "ssprk3"), ("gts", "ssprk3"), ("lts", "rk4")])
def test_run_matches_oracle7(mesh7, initial7, mode, tableau):
    """Two coarse steps (levels 2-4: 4 substeps each) of the configuration, graph-
    captured lts_advance (fused side-1 tiles) against the oracle; the eager phase
    calls give the same state bitwise (same values, same operation order)."""
    om, gm = mesh7
    cfg = config(NAME)
    n = cfg["n_coarse"]
    print(f"[run7] {mode} {tableau} oracle...", flush=True)
    want = so.run(om, initial7, n, mode, sigma=cfg["ko_sigma"], tableau=tableau).reshape(2, om.n_oct, -1)
    md = P.MODE_GTS if mode == "gts" else P.MODE_LTS
    s = P.Sim(gm, "wave", P.FP64, tableau, ko_sigma=cfg["ko_sigma"], device=DEV)
    s.set_state(initial7)
    s.advance(n, md, graph=True, check_finite=True)
    got = s.current()
    assert s.coarse_step == n
    assert rel_err(got.cpu().numpy(), want) < TOL
    e = P.Sim(gm, "wave", P.FP64, tableau, ko_sigma=cfg["ko_sigma"], device=DEV)
    e.set_state(initial7)
    e.advance_unfused(n, md)
    assert torch.equal(e.current(), got)


def test_fp32_rhs_run7(mesh7, initial7):
    """FP32 stencils (FP64 state, RK and time interpolation) stay within FP32
    rounding of the FP64 run."""
    _, gm = mesh7
    outs = {}
    for prec in (P.FP64, P.FP32_RHS):
        s = P.Sim(gm, "wave", prec, "ssprk3", ko_sigma=0.1, device=DEV)
        s.set_state(initial7)
        s.advance(2, P.MODE_LTS)
        outs[prec] = s.current().cpu().numpy()
    assert rel_err(outs[P.FP32_RHS], outs[P.FP64]) < 1e-4


def test_checkpoint_restore7(mesh7, initial7):
    _, gm = mesh7
    a = P.Sim(gm, "wave", P.FP64, "ssprk3", device=DEV)
    a.set_state(initial7)
    a.advance(1, P.MODE_LTS)
    ck = a.checkpoint()
    a.advance(1, P.MODE_LTS)
    b = P.Sim(gm, "wave", P.FP64, "ssprk3", device=DEV)
    b.restore(ck)
    b.advance(1, P.MODE_LTS)
    assert torch.equal(a.current(), b.current())


def test_norms7(mesh7):
    om, gm = mesh7
    a = random_dg((2, om.n_oct, 343), 3)
    b = random_dg((2, om.n_oct, 343), 4)
    r = P.norms(gm, _dev(a), _dev(b), 2)
    w = (2.0 ** (om.L - om.levels)) ** 3
    for f in range(2):
        e = a[f] - b[f]
        l2 = np.sqrt((w * (e ** 2).sum(1)).sum() / (343 * w.sum()))
        assert abs(r["l2"][f] - l2) < 1e-12 * l2
        assert r["linf"][f] == np.abs(e).max()


def test_refusals7(mesh7):
    """The fused stage for Maxwell or on side-2 tiles, batches, the non-linear
    wave and remeshing refuse 7-node meshes with LTS_EUNSUPPORTED."""
    om, gm = mesh7
    U = torch.zeros((2, 2, om.n_oct, 343), dtype=torch.float64, device=DEV)
    K = torch.zeros((4, 2, om.n_oct, 343), dtype=torch.float64, device=DEV)
    Um = torch.zeros((2, 6, om.n_oct, 343), dtype=torch.float64, device=DEV)
    Km = torch.zeros((4, 6, om.n_oct, 343), dtype=torch.float64, device=DEV)
    with pytest.raises(P.LTSError) as e:
        P.fused_stage(gm, Um, Km, P.EQ_MAXWELL, 0.1, 0, 0, P.MODE_LTS, 0)
    assert e.value.status == P._L.EUNSUPPORTED
    gm.set_tile(2)
    try:
        with pytest.raises(P.LTSError) as e:
            P.fused_stage(gm, U, K, P.EQ_WAVE, 0.1, 0, 0, P.MODE_LTS, 0)
        assert e.value.status == P._L.EUNSUPPORTED
    finally:
        gm.set_tile(1)
    s = P.Sim(gm, "wave", P.FP64, "rk4", device=DEV)
    s.set_state(np.zeros((2, om.n_oct, 343)))
    b = P.Batch("wave", P.FP64, "rk4", P.MODE_LTS, capacity=2)
    with pytest.raises(P.LTSError) as e:
        b.attach(s, 1)
    assert e.value.status == P._L.EUNSUPPORTED
    with pytest.raises(P.LTSError) as e:
        P.Sim(gm, "nlwave", P.FP64, "rk4", device=DEV)
    assert e.value.status == P._L.EUNSUPPORTED
    with pytest.raises(P.LTSError) as e:
        P.remesh_indicators(gm, s.current())
    assert e.value.status == P._L.EUNSUPPORTED


def test_wave7_c2_lts_coarse_step_vs_oracle():
    """One whole graph-captured LTS coarse step of the 7^3-node benchmark workload
    (wave7_c2: 75,230 octants, levels 3-8, SSP-RK3, the launch bench.py times)
    against the oracle's full run of it (tests/golden/wave7_c2_lts_step.txt,
    written by make_c2_lts_step.py from oracle/ only): element by element at 4096
    seeded nodes, and the whole state's per-field maximum and sum of squares."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "wave7_c2_lts_step.txt")
    stats, rows = {}, []
    for line in open(path):
        if line.startswith("#"):
            continue
        p = line.split()
        if p[0] in ("max_abs", "sum_sq"):
            stats[(p[0], int(p[1]))] = float(p[2])
        else:
            rows.append((int(p[0]), int(p[1]), float(p[2]), float(p[3])))
    rows = np.array(rows)
    assert len(rows) == 4096
    cfg = config("wave7_c2")
    gm = P.build_mesh(mesh_spec("wave7_c2"))
    lv = gm.leaves()
    U0 = wave_gaussian(lv[:, :3], lv[:, 3], gm.info()["L"], cfg["pulses"], sigma=cfg["sigma"], nodes=N7)
    print("[n7] one LTS coarse step of wave7_c2 vs the oracle's full run", flush=True)
    sim = P.Sim(gm, "wave", P.FP64, cfg["tableau"], ko_sigma=cfg["ko_sigma"], device=DEV)
    sim.set_state(U0)
    sim.advance(1, P.MODE_LTS, graph=True)
    out = sim.current().reshape(2, len(lv), N7 ** 3)
    o = torch.from_numpy(rows[:, 0].astype(np.int64)).to(DEV)
    n = torch.from_numpy(rows[:, 1].astype(np.int64)).to(DEV)
    for f in range(2):
        got = out[f][o, n].cpu().numpy()
        scale = stats[("max_abs", f)]
        assert np.abs(got - rows[:, 2 + f]).max() <= TOL * scale, f
        assert abs(out[f].abs().max().item() - scale) <= TOL * scale, f
        ss = (out[f] * out[f]).sum().item()
        assert abs(ss - stats[("sum_sq", f)]) <= 1e-11 * stats[("sum_sq", f)], f
