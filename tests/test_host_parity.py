"""CPU tests of the library's host side: the shared library loads and exports every
function include/lts.h declares; the C++ mesh builder, unzip map, schedule and
coefficient tables are bit-exact with the oracle (no GPU needed)."""
import ctypes
import os
import re
from fractions import Fraction as Fr

import numpy as np
import pytest

import paper_2011_10570_amd as P
from paper_2011_10570_amd import _lib
from oracle import octree as ot
from oracle import rk
from workloads import config, mesh_spec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "lts.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lts_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 20
    L = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.PROTOTYPES), set(names) ^ set(_lib.PROTOTYPES)


def _oracle_mesh(name):
    return ot.build_mesh(ot.MeshSpec.from_dict(mesh_spec(name)))


@pytest.mark.parametrize("name", ["small", "wave_c1", "nl_small", "nl_c1", "wave7_small"])
def test_mesh_bit_exact(name):
    om = _oracle_mesh(name)
    gm = P.build_mesh(mesh_spec(name))
    lv = gm.leaves()
    assert np.array_equal(lv[:, :3], om.anchors) and np.array_equal(lv[:, 3], om.levels)
    assert np.array_equal(gm.blocks(), om.blocks)
    sched = gm.schedule()
    assert len(sched) == ot.substeps(om)
    for j, got in enumerate(sched):
        assert np.array_equal(got, ot.active_blocks(om, j))


def test_ghost_owner_fixture_library():
    """The library's unzip map gives the owners of tests/golden/ghost_owner.txt."""
    from test_oracle_mesh import map_row, owner_fixture_mesh, owner_fixture_rows
    a, l, L = owner_fixture_mesh()
    gm = P.build_mesh(leaves=np.concatenate([a, l[:, None]], axis=1), L=L)
    blocks = gm.blocks()
    S = 4 * blocks[:, 1] + 7
    off = np.concatenate([[0], np.cumsum(S ** 3)])
    mp = gm.unzip_map()
    for r in owner_fixture_rows():
        b, qx, qy, qz = r[:4]
        assert map_row(mp[off[b]:off[b + 1]], int(blocks[b, 1]), qx, qy, qz) == r[4:9], r


@pytest.mark.parametrize("name", ["small", "wave_c1", "nl_small", "nl_c1", "wave7_small"])
def test_unzip_map_bit_exact(name):
    om = _oracle_mesh(name)
    gm = P.build_mesh(mesh_spec(name))
    got = gm.unzip_map()
    want = np.concatenate([ot.unzip_map(om, b) for b in range(len(om.blocks))])
    assert got.shape == want.shape
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name", ["small", "nl_small", "wave7_small"])
def test_ghost_table_read_boxes(name):
    """The ghost table holds exactly the coarser sources of the oracle's unzip
    map, receiver level = source level + 1 (finest receivers first), and each
    entry's box is the tight bounding box of the half-node points read from it."""
    om = _oracle_mesh(name)
    gm = P.build_mesh(mesh_spec(name))
    want = np.concatenate([ot.unzip_map(om, b) for b in range(len(om.blocks))])
    co = want[want[:, 1] == ot.KIND_COARSE]
    g = gm.ghosts()
    assert len(g) > 0
    assert np.array_equal(np.sort(g[:, 0]), np.unique(co[:, 0]))
    assert np.array_equal(g[:, 1], om.levels[g[:, 0]] + 1)
    assert np.all(np.diff(g[:, 1]) <= 0)
    order = np.argsort(co[:, 0], kind="stable")
    co = co[order]
    starts = np.searchsorted(co[:, 0], g[:, 0])
    ends = np.searchsorted(co[:, 0], g[:, 0], side="right")
    for row, a, e in zip(g, starts, ends):
        pts = co[a:e, 2:5]
        assert np.array_equal(pts.min(0), row[[2, 4, 6]]), row
        assert np.array_equal(pts.max(0), row[[3, 5, 7]]), row


def test_mesh_info_matches_model():
    om = _oracle_mesh("wave_c1")
    info = P.build_mesh(mesh_spec("wave_c1")).info()
    sm = ot.speedup_model(om)
    assert info["node_updates_lts"] == sm["w_lts"] and info["node_updates_gts"] == sm["w_gts"]
    assert abs(info["s_est"] - sm["s_est"]) < 1e-12 * sm["s_est"]
    assert (info["lmin"], info["lmax"], info["n_oct"]) == (om.lmin, om.lmax, om.n_oct)


@pytest.mark.slow
@pytest.mark.parametrize("name", ["wave_c2", "wave7_c2"])
def test_c2_mesh_bit_exact(name):
    """The benchmark meshes (200k leaves of 5^3 nodes; 75k leaves of 7^3 nodes):
    leaves and blocks identical to the oracle's."""
    om = _oracle_mesh(name)
    gm = P.build_mesh(mesh_spec(name))
    lv = gm.leaves()
    assert np.array_equal(lv[:, :3], om.anchors) and np.array_equal(lv[:, 3], om.levels)
    assert np.array_equal(gm.blocks(), om.blocks)


def test_explicit_leaves_and_errors():
    om = _oracle_mesh("small")
    leaves = np.concatenate([om.anchors, om.levels[:, None]], axis=1)
    gm = P.build_mesh(leaves=leaves, L=om.L)
    assert np.array_equal(gm.blocks(), om.blocks)
    # a hole in the tiling is rejected with LTS_EINVAL
    with pytest.raises(P.LTSError) as e:
        P.build_mesh(leaves=leaves[1:], L=om.L)
    assert e.value.status == _lib.EINVAL
    bad = dict(mesh_spec("small"))
    bad["block_cap"] = 3
    with pytest.raises(P.LTSError):
        P.build_mesh(bad)


def test_unbalanced_leaves_get_balanced():
    """An explicit leaf list violating the ghost-reach balance is closed under it,
    exactly as the oracle does."""
    L = 4
    a, l = ot.uniform_leaves(2, L)
    # refine one level-2 leaf twice in its far corner
    keep = np.ones(len(l), bool); keep[5] = False
    ch = ot._children(a[5:6], 2, L)
    gch = ot._children(ch[7:8], 3, L)
    A = np.concatenate([a[keep], ch[:7], gch]); Lv = np.concatenate([l[keep], np.full(7, 3), np.full(8, 4)])
    om = ot.mesh_from_leaves(A, Lv, L)
    gm = P.build_mesh(leaves=np.concatenate([A, Lv[:, None]], 1), L=L)
    lv = gm.leaves()
    assert np.array_equal(lv[:, :3], om.anchors) and np.array_equal(lv[:, 3], om.levels)
    assert len(om.levels) > len(Lv)


@pytest.mark.parametrize("tab,code", [(rk.RK4, P.RK4), (rk.SSPRK3, P.SSPRK3)])
def test_coefficients_match_oracle_rationals(tab, code):
    c = P.coefficients(code)
    W = rk.weight_table(tab)
    for ci in range(4):
        for s in range(tab.p):
            for i in range(tab.p):
                assert c["w"][ci, s, i] == rk.to_float(W[ci][s][i])
    assert np.array_equal(c["b"], rk.b_f64(tab))
    assert np.array_equal(c["a"], rk.a_f64(tab))


def test_tiles_cover_blocks():
    gm = P.build_mesh(mesh_spec("wave_c1"))
    for t in (1, 2, 4):
        gm.set_tile(t)
        tiles = gm.tiles()
        blocks = gm.blocks()
        covered = np.zeros(gm.info()["n_oct"], int)
        for row in tiles:
            first, counts, lev, m, tt = row[:5]
            assert tt == min(m, t)
            for o in range(tt ** 3):
                covered[first + o] += 1
        assert (covered == 1).all()
        # finest level first within each tile side
        for tt in (1, 2, 4):
            assert (np.diff(tiles[tiles[:, 4] == tt][:, 2]) <= 0).all()
    assert (gm.tiles()[:, 4] == 4).sum() == (gm.blocks()[:, 1] == 4).sum() > 0
    with pytest.raises(P.LTSError):
        gm.set_tile(3)


def test_batch_arguments_checked_before_device_use():
    """lts_batch_create rejects bad arguments with LTS_EINVAL without a device."""
    L = _lib.lib()
    h = ctypes.c_void_p()
    for args in ((7, P.FP64, P.RK4, P.MODE_LTS, 4), (P.EQ_WAVE, 9, P.RK4, P.MODE_LTS, 4),
                 (P.EQ_WAVE, P.FP64, 9, P.MODE_LTS, 4), (P.EQ_WAVE, P.FP64, P.RK4, 5, 4),
                 (P.EQ_WAVE, P.FP64, P.RK4, P.MODE_LTS, 0), (P.EQ_WAVE, P.FP64, P.RK4, P.MODE_LTS, 257)):
        assert L.lts_batch_create(*args, ctypes.byref(h)) == _lib.EINVAL
        assert not h.value
    assert L.lts_batch_attach(None, None, 1) == _lib.EINVAL
    assert L.lts_batch_run(None, 1, 1, None) == _lib.EINVAL
    assert L.lts_sim_rounds_left(None) == 0
    L.lts_batch_destroy(None)


def test_launch_shape_defaults_and_validation():
    """lts_set_launch / lts_get_launch (host state only): the defaults, a round
    trip, and rejection of shapes the kernels are not built for."""
    old = P.get_launch()
    try:
        assert old == (512, 65536, 512)
        P.set_launch(256, 4096, 256)
        assert P.get_launch() == (256, 4096, 256)
        for bad in ((128, 4096, 512), (512, 4, 512), (512, 4096, 1024), (768, 4096, 512)):
            with pytest.raises(P.LTSError):
                P.set_launch(*bad)
            assert P.get_launch() == (256, 4096, 256)
    finally:
        P.set_launch(*old)
    assert P.get_launch() == old


def test_batch_launch_shape_defaults_and_validation():
    """lts_set_batch_launch / lts_get_batch_launch: the defaults, a round trip,
    independence from the one-mesh shape, and rejection of unsupported shapes."""
    old, old_one = P.get_batch_launch(), P.get_launch()
    try:
        assert old == (512, 4096)
        P.set_batch_launch(256, 1024)
        assert P.get_batch_launch() == (256, 1024) and P.get_launch() == old_one
        for bad in ((128, 1024), (384, 1024), (1024, 1024), (512, 4), (512, 0)):
            with pytest.raises(P.LTSError):
                P.set_batch_launch(*bad)
            assert P.get_batch_launch() == (256, 1024)
    finally:
        P.set_batch_launch(*old)
    assert P.get_batch_launch() == old


def test_arrays_beyond_32bit_offsets_rejected():
    """The kernels address field arrays with 32-bit element offsets: a simulation
    whose stage arrays (p x F x N x 125 elements) reach 2^31 is refused before any
    device work.  A uniform level-7 mesh (2,097,152 octants) fits the wave
    equation (4 x 2 fields) but not Maxwell (4 x 6 fields)."""
    a, l = ot.uniform_leaves(7, 7)
    gm = P.build_mesh(leaves=np.concatenate([a, l[:, None]], 1), L=7)
    n = gm.info()["n_oct"]
    assert n == 2 ** 21
    assert 4 * 2 * n * 125 < 2 ** 31 <= 4 * 6 * n * 125
    with pytest.raises(P.LTSError, match="32-bit"):
        P.Sim(gm, "maxwell", P.FP64, "rk4", device="cpu")


def test_footprint_counts_ghost_scratch():
    """The serving loop's admission footprint counts the mesh's region of the
    batch ghost-table scratch (F x 729 doubles per coarser ghost source)."""
    from paper_2011_10570_amd import serve
    m = P.Mesh(mesh_spec("wave_c1"))
    info = m.info()
    assert info["ghost_entries"] > 0
    base = info["n_oct"] * 125 * 2 * (16 + 4 * 8) + info["table_bytes"]
    assert serve.footprint_bytes(info, "wave", P.FP64) == base + info["ghost_entries"] * 2 * 729 * 8


def test_bounded_mesh_info():
    """A bounded mesh reports its boundary; an unknown boundary is refused."""
    assert P.build_mesh(mesh_spec("nl_small")).info()["boundary"] == P.BOUNDARY_OUTER
    assert P.build_mesh(mesh_spec("small")).info()["boundary"] == P.BOUNDARY_PERIODIC
    spec = P._L.MeshSpecC()
    spec.l_min, spec.l_max, spec.block_cap, spec.boundary = 2, 3, 4, 7
    h = ctypes.c_void_p()
    assert P.lib().lts_build_mesh(ctypes.byref(spec), ctypes.byref(h)) == _lib.EINVAL


def test_nodes7_mesh_info_and_refusals():
    """A 7-node mesh reports its nodes and the speedup model with 343 nodes per
    octant; the fused stage, batches and remeshing refuse it before device work;
    an unknown node count is refused."""
    om = _oracle_mesh("wave7_small")
    gm = P.build_mesh(mesh_spec("wave7_small"))
    info = gm.info()
    sm = ot.speedup_model(om)
    assert info["nodes"] == 7 and om.nodes == 7
    assert info["node_updates_lts"] == sm["w_lts"] and info["node_updates_gts"] == sm["w_gts"]
    ni = 6
    assert info["unzip_points"] == sum((ni * int(m) + 7) ** 3 for m in om.blocks[:, 1])
    assert P.build_mesh(mesh_spec("small")).info()["nodes"] == 5
    spec = dict(mesh_spec("small"))
    spec["nodes"] = 6
    with pytest.raises(P.LTSError):
        P.build_mesh(spec)


def test_tuner_candidates():
    """Side-1 tiles run 256-thread workgroups whatever the launch shape says, so
    the tuner times one thread count for them; side-4 candidates also vary the
    streaming kernel's threads."""
    from paper_2011_10570_amd import tune
    c = list(tune._candidates([1, 2, 4], [256, 512], [4096, 65536], [512, 256]))
    assert len([x for x in c if x[0] == 1]) == 2
    assert len([x for x in c if x[0] == 2]) == 4
    assert len([x for x in c if x[0] == 4]) == 8
    assert all(x[1] == 256 for x in c if x[0] == 1)
