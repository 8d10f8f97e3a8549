"""CPU tests of bench.py's contract: one GPU only, the roofline's algorithmic
byte count (224 B per FP64 LTS node-update, counted per fused stage) and the
reader of the committed counter summary."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("tile", [1, 2, 4])
def test_stage_accounting_is_224_bytes_per_node_update(tile):
    import paper_2011_10570_amd as P
    from workloads import mesh_spec
    gm = P.build_mesh(mesh_spec("small"))
    gm.set_tile(tile)
    info = gm.info()
    acc = bench.stage_accounting(info, gm.tiles())
    assert acc["alg_bytes"] == 224 * info["node_updates_lts"]
    assert acc["stages"] == 4 * info["n_substeps"]
    # at least one tile launch per stage, at most 3 tile sides and 2 pre-passes
    assert acc["stages"] <= acc["launches"] <= 5 * acc["stages"]


def test_rk4_passes_total_14():
    assert sum(bench.passes_rk4(s) for s in range(4)) == 14


def test_stored_traffic_reader(tmp_path):
    good = tmp_path / "c.md"
    good.write_text(f"traffic_bytes_per_stage: 2.5e+09\nsources_sha256: {bench.source_digest()}\n")
    assert bench.stored_traffic(str(good)) == 2.5e9
    stale = tmp_path / "s.md"
    stale.write_text("traffic_bytes_per_stage: 2.5e+09\nsources_sha256: " + "0" * 64 + "\n")
    assert bench.stored_traffic(str(stale)) is None
    assert bench.stored_traffic(str(tmp_path / "missing.md")) is None


def test_committed_counter_summary_parses():
    txt = open(os.path.join(ROOT, "profiles", "fused_stage_wave_c2_counters.md")).read()
    assert "traffic_bytes_per_stage:" in txt and "sources_sha256:" in txt


def test_analytic_fields_match_oracle():
    """bench.py's torch evaluation of the Gaussian spherical wave (the accuracy
    numbers of every bench line) equals the oracle's closed form on every DG node,
    u and v, including the node at a pulse centre (the r -> 0 limits)."""
    import torch
    from oracle import analytic as an
    from oracle import octree as ot
    from workloads import centre_physical, mesh_spec, node_units, physical
    m = ot.build_mesh(ot.MeshSpec.from_dict(mesh_spec("small")))
    L = m.L
    pulses = [[16, 12, 20], [5, 30, 11]]
    leaves = np.concatenate([m.anchors, m.levels[:, None]], axis=1)
    X = physical(node_units(m.anchors, m.levels, L), L)
    c = np.stack([centre_physical(p, L) for p in pulses])
    r0 = np.sqrt(((X - c[0]) ** 2).sum(-1)).min()
    assert r0 == 0.0          # a node sits on the first centre
    for T in (0.0, 0.0625, 0.3):
        got = bench.analytic_fields(leaves, L, pulses, 0.1, T, "cpu").numpy()
        want = an.gaussian_periodic(X, c, T, 0.1).reshape(2, m.n_oct, 125)
        for f in range(2):
            assert np.abs(got[f] - want[f]).max() <= 1e-12 * np.abs(want[f]).max(), (T, f)
    e = bench.analytic_error(torch.as_tensor(want), leaves, L, pulses, 0.1, 0.3)
    assert e["l2_u"] < 1e-13 * e["l2_exact_u"] and e["l2_v"] < 1e-13 * e["l2_exact_v"]


def test_analytic_fields_nodes7_match_oracle():
    """The same on a 7-node mesh (wave7_small): every node of its 7^3 octants."""
    from oracle import analytic as an
    from oracle import octree as ot
    from workloads import centre_physical, mesh_spec, node_units, physical
    m = ot.build_mesh(ot.MeshSpec.from_dict(mesh_spec("wave7_small")))
    L = m.L
    pulses = [[55, 37, 26]]
    leaves = np.concatenate([m.anchors, m.levels[:, None]], axis=1)
    X = physical(node_units(m.anchors, m.levels, L, nodes=7), L, nodes=7)
    c = np.stack([centre_physical(p, L, nodes=7) for p in pulses])
    for T in (0.0, 0.05):
        got = bench.analytic_fields(leaves, L, pulses, 0.1, T, "cpu", nodes=7).numpy()
        want = an.gaussian_periodic(X, c, T, 0.1).reshape(2, m.n_oct, 343)
        for f in range(2):
            assert np.abs(got[f] - want[f]).max() <= 1e-12 * max(np.abs(want[f]).max(), 1e-300), (T, f)
