"""GPU tests of continuous batching (lts_batch_*): several meshes with different
level ranges advanced together give, for every sim, bitwise the state it reaches
alone; sims join and leave at round boundaries; misuse is rejected."""
import numpy as np
import pytest
import torch

import paper_2011_10570_amd as P
from oracle import solver as so
from workloads import config, mesh_spec, wave_gaussian, maxwell_gaussian

from gpu_common import TOL, oracle_mesh, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
# batch problems of 1.0k-2.6k leaves: level ranges 2-4 and 2-5
SMALL_PROBLEMS = (28, 24, 17, 6)


def _problem(i):
    p = config("batch")["problems"][i]
    return p["mesh"], p["mesh"]["criteria"][0]["center"]


def _state(gm, eq, centre):
    lv = gm.leaves()
    L = gm.info()["L"]
    if eq == "wave":
        return wave_gaussian(lv[:, :3], lv[:, 3], L, [centre], sigma=0.1)
    return maxwell_gaussian(lv[:, :3], lv[:, 3], L, [centre], sigma=0.1)


@pytest.fixture(scope="module")
def meshes():
    """(mesh, tile side, initial state) of the wave cases: the small and C1
    meshes and four batch problems, mixed tile sides."""
    out = []
    for name, tile in (("small", 2), ("wave_c1", 1)):
        gm = P.build_mesh(mesh_spec(name))
        cfg = config(name)
        centre = cfg["pulses"][0] if "pulses" in cfg else cfg["mesh"]["criteria"][0]["center"]
        out.append((gm, tile, _state(gm, "wave", centre)))
    for k, i in enumerate(SMALL_PROBLEMS):
        spec, centre = _problem(i)
        gm = P.build_mesh(spec)
        out.append((gm, 1 + (k % 2), _state(gm, "wave", centre)))
    return out


def _sim(gm, tile, U0, eq="wave", prec=P.FP64, tableau="rk4"):
    gm.set_tile(tile)
    s = P.Sim(gm, eq, prec, tableau, ko_sigma=0.1, device=DEV)
    s.set_state(U0)
    return s


def _alone(gm, tile, U0, n, mode, **kw):
    s = _sim(gm, tile, U0, **kw)
    s.advance(n, mode, graph=True)
    return s.current()


@pytest.mark.parametrize("mode,prec", [(P.MODE_LTS, P.FP64), (P.MODE_GTS, P.FP64), (P.MODE_LTS, P.FP32_RHS)])
def test_batch_equals_alone(meshes, mode, prec):
    print(f"[batch] equals-alone mode={mode} prec={prec}", flush=True)
    want = [_alone(gm, t, U0, 2, mode, prec=prec) for gm, t, U0 in meshes]
    sims = [_sim(gm, t, U0, prec=prec) for gm, t, U0 in meshes]
    P.batch_advance(sims, 2, mode)
    for s, w in zip(sims, want):
        assert s.coarse_step == 2
        assert torch.equal(s.current(), w)


@pytest.mark.parametrize("threads,cap", [(512, 16), (256, 16), (256, 4096), (512, 100000)])
def test_batch_walked_tiles(meshes, threads, cap):
    """A batch under another batch launch shape (a small grid cap: each workgroup
    walks many tiles and ghost entries; 256-thread workgroups) equals the
    default shape, bitwise; the one-mesh launch shape does not affect batches."""
    old, old_one = P.get_batch_launch(), P.get_launch()
    try:
        assert old == (512, 4096)
        sims = [_sim(gm, t, U0) for gm, t, U0 in meshes]
        P.batch_advance(sims, 1, P.MODE_LTS)
        want = [s.current() for s in sims]
        P.set_batch_launch(threads, cap)
        P.set_launch(256, 16, 256)
        sims = [_sim(gm, t, U0) for gm, t, U0 in meshes]
        P.batch_advance(sims, 1, P.MODE_LTS)
        for s, w in zip(sims, want):
            assert torch.equal(s.current(), w)
    finally:
        P.set_batch_launch(*old)
        P.set_launch(*old_one)


def test_tune_batch_bitwise(meshes):
    """The batch autotuner times every candidate, checks each gives bitwise the
    same states (it raises otherwise), applies the fastest, and caches it."""
    from paper_2011_10570_amd import tune
    old = P.get_batch_launch()
    tiles_before = [gm.info()["tile"] for gm, _, _ in meshes]
    try:
        ms = [gm for gm, _, _ in meshes[:4]]
        st = [U0 for _, _, U0 in meshes[:4]]
        tune.clear_cache()
        r = tune.tune_batch(ms, st, threads=(256, 512), max_workgroups=(512, 4096))
        # side 2: 2 thread counts x 2 grid caps; side 1 (always 256 threads): 2 caps
        assert len(r["table"]) == 2 * 2 + 2
        best = r["best"]
        assert P.get_batch_launch() == (best[1], best[2])
        assert all(m.info()["tile"] == best[0] for m in ms)
        r2 = tune.tune_batch(ms, st)
        assert r2["table"] is None and r2["best"] == best
    finally:
        tune.clear_cache()
        P.set_batch_launch(*old)
        for (gm, _, _), t in zip(meshes, tiles_before):
            gm.set_tile(t)


def test_batch_matches_oracle():
    """The small mesh advanced inside a batch against the oracle's LTS driver."""
    om = oracle_mesh("small")
    gm = P.build_mesh(mesh_spec("small"))
    cfg = config("small")
    centre = cfg["pulses"][0] if "pulses" in cfg else cfg["mesh"]["criteria"][0]["center"]
    U0 = wave_gaussian(om.anchors, om.levels, om.L, [centre], sigma=0.1)
    print("[oracle] small lts 2 coarse steps", flush=True)
    want = so.run(om, U0, 2, "lts", sigma=0.1).reshape(2, om.n_oct, 125)
    other = P.build_mesh(mesh_spec("wave_c1"))
    sims = [_sim(gm, 2, U0), _sim(other, 2, _state(other, "wave", centre))]
    P.batch_advance(sims, 2, P.MODE_LTS)
    assert rel_err(sims[0].current().cpu().numpy(), want) < TOL


def test_many_sims_one_mesh():
    """16 sims sharing one mesh, different data: the union is split across
    sims mid-range; each equals its own alone run."""
    gm = P.build_mesh(mesh_spec("small"))
    lv = gm.leaves()
    rng = np.random.default_rng(5)
    states = [wave_gaussian(lv[:, :3], lv[:, 3], gm.info()["L"], [list(rng.integers(0, 64, 3))], sigma=0.15)
              for _ in range(16)]
    want = [_alone(gm, 2, U0, 1, P.MODE_LTS) for U0 in states]
    sims = [_sim(gm, 2, U0) for U0 in states]
    P.batch_advance(sims, 1, P.MODE_LTS)
    for s, w in zip(sims, want):
        assert torch.equal(s.current(), w)


@pytest.mark.parametrize("graph", [True, False])
def test_join_and_leave(meshes, graph):
    """A joins at round 0, B at round 5 (inside A's second coarse step); A leaves
    at a coarse-step boundary and later joins again; every state equals the alone
    run of the same number of coarse steps (graph-captured rounds or not)."""
    (ga, ta, Ua), (gb, tb, Ub) = meshes[1], meshes[4]
    a = _sim(ga, ta, Ua)
    b = _sim(gb, tb, Ub)
    nsub_a = 1 << (ga.info()["lmax"] - ga.info()["lmin"])
    B = P.Batch("wave", P.FP64, "rk4", P.MODE_LTS, capacity=4)
    B.attach(a, 3)
    B.run(5, graph)
    B.attach(b, 2)
    assert B.info()["attached"] == 2
    B.run(2 * nsub_a - 5, graph)     # a is now at a coarse-step boundary (2 done)
    B.detach(a)
    assert a.coarse_step == 2 and a.rounds_left == 0
    assert torch.equal(a.current(), _alone(ga, ta, Ua, 2, P.MODE_LTS))
    B.attach(a, 1)                     # continues from coarse step 2
    done = B.drain(graph)
    assert set(map(id, done)) == {id(a), id(b)}
    assert B.info()["attached"] == 0
    assert a.coarse_step == 3 and b.coarse_step == 2
    assert torch.equal(a.current(), _alone(ga, ta, Ua, 3, P.MODE_LTS))
    assert torch.equal(b.current(), _alone(gb, tb, Ub, 2, P.MODE_LTS))
    # a batch-advanced sim continues with lts_advance from where it stopped
    a.advance(1, P.MODE_LTS)
    assert torch.equal(a.current(), _alone(ga, ta, Ua, 4, P.MODE_LTS))


@pytest.mark.parametrize("tile", [1, 2])
def test_batch_maxwell(tile):
    """Batched Maxwell (side-1 or side-2 tiles) equals the sims advanced alone
    on side-1 tiles, bitwise."""
    out = []
    for name in ("small", "wave_c1"):
        gm = P.build_mesh(mesh_spec(name))
        cfg = config(name)
        centre = cfg["pulses"][0] if "pulses" in cfg else cfg["mesh"]["criteria"][0]["center"]
        out.append((gm, _state(gm, "maxwell", centre)))
    want = [_alone(gm, 1, U0, 1, P.MODE_LTS, eq="maxwell") for gm, U0 in out]
    sims = [_sim(gm, tile, U0, eq="maxwell") for gm, U0 in out]
    P.batch_advance(sims, 1, P.MODE_LTS)
    for s, w in zip(sims, want):
        assert torch.equal(s.current(), w)


def test_batch_misuse(meshes):
    gm, t, U0 = meshes[0]
    B = P.Batch("wave", P.FP64, "rk4", P.MODE_LTS, capacity=1)
    mx = _sim(gm, 1, _state(gm, "maxwell", [32, 32, 32]), eq="maxwell")
    with pytest.raises(P.LTSError):
        B.attach(mx, 1)                 # another equation
    a = _sim(gm, t, U0)
    B.attach(a, 2)
    with pytest.raises(P.LTSError):
        B.attach(a, 1)                  # already attached
    c = _sim(meshes[1][0], meshes[1][1], meshes[1][2])
    with pytest.raises(P.LTSError):
        B.attach(c, 1)                  # full
    with pytest.raises(P.LTSError):
        a.advance(1, P.MODE_LTS)        # driven by the batch
    with pytest.raises(P.LTSError):
        gm.set_tile(3 - t)              # its tables are in use
    B.run(1)
    with pytest.raises(P.LTSError):
        B.detach(a)                     # inside a coarse step
    B.drain()
    assert a.coarse_step == 2
    gm.set_tile(3 - t)
    gm.set_tile(t)
    # streamed 4^3 blocks are not batched
    g4, t4, U4 = meshes[1]
    d = _sim(g4, 4, U4)
    with pytest.raises(P.LTSError):
        B.attach(d, 1)
    g4.set_tile(t4)
