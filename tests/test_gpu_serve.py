"""GPU tests of the serving loop and the autotuner: every request served in the
wave/Maxwell mix, under a memory budget that forces queueing, ends in bitwise
the state it reaches alone; tuned launch shapes do not change results."""
import pytest
import torch

import paper_2011_10570_amd as P
from paper_2011_10570_amd import serve, tune
from workloads import config, mesh_spec

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _requests():
    small = mesh_spec("small")
    c1 = mesh_spec("wave_c1")
    probs = config("batch")["problems"]
    rows = [("wave", small, [18, 12, 9], 2), ("maxwell", small, [20, 10, 12], 1),
            ("wave", c1, [36, 25, 17], 1), ("maxwell", c1, [30, 20, 40], 1),
            ("wave", probs[28]["mesh"], probs[28]["mesh"]["criteria"][0]["center"], 1),
            ("maxwell", probs[24]["mesh"], probs[24]["mesh"]["criteria"][0]["center"], 1),
            ("wave", probs[6]["mesh"], probs[6]["mesh"]["criteria"][0]["center"], 1)]
    return [serve.Request(i, eq, spec, c, n) for i, (eq, spec, c, n) in enumerate(rows)]


def _alone(req):
    m = P.Mesh(req.mesh_spec)
    m.set_tile(2 if req.equation == "wave" else 1)
    s = P.Sim(m, req.equation, P.FP64, "rk4", ko_sigma=0.1, device=DEV)
    s.set_state(serve.initial_state(m, req.equation, req.centre, req.sigma, DEV))
    s.advance(req.n_coarse, P.MODE_LTS)
    return s.current()


def test_served_equals_alone():
    reqs = _requests()
    # a budget of twice the largest footprint: most requests wait for others to leave
    fps = []
    for r in reqs:
        m = P.Mesh(r.mesh_spec)
        fps.append(serve.footprint_bytes(m.info(), r.equation, P.FP64))
    srv = serve.Server(2 * max(fps), keep_state=True, tick_rounds=3, device=DEV)
    stats = srv.run(reqs)
    srv.close()
    print("[serve]", stats, flush=True)
    assert stats["requests"] == len(reqs)
    assert stats["peak_resident_bytes"] <= stats["budget_bytes"]
    assert stats["p50_time_to_t_s"] <= stats["p99_time_to_t_s"]
    assert all(r.finished >= r.admitted >= r.arrival for r in reqs)
    # some request had to wait for an earlier one to leave
    assert max(r.admitted for r in reqs) >= min(r.finished for r in reqs)
    for r in reqs:
        assert torch.equal(r.state, _alone(r)), r.rid


def test_served_with_arrivals():
    """Staggered arrivals (a few ms apart): the loop idles, admits and finishes."""
    reqs = _requests()[:4]
    for i, r in enumerate(reqs):
        r.arrival = 0.003 * i
    srv = serve.Server(8 << 30, keep_state=True, device=DEV)
    stats = srv.run(reqs)
    srv.close()
    assert stats["requests"] == 4 and stats["wave"] == 2 and stats["maxwell"] == 2
    for r in reqs:
        assert torch.equal(r.state, _alone(r)), r.rid


def test_serve_refuses_oversize_and_cancels():
    """A request larger than the whole budget is refused with a status (the rest
    is served); a cancelled request leaves (before admission, or at its next
    coarse-step boundary) and the others still end bitwise as alone."""
    reqs = _requests()[:4]
    fps = [serve.footprint_bytes(P.Mesh(r.mesh_spec).info(), r.equation, P.FP64) for r in reqs]
    probs = config("batch")["problems"]
    big = serve.Request(10, "wave", probs[35]["mesh"], probs[35]["mesh"]["criteria"][0]["center"], 1)
    big_fp = serve.footprint_bytes(P.Mesh(big.mesh_spec).info(), "wave", P.FP64)
    budget = max(fps) * 2
    assert big_fp > budget
    early = serve.Request(11, "wave", mesh_spec("small"), [18, 12, 9], 1, cancel_after=0.0)
    late = serve.Request(12, "wave", mesh_spec("wave_c1"), [36, 25, 17], 3, cancel_after=0.002)
    srv = serve.Server(budget, keep_state=True, tick_rounds=1, device=DEV)
    stats = srv.run(reqs + [big, early, late])
    srv.close()
    print("[serve]", stats, flush=True)
    assert big.status == "rejected" and stats["rejected"] == 1
    assert early.status == "cancelled" and late.status == "cancelled"
    assert stats["done"] == len(reqs) and stats["peak_resident_bytes"] <= budget
    for r in reqs:
        assert r.status == "done"
        assert torch.equal(r.state, _alone(r)), r.rid


def test_autotuner_applies_fastest_and_keeps_results():
    from workloads import wave_gaussian_torch
    m = P.Mesh(mesh_spec("wave_c1"))
    U0 = wave_gaussian_torch(m.leaves(), m.info()["L"], [[36, 25, 17]], device=DEV)
    old = P.get_launch()
    try:
        res = tune.tune(m, U0, tiles=(1, 2, 4), threads=(256, 512), max_workgroups=(512, 4096),
                        stream_threads=(256, 512), reps=1, device=DEV, use_cache=False)
        assert len(res["table"]) == 2 + 4 + 8   # side 1 always runs 256 threads
        best = res["best"]
        assert res["ms"] == min(ms for _, ms in res["table"])
        assert m.info()["tile"] == best[0] and P.get_launch() == (best[1], best[2], best[3])
        res2 = tune.tune(m, U0, device=DEV)          # cached: applies without timing
        assert res2["table"] is None or res2["best"] is not None
    finally:
        P.set_launch(*old)
        tune.clear_cache()


def test_batch_throughput_runs():
    probs = config("batch")["problems"][:6]
    r = serve.batch_throughput(probs, 1, device=DEV)
    assert r["problems"] == 6 and r["node_updates"] > 0 and r["node_updates_per_s"] > 0
