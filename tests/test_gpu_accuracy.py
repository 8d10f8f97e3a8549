"""The analogue of the paper's LTS/GTS accuracy experiment with increasing
spacetime resolution (Sec. 4.3, fig. accu_d8): the linear wave travelling along
x, third-order RK (SSP-RK3) on 7^3-node octants, adaptive meshes of levels
l..l+2 refined around a ball (most octants at the two coarser levels), every
level one finer at each resolution and the same final time.  Both LTS and GTS
converge at the scheme's third order against the analytic solution.  The error
is the time error of the coarsest octants, which LTS steps with a 2^(lmax-lmin)
= 4 times larger dt than GTS: the LTS error is up to 4^3 = 64 times GTS's, and
the test bounds the ratio by 80."""
import json

import numpy as np
import pytest

import paper_2011_10570_amd as P
from oracle import analytic as an
from workloads import node_units, physical, wave_plane

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N7 = 7


def _spec(lmin, L, r=0.3):
    """7-node mesh of levels lmin..L: a ball of radius r (physical) around the
    origin refined to L."""
    n_u = 6 * (1 << L)
    c = n_u // 2
    r2 = [-1] * L
    for lev in range(lmin, L):
        r2[lev] = int((r * n_u / 2) ** 2)
    return {"l_min": lmin, "l_max": L, "block_cap": 4, "nodes": 7,
            "criteria": [{"kind": "ball", "center": [c, c, c], "r2": r2}]}


def _error(gm, mode, n_coarse, tableau="ssprk3"):
    lv = gm.leaves()
    info = gm.info()
    L = info["L"]
    s = P.Sim(gm, "wave", P.FP64, tableau, ko_sigma=0.0, device=DEV)
    s.set_state(wave_plane(lv[:, :3], lv[:, 3], L, (1, 0, 0), nodes=N7))
    s.advance(n_coarse, mode)
    out = s.current().cpu().numpy().reshape(2, len(lv), N7, N7, N7)
    T = n_coarse * 0.25 * (2.0 ** (1 - info["lmin"]) / 6.0)
    X = physical(node_units(lv[:, :3], lv[:, 3], L, nodes=N7), L, nodes=N7)
    ex = an.plane_wave(X, (1, 0, 0), T)
    l2, linf = an.norms(out - ex, lv[:, 3], L)
    return float(l2[0]), float(linf[0]), T


def test_lts_gts_convergence_rk3():
    rows = []
    for lmin in (2, 3, 4):
        gm = P.build_mesh(_spec(lmin, lmin + 2))
        info = gm.info()
        assert (info["lmin"], info["lmax"]) == (lmin, lmin + 2)
        nco = 8 << (lmin - 2)          # the same T = 1/6 at every resolution
        el, eli, T = _error(gm, P.MODE_LTS, nco)
        eg, egi, _ = _error(gm, P.MODE_GTS, nco)
        rows.append({"levels": [lmin, lmin + 2], "octants": info["n_oct"], "T": T, "lts_l2": el, "gts_l2": eg,
                     "lts_linf": eli, "gts_linf": egi})
    print(json.dumps(rows), flush=True)
    for k in ("lts_l2", "gts_l2"):
        orders = [np.log2(a[k] / b[k]) for a, b in zip(rows, rows[1:])]
        assert orders[0] >= 2.4 and orders[-1] >= 2.7, (k, orders)   # pre-asymptotic, then third order
    for r in rows:
        assert r["lts_l2"] <= 80 * r["gts_l2"], r
