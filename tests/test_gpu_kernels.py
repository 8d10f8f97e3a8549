"""GPU parity of the phase kernels (unzip, rhs, zip, rk_stage, fused stage) with the
oracle, called through the C ABI on seeded random states."""
import numpy as np
import pytest
import torch

import paper_2011_10570_amd as P
from oracle import fd
from oracle import octree as ot
from workloads import mesh_spec, random_dg

from gpu_common import TOL, oracle_mesh, positioned_state, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def meshes():
    out = {}
    for name in ("small", "wave_c1"):
        out[name] = (oracle_mesh(name), P.build_mesh(mesh_spec(name)))
    return out


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


CASES = [("wave_c1", "lts", 0, 0), ("wave_c1", "lts", 1, 1), ("wave_c1", "lts", 2, 2), ("wave_c1", "lts", 3, 3),
         ("wave_c1", "gts", 1, 2), ("small", "lts", 1, 1), ("small", "gts", 0, 0)]


@pytest.mark.parametrize("name,mode,n,j", CASES)
@pytest.mark.parametrize("stage", [0, 1, 2, 3])
def test_unzip(meshes, name, mode, n, j, stage):
    om, gm = meshes[name]
    print(f"[unzip] {name} {mode} n={n} j={j} s={stage}", flush=True)
    st, act = positioned_state(om, 2, mode, n, j, seed=10 * n + j)
    S = 4 * om.blocks[act, 1] + 7
    tot = int((S ** 3).sum())
    U, K = _dev(st.U), _dev(st.K)
    out = torch.full((2, tot), np.nan, dtype=torch.float64, device=DEV)
    md = P.MODE_GTS if mode == "gts" else P.MODE_LTS
    P.unzip(gm, U, K, stage, j, md, n, None, out)
    got = out.cpu().numpy()
    want = np.concatenate([st.unzip(int(b), stage).reshape(2, -1) for b in act], axis=1)
    assert rel_err(got, want) < TOL


def test_unzip_explicit_list_and_empty(meshes):
    om, gm = meshes["wave_c1"]
    st, act = positioned_state(om, 2, "lts", 0, 0, seed=3)
    ids = act[::-7][:5]
    S = 4 * om.blocks[ids, 1] + 7
    out = torch.zeros((2, int((S ** 3).sum())), dtype=torch.float64, device=DEV)
    P.unzip(gm, _dev(st.U), _dev(st.K), 2, 0, P.MODE_LTS, 0, ids, out)
    want = np.concatenate([st.unzip(int(b), 2).reshape(2, -1) for b in ids], axis=1)
    assert rel_err(out.cpu().numpy(), want) < TOL
    # empty list: no work, no error
    P.unzip(gm, _dev(st.U), _dev(st.K), 2, 0, P.MODE_LTS, 0, [], out)
    torch.cuda.synchronize()


@pytest.mark.parametrize("eq", ["wave", "maxwell"])
def test_rhs(meshes, eq):
    om, gm = meshes["wave_c1"]
    F = 2 if eq == "wave" else 6
    ids = np.arange(len(om.blocks))
    S = 4 * om.blocks[ids, 1] + 7
    G = 4 * om.blocks[ids, 1] + 1
    pad = random_dg((F, int((S ** 3).sum())), 5)
    out = torch.zeros((F, int((G ** 3).sum())), dtype=torch.float64, device=DEV)
    P.rhs(gm, P.EQ_WAVE if eq == "wave" else P.EQ_MAXWELL, 0.1, _dev(pad), P.FP64, ids, out)
    rfun = fd.rhs_wave if eq == "wave" else fd.rhs_maxwell
    po, want = 0, []
    for b, s in zip(ids, S):
        h = 2.0 ** (-int(om.blocks[b, 2]) - 1)
        want.append(rfun(pad[:, po:po + s ** 3].reshape(F, s, s, s), h, 0.1).reshape(F, -1))
        po += s ** 3
    assert rel_err(out.cpu().numpy(), np.concatenate(want, axis=1)) < TOL


def test_zip(meshes):
    om, gm = meshes["wave_c1"]
    ids = np.arange(0, len(om.blocks), 2)
    G = 4 * om.blocks[ids, 1] + 1
    kb = random_dg((2, int((G ** 3).sum())), 8)
    N = om.n_oct
    out = torch.full((2, N, 125), 7.0, dtype=torch.float64, device=DEV)
    P.zip(gm, 2, P.FP64, _dev(kb), ids, out)
    st, _ = positioned_state(om, 2, "lts", 0, 0, seed=1)
    want = np.full((2, N, 5, 5, 5), 7.0)
    go = 0
    for b, g in zip(ids, G):
        st.zip_into(int(b), kb[:, go:go + g ** 3].reshape(2, g, g, g), want)
        go += g ** 3
    assert np.array_equal(out.cpu().numpy(), want.reshape(2, N, 125))   # pure copies: bitwise


@pytest.mark.parametrize("mode,n,j", [("lts", 0, 0), ("lts", 1, 3), ("gts", 2, 1)])
def test_rk_update(meshes, mode, n, j):
    om, gm = meshes["wave_c1"]
    st, act = positioned_state(om, 2, mode, n, j, seed=21)
    U, K = _dev(st.U), _dev(st.K)
    md = P.MODE_GTS if mode == "gts" else P.MODE_LTS
    P.rk_stage(gm, U, K, [1 / 6, 1 / 3, 1 / 3, 1 / 6], j, md, n, None, None)
    st.rk_update(act)
    assert rel_err(U.cpu().numpy().reshape(2, 2, -1), st.U.reshape(2, 2, -1)) < TOL


@pytest.mark.parametrize("tile", [1, 2, 4])
@pytest.mark.parametrize("mode,n,j", [("lts", 0, 0), ("lts", 0, 1), ("lts", 1, 2), ("lts", 3, 3), ("gts", 1, 1)])
@pytest.mark.parametrize("stage", [0, 1, 3])
def test_fused_stage(meshes, tile, mode, n, j, stage):
    """One fused launch == oracle unzip + rhs + zip (+ RK update at the last stage)."""
    om, gm = meshes["wave_c1"]
    gm.set_tile(tile)
    print(f"[fused] tile={tile} {mode} n={n} j={j} s={stage}", flush=True)
    st, act = positioned_state(om, 2, mode, n, j, seed=100 + 10 * j + stage)
    U, K = _dev(st.U), _dev(st.K)
    k_in = K.clone()
    md = P.MODE_GTS if mode == "gts" else P.MODE_LTS
    P.fused_stage(gm, U, K, P.EQ_WAVE, 0.1, stage, j, md, n)
    st.stage(act, stage, fd.rhs_wave, 0.1)
    if stage == 3:
        st.rk_update(act)
    if mode == "gts" and stage == 3:
        # GTS does not store the last stage (no ghost relation reads it)
        assert torch.equal(K.reshape(4, -1)[stage], k_in.reshape(4, -1)[stage])
    else:
        assert rel_err(K.cpu().numpy().reshape(4, 2, -1)[stage], st.K[stage].reshape(2, -1)) < TOL
    assert rel_err(U.cpu().numpy().reshape(2, 2, -1).transpose(1, 0, 2), st.U.reshape(2, 2, -1).transpose(1, 0, 2)) < TOL
    gm.set_tile(2)


def test_norms_and_copy(meshes):
    om, gm = meshes["wave_c1"]
    a = random_dg((2, om.n_oct, 125), 3)
    b = random_dg((2, om.n_oct, 125), 4)
    r = P.norms(gm, _dev(a), _dev(b), 2)
    w = (2.0 ** (om.L - om.levels)) ** 3
    for f in range(2):
        e = a[f] - b[f]
        l2 = np.sqrt((w * (e ** 2).sum(1)).sum() / (125 * w.sum()))
        assert abs(r["l2"][f] - l2) < 1e-12 * l2
        assert r["linf"][f] == np.abs(e).max()
    assert r["nonfinite"] == 0
    a[1, 3, 7] = np.nan
    assert P.norms(gm, _dev(a), None, 2)["nonfinite"] == 1
    src = torch.arange(1 << 16, dtype=torch.float64, device=DEV)
    dst = torch.zeros_like(src)
    P.copy_probe(src, dst, src.numel() * 8)
    assert torch.equal(src, dst)
