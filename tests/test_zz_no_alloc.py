"""lts_fused_stage_noalloc (the entry point for callers that cannot allocate):
its output equals lts_fused_stage's, bitwise, on two calls in a row, the second
on a smaller mesh, through the C ABI."""
import numpy as np
import pytest
import torch

import paper_2011_10570_amd as P
from workloads import config, mesh_spec, random_dg

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _case(name, stage, j, mode, n, seed):
    gm = P.build_mesh(mesh_spec(name))
    N = gm.info()["n_oct"]
    U = torch.from_numpy(random_dg((2, 2, N, 125), seed)).to(DEV)
    K = torch.from_numpy(random_dg((4, 2, N, 125), seed + 1, 0.5)).to(DEV)
    ko = config(name)["ko_sigma"]
    U1, K1 = U.clone(), K.clone()
    print(f"[noalloc] {name} stage={stage} j={j} mode={mode} n={n}", flush=True)
    P.fused_stage(gm, U1, K1, P.EQ_WAVE, ko, stage, j, mode, n)          # uploads the tables too
    U2, K2 = U.clone(), K.clone()
    P.fused_stage_noalloc(gm, U2, K2, P.EQ_WAVE, ko, stage, j, mode, n)
    torch.cuda.synchronize()
    return (U1, K1), (U2, K2)


def test_noalloc_equals_fused_stage_two_calls_second_smaller():
    # first call: C1 mesh (596 octants), last stage of substep 1 (RK update,
    # coarser ghosts one fine step later); second: the small mesh (148 octants)
    for name, stage, j, mode, n in (("wave_c1", 3, 1, P.MODE_LTS, 1), ("small", 1, 0, P.MODE_LTS, 2)):
        (U1, K1), (U2, K2) = _case(name, stage, j, mode, n, 900 + stage)
        assert torch.equal(K1, K2), name
        assert torch.equal(U1, U2), name


def test_noalloc_rejects_unuploaded_mesh():
    gm = P.build_mesh(mesh_spec("small"))
    N = gm.info()["n_oct"]
    U = torch.zeros((2, 2, N, 125), dtype=torch.float64, device=DEV)
    K = torch.zeros((4, 2, N, 125), dtype=torch.float64, device=DEV)
    with pytest.raises(P.LTSError) as e:
        P.fused_stage_noalloc(gm, U, K, P.EQ_WAVE, 0.1, 0, 0, P.MODE_LTS, 0)
    assert e.value.status == 1
