"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np

from oracle import octree as ot
from oracle import solver as so
from workloads import config, mesh_spec, random_dg, wave_gaussian

TOL = 1e-12   # FP64 parity: max |gpu - oracle| / max |oracle| per field


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    F = want.shape[0]
    out = []
    for f in range(F):
        den = max(np.abs(want[f]).max(), 1e-300)
        out.append(np.abs(got[f] - want[f]).max() / den)
    return max(out)


def oracle_mesh(name):
    return ot.build_mesh(ot.MeshSpec.from_dict(mesh_spec(name)))


def positioned_state(mesh, nfields, mode, n, j, seed, tableau="rk4"):
    """Oracle state whose step records sit at substep j of coarse step n (records of
    B_j just opened), filled with seeded random U (both buffers) and K."""
    st = so.State(mesh, nfields, tableau, mode)
    nsub = ot.substeps(mesh)
    for c in range(n):
        for jj in range(nsub):
            st.close_records(st.open_records(jj))
    for jj in range(j):
        st.close_records(st.open_records(jj))
    act = st.open_records(j)
    st.U[:] = random_dg(st.U.shape, seed)
    st.K[:] = random_dg(st.K.shape, seed + 1, 0.5)
    return st, act


def padded_sizes(blocks, ids):
    S = 4 * blocks[ids, 1] + 7
    G = 4 * blocks[ids, 1] + 1
    return S, G


def oracle_c1_at_T(mode):
    """The oracle's whole C1 run (Gaussian pulse, 8 coarse steps to T) in one mode;
    a plain function so that a process pool can run the two modes side by side."""
    om = oracle_mesh("wave_c1")
    cfg = config("wave_c1")
    U0 = wave_gaussian(om.anchors, om.levels, om.L, cfg["pulses"], sigma=cfg["sigma"])
    return so.run(om, U0, cfg["n_coarse"], mode, sigma=cfg["ko_sigma"]).reshape(2, om.n_oct, 125)
