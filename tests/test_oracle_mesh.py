"""Pins of the oracle's octree, blocks, unzip map and schedule: the paper's worked
figures (fig. oct_to_blocks, fig. blk_loop), eqs. w_nuts / w_uts, brute-force checks
on small inputs and exactness of the padding on polynomials."""
import os

import numpy as np
import pytest

from oracle import octree as ot
from oracle import solver as so
from workloads import mesh_spec, consistent_random_dg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _fig_tree():
    """3D analog of fig. oct_to_blocks: root -> level 1, children 1 and 6 -> level 2."""
    L = 2
    a, l = ot.uniform_leaves(1, L)
    al, ll = [], []
    for i, an in enumerate(a):
        if i in (1, 6):
            al.append(ot._children(an[None, :], 1, L)); ll.append(np.full(8, 2))
        else:
            al.append(an[None, :]); ll.append(np.array([1]))
    return np.concatenate(al), np.concatenate(ll), L


def _read_fixture(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_oct_to_blocks_fixture():
    a, l, L = _fig_tree()
    m = ot.mesh_from_leaves(a, l, L, cap=4, do_balance=False)
    got = {}
    for row in m.blocks:
        key = (int(row[2]), int(row[1]))
        got[key] = got.get(key, 0) + 1
    want = {(int(r[0]), int(r[1])): int(r[2]) for r in _read_fixture("oct_to_blocks.txt")}
    assert got == want


def owner_fixture_mesh():
    """The mesh of tests/golden/ghost_owner.txt: L = 2, level-1 octants with the
    one at the origin refined once (15 leaves, 8 blocks)."""
    L = 2
    a, l = ot.uniform_leaves(1, L)
    al, ll = [], []
    for an_, lv in zip(a, l):
        if (an_ == 0).all():
            al.append(ot._children(an_[None, :], 1, L)); ll.append(np.full(8, 2))
        else:
            al.append(an_[None, :]); ll.append(np.array([1]))
    return np.concatenate(al), np.concatenate(ll), L


def owner_fixture_rows():
    return [[int(v) for v in r[:9]] for r in
            ([x for x in line.split("#")[0].split()] for line in open(os.path.join(GOLD, "ghost_owner.txt")))
            if len(r) >= 9]


def map_row(mp, m, qx, qy, qz):
    S = 4 * m + 7
    return mp[((qz + 3) * S + (qy + 3)) * S + (qx + 3)].tolist()


def test_ghost_owner_fixture():
    """The unzip map's owner of face, edge and corner points equals the hand
    derivation of tests/golden/ghost_owner.txt (Sec. 3.3, fig. unzip)."""
    a, l, L = owner_fixture_mesh()
    m = ot.mesh_from_leaves(a, l, L, cap=4, do_balance=True)
    assert m.n_oct == 15 and len(m.blocks) == 8
    rows = owner_fixture_rows()
    assert len(rows) == 13
    for r in rows:
        b, qx, qy, qz = r[:4]
        assert map_row(ot.unzip_map(m, b), int(m.blocks[b, 1]), qx, qy, qz) == r[4:9], r


@pytest.fixture(scope="module")
def small_mesh():
    return ot.build_mesh(ot.MeshSpec.from_dict(mesh_spec("small")))


@pytest.fixture(scope="module")
def c1_mesh():
    return ot.build_mesh(ot.MeshSpec.from_dict(mesh_spec("wave_c1")))


def _random_tree(seed, L=4, lmin=1, p=0.35):
    rng = np.random.default_rng(seed)
    a, l = ot.uniform_leaves(lmin, L)
    for lev in range(lmin, L):
        sel = (l == lev) & (rng.random(len(l)) < p)
        if not sel.any():
            continue
        ch = ot._children(a[sel], lev, L)
        a = np.concatenate([a[~sel], ch]); l = np.concatenate([l[~sel], np.full(len(ch), lev + 1)])
    return ot._sort(a, l)


def _naive_balance(a, l, L):
    """Straightforward closure: repeatedly split the first violating leaf found by
    an O(N^2) scan (independent of the oracle's grid/max-filter implementation)."""
    a, l = a.copy(), l.copy()
    n = 4 * (1 << L)
    while True:
        lo = 4 * a
        hi = lo + 4 * (1 << (L - l))[:, None]
        hit = -1
        for i in range(len(l)):
            cand = np.nonzero(l >= l[i] + 2)[0]
            if len(cand) == 0:
                continue
            gap = np.full((len(cand), 3), 10 ** 9)
            for k in (-1, 0, 1):
                gap = np.minimum(gap, np.maximum(0, np.maximum(lo[cand] + k * n - hi[i], lo[i] - (hi[cand] + k * n))))
            if (gap.max(axis=1) <= 3 * (1 << (L - l[i]))).any():
                hit = i
                break
        if hit < 0:
            return ot._sort(a, l)
        ch = ot._children(a[hit:hit + 1], int(l[hit]), L)
        keep = np.arange(len(l)) != hit
        a = np.concatenate([a[keep], ch]); l = np.concatenate([l[keep], np.full(8, l[hit] + 1)])


@pytest.mark.parametrize("seed,L,lmin,p", [(0, 4, 1, 0.35), (1, 4, 1, 0.35), (2, 4, 1, 0.35), (3, 4, 1, 0.35),
                                            (4, 5, 2, 0.02), (5, 5, 2, 0.03), (6, 5, 2, 0.015)])
def test_balance_equals_naive_closure(seed, L, lmin, p):
    """Dense trees exercise plain 2:1 contact, sparse deep trees the 3 h reach."""
    a, l = _random_tree(seed, L, lmin, p)
    ba, bl = ot.balance(a, l, L)
    na, nl = _naive_balance(a, l, L)
    assert np.array_equal(ba, na) and np.array_equal(bl, nl)
    assert ot.is_balanced_bruteforce(ba, bl, L)


@pytest.mark.parametrize("seed", [0, 1])
def test_balance_minimal(seed):
    """Merging any family of eight siblings created by the balance violates it."""
    a, l = _random_tree(seed)
    ba, bl = ot.balance(a, l, 4)
    before = {(int(x), int(y), int(z), int(v)) for (x, y, z), v in zip(a, l)}
    L = 4
    seen = set()
    for i, (an, lev) in enumerate(zip(ba, bl)):
        key = (int(an[0]), int(an[1]), int(an[2]), int(lev))
        if key in before or lev == 0:
            continue
        s = 1 << (L - lev + 1)
        parent = tuple(int(v) for v in (an // s) * s)
        if (parent, lev) in seen:
            continue
        seen.add((parent, lev))
        sib = [j for j in range(len(bl)) if bl[j] == lev and tuple(int(v) for v in (ba[j] // s) * s) == parent]
        if len(sib) != 8:
            continue
        keep = np.ones(len(bl), bool); keep[sib] = False
        ma = np.concatenate([ba[keep], np.array([parent])]); ml = np.concatenate([bl[keep], [lev - 1]])
        assert not ot.is_balanced_bruteforce(ma, ml, L)


def test_tiling_and_balance(small_mesh, c1_mesh):
    for m in (small_mesh, c1_mesh):
        vol = ((1 << (m.L - m.levels)) ** 3).sum()
        assert vol == 8 ** m.L
        g = ot.level_grid(m.anchors, m.levels, m.L)
        assert (g >= 0).all()
        assert ot.is_balanced_bruteforce(m.anchors, m.levels, m.L)
    assert 500 < c1_mesh.n_oct < 1700 and (c1_mesh.lmin, c1_mesh.lmax) == (2, 4)


def test_blocks_uniform_aligned_maximal(c1_mesh):
    m = c1_mesh
    g = ot.level_grid(m.anchors, m.levels, m.L)
    covered = np.zeros(m.n_oct, bool)
    for first, mm, lev, x, y, z in m.blocks:
        s = 1 << (m.L - lev)
        span = mm * s
        assert x % span == 0 and y % span == 0 and z % span == 0 and mm <= m.cap
        assert (g[x:x + span, y:y + span, z:z + span] == lev).all()
        octs = np.arange(first, first + mm ** 3)
        assert (m.levels[octs] == lev).all() and not covered[octs].any()
        covered[octs] = True
        if mm < m.cap and lev > 0:
            ps = 2 * span
            px, py, pz = (x // ps) * ps, (y // ps) * ps, (z // ps) * ps
            assert not (g[px:px + ps, py:py + ps, pz:pz + ps] == lev).all()
    assert covered.all()


def test_unzip_map_geometry(small_mesh, c1_mesh):
    """Every padded point's source leaf contains the point, one level apart at most,
    and the stored position is the point in the source's node units."""
    for m in (small_mesh, c1_mesh):
        n = 4 * (1 << m.L)
        for b in range(0, len(m.blocks), max(1, len(m.blocks) // 40)):
            first, mm, lev = (int(v) for v in m.blocks[b, :3])
            s = 1 << (m.L - lev)
            mp = ot.unzip_map(m, b)
            q = np.arange(-3, 4 * mm + 4)
            Qz, Qy, Qx = np.meshgrid(q, q, q, indexing="ij")
            Q = np.stack([Qx.ravel(), Qy.ravel(), Qz.ravel()], 1)
            X = (4 * m.blocks[b, 3:6] + Q * s) % n
            leaf, kind, pos2 = mp[:, 0], mp[:, 1], mp[:, 2:5]
            sl = 1 << (m.L - m.levels[leaf])
            Xs = (4 * m.anchors[leaf] + pos2 * sl[:, None] // 2) % n
            assert np.array_equal(X, Xs)
            dl = m.levels[leaf] - lev
            assert ((kind == ot.KIND_OWN) <= (dl == 0)).all()
            assert ((kind == ot.KIND_SAME) <= (dl == 0)).all()
            assert ((kind == ot.KIND_FINE) <= (dl == 1)).all()
            assert ((kind == ot.KIND_COARSE) <= (dl == -1)).all()
            own = kind == ot.KIND_OWN
            assert ((leaf[own] >= first) & (leaf[own] < first + mm ** 3)).all()
            assert (pos2[kind != ot.KIND_COARSE] % 2 == 0).all()
            assert ((pos2 >= 0) & (pos2 <= 8)).all()


def _open_records(st):
    for b in range(len(st.mesh.blocks)):
        st.rec_par[b] = st.cur_par[b]
        st.rec_t0[b] = st.cur_t[b]


def test_zip_unzip_identity(c1_mesh):
    """zip(unzip(U)) == U bitwise for DG data whose duplicated nodes agree."""
    m = c1_mesh
    U = consistent_random_dg(m.anchors, m.levels, m.L, 2, seed=3)
    st = so.State(m, 2, "rk4", "lts")
    st.set_initial(U)
    _open_records(st)
    out = np.zeros_like(U)
    for b in range(len(m.blocks)):
        pad = st.unzip(b, 0)                       # stage 1: Y = U0 for every case
        mm = int(m.blocks[b, 1])
        st.zip_into(b, pad[:, 3:3 + 4 * mm + 1, 3:3 + 4 * mm + 1, 3:3 + 4 * mm + 1], out)
    assert np.array_equal(out, U)


def _poly(X, L):
    x = -1 + 2 * X[..., 0] / (4 * (1 << L)); y = -1 + 2 * X[..., 1] / (4 * (1 << L))
    z = -1 + 2 * X[..., 2] / (4 * (1 << L))
    return 0.3 + x ** 4 * y ** 3 - 2 * z ** 4 * x + y ** 2 * z ** 3, x ** 3 - y * z ** 4 + 0.5


@pytest.mark.parametrize("second_fine_step", [False, True])
def test_unzip_polynomial_exact(c1_mesh, second_fine_step):
    """Padding of tensor-degree-4 polynomial data is exact (injection and Q4
    interpolation), and the time case of every source is the right one:
    with U0 = P and all stages K_i = Q, Y_s = P + dt_r (delta + c_s) Q."""
    from workloads import node_units
    m = c1_mesh
    Xn = node_units(m.anchors, m.levels, m.L)
    P, Q = _poly(Xn, m.L)
    st = so.State(m, 1, "rk4", "lts")
    st.set_initial(P[None])
    st.K[:] = Q[None, None]
    _open_records(st)
    fine = m.lmax
    if second_fine_step:
        for b in range(len(m.blocks)):
            if m.blocks[b, 2] == fine:
                st.rec_t0[b] = st.dt_ticks[b]
    c = [0.0, 0.5, 0.5, 1.0]
    n_u = 4 * (1 << m.L)
    checked = 0
    for b in range(len(m.blocks)):
        first, mm, lev = (int(v) for v in m.blocks[b, :3])
        if second_fine_step and lev != fine:
            continue
        s = 1 << (m.L - lev)
        lo = 4 * m.blocks[b, 3:6] - 3 * s
        hi = 4 * m.blocks[b, 3:6] + (4 * mm + 3) * s
        if (lo < 0).any() or (hi > n_u).any():
            continue                                   # padding wraps: polynomial not periodic
        q = np.arange(-3, 4 * mm + 4)
        Qz, Qy, Qx = np.meshgrid(q, q, q, indexing="ij")
        X = 4 * m.blocks[b, 3:6][None, None, None, :] + np.stack([Qx, Qy, Qz], -1) * s
        Pp, Qp = _poly(X, m.L)
        mp = ot.unzip_map(m, b)
        srcb = m.block_of_leaf[mp[:, 0]]
        delta = ((st.rec_t0[b] - st.rec_t0[srcb]) / st.dt_ticks[b]).reshape(Pp.shape)
        dt = st.dt_phys(b)
        for stage in range(4):
            pad = st.unzip(b, stage)[0]
            want = Pp + dt * (delta + c[stage]) * Qp
            assert np.abs(pad - want).max() < 1e-12 * max(1.0, np.abs(want).max()), (b, stage)
        checked += 1
    assert checked > 5


def test_blk_loop_schedule(c1_mesh):
    """fig. blk_loop: B_0 = {b_h, b_2h, b_4h}, B_1 = {b_h}, B_2 = {b_h, b_2h}, B_3 = {b_h}."""
    m = c1_mesh
    assert m.lmax - m.lmin == 2
    name = {m.lmax: "b_h", m.lmax - 1: "b_2h", m.lmax - 2: "b_4h"}
    for row in _read_fixture("blk_loop.txt"):
        j = int(row[0])
        act = ot.active_blocks(m, j)
        got = {name[int(l)] for l in np.unique(m.blocks[act, 2])}
        assert got == set(row[1:])
        # every block of the named levels is evolved, none other
        lev_ok = np.isin(m.blocks[:, 2], [k for k, v in name.items() if v in row[1:]])
        assert np.array_equal(np.sort(act), np.nonzero(lev_ok)[0])


def test_work_counts_equal_eq_w_nuts(c1_mesh, small_mesh):
    """Node-updates per coarsest step: LTS = eq. w_nuts, GTS = eq. w_uts."""
    for m in (c1_mesh, small_mesh):
        sm = ot.speedup_model(m)
        nodes = 125 * m.blocks[:, 1] ** 3
        lts = sum(int(nodes[ot.active_blocks(m, j)].sum()) for j in range(ot.substeps(m)))
        gts = sum(int(nodes[ot.active_blocks(m, j, "gts")].sum()) for j in range(ot.substeps(m)))
        assert lts == sm["w_lts"] and gts == sm["w_gts"]
        assert 1.0 <= sm["s_est"] <= sm["s_max"]
