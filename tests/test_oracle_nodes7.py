"""Pins of the oracle with 7^3 nodes per octant (the paper's discretisation, used
for its scaling runs, with 2:1 balance; Sec. 4.5 and the mesh-generation figure):
2:1 balance against an independent closure, the unzip map's geometry and its
mid-plane tie rule (hand-derived rows), exact padding of tensor degree-6
polynomials, zip/unzip identity, the Fourier closed form on uniform meshes
(classic RK4 and SSP-RK3), convergence order, and LTS vs GTS agreement."""
import numpy as np
import pytest

from oracle import analytic as an
from oracle import octree as ot
from oracle import solver as so
from workloads import consistent_random_dg, node_units, physical, wave_plane

N7 = 7


def _uniform7(level, L=None):
    L = level if L is None else L
    a, l = ot.uniform_leaves(level, L)
    return ot.mesh_from_leaves(a, l, L, cap=4, do_balance=False, nodes=N7)


def _adaptive7(lmin, L, c=(0.1, 0.05, -0.1), r=0.45, boundary="periodic"):
    """Levels lmin..L with a ball of radius r (physical) refined to L, 7 nodes."""
    n_u = 6 * (1 << L)
    cc = [int(round((v + 1) / 2 * n_u)) for v in c]
    r2 = [-1] * L
    for lev in range(lmin, L):
        r2[lev] = int((r * n_u / 2) ** 2)
    spec = ot.MeshSpec(lmin, L, [ot.Criterion("ball", tuple(cc), r2=r2)], 4, boundary, N7)
    return ot.build_mesh(spec)


ADAPT = dict(lmin=2, L=4, c=(0.3, 0.4, 0.45), r=0.1)     # levels 2-4, 176 octants


@pytest.fixture(scope="module")
def mesh7():
    m = _adaptive7(**ADAPT)
    assert (m.lmin, m.lmax) == (2, 4)
    return m


# ----------------------------------------------------------------------------- balance
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


def _naive_21(a, l, L):
    """2:1 closure by O(N^2) scans: split the first leaf that touches (closed
    boxes, periodic images) a leaf two or more levels finer, until none does."""
    a, l = a.copy(), l.copy()
    n = 1 << L                                     # level-L cells per side
    while True:
        lo = a
        hi = lo + (1 << (L - l))[:, None]
        hit = -1
        for i in range(len(l)):
            cand = np.nonzero(l >= l[i] + 2)[0]
            if len(cand) == 0:
                continue
            gap = np.full((len(cand), 3), 10 ** 9)
            for k in (-1, 0, 1):
                gap = np.minimum(gap, np.maximum(0, np.maximum(lo[cand] + k * n - hi[i], lo[i] - (hi[cand] + k * n))))
            if (gap.max(axis=1) == 0).any():
                hit = i
                break
        if hit < 0:
            return ot._sort(a, l)
        ch = ot._children(a[hit:hit + 1], int(l[hit]), L)
        keep = np.arange(len(l)) != hit
        a = np.concatenate([a[keep], ch]); l = np.concatenate([l[keep], np.full(8, l[hit] + 1)])


@pytest.mark.parametrize("seed,L,lmin,p", [(0, 4, 1, 0.35), (1, 4, 1, 0.35), (4, 5, 2, 0.02), (5, 5, 2, 0.03)])
def test_balance_21_equals_naive_closure(seed, L, lmin, p):
    a, l = _random_tree(seed, L, lmin, p)
    ba, bl = ot.balance(a, l, L, nodes=N7)
    na, nl = _naive_21(a, l, L)
    assert np.array_equal(ba, na) and np.array_equal(bl, nl)
    assert ot.is_balanced_bruteforce(ba, bl, L, nodes=N7)
    # the ghost-reach balance of 5-node octants refines at least as much
    ga, gl = ot.balance(a, l, L, nodes=5)
    assert len(gl) >= len(bl)


def _refined_corner(child_anchor):
    """Bounded domain, L = 4: level-1 leaves (8 level-4 cells wide), leaf (0,0,0)
    split into level-2 children (4 cells) and the child at `child_anchor` split
    again into level-3 leaves (2 cells)."""
    L = 4
    a, l = ot.uniform_leaves(1, L)
    k = int(np.nonzero((a == [0, 0, 0]).all(1))[0][0])
    ch = ot._children(a[k:k + 1], 1, L)
    i = int(np.nonzero((ch == child_anchor).all(1))[0][0])
    gch = ot._children(ch[i:i + 1], 2, L)
    A = np.concatenate([np.delete(a, k, 0), np.delete(ch, i, 0), gch])
    Lv = np.concatenate([np.full(7, 1), np.full(7, 2), np.full(8, 3)])
    return ot._sort(A, Lv) + (L,)


def _has(a, l, anchor, lev):
    return any((x == anchor).all() and v == lev for x, v in zip(a, l))


def test_balance_21_hand_cases():
    """Level-3 leaves filling [0, 4)^3: the nearest level-1 leaves start at 8, a gap
    of half a level-1 octant.  2:1 balance keeps them (no contact); the ghost reach
    of 5-node octants (3/4 of a level-1 octant) splits them.  Level-3 leaves filling
    [4, 8)^3: the level-1 leaf at (8, 8, 8) touches the level-3 leaf at (6, 6, 6) at
    one corner point only, and 2:1 balance splits it."""
    A, Lv, L = _refined_corner([0, 0, 0])
    ba, bl = ot.balance(A, Lv, L, periodic=False, nodes=N7)
    assert np.array_equal(ba, A) and np.array_equal(bl, Lv)
    ga, gl = ot.balance(A, Lv, L, periodic=False, nodes=5)
    for anchor in ([8, 0, 0], [0, 8, 0], [8, 8, 0], [8, 8, 8]):
        assert _has(A, Lv, anchor, 1) and not _has(ga, gl, anchor, 1), anchor
    A, Lv, L = _refined_corner([4, 4, 4])
    ba, bl = ot.balance(A, Lv, L, periodic=False, nodes=N7)
    assert _has(A, Lv, [8, 8, 8], 1) and not _has(ba, bl, [8, 8, 8], 1)
    assert ot.is_balanced_bruteforce(ba, bl, L, periodic=False, nodes=N7)


# ----------------------------------------------------------------------------- unzip map
def test_unzip_map_geometry7(mesh7):
    """Every padded point's source leaf holds the point at the stored position, one
    level apart at most; FINE sources touch the block (the only children that
    2:1 balance keeps leaves)."""
    m = mesh7
    n = 6 * (1 << m.L)
    for b in range(len(m.blocks)):
        first, mm, lev = (int(v) for v in m.blocks[b, :3])
        s = 1 << (m.L - lev)
        mp = ot.unzip_map(m, b)
        q = np.arange(-3, 6 * mm + 4)
        assert len(mp) == len(q) ** 3
        Qz, Qy, Qx = np.meshgrid(q, q, q, indexing="ij")
        Q = np.stack([Qx.ravel(), Qy.ravel(), Qz.ravel()], 1)
        X = (6 * m.blocks[b, 3:6] + Q * s) % n
        leaf, kind, pos2 = mp[:, 0], mp[:, 1], mp[:, 2:5]
        sl = 1 << (m.L - m.levels[leaf])
        Xs = (6 * m.anchors[leaf] + pos2 * sl[:, None] // 2) % n
        assert np.array_equal(X, Xs)
        dl = m.levels[leaf] - lev
        assert ((kind == ot.KIND_OWN) <= (dl == 0)).all()
        assert ((kind == ot.KIND_SAME) <= (dl == 0)).all()
        assert ((kind == ot.KIND_FINE) <= (dl == 1)).all()
        assert ((kind == ot.KIND_COARSE) <= (dl == -1)).all()
        assert ((pos2 >= 0) & (pos2 <= 12)).all()
        assert (pos2[kind != ot.KIND_COARSE] % 2 == 0).all()
        fine = np.nonzero(kind == ot.KIND_FINE)[0]
        if len(fine):
            # a fine source's closed box meets the block's closed box
            blo = 6 * m.blocks[b, 3:6]
            bhi = blo + 6 * mm * s
            flo = 6 * m.anchors[leaf[fine]]
            fhi = flo + 6 * sl[fine][:, None]
            gap = np.full((len(fine), 3), 10 ** 9)
            for k in (-1, 0, 1):
                gap = np.minimum(gap, np.maximum(0, np.maximum(flo + k * n - bhi, blo - (fhi + k * n))))
            assert (gap.max(axis=1) == 0).all(), b


def _two_level_mesh():
    """Periodic L = 2, every level-1 leaf except the one at anchor (2, 0, 0)
    (level-2 units) refined to level 2; 7 nodes per side."""
    L = 2
    a, l = ot.uniform_leaves(1, L)
    keep = ~(a == [2, 0, 0]).all(1)
    ch = ot._children(a[keep], 1, L)
    A = np.concatenate([a[~keep], ch]); Lv = np.concatenate([[1], np.full(len(ch), 2)])
    return ot.mesh_from_leaves(A, Lv, L, cap=1, do_balance=False, nodes=N7)


def test_unzip_map_hand_rows7():
    """Rows worked out by hand from the ownership rule.  Mesh: the level-1 leaf C
    at level-2 anchor (2, 0, 0) (node units 12..24 on x, 0..12 on y, z) and
    level-2 leaves elsewhere.  Block of the level-2 leaf R at anchor (1, 0, 0)
    (x nodes 6..12, spacing 1): its upper x padding Q = 7, 8, 9 lies in the
    receiver-level cell 1 along x, the lower half of C, which is coarser:
    position (6 * beta + nu) / 2 with beta = 0 (x), nu = 1, 2, 3 -> 2 px = 1, 2, 3.
    Block of C (m = 1, level 1, spacing 2): its lower x padding Q = -3..-1 lies in
    level-1 cell -1 (x nodes 6..12 ... 0..12), nu = Q + 6 = 3, 4, 5.  That cell is
    8 level-2 leaves; the near child along x is c = 1 (anchor x = 1), also on the
    mid-plane nu = 3 (x = 6, shared with the far child at anchor x = 0), at fine
    node 2 nu - 6 = 0, 2, 4.  Its upper x padding Q = 7..9 (x = 26, 28, 30, wrapping
    to 2, 4, 6) lies in cell 1 = level-1 cell 0 (periodic), nu = 1, 2, 3: near child
    c = 0 (anchor x = 0) also at nu = 3 (x = 6, the far child's face), fine node
    2 nu = 2, 4, 6."""
    m = _two_level_mesh()
    L = m.L

    def leaf_at(ax, ay, az, lev):
        return m._lookup[(lev, ax, ay, az)]

    def row(b, qx, qy, qz):
        mm = int(m.blocks[b, 1])
        S = 6 * mm + 7
        mp = ot.unzip_map(m, b)
        return tuple(int(v) for v in mp[((qz + 3) * S + (qy + 3)) * S + (qx + 3)])

    C = leaf_at(2, 0, 0, 1)
    R = leaf_at(1, 0, 0, 2)
    bC = int(m.block_of_leaf[C])
    bR = int(m.block_of_leaf[R])
    assert m.blocks[bC, 1] == 1 and m.blocks[bR, 1] == 1
    # receiver R (level 2), y = z = node 2 of R
    for Q, p2 in ((7, 1), (8, 2), (9, 3)):
        assert row(bR, Q, 2, 2) == (C, ot.KIND_COARSE, p2, 2, 2), Q
    # receiver C (level 1), y = z = node 2 of C (level-2 nodes y = z = 4: in the
    # lower level-2 children along y and z, fine node 4 -> 2 * 4 = 8 in 2x units)
    for Q, nu in ((-3, 3), (-2, 4), (-1, 5)):
        fine = leaf_at(1, 0, 0, 2)              # near child along x, y, z = 0
        assert row(bC, Q, 2, 2) == (fine, ot.KIND_FINE, 2 * (2 * nu - 6), 8, 8), Q
    for Q, nu in ((7, 1), (8, 2), (9, 3)):
        fine = leaf_at(0, 0, 0, 2)              # wraps: near child along x is c = 0
        assert row(bC, Q, 2, 2) == (fine, ot.KIND_FINE, 4 * nu, 8, 8), Q
    # a diagonal padding cell, on the mid-plane of x and y: Q = (-3, -3, 2) is in
    # level-1 cell (0, -1, 0) = (0, 1, 0) after wrapping, nu = (3, 3, 2).  Near
    # children: c_x = 1 and c_y = 1 (cells below the block), c_z = 0 (nu < 3):
    # level-2 anchor (2*0 + 1, 2*1 + 1, 0) = (1, 3, 0), fine node (0, 0, 4)
    fine = leaf_at(1, 3, 0, 2)
    assert row(bC, -3, -3, 2) == (fine, ot.KIND_FINE, 0, 0, 8)


def _poly6(X, L):
    n_u = 6 * (1 << L)
    x, y, z = (-1 + 2 * X[..., d] / n_u for d in range(3))
    return 0.3 + x ** 6 * y ** 5 - 2 * z ** 6 * x + y ** 2 * z ** 3, x ** 5 - y * z ** 6 + 0.5


def _open_records(st):
    for b in range(len(st.mesh.blocks)):
        st.rec_par[b] = st.cur_par[b]
        st.rec_t0[b] = st.cur_t[b]


@pytest.mark.parametrize("second_fine_step", [False, True])
def test_unzip_polynomial_exact7(second_fine_step):
    """Padding of tensor-degree-6 polynomial data is exact (injection and degree-6
    interpolation), with the time case of every source: U0 = P, K_i = Q give
    Y_s = P + dt_r (delta + c_s) Q.  Bounded mesh: nothing wraps."""
    m = _adaptive7(**ADAPT, boundary="outer")
    Xn = node_units(m.anchors, m.levels, m.L, nodes=N7)
    P, Q = _poly6(Xn, m.L)
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
    checked = coarse_pts = 0
    for b in range(len(m.blocks)):
        first, mm, lev = (int(v) for v in m.blocks[b, :3])
        if second_fine_step and lev != fine:
            continue
        s = 1 << (m.L - lev)
        q = np.arange(-3, 6 * mm + 4)
        Qz, Qy, Qx = np.meshgrid(q, q, q, indexing="ij")
        X = 6 * m.blocks[b, 3:6][None, None, None, :] + np.stack([Qx, Qy, Qz], -1) * s
        Pp, Qp = _poly6(X, m.L)
        mp = ot.unzip_map(m, b)
        has = (mp[:, 1] != ot.KIND_NONE).reshape(Pp.shape)
        coarse_pts += int((mp[:, 1] == ot.KIND_COARSE).sum())
        srcb = m.block_of_leaf[np.maximum(mp[:, 0], 0)]
        delta = ((st.rec_t0[b] - st.rec_t0[srcb]) / st.dt_ticks[b]).reshape(Pp.shape)
        dt = st.dt_phys(b)
        for stage in range(4):
            pad = st.unzip(b, stage)[0]
            want = Pp + dt * (delta + c[stage]) * Qp
            err = np.abs(pad - want)[has].max()
            assert err < 1e-12 * max(1.0, np.abs(want).max()), (b, stage, err)
        checked += 1
    assert checked >= (3 if second_fine_step else 6) and coarse_pts > 0


def test_zip_unzip_identity7(mesh7):
    """zip(unzip(U)) == U bitwise for DG data whose duplicated nodes agree."""
    m = mesh7
    U = consistent_random_dg(m.anchors, m.levels, m.L, 2, seed=5, nodes=N7)
    st = so.State(m, 2, "rk4", "lts")
    st.set_initial(U)
    _open_records(st)
    out = np.zeros_like(U)
    for b in range(len(m.blocks)):
        pad = st.unzip(b, 0)
        mm = int(m.blocks[b, 1])
        g = 6 * mm + 1
        st.zip_into(b, pad[:, 3:3 + g, 3:3 + g, 3:3 + g], out)
    assert np.array_equal(out, U)


# ----------------------------------------------------------------------------- time stepping
@pytest.mark.parametrize("tableau,order", [("rk4", 4), ("ssprk3", 3)])
@pytest.mark.parametrize("n,sigma", [((1, 2, 0), 0.1), ((2, 1, 1), 0.3)])
def test_fourier_mode_closed_form7(n, sigma, tableau, order):
    """On a uniform periodic 7-node mesh the scheme is the uniform-grid scheme with
    h = 2^(1-l) / 6: cos(pi n.x) evolves by R(dt M)^N exactly (to rounding)."""
    m = _uniform7(1)
    X = physical(node_units(m.anchors, m.levels, m.L, nodes=N7), m.L, nodes=N7)
    ph = np.pi * (X * np.asarray(n)).sum(-1)
    U0 = np.stack([np.cos(ph), np.zeros_like(ph)])
    nsteps = 3
    out = so.run(m, U0, nsteps, "lts", sigma=sigma, tableau=tableau)
    h = ot.h_level(1, N7)
    assert h == 1.0 / 6.0 and ot.dt_level(1, N7) == 0.25 * (1.0 / 6.0)
    amp = an.fourier_mode_solution(order, n, h, ot.dt_level(1, N7), nsteps, sigma)
    want = np.stack([amp[0] * np.cos(ph), amp[1] * np.cos(ph)])
    assert np.abs(out - want).max() <= 1e-13 * max(1.0, np.abs(want).max())


def _plane_error7(m, n_coarse, mode, n=(1, 1, 0), tableau="rk4"):
    U0 = wave_plane(m.anchors, m.levels, m.L, n, nodes=N7)
    out = so.run(m, U0, n_coarse, mode, sigma=0.0, tableau=tableau)
    T = n_coarse * ot.dt_level(m.lmin, N7)
    X = physical(node_units(m.anchors, m.levels, m.L, nodes=N7), m.L, nodes=N7)
    return out, an.norms(out - an.plane_wave(X, n, T), m.levels, m.L)[0][0]


def test_convergence_uniform7():
    """Plane wave, uniform levels 1 and 2, same T: observed order >= 3.5 (RK4,
    sixth-order space)."""
    e1 = _plane_error7(_uniform7(1), 2, "gts")[1]
    e2 = _plane_error7(_uniform7(2), 4, "gts")[1]
    assert np.log2(e1 / e2) >= 3.5, (e1, e2)


def test_lts_vs_gts_adaptive7(mesh7):
    """LTS and GTS on the adaptive 7-node mesh (levels 2-4): both within 25 % of
    the plane-wave error of a uniform run at the coarsest level (the level-2
    octants dominate the error; GTS steps them with a quarter of LTS's step), and
    their difference below the larger of the two errors (truncation-order
    agreement, Sec. 4.3)."""
    m = mesh7
    for tableau in ("rk4", "ssprk3"):
        a, ea = _plane_error7(m, 1, "lts", tableau=tableau)
        g, eg = _plane_error7(m, 1, "gts", tableau=tableau)
        d = an.norms(a - g, m.levels, m.L)[0][0]
        eu = _plane_error7(_uniform7(2), 1, "gts", tableau=tableau)[1]
        assert d <= max(ea, eg) and ea <= 1.25 * eu and eg <= 1.25 * eu, (tableau, d, ea, eg, eu)


def test_speedup_model7(mesh7):
    """alpha_l counts 7^3 nodes per octant in eqs. w_nuts / w_uts."""
    sm = ot.speedup_model(mesh7)
    assert sum(sm["alpha"]) == 343 * mesh7.n_oct
