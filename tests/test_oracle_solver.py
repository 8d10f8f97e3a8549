"""Pins of the oracle's time stepping: closed-form Fourier solution on uniform
meshes, LTS == GTS where only one level exists, analytic solutions and convergence
order, LTS vs GTS agreement at truncation order (Sec. 4.3)."""
import numpy as np
import pytest

from oracle import analytic as an
from oracle import octree as ot
from oracle import solver as so
from workloads import centre_physical, mesh_spec, node_units, physical, wave_gaussian, wave_plane


def _uniform(level, L=None):
    L = level if L is None else L
    a, l = ot.uniform_leaves(level, L)
    return ot.mesh_from_leaves(a, l, L, cap=4, do_balance=False)


def test_uniform_lts_equals_gts_bitwise():
    m = _uniform(2)
    U0 = wave_plane(m.anchors, m.levels, m.L, (1, 2, 0))
    a = so.run(m, U0, 2, "lts", sigma=0.1)
    b = so.run(m, U0, 2, "gts", sigma=0.1)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("tableau,order", [("rk4", 4), ("ssprk3", 3)])
@pytest.mark.parametrize("n,sigma", [((1, 2, 0), 0.1), ((3, 1, 1), 0.0), ((2, 2, 2), 0.3)])
def test_fourier_mode_closed_form(n, sigma, tableau, order):
    """u0 = cos(pi n.x), v0 = 0 on a uniform periodic level-2 mesh evolves as
    R(dt M)^N applied to (1, 0) times cos(pi n.x), R the stability polynomial of
    the tableau (classic RK4: exp truncated at 4; SSP-RK3: at 3)."""
    m = _uniform(2)
    X = physical(node_units(m.anchors, m.levels, m.L), m.L)
    ph = np.pi * (X * np.asarray(n)).sum(-1)
    U0 = np.stack([np.cos(ph), np.zeros_like(ph)])
    nsteps = 3
    out = so.run(m, U0, nsteps, "lts", sigma=sigma, tableau=tableau)
    h = 2.0 ** (-2 - 1)
    amp = an.fourier_mode_solution(order, n, h, ot.dt_level(2), nsteps, sigma)
    want = np.stack([amp[0] * np.cos(ph), amp[1] * np.cos(ph)])
    assert np.abs(out - want).max() <= 1e-13 * max(1.0, np.abs(want).max())


def test_gaussian_analytic_initial_data_matches_generator():
    m = _uniform(2)
    c = [17, 9, 20]
    U0 = wave_gaussian(m.anchors, m.levels, m.L, [c], sigma=0.1)
    X = physical(node_units(m.anchors, m.levels, m.L), m.L)
    ex = an.gaussian_periodic(X, centre_physical(c, m.L)[None], 0.0, 0.1)
    assert np.abs(U0 - ex).max() < 1e-14


def test_gaussian_analytic_solves_wave_equation():
    """Finite-difference check of u_t = v and v_t = Lap u for the spherical-wave
    formula at points near and away from the centre."""
    rng = np.random.default_rng(0)
    c = np.array([0.1, -0.2, 0.05])
    pts = c + rng.uniform(-0.3, 0.3, size=(20, 3))
    pts[0] = c + 1e-6
    t, e = 0.13, 1e-4
    u = lambda x, t: an.gaussian_periodic(x, c[None], t, 0.1)[0]
    v = lambda x, t: an.gaussian_periodic(x, c[None], t, 0.1)[1]
    ut = (u(pts, t + e) - u(pts, t - e)) / (2 * e)
    assert np.abs(ut - v(pts, t)).max() < 1e-5 * max(1.0, np.abs(ut).max())
    vt = (v(pts, t + e) - v(pts, t - e)) / (2 * e)
    lap = np.zeros(len(pts))
    for d in range(3):
        sh = np.zeros(3); sh[d] = e
        lap += (u(pts + sh, t) - 2 * u(pts, t) + u(pts - sh, t)) / e ** 2
    assert np.abs(vt - lap).max() < 2e-3 * np.abs(vt).max()


def test_standing_wave_matches_1d_form():
    """u0 = cos(pi x), v0 = 0 is the paper's 1D solution (f(x - t) + f(x + t)) / 2
    with f = cos(pi .) (Sec. 4.2); the oracle's 3D run on a uniform level-3 mesh
    reproduces it at T to the scheme's error, and the error falls at order >= 3.5
    from level 2 to level 3."""
    errs = []
    for lev in (2, 3):
        m = _uniform(lev)
        X = physical(node_units(m.anchors, m.levels, m.L), m.L)
        U0 = np.stack([np.cos(np.pi * X[..., 0]), np.zeros(X.shape[:-1])])
        nc = 1 << (lev - 2)
        out = so.run(m, U0, nc, "gts", sigma=0.0)
        T = nc * ot.dt_level(m.lmin)
        f = lambda s: np.cos(np.pi * s)
        ex_u = an.wave_1d(X[..., 0], f, T)
        ex_v = 0.5 * (np.pi * np.sin(np.pi * (X[..., 0] - T)) - np.pi * np.sin(np.pi * (X[..., 0] + T)))
        errs.append(an.norms(out - np.stack([ex_u, ex_v]), m.levels, m.L)[0])
        assert np.abs(out[0] - ex_u).max() < 1e-5
    assert np.log2(errs[0] / errs[1]).min() >= 3.5, errs


def test_norms_volume_weighted():
    """The discrete l2 norm (Sec. 4.3) weights each octant by its volume: an error
    that is constant per octant gives the root of the volume-weighted mean square,
    whose weights are fixed by geometry alone (a level-l octant is 8^-l of the
    domain); the max norm is the largest magnitude."""
    m = ot.build_mesh(ot.MeshSpec.from_dict(mesh_spec("small")))
    rng = np.random.default_rng(5)
    c = rng.standard_normal((2, m.n_oct))
    err = np.broadcast_to(c[:, :, None, None, None], (2, m.n_oct, 5, 5, 5))
    vol = np.array([8.0 ** -int(l) for l in m.levels])
    assert abs(vol.sum() - 1.0) < 1e-15
    l2, linf = an.norms(err, m.levels, m.L)
    for f in range(2):
        assert abs(l2[f] - np.sqrt((vol * c[f] ** 2).sum())) < 1e-14 * l2[f]
        assert linf[f] == np.abs(c[f]).max()
    # one non-zero node of one level-l octant: l2^2 = 8^-l e^2 / 125
    e = np.zeros((1, m.n_oct, 5, 5, 5))
    o = int(np.argmax(m.levels))
    e[0, o, 2, 1, 3] = 3.0
    assert abs(an.norms(e, m.levels, m.L)[0][0] - np.sqrt(vol[o] * 9.0 / 125.0)) < 1e-15


def _plane_error(m, n_coarse, mode, n=(1, 1, 0), sigma=0.0):
    U0 = wave_plane(m.anchors, m.levels, m.L, n)
    out = so.run(m, U0, n_coarse, mode, sigma=sigma)
    T = n_coarse * ot.dt_level(m.lmin)
    X = physical(node_units(m.anchors, m.levels, m.L), m.L)
    ex = an.plane_wave(X, n, T)
    return out, an.norms(out - ex, m.levels, m.L)[0][0]


def test_convergence_uniform():
    """Observed order >= 3.5 for the plane wave, uniform levels 2, 3, 4, same T."""
    errs = []
    for lev in (2, 3, 4):
        m = _uniform(lev)
        _, e = _plane_error(m, 1 << (lev - 2), "gts")
        errs.append(e)
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= 3.5, (errs, rates)


def _adaptive(lmin, L, c=(0.1, 0.05, -0.1), r=0.45):
    """Levels lmin..L with a ball of radius r (physical) refined to L."""
    n_u = 4 * (1 << L)
    cc = [int(round((v + 1) / 2 * n_u)) for v in c]
    r2 = [-1] * L
    for lev in range(lmin, L):
        r2[lev] = int((r * n_u / 2) ** 2)
    spec = ot.MeshSpec(lmin, L, [ot.Criterion("ball", tuple(cc), r2=r2)], 4)
    return ot.build_mesh(spec)


@pytest.mark.slow
def test_lts_vs_gts_adaptive():
    """LTS and GTS agree at truncation order: on an adaptive mesh their difference
    is below GTS's own error, and it falls at order >= 3.5 when every level is
    refined once (same final time)."""
    diffs, errs = [], []
    for lmin in (2, 3):
        m = _adaptive(lmin, lmin + 1)
        assert m.lmax - m.lmin == 1
        nc = 1 << (lmin - 2)
        a, ea = _plane_error(m, nc, "lts")
        g, eg = _plane_error(m, nc, "gts")
        d = an.norms(a - g, m.levels, m.L)[0][0]
        assert d <= eg
        diffs.append(d); errs.append((ea, eg))
    assert np.log2(diffs[0] / diffs[1]) >= 3.5, (diffs, errs)
    assert np.log2(errs[0][0] / errs[1][0]) >= 3.5, errs
