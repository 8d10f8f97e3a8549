"""Pins of the oracle's Maxwell parts: the closed-form solutions solve vacuum
Maxwell and are divergence free (checked by independent finite differences), the
Gaussian-potential solution starts from the seeded initial data, and the oracle's
Maxwell time stepping converges to it (RK4 at order >= 3.5, SSP-RK3 >= 2.5 on
uniform meshes) with LTS at truncation order from GTS on an adaptive mesh."""
import numpy as np
import pytest

from oracle import analytic as an
from oracle import octree as ot
from oracle import solver as so
from workloads import centre_physical, maxwell_gaussian, node_units, physical

SIG = 0.1


def _d(f, x, axis, e):
    """Fourth-order central difference of f along axis at x."""
    sh = np.zeros(3)
    sh[axis] = e
    return (-f(x + 2 * sh) + 8 * f(x + sh) - 8 * f(x - sh) + f(x - 2 * sh)) / (12 * e)


def _dt(f, x, t, e):
    return (-f(x, t + 2 * e) + 8 * f(x, t + e) - 8 * f(x, t - e) + f(x, t - 2 * e)) / (12 * e)


def _curl(F, x, e, off):
    """curl of the 3-vector fields F[off:off+3] at x."""
    def comp(i):
        return lambda y: F(y)[off + i]
    return np.stack([_d(comp(2), x, 1, e) - _d(comp(1), x, 2, e),
                     _d(comp(0), x, 2, e) - _d(comp(2), x, 0, e),
                     _d(comp(1), x, 0, e) - _d(comp(0), x, 1, e)])


def _div(F, x, e, off):
    return sum(_d(lambda y, i=i: F(y)[off + i], x, i, e) for i in range(3))


def _points():
    rng = np.random.default_rng(7)
    c = np.array([0.1, -0.2, 0.05])
    pts = c + rng.uniform(-0.3, 0.3, size=(24, 3))
    # on both sides of the series cutoff (0.5 sigma), near the centre and at it
    pts[0] = c + np.array([1e-7, 0.0, 0.0])
    pts[1] = c + np.array([0.0, 0.3, 0.1]) * SIG
    pts[2] = c + np.array([0.49, 0.0, 0.0]) * SIG
    pts[3] = c + np.array([0.0, 0.0, 0.51]) * SIG
    pts[4] = c + np.array([0.2, 0.2, 0.3]) * SIG
    return c, pts


@pytest.mark.parametrize("t", [0.0, 0.06, 0.17])
def test_maxwell_gaussian_solves_maxwell(t):
    c, pts = _points()
    F = lambda y, tt=t: an.maxwell_gaussian(y, c[None], tt, SIG)
    G = lambda y, tt: an.maxwell_gaussian(y, c[None], tt, SIG)
    e = 1e-3
    E_t = _dt(lambda y, tt: G(y, tt)[0:3], pts, t, e)
    B_t = _dt(lambda y, tt: G(y, tt)[3:6], pts, t, e)
    cB = _curl(F, pts, e, 3)
    cE = _curl(F, pts, e, 0)
    scale = max(np.abs(cB).max(), np.abs(cE).max())
    assert np.abs(E_t - cB).max() < 1e-6 * scale
    assert np.abs(B_t + cE).max() < 1e-6 * scale
    assert np.abs(_div(F, pts, e, 0)).max() < 1e-6 * scale
    assert np.abs(_div(F, pts, e, 3)).max() < 1e-6 * scale


def test_maxwell_gaussian_initial_data_matches_generator():
    """t = 0: E = curl(z g), B = 0 -- the seeded serving data."""
    a, l = ot.uniform_leaves(2, 3)
    L = 3
    cc = [29, 13, 40]
    got = maxwell_gaussian(a, l, L, [cc], sigma=SIG)
    X = physical(node_units(a, l, L), L)
    want = an.maxwell_gaussian(X, centre_physical(cc, L)[None], 0.0, SIG)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_maxwell_plane_solves_maxwell():
    rng = np.random.default_rng(3)
    pts = rng.uniform(-1, 1, size=(16, 3))
    n, e0 = (1, 2, 0), np.array([2.0, -1.0, 0.5])
    F = lambda y, tt=0.3: an.maxwell_plane(y, n, e0, tt)
    G = lambda y, tt: an.maxwell_plane(y, n, e0, tt)
    e = 1e-3
    assert np.abs(_dt(lambda y, tt: G(y, tt)[0:3], pts, 0.3, e) - _curl(F, pts, e, 3)).max() < 1e-6
    assert np.abs(_dt(lambda y, tt: G(y, tt)[3:6], pts, 0.3, e) + _curl(F, pts, e, 0)).max() < 1e-6
    assert np.abs(_div(F, pts, e, 0)).max() < 1e-8 and np.abs(_div(F, pts, e, 3)).max() < 1e-8


def _uniform(level):
    a, l = ot.uniform_leaves(level, level)
    return ot.mesh_from_leaves(a, l, level, cap=4, do_balance=False)


def _maxwell_error(m, n_coarse, mode, tableau, sigma_g=0.3):
    c = np.array([0.05, -0.1, 0.15])
    X = physical(node_units(m.anchors, m.levels, m.L), m.L)
    U0 = an.maxwell_gaussian(X, c[None], 0.0, sigma_g)
    out = so.run(m, U0, n_coarse, mode, equation="maxwell", tableau=tableau, sigma=0.0)
    T = n_coarse * ot.dt_level(m.lmin)
    ex = an.maxwell_gaussian(X, c[None], T, sigma_g)
    return an.norms(out - ex, m.levels, m.L)[0]


@pytest.mark.slow
def test_maxwell_convergence_uniform():
    """The oracle's Maxwell RK4 stepping converges to the closed form at order
    >= 3.5 on uniform meshes of levels 2, 3, 4 (same T) in every field."""
    errs = []
    for lev in (2, 3, 4):
        m = _uniform(lev)
        errs.append(_maxwell_error(m, 1 << (lev - 2), "gts", "rk4"))
    errs = np.array(errs)                                     # [level, field]
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates.min() >= 3.5, (errs, rates)


@pytest.mark.slow
def test_maxwell_convergence_ssprk3():
    """SSP-RK3 (the paper's third-order scheme) converges at order >= 2.5."""
    errs = np.array([_maxwell_error(_uniform(lev), 1 << (lev - 2), "gts", "ssprk3") for lev in (2, 3, 4)])
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates.min() >= 2.5, (errs, rates)


def test_maxwell_lts_vs_gts_adaptive():
    """On a two-level mesh, Maxwell LTS differs from GTS by less than GTS's own
    error against the closed form, in every field (LTS at truncation order)."""
    from test_oracle_solver import _adaptive
    m = _adaptive(2, 3)
    assert m.lmax - m.lmin == 1
    c = np.array([0.05, -0.1, 0.15])
    X = physical(node_units(m.anchors, m.levels, m.L), m.L)
    U0 = an.maxwell_gaussian(X, c[None], 0.0, 0.3)
    a = so.run(m, U0, 1, "lts", equation="maxwell", sigma=0.0)
    g = so.run(m, U0, 1, "gts", equation="maxwell", sigma=0.0)
    ex = an.maxwell_gaussian(X, c[None], ot.dt_level(m.lmin), 0.3)
    d = an.norms(a - g, m.levels, m.L)[0]
    eg = an.norms(g - ex, m.levels, m.L)[0]
    assert (d < eg).all(), (d, eg)
