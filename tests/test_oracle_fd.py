"""Pins of the oracle's stencils and interpolant against exactness properties fixed
by the mathematics (Sec. 3.3: high-order FD on padded blocks, c->f interpolation)."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import fd

H = 0.125


def _cube(fun, m=1, h=H, x0=0.3):
    """Padded cube f[z, y, x] of a function on a grid of spacing h."""
    S = 4 * m + 7
    g = x0 + h * (np.arange(S) - 3)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return fun(x, y, z), (x, y, z)


def _inner(a, m=1):
    sl = slice(3, 3 + 4 * m + 1)
    return a[sl, sl, sl]


@pytest.mark.parametrize("d", range(0, 8))
def test_laplacian_exact_to_degree_7(d):
    f, (x, y, z) = _cube(lambda x, y, z: x ** d + 0.5 * y ** d - z ** d)
    ex = d * (d - 1) * (x ** (d - 2) + 0.5 * y ** (d - 2) - z ** (d - 2)) if d >= 2 else 0 * x
    assert np.abs(fd.laplacian6(f, H) - _inner(ex)).max() <= 1e-9 * max(1.0, np.abs(_inner(ex)).max())


def test_laplacian_degree_8_error():
    """x^8: the sixth-order stencil's error is h^6 sum_k c_k k^8 = 72 h^6 exactly."""
    f, (x, y, z) = _cube(lambda x, y, z: x ** 8, x0=0.0)
    err = fd.laplacian6(f, H) - _inner(56 * x ** 6)
    assert np.allclose(err, 72 * H ** 6, rtol=1e-9, atol=0)


@pytest.mark.parametrize("d", range(0, 7))
def test_first_derivative_exact_to_degree_6(d):
    f, (x, y, z) = _cube(lambda x, y, z: y ** d)
    ex = d * y ** (d - 1) if d >= 1 else 0 * y
    assert np.abs(fd.d1_6(f, H, fd.AX_Y) - _inner(ex)).max() <= 1e-10 * max(1.0, np.abs(_inner(ex)).max())


def test_first_derivative_degree_7_error():
    f, (x, y, z) = _cube(lambda x, y, z: z ** 7, x0=0.0)
    err = fd.d1_6(f, H, fd.AX_Z) - _inner(7 * z ** 6)
    assert np.allclose(err, 36 * H ** 6, rtol=1e-9, atol=0)


@pytest.mark.parametrize("d", range(0, 6))
def test_ko_annihilates_degree_5(d):
    f, _ = _cube(lambda x, y, z: x ** d + y ** d * z)
    assert np.abs(fd.ko6(f, H, 0.1)).max() <= 1e-12


def test_ko_degree_6_value_and_sign():
    """delta^6 x^6 = 720 h^6, so KO(x^6) = sigma/(64 h) 720 h^6; the symbol at the
    Nyquist mode is -64 per axis (dissipative)."""
    f, _ = _cube(lambda x, y, z: x ** 6, x0=0.0)
    assert np.allclose(fd.ko6(f, H, 0.1), 0.1 / (64 * H) * 720 * H ** 6, rtol=1e-9)
    k = np.arange(-3, 4)
    assert np.isclose((fd.KO * np.cos(np.pi * k)).sum(), -64.0)


def test_lagrange_half_weights():
    assert fd.lagrange_weights_fr(Fr(1, 2)) == [Fr(35, 128), Fr(140, 128), Fr(-70, 128), Fr(28, 128), Fr(-5, 128)]
    assert fd.lagrange_weights_fr(Fr(3, 2)) == [Fr(-5, 128), Fr(60, 128), Fr(90, 128), Fr(-20, 128), Fr(3, 128)]


@pytest.mark.parametrize("d", range(0, 5))
def test_lagrange_exact_to_degree_4(d):
    for xi2 in range(9):
        w = fd.lagrange_weights_fr(Fr(xi2, 2))
        assert sum(wk * Fr(k) ** d for k, wk in enumerate(w)) == Fr(xi2, 2) ** d


def test_rhs_wave_on_polynomials():
    """u = x^2 y + z^4, v = x^3: du = v + KO(u) = v, dv = Lap u + KO(v) = 2y + 12 z^2."""
    u, (x, y, z) = _cube(lambda x, y, z: x ** 2 * y + z ** 4)
    v, _ = _cube(lambda x, y, z: x ** 3)
    out = fd.rhs_wave(np.stack([u, v]), H, 0.1)
    assert np.abs(out[0] - _inner(x ** 3)).max() < 1e-12
    assert np.abs(out[1] - _inner(2 * y + 12 * z ** 2)).max() < 1e-10


def test_rhs_maxwell_on_polynomials():
    """E = (y^2, z^3, x^4), B = (z, x^2 y, 0): curl B = (0, 1, 2 x y),
    curl E = (-3 z^2, -4 x^3, -2 y)."""
    c = lambda f: _cube(f)[0]
    x, y, z = _cube(lambda x, y, z: x)[1]
    P = np.stack([c(lambda x, y, z: y ** 2), c(lambda x, y, z: z ** 3), c(lambda x, y, z: x ** 4),
                  c(lambda x, y, z: z + 0 * x), c(lambda x, y, z: x ** 2 * y), c(lambda x, y, z: 0 * x)])
    out = fd.rhs_maxwell(P, H, 0.1)
    exp = [0 * x, 1 + 0 * x, 2 * x * y, 3 * z ** 2, 4 * x ** 3, 2 * y]
    for f in range(6):
        assert np.abs(out[f] - _inner(exp[f])).max() < 1e-10, f
