"""Closed-form solutions and discrete norms (test infrastructure only).

Paper passages:
  * eq. lsm with c = 0 (Sec. 4.2): the linear wave equation, first order in time
    (eqs. chi, phi); its 1D solution chi = (f(x - t) + f(x + t)) / 2.
  * Sec. 4.3: accuracy is measured as the discrete l2 error against the analytic
    solution.  Reading: the l2 norm is volume weighted over the DG nodes,
    sqrt(sum_o W_o^3 sum_n e^2 / (125 sum_o W_o^3)), W_o the octant width.

The Gaussian pulse u0 = A exp(-r^2/(2 sigma^2)), v0 = 0 evolves as the spherical
wave u = (phi(r+t) + phi(r-t)) / (2r), phi(xi) = xi g(xi) (d'Alembert applied to
r u); on the periodic domain the 27 nearest images are summed.

For a Fourier mode on a uniform periodic grid the discrete scheme has a closed
form: with the symbols lam (sixth-order Laplacian) and kap (Kreiss-Oliger term)
the semi-discrete system is d/dt (u^, v^) = [[kap, 1], [lam, kap]] (u^, v^), and
one RK step multiplies by the stability polynomial R(dt M).
"""
from __future__ import annotations

from math import factorial

import numpy as np

from .fd import D2, KO

IMAGES = np.array([(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)], dtype=np.float64) * 2.0


# ----------------------------------------------------------------------------- Gaussian
def _g(xi, sigma, amp):
    return amp * np.exp(-xi * xi / (2.0 * sigma * sigma))


def _phi(xi, sigma, amp):
    return xi * _g(xi, sigma, amp)


def _dphi(xi, sigma, amp):
    return _g(xi, sigma, amp) * (1.0 - xi * xi / sigma ** 2)


def _d2phi(xi, sigma, amp):
    s2 = sigma * sigma
    return _g(xi, sigma, amp) * (xi ** 3 / s2 ** 2 - 3.0 * xi / s2)


def _d3phi(xi, sigma, amp):
    s2 = sigma * sigma
    return _g(xi, sigma, amp) * (-xi ** 4 / s2 ** 3 + 6.0 * xi * xi / s2 ** 2 - 3.0 / s2)


def spherical_wave(x: np.ndarray, centre: np.ndarray, t: float, sigma: float, amp: float = 1.0):
    """(u, v) of a Gaussian pulse at rest at time t, one image.  x: [..., 3]."""
    d = x - centre
    r = np.sqrt((d * d).sum(axis=-1))
    small = r < 1e-4
    rs = np.where(small, 1.0, r)
    u = (_phi(rs + t, sigma, amp) + _phi(rs - t, sigma, amp)) / (2.0 * rs)
    v = (_dphi(rs + t, sigma, amp) - _dphi(rs - t, sigma, amp)) / (2.0 * rs)
    # r -> 0: u = phi'(t) + r^2 phi'''(t)/6, v = phi''(t) (+O(r^2))
    u0 = _dphi(t, sigma, amp) + r * r * _d3phi(t, sigma, amp) / 6.0
    v0 = _d2phi(t, sigma, amp)
    return np.where(small, u0, u), np.where(small, v0, v)


def gaussian_periodic(x: np.ndarray, centres: np.ndarray, t: float, sigma: float, amp: float = 1.0):
    u = np.zeros(x.shape[:-1])
    v = np.zeros(x.shape[:-1])
    for c in np.atleast_2d(centres):
        for im in IMAGES:
            du, dv = spherical_wave(x, c + im, t, sigma, amp)
            u += du
            v += dv
    return np.stack([u, v])


def plane_wave(x: np.ndarray, n, t: float):
    k = np.pi * np.asarray(n, dtype=np.float64)
    w = np.linalg.norm(k)
    ph = (x * k).sum(axis=-1) - w * t
    return np.stack([np.sin(ph), -w * np.cos(ph)])


def wave_1d(x: np.ndarray, f, t: float):
    """The paper's 1D form (Sec. 4.2): chi = (f(x - t) + f(x + t)) / 2."""
    return 0.5 * (f(x - t) + f(x + t))


# ----------------------------------------------------------------------------- Fourier
def symbol_d2(theta: float) -> float:
    """sum_j D2_j e^{i j theta} (real) for the sixth-order second derivative."""
    return float(sum(D2[j + 3] * np.cos(j * theta) for j in range(-3, 4)))


def symbol_ko(theta: float) -> float:
    return float(sum(KO[j + 3] * np.cos(j * theta) for j in range(-3, 4)))


def rk_polynomial(order: int, z: np.ndarray) -> np.ndarray:
    """Stability function of a p-stage RK method of order p = p on linear problems
    (classic RK4, SSP-RK3): the truncated exponential sum_{j<=p} Z^j / j!."""
    n = z.shape[0]
    R = np.eye(n)
    term = np.eye(n)
    for j in range(1, order + 1):
        term = term @ z / j
        R = R + term
    return R


def fourier_mode_solution(order: int, n, h: float, dt: float, nsteps: int, sigma_ko: float):
    """Amplitudes (u^, v^) after nsteps of the fully discrete scheme for
    u0 = cos(pi n . x), v0 = 0 on a uniform periodic grid of spacing h."""
    lam = sum(symbol_d2(np.pi * nd * h) for nd in n) / (h * h)
    kap = sigma_ko / (64.0 * h) * sum(symbol_ko(np.pi * nd * h) for nd in n)
    M = np.array([[kap, 1.0], [lam, kap]])
    R = rk_polynomial(order, dt * M)
    y = np.array([1.0, 0.0])
    for _ in range(nsteps):
        y = R @ y
    return y


# ----------------------------------------------------------------------------- norms
def norms(err: np.ndarray, levels: np.ndarray, L: int):
    """Per field volume-weighted l2 and max norms of err [F][N][5][5][5]."""
    w = (2.0 ** (L - np.asarray(levels, dtype=np.float64))) ** 3
    e2 = (err.reshape(err.shape[0], err.shape[1], -1) ** 2).sum(axis=2)      # [F, N]
    l2 = np.sqrt((e2 * w[None, :]).sum(axis=1) / (125.0 * w.sum()))
    linf = np.abs(err).reshape(err.shape[0], -1).max(axis=1)
    return l2, linf
