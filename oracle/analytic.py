"""Closed-form solutions and discrete norms (test infrastructure only).

Paper passages:
  * eq. lsm with c = 0 (Sec. 4.2): the linear wave equation, first order in time
    (eqs. chi, phi); its 1D solution chi = (f(x - t) + f(x + t)) / 2.
  * Sec. 4.3: accuracy is measured as the discrete l2 error against the analytic
    solution.  Reading: the l2 norm is volume weighted over the DG nodes,
    sqrt(sum_o W_o^3 sum_n e^2 / (n^3 sum_o W_o^3)), W_o the octant width, n^3 nodes per octant.

The Gaussian pulse u0 = A exp(-r^2/(2 sigma^2)), v0 = 0 evolves as the spherical
wave u = (phi(r+t) + phi(r-t)) / (2r), phi(xi) = xi g(xi) (d'Alembert applied to
r u); on the periodic domain the 27 nearest images are summed.

Vacuum Maxwell (the serving mix's second equation; not in the paper): with Psi
the Gaussian spherical wave above and Phi the wave solution with Phi(0) = 0,
Phi_t(0) = g, i.e. Phi = sigma^2 (g(r - t) - g(r + t)) / (2 r) (so Phi_t = Psi and
Lap Phi = Psi_t),
    E = curl(z Psi) = (d_y Psi, -d_x Psi, 0),   B = -grad(d_z Phi) + z Psi_t
solves dE/dt = curl B, dB/dt = -curl E with div E = div B = 0, and starts from
E = curl(z g), B = 0.  A plane wave E = e sin(k.x - |k| t), B = (k/|k| x e)
sin(k.x - |k| t), e.k = 0, is the second closed form.

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


# ----------------------------------------------------------------------------- Maxwell
def _gauss_derivs(xi, sigma, amp, nmax):
    """g^(n)(xi), n = 0..nmax, for g = amp exp(-xi^2 / (2 sigma^2)):
    g^(n) = (-1/sigma)^n He_n(xi/sigma) g with the probabilists' Hermite
    polynomials He_0 = 1, He_1 = x, He_(n+1) = x He_n - n He_(n-1)."""
    x = xi / sigma
    g = amp * np.exp(-0.5 * x * x)
    he = [np.ones_like(x), x]
    for n in range(1, nmax):
        he.append(x * he[n] - n * he[n - 1])
    return [(-1.0 / sigma) ** n * he[n] * g for n in range(nmax + 1)]


#: radius below which the radial factors are summed as Taylor series (in sigma)
_SERIES_R = 0.5
_SERIES_K = 16


def _radial_factors(r, t, sigma, amp):
    """Radial factors of one image at distance r: Psi_r / r, Psi_t, Phi_r / r and
    (Phi_rr - Phi_r / r) / r^2, for Psi = N / (2r), N = phi(r+t) + phi(r-t),
    phi = xi g, and Phi = M / (2r), M = sigma^2 (g(r-t) - g(r+t)).

    With N' etc. the r-derivatives: Psi_r / r = (r N' - N) / (2 r^3) and
    (Phi_rr - Phi_r/r) / r^2 = (r^2 M'' - 3 r M' + 3 M) / (2 r^5).  Near r = 0 these
    cancel; there the odd series N = sum_k n_k r^(2k+1) gives
    sum_(k>=1) k n_k r^(2k-2) and sum_(k>=2) 2k(k-1) n_k r^(2k-4)."""
    r = np.asarray(r, dtype=np.float64)
    out = [np.zeros_like(r) for _ in range(4)]
    far = r >= _SERIES_R * sigma
    if far.any():
        rf = r[far]
        gp = _gauss_derivs(rf + t, sigma, amp, 3)
        gm = _gauss_derivs(rf - t, sigma, amp, 3)
        # phi^(n) = xi g^(n) + n g^(n-1)
        def ph(gd, xi, n):
            return xi * gd[n] + (n * gd[n - 1] if n > 0 else 0.0)
        N = ph(gp, rf + t, 0) + ph(gm, rf - t, 0)
        N1 = ph(gp, rf + t, 1) + ph(gm, rf - t, 1)
        V = ph(gp, rf + t, 1) - ph(gm, rf - t, 1)          # phi'(r+t) - phi'(r-t)
        s2 = sigma * sigma
        M = s2 * (gm[0] - gp[0])
        M1 = s2 * (gm[1] - gp[1])
        M2 = s2 * (gm[2] - gp[2])
        out[0][far] = (rf * N1 - N) / (2.0 * rf ** 3)
        out[1][far] = V / (2.0 * rf)
        out[2][far] = (rf * M1 - M) / (2.0 * rf ** 3)
        out[3][far] = (rf * rf * M2 - 3.0 * rf * M1 + 3.0 * M) / (2.0 * rf ** 5)
    near = ~far
    if near.any():
        from math import factorial
        rn = r[near]
        K = _SERIES_K
        tt = np.full_like(rn, float(t))
        gd = _gauss_derivs(tt, sigma, amp, 2 * K + 5)
        s2 = sigma * sigma

        def phd(n):                                      # phi^(n)(t) = t g^(n) + n g^(n-1)
            return tt * gd[n] + n * gd[n - 1]

        def n_(k):                                       # N = sum_k n_k r^(2k+1)
            return 2.0 * phd(2 * k + 1) / float(factorial(2 * k + 1))

        def m_(k):                                       # M = sum_k m_k r^(2k+1)
            return -2.0 * s2 * gd[2 * k + 1] / float(factorial(2 * k + 1))

        def v_(k):                                       # Psi_t = sum_k v_k r^(2k)
            return phd(2 * k + 2) / float(factorial(2 * k + 1))

        coef = [[(j + 1) * n_(j + 1) for j in range(K + 1)],
                [v_(j) for j in range(K + 1)],
                [(j + 1) * m_(j + 1) for j in range(K + 1)],
                [2.0 * (j + 2) * (j + 1) * m_(j + 2) for j in range(K + 1)]]
        r2 = rn * rn
        for i in range(4):
            acc = np.zeros_like(rn)
            for j in range(K, -1, -1):                   # Horner in r^2
                acc = acc * r2 + coef[i][j]
            out[i][near] = acc
    return out


def maxwell_gaussian(x: np.ndarray, centres: np.ndarray, t: float, sigma: float, amp: float = 1.0):
    """(E, B) = [6, ...] of the Gaussian-potential Maxwell solution at time t, summed
    over the pulses and their 27 nearest periodic images.  x: [..., 3]."""
    out = np.zeros((6,) + x.shape[:-1])
    for c in np.atleast_2d(centres):
        for im in IMAGES:
            d = x - (c + im)
            r = np.sqrt((d * d).sum(axis=-1))
            p_psi, psi_t, s_phi, q_phi = _radial_factors(r, t, sigma, amp)
            dx, dy, dz = d[..., 0], d[..., 1], d[..., 2]
            out[0] += p_psi * dy
            out[1] -= p_psi * dx
            out[3] -= q_phi * dx * dz
            out[4] -= q_phi * dy * dz
            out[5] += psi_t - (q_phi * dz * dz + s_phi)
    return out


def maxwell_plane(x: np.ndarray, n, e, t: float):
    """E = e sin(k.x - |k| t), B = (k/|k| x e) sin(k.x - |k| t), k = pi n, e.k = 0."""
    k = np.pi * np.asarray(n, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    w = np.linalg.norm(k)
    bvec = np.cross(k / w, e)
    s = np.sin((x * k).sum(axis=-1) - w * t)
    return np.stack([e[i] * s for i in range(3)] + [bvec[i] * s for i in range(3)])


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
    """Per field volume-weighted l2 and max norms of err [F][N][n][n][n]."""
    w = (2.0 ** (L - np.asarray(levels, dtype=np.float64))) ** 3
    e2 = (err.reshape(err.shape[0], err.shape[1], -1) ** 2).sum(axis=2)      # [F, N]
    nn = err.reshape(err.shape[0], err.shape[1], -1).shape[2]                 # nodes per octant
    l2 = np.sqrt((e2 * w[None, :]).sum(axis=1) / (nn * w.sum()))
    linf = np.abs(err).reshape(err.shape[0], -1).max(axis=1)
    return l2, linf


def nlwave_radial(profile, T: float, r_max: float = 2.0, n: int = 2000, c_nl: float = 1.0):
    """Spherically symmetric solution of the non-linear wave (Sec. 4.2, eqs. lsm,
    chi, phi) from chi(r, 0) = profile(r), chi_t(r, 0) = 0, by a method independent
    of the octree solver: with u = r chi the radial equation reads
        u_tt = u_rr - c sin(2 u / r) / r,   u odd in r (u(0) = 0),
    discretised with sixth-order centred differences on r_i = i dr (odd reflection
    at r = 0, zero beyond r_max, which the data must not reach by T) and classic RK4
    with dt = dr / 4.  Returns (r, chi(r, T)) on the grid r_i, i >= 1."""
    dr = r_max / n
    r = dr * np.arange(n + 1)
    u = r * profile(r)
    u[0] = 0.0
    w = np.zeros_like(u)
    c2 = np.array([1 / 90, -3 / 20, 3 / 2, -49 / 18, 3 / 2, -3 / 20, 1 / 90])

    def acc(u):
        ext = np.concatenate([-u[3:0:-1], u, np.zeros(3)])        # odd at r = 0
        urr = sum(c2[k] * ext[k:k + n + 1] for k in range(7)) / (dr * dr)
        src = np.zeros_like(u)
        src[1:] = np.sin(2.0 * u[1:] / r[1:]) / r[1:]
        return urr - c_nl * src

    dt = dr / 4.0
    steps = int(round(T / dt))
    assert abs(steps * dt - T) < 1e-12 * max(T, 1.0)
    for _ in range(steps):
        k1u, k1w = w, acc(u)
        k2u, k2w = w + 0.5 * dt * k1w, acc(u + 0.5 * dt * k1u)
        k3u, k3w = w + 0.5 * dt * k2w, acc(u + 0.5 * dt * k2u)
        k4u, k4w = w + dt * k3w, acc(u + dt * k3u)
        u = u + dt / 6.0 * (k1u + 2 * k2u + 2 * k3u + k4u)
        w = w + dt / 6.0 * (k1w + 2 * k2w + 2 * k3w + k4w)
    return r[1:], u[1:] / r[1:]
