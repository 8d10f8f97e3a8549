"""Finite-difference stencils and the c->f interpolant (test infrastructure only).

The paper uses high-order central differences on padded blocks (Sec. 3.3) but
prints no stencil.  Readings:
  * second derivative: sixth-order central, weights (1/90, -3/20, 3/2, -49/18,
    3/2, -3/20, 1/90) / h^2 per axis;
  * first derivative:  sixth-order central, (-1/60, 3/20, -3/4, 0, 3/4, -3/20,
    1/60) / h;
  * Kreiss-Oliger dissipation (not in the paper): + sigma/(64 h) * (1, -6, 15,
    -20, 15, -6, 1) per axis, i.e. sigma h^5 / 64 * D+^3 D-^3, which is
    non-positive in Fourier space (dissipative) and fits three ghost layers;
  * coarse->fine interpolation (Sec. 3.3 "coarser to finer interpolation"):
    tensor degree-4 Lagrange on the coarse leaf's own 5 nodes per axis.
All weights are exact rationals converted by one correctly rounded division.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from typing import List

import numpy as np

D2_FR = [Fr(1, 90), Fr(-3, 20), Fr(3, 2), Fr(-49, 18), Fr(3, 2), Fr(-3, 20), Fr(1, 90)]
D1_FR = [Fr(-1, 60), Fr(3, 20), Fr(-3, 4), Fr(0), Fr(3, 4), Fr(-3, 20), Fr(1, 60)]
KO_FR = [Fr(1), Fr(-6), Fr(15), Fr(-20), Fr(15), Fr(-6), Fr(1)]

D2 = np.array([float(x) for x in D2_FR])
D1 = np.array([float(x) for x in D1_FR])
KO = np.array([float(x) for x in KO_FR])


def lagrange_weights_fr(xi: Fr, n: int = 5) -> List[Fr]:
    """Weights of the degree n-1 Lagrange interpolant on nodes 0..n-1 at xi."""
    xi = Fr(xi)
    w = []
    for k in range(n):
        num, den = Fr(1), Fr(1)
        for m in range(n):
            if m != k:
                num *= xi - m
                den *= k - m
        w.append(num / den)
    return w


def lagrange_weights(xi2: int) -> np.ndarray:
    """float64 weights for the position xi = xi2 / 2 (xi2 integer in [0, 8])."""
    return np.array([float(x) for x in lagrange_weights_fr(Fr(int(xi2), 2))])


def _axis_stencil(f: np.ndarray, w: np.ndarray, axis: int, m4: int) -> np.ndarray:
    """sum_k w[k] f[.. c+k-3 ..] on the interior [3, 3+m4] of a padded axis."""
    out = None
    for k in range(7):
        if w[k] == 0.0:
            continue
        sl = [slice(3, 3 + m4 + 1)] * 3
        sl[axis] = slice(k, k + m4 + 1)
        term = w[k] * f[tuple(sl)]
        out = term if out is None else out + term
    return out


def laplacian6(f: np.ndarray, h: float) -> np.ndarray:
    """Sixth-order Laplacian on the interior of a padded cube f[z, y, x]."""
    m4 = f.shape[0] - 7
    return sum(_axis_stencil(f, D2, ax, m4) for ax in range(3)) / (h * h)


def d1_6(f: np.ndarray, h: float, axis: int) -> np.ndarray:
    m4 = f.shape[0] - 7
    return _axis_stencil(f, D1, axis, m4) / h


def ko6(f: np.ndarray, h: float, sigma: float) -> np.ndarray:
    m4 = f.shape[0] - 7
    return (sigma / (64.0 * h)) * sum(_axis_stencil(f, KO, ax, m4) for ax in range(3))


AX_X, AX_Y, AX_Z = 2, 1, 0   # array axes of a [z, y, x] cube


def rhs_wave(padded: np.ndarray, h: float, sigma: float) -> np.ndarray:
    """First-order-in-time wave system (eqs. chi, phi with c = 0):
    du/dt = v + KO(u),  dv/dt = Lap u + KO(v).  padded: [2, S, S, S]."""
    u, v = padded[0], padded[1]
    m4 = u.shape[0] - 7
    inner = (slice(3, 3 + m4 + 1),) * 3
    du = v[inner] + ko6(u, h, sigma)
    dv = laplacian6(u, h) + ko6(v, h, sigma)
    return np.stack([du, dv])


def rhs_maxwell(padded: np.ndarray, h: float, sigma: float) -> np.ndarray:
    """Vacuum Maxwell, fields (Ex, Ey, Ez, Bx, By, Bz):
    dE/dt = curl B + KO(E),  dB/dt = -curl E + KO(B)."""
    Ex, Ey, Ez, Bx, By, Bz = padded

    def curl(Fx, Fy, Fz):
        return (d1_6(Fz, h, AX_Y) - d1_6(Fy, h, AX_Z),
                d1_6(Fx, h, AX_Z) - d1_6(Fz, h, AX_X),
                d1_6(Fy, h, AX_X) - d1_6(Fx, h, AX_Y))

    cB = curl(Bx, By, Bz)
    cE = curl(Ex, Ey, Ez)
    out = [cB[0] + ko6(Ex, h, sigma), cB[1] + ko6(Ey, h, sigma), cB[2] + ko6(Ez, h, sigma),
           -cE[0] + ko6(Bx, h, sigma), -cE[1] + ko6(By, h, sigma), -cE[2] + ko6(Bz, h, sigma)]
    return np.stack(out)


EQUATIONS = {"wave": (2, rhs_wave), "maxwell": (6, rhs_maxwell)}
