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
    tensor degree n-1 Lagrange on the coarse leaf's own n nodes per axis (n = 5
    or 7 nodes per octant side);
  * on a bounded domain (the non-linear wave with radiative boundary of
    Sec. 4.2): centred stencils of reduced order next to the faces and one-sided
    fourth-order first differences on them (the paper gives the radiative
    condition, not its discretisation).
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


def lagrange_weights(xi2: int, n: int = 5) -> np.ndarray:
    """float64 weights on nodes 0..n-1 for the position xi = xi2 / 2 (xi2 integer
    in [0, 2n-2])."""
    return np.array([float(x) for x in lagrange_weights_fr(Fr(int(xi2), 2), n)])


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


def rhs_wave(padded: np.ndarray, h: float, sigma: float, geo: dict = None) -> np.ndarray:
    """First-order-in-time wave system (eqs. chi, phi with c = 0):
    du/dt = v + KO(u),  dv/dt = Lap u + KO(v).  padded: [2, S, S, S]."""
    u, v = padded[0], padded[1]
    m4 = u.shape[0] - 7
    inner = (slice(3, 3 + m4 + 1),) * 3
    du = v[inner] + ko6(u, h, sigma)
    dv = laplacian6(u, h) + ko6(v, h, sigma)
    return np.stack([du, dv])


def rhs_maxwell(padded: np.ndarray, h: float, sigma: float, geo: dict = None) -> np.ndarray:
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


# ----------------------------------------------------------------------------- outer boundary
# Stencils that stay inside a bounded domain.  On a bounded domain a grid point
# at d grid steps from the nearest face (per axis) uses the widest centred
# stencil that fits: sixth order for d >= 3, fourth for d = 2, second for d = 1;
# Kreiss-Oliger only along axes with d >= 3.  A point on a face (d = 0) takes the
# radiative condition instead of the evolution equation, with one-sided
# fourth-order first differences along the axes where it sits on a face.
D2_4_FR = [Fr(0), Fr(-1, 12), Fr(4, 3), Fr(-5, 2), Fr(4, 3), Fr(-1, 12), Fr(0)]
D2_2_FR = [Fr(0), Fr(0), Fr(1), Fr(-2), Fr(1), Fr(0), Fr(0)]
D1_4_FR = [Fr(0), Fr(1, 12), Fr(-2, 3), Fr(0), Fr(2, 3), Fr(-1, 12), Fr(0)]
D1_2_FR = [Fr(0), Fr(0), Fr(-1, 2), Fr(0), Fr(1, 2), Fr(0), Fr(0)]
D1_SIDE_FR = [Fr(-25, 12), Fr(4), Fr(-3), Fr(4, 3), Fr(-1, 4)]    # offsets 0..4 into the domain
D2_4, D2_2 = (np.array([float(x) for x in w]) for w in (D2_4_FR, D2_2_FR))
D1_4, D1_2 = (np.array([float(x) for x in w]) for w in (D1_4_FR, D1_2_FR))
D1_SIDE = np.array([float(x) for x in D1_SIDE_FR])

#: exponents k of the radiative condition (f - f0 ~ 1/r^k far out), f0 = 0
RADIATIVE_K = (1.0, 2.0)


def face_distance(geo: dict, G: int):
    """Per axis (x, y, z): grid steps from each block grid point to the nearest
    outer face (a large number on a periodic domain), and the side of the face a
    point on it lies on (+1 low face, -1 high face, 0 otherwise)."""
    X0, w, Nu = geo["X0"], geo["w"], geo["Nu"]
    dist, side = [], []
    for a in range(3):
        X = X0[a] + w * np.arange(G, dtype=np.int64)
        if geo["periodic"]:
            dist.append(np.full(G, 1 << 20, dtype=np.int64))
            side.append(np.zeros(G, dtype=np.int64))
        else:
            dist.append(np.minimum(X, Nu - X) // w)
            side.append(np.where(X == 0, 1, np.where(X == Nu, -1, 0)))
    return dist, side


def node_coordinates(geo: dict, G: int):
    """Physical coordinates x = -1 + 2 X / Nu of the block grid along x, y, z."""
    return [-1.0 + 2.0 * (geo["X0"][a] + geo["w"] * np.arange(G, dtype=np.int64)) / geo["Nu"] for a in range(3)]


def _select_axis(values: dict, d: np.ndarray, axis: int, G: int):
    """Per grid point, the entry of `values` (keyed by minimum distance 3, 2, 1)
    chosen by the point's distance d along the array axis `axis`."""
    shape = [1, 1, 1]
    shape[axis] = G
    dd = d.reshape(shape)
    out = np.where(dd >= 3, values[3], np.where(dd == 2, values[2], values[1]))
    return out


def _one_sided(f: np.ndarray, axis: int, m4: int, side: int) -> np.ndarray:
    """Fourth-order one-sided first difference (times h) along `axis` on the block
    grid: forward (side +1, offsets 0..4) or backward (side -1, offsets 0..-4).
    The padded cube is extended by zeros so that every grid point has a window;
    only the face points, whose window lies inside the domain, are used."""
    ext = np.pad(f, [(4, 4) if a == axis else (0, 0) for a in range(3)])
    out = 0.0
    for k in range(5):
        sl = [slice(3, 3 + m4 + 1)] * 3
        start = 4 + 3 + side * k
        sl[axis] = slice(start, start + m4 + 1)
        out = out + (side * D1_SIDE[k]) * ext[tuple(sl)]
    return out


def _d1_bounded(f, h, axis, m4, dist, side):
    """First derivative along array axis `axis` with the bounded-domain stencils:
    centred of the widest order that fits, one-sided on the faces."""
    G = m4 + 1
    c = {3: _axis_stencil(f, D1, axis, m4), 2: _axis_stencil(f, D1_4, axis, m4), 1: _axis_stencil(f, D1_2, axis, m4)}
    out = _select_axis(c, dist, axis, G)
    if (side != 0).any():
        shape = [1, 1, 1]
        shape[axis] = G
        sd = side.reshape(shape)
        out = np.where(sd > 0, _one_sided(f, axis, m4, 1), np.where(sd < 0, _one_sided(f, axis, m4, -1), out))
    return out / h


def rhs_nlwave(padded: np.ndarray, h: float, sigma: float, geo: dict, c_nl: float = 1.0) -> np.ndarray:
    """Non-linear wave system of Sec. 4.2 (eqs. lsm, chi, phi):
        dchi/dt = phi + KO(chi),
        dphi/dt = Lap chi - c sin(2 chi) / r^2 + KO(phi),   r = |x|,
    with c != 0 the node r = 0 holding the regularity condition chi = 0 (a
    regular solution of the source behaves like chi ~ a(t) r there, so its
    state does not change; the data must vanish there); on a bounded domain
    the widest centred stencils that fit near the
    faces, and on the faces the radiative (outgoing-wave) condition
        df/dt = -(x . grad f) / r - k f / r,   k = 1 (chi), 2 (phi), f0 = 0.
    padded: [2, S, S, S]; geo: block geometry (solver.State.geometry)."""
    chi, phi = padded[0], padded[1]
    m4 = chi.shape[0] - 7
    G = m4 + 1
    inner = (slice(3, 3 + m4 + 1),) * 3
    dist, side = face_distance(geo, G)          # per axis x, y, z
    arr_axis = (AX_X, AX_Y, AX_Z)
    lap = 0.0
    ko_c = 0.0
    ko_p = 0.0
    for A in range(3):                 # array axes z, y, x (the order of rhs_wave's sums)
        a = arr_axis.index(A)
        c2 = {3: _axis_stencil(chi, D2, A, m4), 2: _axis_stencil(chi, D2_4, A, m4), 1: _axis_stencil(chi, D2_2, A, m4)}
        lap = lap + _select_axis(c2, dist[a], A, G)
        kc = _axis_stencil(chi, KO, A, m4)
        kp = _axis_stencil(phi, KO, A, m4)
        zero = np.zeros_like(kc)
        ko_c = ko_c + _select_axis({3: kc, 2: zero, 1: zero}, dist[a], A, G)
        ko_p = ko_p + _select_axis({3: kp, 2: zero, 1: zero}, dist[a], A, G)
    x1 = node_coordinates(geo, G)
    xz, xy, xx = np.meshgrid(x1[2], x1[1], x1[0], indexing="ij")
    r2 = xx * xx + xy * xy + xz * xz
    c = chi[inner]
    lapn = lap / (h * h)
    src = np.where(r2 > 0.0, np.sin(2.0 * c) / np.where(r2 > 0.0, r2, 1.0), 0.0)
    kos = sigma / (64.0 * h)
    dchi = phi[inner] + kos * ko_c
    dphi = lapn - c_nl * src + kos * ko_p
    if c_nl != 0.0:
        # the node r = 0 holds the regularity condition of the source, chi = 0:
        # its state does not change
        dchi = np.where(r2 > 0.0, dchi, 0.0)
        dphi = np.where(r2 > 0.0, dphi, 0.0)
    # points on a face: radiative condition
    on_face = np.zeros((G, G, G), dtype=bool)
    for a in range(3):
        shape = [1, 1, 1]
        shape[arr_axis[a]] = G
        on_face |= (dist[a] == 0).reshape(shape)
    if on_face.any():
        r = np.sqrt(r2)
        xs = (xx, xy, xz)
        for f_idx, (fld, k) in enumerate(((chi, RADIATIVE_K[0]), (phi, RADIATIVE_K[1]))):
            xgrad = 0.0
            for a in range(3):
                xgrad = xgrad + xs[a] * _d1_bounded(fld, h, arr_axis[a], m4, dist[a], side[a])
            rad = -xgrad / np.where(on_face, r, 1.0) - k * fld[inner] / np.where(on_face, r, 1.0)
            if f_idx == 0:
                dchi = np.where(on_face, rad, dchi)
            else:
                dphi = np.where(on_face, rad, dphi)
    return np.stack([dchi, dphi])


EQUATIONS = {"wave": (2, rhs_wave), "maxwell": (6, rhs_maxwell), "nlwave": (2, rhs_nlwave)}
