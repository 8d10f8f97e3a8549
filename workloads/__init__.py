"""Seeded synthetic inputs shared by the library's tests/benchmarks and the oracle.

This package holds no arithmetic of the method (no stencil, interpolation,
time-stepping or mesh logic).  It provides
  * the frozen mesh specifications of the benchmark configurations (integer
    refinement radii in node units, calibrated once by ``calibrate.py`` beside
    this file and then stored here),
  * seeded pulse centres,
  * initial data evaluated at octant-local node coordinates of a given leaf list
    (Gaussian pulse, plane wave, divergence-free Maxwell data, the non-linear
    wave's shell),
  * seeded random DG arrays for kernel unit tests.

Coordinates: level-L node units, N_u = ni * 2^L per side, x = -1 + 2 X / N_u,
with n = 5 (default) or 7 nodes per octant side and ni = n - 1; a leaf (anchor a
in level-L octant units, level l) has nodes ni a + i 2^(L-l), i = 0..ni.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------- coordinates
def node_units(anchors: np.ndarray, levels: np.ndarray, L: int, nodes: int = 5) -> np.ndarray:
    """Integer node coordinates [N, n, n, n, 3] (x, y, z), node index [k][j][i]."""
    anchors = np.asarray(anchors, dtype=np.int64)
    s = (1 << (L - np.asarray(levels, dtype=np.int64)))
    i = np.arange(nodes, dtype=np.int64)
    k_, j_, i_ = np.meshgrid(i, i, i, indexing="ij")
    loc = np.stack([i_, j_, k_], axis=-1)[None]                   # [1,n,n,n,3]
    return (nodes - 1) * anchors[:, None, None, None, :] + loc * s[:, None, None, None, None]


def physical(X: np.ndarray, L: int, nodes: int = 5) -> np.ndarray:
    return -1.0 + 2.0 * X.astype(np.float64) / float((nodes - 1) * (1 << L))


def centre_from_seed(seed: int, L: int, lo: float = -0.5, hi: float = 0.5, nodes: int = 5) -> List[int]:
    """Pulse centre ~ U([lo, hi]^3) from numpy's default_rng(seed), snapped to node units."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(lo, hi, size=3)
    n = (nodes - 1) * (1 << L)
    return [int(round((v + 1.0) * 0.5 * n)) % n for v in x]


def centre_physical(c: Sequence[int], L: int, nodes: int = 5) -> np.ndarray:
    return -1.0 + 2.0 * np.asarray(c, dtype=np.float64) / float((nodes - 1) * (1 << L))


IMAGES = np.array([(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)], dtype=np.float64) * 2.0


# ----------------------------------------------------------------------------- initial data
def gaussian(x: np.ndarray, centres: np.ndarray, sigma: float, amp: float = 1.0) -> np.ndarray:
    """sum over pulses and the 27 nearest periodic images of amp exp(-r^2 / (2 sigma^2))."""
    out = np.zeros(x.shape[:-1])
    for c in np.atleast_2d(centres):
        for im in IMAGES:
            d = x - (c + im)
            out += amp * np.exp(-(d * d).sum(axis=-1) / (2.0 * sigma * sigma))
    return out


def wave_gaussian(anchors, levels, L, centres_nu, sigma=0.1, amp=1.0, nodes: int = 5) -> np.ndarray:
    """Wave-equation data (u, v) = (Gaussian, 0): [2, N, n, n, n]."""
    x = physical(node_units(anchors, levels, L, nodes), L, nodes)
    c = np.stack([centre_physical(cc, L, nodes) for cc in centres_nu])
    u = gaussian(x, c, sigma, amp)
    return np.stack([u, np.zeros_like(u)])


def wave_plane(anchors, levels, L, n=(1, 0, 0), nodes: int = 5) -> np.ndarray:
    """(u, v) = (sin(k.x), -|k| cos(k.x)), k = pi n: a periodic travelling wave."""
    x = physical(node_units(anchors, levels, L, nodes), L, nodes)
    k = np.pi * np.asarray(n, dtype=np.float64)
    ph = (x * k).sum(axis=-1)
    return np.stack([np.sin(ph), -np.linalg.norm(k) * np.cos(ph)])


def maxwell_gaussian(anchors, levels, L, centres_nu, sigma=0.1, amp=1.0) -> np.ndarray:
    """E = curl(z psi) = (d_y psi, -d_x psi, 0), B = 0 with psi a Gaussian: [6, N, 5, 5, 5]."""
    x = physical(node_units(anchors, levels, L), L)
    ex = np.zeros(x.shape[:-1])
    ey = np.zeros(x.shape[:-1])
    for cc in centres_nu:
        c = centre_physical(cc, L)
        for im in IMAGES:
            d = x - (c + im)
            g = amp * np.exp(-(d * d).sum(axis=-1) / (2.0 * sigma * sigma))
            ex += -d[..., 1] / (sigma * sigma) * g
            ey += d[..., 0] / (sigma * sigma) * g
    z = np.zeros_like(ex)
    return np.stack([ex, ey, z, z, z.copy(), z.copy()])


def nlwave_shell(anchors, levels, L, radius=0.5, sigma=0.1, amp=1.0) -> np.ndarray:
    """Non-linear wave data (chi, phi) = (amp (r/R)^2 exp(-(r - R)^2 / (2 sigma^2)), 0),
    r = |x|: a spherical shell around the origin (no images), even in r and
    vanishing at r = 0 like r^2, as a regular solution does: [2, N, 5, 5, 5]."""
    x = physical(node_units(anchors, levels, L), L)
    r2 = (x * x).sum(axis=-1)
    chi = shell_profile(np.sqrt(r2), radius, sigma, amp)
    return np.stack([chi, np.zeros_like(chi)])


def shell_profile(r, radius=0.5, sigma=0.1, amp=1.0):
    """The radial profile of nlwave_shell."""
    r = np.asarray(r, dtype=np.float64)
    return amp * (r / radius) ** 2 * np.exp(-(r - radius) ** 2 / (2.0 * sigma * sigma))


def random_dg(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape) * scale


def consistent_random_dg(anchors, levels, L, nfields: int, seed: int, nodes: int = 5) -> np.ndarray:
    """Random smooth-free data whose duplicated DG nodes agree: a random value per
    distinct node coordinate (hash of the integer coordinate)."""
    X = node_units(anchors, levels, L, nodes)
    n = (nodes - 1) * (1 << L)
    key = (X[..., 0] % n) + n * ((X[..., 1] % n) + n * (X[..., 2] % n))
    out = []
    for f in range(nfields):
        rng = np.random.default_rng(seed * 1000 + f)
        uniq, inv = np.unique(key.ravel(), return_inverse=True)
        vals = rng.standard_normal(len(uniq))
        out.append(vals[inv.reshape(-1)].reshape(key.shape))
    return np.stack(out)


# ----------------------------------------------------------------------------- configurations
def _load_specs() -> Dict[str, dict]:
    with open(os.path.join(_HERE, "specs.json")) as f:
        return json.load(f)


def mesh_spec(name: str) -> dict:
    """Frozen mesh specification (dict) of a named configuration."""
    return _load_specs()[name]["mesh"]


def config(name: str) -> dict:
    return _load_specs()[name]


def config_names() -> List[str]:
    return list(_load_specs().keys())


def _nodes_torch(leaves: np.ndarray, L: int, device, nodes: int = 5):
    """Physical coordinates [N, n^3, 3] of every DG node (torch, float64)."""
    import torch
    lv = torch.as_tensor(np.asarray(leaves), dtype=torch.int64, device=device)
    s = torch.bitwise_left_shift(torch.ones_like(lv[:, 3]), L - lv[:, 3]).to(torch.float64)
    i = torch.arange(nodes, dtype=torch.float64, device=device)
    k_, j_, i_ = torch.meshgrid(i, i, i, indexing="ij")
    loc = torch.stack([i_, j_, k_], -1).reshape(nodes ** 3, 3)
    X = float(nodes - 1) * lv[:, None, :3].to(torch.float64) + loc[None] * s[:, None, None]       # [N,n^3,3]
    return -1.0 + 2.0 * X / float((nodes - 1) * (1 << L))


def wave_gaussian_torch(leaves: np.ndarray, L: int, centres_nu, sigma=0.1, amp=1.0, device="cuda", nodes: int = 5):
    """Same data as wave_gaussian, evaluated with torch on `device` (large meshes).
    leaves: int [N, 4] (anchor x, y, z, level).  Returns [2, N, n^3] float64."""
    import torch
    x = _nodes_torch(leaves, L, device, nodes)
    u = torch.zeros(x.shape[:2], dtype=torch.float64, device=device)
    ims = torch.as_tensor(IMAGES, device=device)
    for cc in centres_nu:
        c = torch.as_tensor(centre_physical(cc, L, nodes), device=device)
        for im in ims:
            d = x - (c + im)
            u += amp * torch.exp(-(d * d).sum(-1) / (2.0 * sigma * sigma))
    return torch.stack([u, torch.zeros_like(u)])


def maxwell_gaussian_torch(leaves: np.ndarray, L: int, centres_nu, sigma=0.1, amp=1.0, device="cuda"):
    """Same data as maxwell_gaussian with torch: [6, N, 125] float64."""
    import torch
    x = _nodes_torch(leaves, L, device)
    ex = torch.zeros(x.shape[:2], dtype=torch.float64, device=device)
    ey = torch.zeros_like(ex)
    ims = torch.as_tensor(IMAGES, device=device)
    for cc in centres_nu:
        c = torch.as_tensor(centre_physical(cc, L), device=device)
        for im in ims:
            d = x - (c + im)
            g = amp * torch.exp(-(d * d).sum(-1) / (2.0 * sigma * sigma))
            ex += -d[..., 1] / (sigma * sigma) * g
            ey += d[..., 0] / (sigma * sigma) * g
    z = torch.zeros_like(ex)
    return torch.stack([ex, ey, z, z.clone(), z.clone(), z.clone()])
