"""Remeshing at coarse-step boundaries (test infrastructure only).

Paper passages:
  * Sec. 3.2.2 (construction and refinement): the octree follows a wavelet
    criterion -- the wavelet coefficient measures the failure of a field to be
    interpolated from the coarser level, and refinement stops where it is below
    a tolerance eps.
  * Sec. 5 (conclusions): remeshing is a global operation, done when all blocks
    are synchronised in time (a coarse-step boundary of Alg. 2), after which
    the state is carried to the new octree.

Readings (the paper names the criterion but not its discretisation):
  * wavelet indicator of an octant with node values v (5 per axis): the largest
    |v - I2 v| over fields and over the nodes that are not on its every-second-
    node grid, I2 the tensor degree-2 Lagrange interpolant of the 3^3 nodes at
    positions 0, 2, 4 (the octant seen from one level coarser);
  * a leaf of level < l_max splits where its indicator exceeds eps;
  * a complete family of 8 sibling leaves (level > l_min, none splitting) merges
    where the indicator of the parent octant is below eps / 4 (the parent's 5^3
    nodes are nodes of its children; the margin keeps a merged parent from
    splitting again at the next remesh);
  * the result is closed under the ghost-reach balance (octree.balance);
  * intergrid transfer: a new leaf inside an old leaf takes the old leaf's
    tensor degree-4 Lagrange interpolant at its nodes (a copy when the levels
    agree); a new leaf that is the union of 8 old leaves one level finer takes
    the coincident child nodes (injection: node i of the parent is node
    2 (i - 2c) of child c = min(i >> 1, 1) per axis).
The state at a coarse-step boundary is all that is carried: every level starts a
new step there, so no stored RK stage is read across it.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from typing import Tuple

import numpy as np

from .fd import lagrange_weights_fr
from .octree import Mesh, _children, _sort, balance, build_blocks, morton_key

#: degree-2 interpolation from nodes 0, 2, 4 to positions 0..4 (exact rationals)
I2_FR = [[Fr(1), Fr(0), Fr(0)], [Fr(3, 8), Fr(3, 4), Fr(-1, 8)], [Fr(0), Fr(1), Fr(0)],
         [Fr(-1, 8), Fr(3, 4), Fr(3, 8)], [Fr(0), Fr(0), Fr(1)]]
I2 = np.array([[float(x) for x in row] for row in I2_FR])


def wavelet_indicator(v: np.ndarray) -> np.ndarray:
    """Indicator of octants with node values v [..., F, 5, 5, 5] ([k][j][i]):
    max over fields and non-even nodes of |v - I2 v| (I2 from the 27 even nodes)."""
    e = v[..., 0::2, 0::2, 0::2]                                       # [.., F, 3, 3, 3]
    t = np.einsum("ia,...cba->...cbi", I2, e)                          # x
    t = np.einsum("jb,...cbi->...cji", I2, t)                          # y
    t = np.einsum("kc,...cji->...kji", I2, t)                          # z
    d = np.abs(v - t)
    return d.reshape(d.shape[:-4] + (-1,)).max(axis=-1)


def parent_values(children: np.ndarray) -> np.ndarray:
    """Node values of the parent of 8 sibling leaves [8, F, 5, 5, 5] (Morton child
    order): node i of the parent is node 2 (i - 2c) of child c = min(i >> 1, 1)."""
    F = children.shape[1]
    out = np.empty((F, 5, 5, 5))
    for k in range(5):
        for j in range(5):
            for i in range(5):
                cx, cy, cz = min(i >> 1, 1), min(j >> 1, 1), min(k >> 1, 1)
                c = cx + 2 * cy + 4 * cz
                out[:, k, j, i] = children[c][:, 2 * (k - 2 * cz), 2 * (j - 2 * cy), 2 * (i - 2 * cx)]
    return out


def families(mesh: Mesh):
    """First leaf index of every complete family of 8 same-level siblings."""
    out = []
    a, l = mesh.anchors, mesh.levels
    for i in range(mesh.n_oct - 7):
        lev = int(l[i])
        if lev == 0:
            continue
        s = 1 << (mesh.L - lev)
        if (a[i] % (2 * s)).any() or (l[i:i + 8] != lev).any():
            continue
        ok = True
        for c in range(8):
            off = np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1]) * s
            if not np.array_equal(a[i + c], a[i] + off):
                ok = False
                break
        if ok:
            out.append(i)
    return np.array(out, dtype=np.int64)


def indicators(mesh: Mesh, state: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(leaf indicator [N], family first leaves [M], family indicator [M]) of a
    state [F][N][5][5][5]."""
    v = np.moveaxis(state, 0, 1)                                        # [N, F, 5,5,5]
    leaf = wavelet_indicator(v)
    fam = families(mesh)
    fw = np.array([wavelet_indicator(parent_values(v[f:f + 8])) for f in fam])
    return leaf, fam, fw


def remesh(mesh: Mesh, state: np.ndarray, eps: float, l_min: int, l_max: int) -> Mesh:
    """The new octree of a state (readings in the module doc)."""
    leaf, fam, fw = indicators(mesh, state)
    L = mesh.L
    split = (mesh.levels < l_max) & (leaf > eps)
    merge = np.zeros(mesh.n_oct, dtype=bool)
    for f, w in zip(fam, fw):
        if mesh.levels[f] > l_min and w < eps / 4 and not split[f:f + 8].any():
            merge[f:f + 8] = True
    keep = ~(split | merge)
    a_new = [mesh.anchors[keep]]
    l_new = [mesh.levels[keep]]
    for lev in np.unique(mesh.levels[split]):
        sel = split & (mesh.levels == lev)
        ch = _children(mesh.anchors[sel], int(lev), L)
        a_new.append(ch)
        l_new.append(np.full(len(ch), lev + 1, np.int64))
    mf = [f for f in fam if merge[f]]
    if mf:
        a_new.append(mesh.anchors[mf])
        l_new.append(mesh.levels[mf] - 1)
    a, l = _sort(np.concatenate(a_new), np.concatenate(l_new))
    a, l = balance(a, l, L, mesh.periodic)
    return Mesh(L, a, l, build_blocks(a, l, L, mesh.cap), mesh.cap, mesh.periodic)


def transfer(old: Mesh, new: Mesh, state: np.ndarray) -> np.ndarray:
    """Intergrid transfer of a state [F][N_old][5][5][5] to the new octree."""
    F = state.shape[0]
    L = old.L
    out = np.empty((F, new.n_oct, 5, 5, 5))
    key_old = morton_key(old.anchors[:, 0], old.anchors[:, 1], old.anchors[:, 2])
    for n in range(new.n_oct):
        a, l = new.anchors[n], int(new.levels[n])
        # the old leaf holding the new leaf's anchor cell
        k = morton_key(a[0], a[1], a[2])
        o = int(np.searchsorted(key_old, k, side="right")) - 1
        lo = int(old.levels[o])
        if lo <= l:
            s_old = 1 << (L - lo)
            s_new = 1 << (L - l)
            w = []
            for d in range(3):
                pos = [Fr(int(4 * a[d] + i * s_new - 4 * old.anchors[o][d]), s_old) for i in range(5)]
                w.append(np.array([[float(x) for x in lagrange_weights_fr(p)] for p in pos]))   # [5 new, 5 old]
            v = state[:, o]                                                # [F, 5,5,5] (k, j, i)
            t = np.einsum("ia,fcba->fcbi", w[0], v)
            t = np.einsum("jb,fcbi->fcji", w[1], t)
            t = np.einsum("kc,fcji->fkji", w[2], t)
            out[:, n] = t
        else:
            if lo != l + 1:
                raise ValueError("a new leaf merges leaves more than one level finer")
            out[:, n] = parent_values(np.moveaxis(state[:, o:o + 8], 1, 0))
    return out
