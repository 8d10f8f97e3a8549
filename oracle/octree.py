"""Linear octree, balance, blocks, unzip map and LTS schedule (test infrastructure only).

Paper passages:
  * Sec. 3.2 (octree on [0, 2^L]^3): axis-aligned linear octree, leaves sorted along
    a space-filling curve.  One GPU has no partition, so Morton order is used.
  * Sec. 3.2.2 (construction/refinement): refine while a criterion holds.  The
    paper's wavelet criterion is replaced by integer geometric criteria so that
    meshes are bit-exact (ball / annulus around a point).
  * Sec. 3.2.3 (2:1 balance).  Octants carry n^3 nodes, n = 5 or 7 (the paper's
    runs use 7^3, Sec. 4.5 / fig. of the mesh generation).  The three ghost layers
    of the sixth-order stencils reach 3/(n-1) of a neighbouring octant: half of it
    for n = 7, where the paper's 2:1 balance (face, edge and corner) keeps every
    ghost source within one level of the receiver, as the time-gap argument of
    Sec. 3.6.3 assumes.  For n = 5 the reach is 3/4 of an octant, so the balance
    is extended to ghost reach: a leaf of level l is split when a leaf of level
    >= l+2 lies within three grid spacings of it.
  * Sec. 3.2.5 + fig. oct_to_blocks (octree to block decomposition): a block is a
    maximal uniformly refined sub-tree, split into aligned cubes of at most
    ``cap`` octants per side.
  * Sec. 3.3 + fig. unzip: padded blocks; coarse->fine interpolation and
    fine->coarse injection for the padding.
  * Sec. 3.6.3 + fig. blk_loop: level-frequency schedule.
  * Sec. 3.7, eqs. w_nuts, w_uts, invS: speedup model.

Geometry (integer "node units" at the finest level L of the spec), with
n nodes per octant side and ni = n - 1 intervals:
  domain [-1, 1]^3, periodic (default) or bounded by the outer faces (boundary
  "outer", the radiative boundary of Sec. 4.2); N_u = ni * 2^L node units per
  side, x = -1 + 2 X / N_u.
  A leaf has an anchor a (in level-L octant units, a multiple of s = 2^(L-l)) and a
  level l; its n nodes per axis sit at ni a + i s, i = 0..ni; spacing
  h_l = 2^(1-l) / ni (2^(-l-1) for n = 5).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
from scipy.ndimage import maximum_filter1d

NODES = 5          # default nodes per octant side (5 or 7)
GHOST = 3          # ghost layers of the sixth-order stencils

KIND_OWN, KIND_SAME, KIND_FINE, KIND_COARSE, KIND_NONE = 0, 1, 2, 3, 4   # NONE: outside the domain


# ----------------------------------------------------------------------------- Morton
def morton_key(ax, ay, az) -> np.ndarray:
    """Bit-interleaved key, x in the lowest bit (child index x + 2y + 4z)."""
    ax = np.asarray(ax, dtype=np.int64)
    ay = np.asarray(ay, dtype=np.int64)
    az = np.asarray(az, dtype=np.int64)
    key = np.zeros(np.broadcast(ax, ay, az).shape, dtype=np.int64)
    for b in range(20):
        key |= ((ax >> b) & 1) << (3 * b)
        key |= ((ay >> b) & 1) << (3 * b + 1)
        key |= ((az >> b) & 1) << (3 * b + 2)
    return key


# ----------------------------------------------------------------------------- spec
@dataclass
class Criterion:
    """Refinement criterion around an integer centre (node units at level L).

    kind "ball":    refine a level-l leaf if dmin^2 < r2[l].
    kind "annulus": refine if rlo2[l] < dmax^2 and dmin^2 < rhi2[l]  (the leaf
                    meets the shell where a Gaussian's gradient is large).
    dmin / dmax are the smallest / largest periodic distances from the centre to
    the leaf's closed box.  A negative radius entry never refines.
    """
    kind: str
    center: Tuple[int, int, int]
    r2: Sequence[int] = ()
    rlo2: Sequence[int] = ()
    rhi2: Sequence[int] = ()


@dataclass
class MeshSpec:
    l_min: int
    l_max: int
    criteria: List[Criterion] = field(default_factory=list)
    block_cap: int = 4
    boundary: str = "periodic"      # "periodic" or "outer"
    nodes: int = NODES              # nodes per octant side: 5 or 7

    @property
    def periodic(self) -> bool:
        return self.boundary == "periodic"

    @staticmethod
    def from_dict(d: dict) -> "MeshSpec":
        crit = []
        for c in d.get("criteria", []):
            crit.append(Criterion(kind=c["kind"], center=tuple(int(v) for v in c["center"]),
                                  r2=tuple(c.get("r2", ())), rlo2=tuple(c.get("rlo2", ())),
                                  rhi2=tuple(c.get("rhi2", ()))))
        b = d.get("boundary", "periodic")
        if b not in ("periodic", "outer"):
            raise ValueError(f"unknown boundary {b}")
        n = int(d.get("nodes", NODES))
        if n not in (5, 7):
            raise ValueError(f"nodes per octant side must be 5 or 7, not {n}")
        return MeshSpec(int(d["l_min"]), int(d["l_max"]), crit, int(d.get("block_cap", 4)), b, n)


def _periodic_min_dist(lo, hi, c, n):
    """Per-axis smallest periodic distance from c to the closed interval [lo, hi]."""
    best = None
    for k in (-1, 0, 1):
        d = np.maximum(0, np.maximum(lo + k * n - c, c - (hi + k * n)))
        best = d if best is None else np.minimum(best, d)
    return best


def _periodic_point_dist(x, c, n):
    d = np.abs(x - c) % n
    return np.minimum(d, n - d)


def _periodic_max_dist(lo, hi, c, n):
    """Per-axis largest periodic distance from c to a point of [lo, hi].

    The periodic distance to c peaks (value n/2) at the antipode c + n/2; if the
    antipode lies in the interval that is the maximum, else an end point is.
    """
    anti = (c + n // 2) % n
    # antipode (or one of its images) inside [lo, hi]?
    inside = np.zeros(np.broadcast(lo, hi).shape, dtype=bool)
    for k in (-1, 0, 1):
        a = anti + k * n
        inside |= (lo <= a) & (a <= hi)
    ends = np.maximum(_periodic_point_dist(lo, c, n), _periodic_point_dist(hi, c, n))
    return np.where(inside, n // 2, ends)


def criterion_holds(crit: Criterion, anchors: np.ndarray, level: int, L: int, periodic: bool = True,
                    nodes: int = NODES) -> np.ndarray:
    """Evaluate a criterion for leaves of one level (Sec. 3.2.2, reading in module doc).
    Distances are periodic (nearest image) or, for a bounded domain, plain, in the
    node units of a mesh of `nodes` nodes per octant side."""
    if len(anchors) == 0:
        return np.zeros(0, dtype=bool)
    ni = nodes - 1
    n = ni * (1 << L)
    s = 1 << (L - level)
    lo = ni * anchors.astype(np.int64)
    hi = lo + ni * s
    c = np.asarray(crit.center, dtype=np.int64)[None, :]
    if periodic:
        dmin2 = (_periodic_min_dist(lo, hi, c, n) ** 2).sum(axis=1)
    else:
        dmin2 = (np.maximum(0, np.maximum(lo - c, c - hi)) ** 2).sum(axis=1)
    if crit.kind == "ball":
        r2 = crit.r2[level] if level < len(crit.r2) else -1
        if r2 < 0:
            return np.zeros(len(anchors), dtype=bool)
        return dmin2 < r2
    if crit.kind == "annulus":
        rlo2 = crit.rlo2[level] if level < len(crit.rlo2) else -1
        rhi2 = crit.rhi2[level] if level < len(crit.rhi2) else -1
        if rhi2 < 0:
            return np.zeros(len(anchors), dtype=bool)
        if periodic:
            dmax2 = (_periodic_max_dist(lo, hi, c, n) ** 2).sum(axis=1)
        else:
            dmax2 = (np.maximum(np.abs(lo - c), np.abs(hi - c)) ** 2).sum(axis=1)
        return (rlo2 < dmax2) & (dmin2 < rhi2)
    raise ValueError(f"unknown criterion kind {crit.kind}")


# ----------------------------------------------------------------------------- leaves
def _children(anchors: np.ndarray, level: int, L: int) -> np.ndarray:
    h = 1 << (L - level - 1)
    out = []
    for c in range(8):
        off = np.array([(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1], dtype=np.int64) * h
        out.append(anchors + off[None, :])
    return np.concatenate(out, axis=0) if len(anchors) else np.zeros((0, 3), np.int64)


def _sort(anchors: np.ndarray, levels: np.ndarray):
    key = morton_key(anchors[:, 0], anchors[:, 1], anchors[:, 2])
    order = np.argsort(key, kind="stable")
    return anchors[order], levels[order]


def uniform_leaves(level: int, L: int) -> Tuple[np.ndarray, np.ndarray]:
    n = 1 << level
    s = 1 << (L - level)
    g = np.arange(n, dtype=np.int64) * s
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    anchors = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    return _sort(anchors, np.full(len(anchors), level, dtype=np.int64))


def refine(spec: MeshSpec) -> Tuple[np.ndarray, np.ndarray]:
    """Uniform tree at l_min, then split every leaf whose criterion holds, level by level."""
    L = spec.l_max
    anchors, levels = uniform_leaves(spec.l_min, L)
    keep_a, keep_l = [], []
    cur = anchors
    for lev in range(spec.l_min, L + 1):
        if lev == L or not spec.criteria:
            keep_a.append(cur); keep_l.append(np.full(len(cur), lev, np.int64))
            break
        split = np.zeros(len(cur), dtype=bool)
        for crit in spec.criteria:
            split |= criterion_holds(crit, cur, lev, L, spec.periodic, spec.nodes)
        keep_a.append(cur[~split]); keep_l.append(np.full(int((~split).sum()), lev, np.int64))
        cur = _children(cur[split], lev, L)
        if len(cur) == 0:
            break
    anchors = np.concatenate(keep_a, axis=0)
    levels = np.concatenate(keep_l)
    return _sort(anchors, levels)


def level_grid(anchors: np.ndarray, levels: np.ndarray, L: int) -> np.ndarray:
    """Cell grid at level L: level of the leaf covering each cell, indexed [x, y, z]."""
    n = 1 << L
    g = np.full((n, n, n), -1, dtype=np.int16)
    for a, l in zip(anchors, levels):
        s = 1 << (L - int(l))
        g[a[0]:a[0] + s, a[1]:a[1] + s, a[2]:a[2] + s] = l
    if (g < 0).any():
        raise ValueError("leaves do not tile the domain")
    return g


def _window_max(grid: np.ndarray, s: int, periodic: bool = True, reach: bool = True) -> np.ndarray:
    """max over cells [a-1-f, a+s+f]^3 around every anchor a.

    reach (5 nodes per side): f = floor(3 s / 4); these are exactly the level-L
    cells whose closed box meets the closed box of a level-l leaf (width 4 s node
    units) grown by 3 h_l = 3 s node units.  Without reach (2:1 balance, 7 nodes
    per side): f = 0, the cells whose closed box meets the leaf's.  A centred
    window of even size s + 2f + 2 read at a + s/2 covers that range.  A bounded
    domain has no cells beyond its faces (padding -1 is below every level).
    """
    f = (3 * s) // 4 if reach else 0
    size = s + 2 * f + 2
    out = grid
    for ax in range(3):
        if not periodic:
            out = maximum_filter1d(out, size=size, axis=ax, mode="constant", cval=-1)
        elif size >= out.shape[ax]:
            # the window covers the whole period: the axis-wise maximum
            out = np.broadcast_to(out.max(axis=ax, keepdims=True), out.shape).copy()
        else:
            out = maximum_filter1d(out, size=size, axis=ax, mode="wrap")
    return out


def balance(anchors: np.ndarray, levels: np.ndarray, L: int, periodic: bool = True,
            nodes: int = NODES) -> Tuple[np.ndarray, np.ndarray]:
    """Balance (Sec. 3.2.3).  5 nodes per side: ghost-reach balance, split any leaf
    a of level l for which some leaf of level >= l+2 has periodic Chebyshev box
    distance <= 3 h_l.  7 nodes per side: 2:1 balance, the same with distance 0
    (a leaf of level >= l+2 touching a at a face, edge or corner).

    Iterated to the fixpoint.  Every split is forced in any balanced refinement of
    the current tree, so the result is the unique minimal balanced refinement.
    """
    anchors = anchors.copy()
    levels = levels.copy()
    n = 1 << L
    while True:
        grid = level_grid(anchors, levels, L)
        changed = False
        new_a, new_l = [], []
        split_mask = np.zeros(len(levels), dtype=bool)
        for lev in range(int(levels.min()), L - 1):
            sel = np.nonzero(levels == lev)[0]
            if len(sel) == 0:
                continue
            s = 1 << (L - lev)
            wm = _window_max(grid, s, periodic, nodes == 5)
            pos = (anchors[sel] + s // 2) % n
            mx = wm[pos[:, 0], pos[:, 1], pos[:, 2]]
            split_mask[sel[mx >= lev + 2]] = True
        if split_mask.any():
            changed = True
            keep = ~split_mask
            new_a.append(anchors[keep]); new_l.append(levels[keep])
            for lev in np.unique(levels[split_mask]):
                sel = split_mask & (levels == lev)
                ch = _children(anchors[sel], int(lev), L)
                new_a.append(ch); new_l.append(np.full(len(ch), lev + 1, np.int64))
            anchors, levels = _sort(np.concatenate(new_a), np.concatenate(new_l))
        if not changed:
            return anchors, levels


def is_balanced_bruteforce(anchors: np.ndarray, levels: np.ndarray, L: int, periodic: bool = True,
                           nodes: int = NODES) -> bool:
    """O(N^2) check of the balance predicate (for small meshes in tests)."""
    ni = nodes - 1
    n = ni * (1 << L)
    lo = ni * anchors.astype(np.int64)
    w = ni * (1 << (L - levels.astype(np.int64)))
    hi = lo + w[:, None]
    for a in range(len(levels)):
        h = 1 << (L - int(levels[a]))
        cand = levels >= levels[a] + 2
        if not cand.any():
            continue
        gap = np.zeros((int(cand.sum()), 3), dtype=np.int64) + 10 ** 9
        for k in ((-1, 0, 1) if periodic else (0,)):
            g = np.maximum(0, np.maximum(lo[cand] + k * n - hi[a], lo[a] - (hi[cand] + k * n)))
            gap = np.minimum(gap, g)
        if (gap.max(axis=1) <= (3 * h if nodes == 5 else 0)).any():
            return False
    return True


# ----------------------------------------------------------------------------- mesh
@dataclass
class Mesh:
    L: int                      # finest resolution of the coordinates (spec l_max)
    anchors: np.ndarray         # [N, 3] level-L octant units, Morton sorted
    levels: np.ndarray          # [N]
    blocks: np.ndarray          # [B, 6] first_leaf, m, level, ax, ay, az (level-L units)
    cap: int
    periodic: bool = True       # False: bounded by the outer faces of [-1, 1]^3
    nodes: int = NODES          # nodes per octant side (5 or 7)

    @property
    def ni(self) -> int:
        """Node intervals per octant side."""
        return self.nodes - 1

    @property
    def n_oct(self) -> int:
        return len(self.levels)

    @property
    def lmin(self) -> int:
        return int(self.levels.min())

    @property
    def lmax(self) -> int:
        return int(self.levels.max())

    def __post_init__(self):
        self._lookup = {}
        for i, (a, l) in enumerate(zip(self.anchors, self.levels)):
            self._lookup[(int(l), int(a[0]), int(a[1]), int(a[2]))] = i
        self.block_of_leaf = np.full(self.n_oct, -1, dtype=np.int64)
        for b, row in enumerate(self.blocks):
            first, m = int(row[0]), int(row[1])
            self.block_of_leaf[first:first + m ** 3] = b
        assert (self.block_of_leaf >= 0).all()

    def find(self, level: int, cell) -> int:
        """Leaf index of the octant at `level` with level-`level` coordinates `cell`
        (wrapped periodically; outside a bounded domain: -1), or -1."""
        n = 1 << level
        s = 1 << (self.L - level)
        if not self.periodic and any(int(v) < 0 or int(v) >= n for v in cell):
            return -1
        key = (level, (int(cell[0]) % n) * s, (int(cell[1]) % n) * s, (int(cell[2]) % n) * s)
        return self._lookup.get(key, -1)


def build_blocks(anchors: np.ndarray, levels: np.ndarray, L: int, cap: int) -> np.ndarray:
    """Octree-to-block decomposition (Sec. 3.2.5, fig. oct_to_blocks).

    For every leaf find its largest ancestor whose sub-tree is uniformly refined
    at the leaf's level; that sub-tree, split into aligned cubes of side
    min(side, cap) leaves, gives the blocks.  Blocks are ordered by Morton key.
    """
    grid = level_grid(anchors, levels, L)
    n = 1 << L
    # uni[k] : the single leaf level found in every level-k cell, -1 if mixed
    uni = {L: grid.astype(np.int16)}
    for k in range(L - 1, -1, -1):
        c = uni[k + 1]
        sub = [c[dx::2, dy::2, dz::2] for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)]
        same = np.ones_like(sub[0], dtype=bool)
        for t in sub[1:]:
            same &= (t == sub[0])
        uni[k] = np.where(same, sub[0], -1).astype(np.int16)
    rows = {}
    for i, (a, l) in enumerate(zip(anchors, levels)):
        l = int(l)
        kstar = l
        for k in range(l - 1, -1, -1):
            sk = 1 << (L - k)
            if uni[k][a[0] // sk, a[1] // sk, a[2] // sk] == l:
                kstar = k
            else:
                break
        side = 1 << (l - kstar)
        m = min(side, cap)
        span = m * (1 << (L - l))
        ba = (a // span) * span
        key = (l, int(ba[0]), int(ba[1]), int(ba[2]))
        rows.setdefault(key, (m, i))
        rows[key] = (m, min(rows[key][1], i))
    out = []
    for (l, x, y, z), (m, first) in rows.items():
        out.append((first, m, l, x, y, z))
    out.sort(key=lambda r: r[0])
    blk = np.array(out, dtype=np.int64).reshape(-1, 6)
    return blk


def build_mesh(spec: MeshSpec) -> Mesh:
    """Refinement, balance, blocks (Sec. 3.2.2 -> 3.2.3 -> 3.2.5)."""
    a, l = refine(spec)
    a, l = balance(a, l, spec.l_max, spec.periodic, spec.nodes)
    blk = build_blocks(a, l, spec.l_max, spec.block_cap)
    return Mesh(spec.l_max, a, l, blk, spec.block_cap, spec.periodic, spec.nodes)


def mesh_from_leaves(anchors, levels, L: int, cap: int = 4, do_balance: bool = True, periodic: bool = True,
                     nodes: int = NODES) -> Mesh:
    a = np.asarray(anchors, dtype=np.int64).reshape(-1, 3)
    l = np.asarray(levels, dtype=np.int64).reshape(-1)
    a, l = _sort(a, l)
    level_grid(a, l, L)  # validates the tiling
    if do_balance:
        a, l = balance(a, l, L, periodic, nodes)
    return Mesh(L, a, l, build_blocks(a, l, L, cap), cap, periodic, nodes)


# ----------------------------------------------------------------------------- unzip map
def block_octants(mesh: Mesh, b: int) -> np.ndarray:
    """Leaf indices of block b in lexicographic (oi, oj, ok) order, shape [m, m, m] as [ok, oj, oi]."""
    first, m = int(mesh.blocks[b, 0]), int(mesh.blocks[b, 1])
    o = np.arange(m)
    ok, oj, oi = np.meshgrid(o, o, o, indexing="ij")
    return first + morton_key(oi, oj, ok)


def unzip_map(mesh: Mesh, b: int) -> np.ndarray:
    """Canonical source of every padded point of block b (Sec. 3.3, fig. unzip).

    Returns int64 [S^3, 5] rows (leaf, kind, 2*px, 2*py, 2*pz), S = ni m + 7
    (ni = nodes - 1 intervals per octant side), points in lexicographic order of
    Q in [-3, ni m + 3]^3 with x fastest; (px, py, pz) is the position in the
    source leaf's node units (half-integers only for kind COARSE).

    Ownership rule (the paper is silent on points shared by several leaves), per
    axis on the receiver-level grid (node spacing h_lam, ni per octant):
      cell = -1 if Q < 0;  min(Q // ni, m-1) if 0 <= Q <= ni m;  m if Q > ni m,
      nu = Q - ni cell in [0, ni],
    i.e. the block's closed box is cut along its own octant grid (its upper faces
    belong to its last octants) and outside it the cells are half-open.  The
    receiver-level cell (cx, cy, cz) is then
      * one of the block's octants (OWN): node nu;
      * one same-level leaf (SAME): node nu;
      * leaves one level finer (FINE): per axis a child c and the fine node
        2 (nu - c ni/2) (injection of the coincident fine node).  5 nodes:
        c = min(nu >> 1, 1), and all 8 children are leaves.  7 nodes: c = 1 if
        nu > 3, 0 if nu < 3, and on the mid-plane nu = 3 the child next to the
        block (c = 1 below it, 0 above): the children next to the block are the
        ones that 2:1 balance keeps leaves (the others may be refined further);
      * one octant (child bits beta) of a leaf one level coarser (COARSE): position
        (ni beta + nu) / 2 in its node units (interpolated when odd);
      * on a bounded domain, a cell beyond the outer faces (NONE, leaf -1): the
        block's stencils there switch to the boundary closure and read no value.
    """
    first, m, lev = int(mesh.blocks[b, 0]), int(mesh.blocks[b, 1]), int(mesh.blocks[b, 2])
    ni = mesh.ni
    s = 1 << (mesh.L - lev)
    base = mesh.blocks[b, 3:6] // s          # block anchor in level-lev units
    S = ni * m + 7
    q = np.arange(-3, ni * m + 4, dtype=np.int64)
    Qz, Qy, Qx = np.meshgrid(q, q, q, indexing="ij")
    Q = np.stack([Qx.ravel(), Qy.ravel(), Qz.ravel()], axis=1)  # [S^3, 3]
    cell = np.where(Q < 0, -1, np.where(Q <= ni * m, np.minimum(Q // ni, m - 1), m))
    nu = Q - ni * cell
    out = np.zeros((S ** 3, 5), dtype=np.int64)
    inside = ((cell >= 0) & (cell <= m - 1)).all(axis=1)
    if not mesh.periodic:
        # a bounded domain: points beyond its outer faces have no source
        n = 1 << lev
        gc = base[None, :] + cell
        outside = ((gc < 0) | (gc >= n)).any(axis=1)
        out[outside, 0] = -1
        out[outside, 1] = KIND_NONE
        out[outside, 2:5] = 2 * nu[outside]
    else:
        outside = np.zeros(len(Q), dtype=bool)
    oc = cell[inside]
    out[inside, 0] = first + morton_key(oc[:, 0], oc[:, 1], oc[:, 2])
    out[inside, 1] = KIND_OWN
    out[inside, 2:5] = 2 * nu[inside]
    gi = np.nonzero(~inside & ~outside)[0]
    cells = base[None, :] + cell[gi]
    nug = nu[gi]
    below = cell[gi] < 0                      # per axis: the cell lies below the block
    uniq, inv = np.unique(cells, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    for u_i, c in enumerate(uniq):
        rows = gi[inv == u_i]
        nur = nug[inv == u_i]
        blw = below[inv == u_i]
        same = mesh.find(lev, c)
        if same >= 0:
            out[rows, 0] = same
            out[rows, 1] = KIND_SAME
            out[rows, 2:5] = 2 * nur
            continue
        coarse = mesh.find(lev - 1, c >> 1) if lev > 0 else -1
        if coarse >= 0:
            beta = np.asarray(c) & 1
            out[rows, 0] = coarse
            out[rows, 1] = KIND_COARSE
            out[rows, 2:5] = ni * beta[None, :] + nur
            continue
        if ni == 4:
            # the padding reaches 3/4 into the cell: all 8 children are leaves
            ch0 = mesh.find(lev + 1, 2 * c)
            if ch0 < 0:
                raise ValueError(f"unbalanced mesh: no ghost source for block {b} cell {c}")
            for k in range(8):
                cc = 2 * c + np.array([k & 1, (k >> 1) & 1, (k >> 2) & 1])
                if mesh.find(lev + 1, cc) != ch0 + k:
                    raise ValueError(f"unbalanced mesh: cell {c} of block {b} is not 8 finer leaves")
            cb = np.minimum(nur >> 1, 1)
            out[rows, 0] = ch0 + cb[:, 0] + 2 * cb[:, 1] + 4 * cb[:, 2]
        else:
            # the padding reaches half-way into the cell: only the children next to
            # the block are read, and 2:1 balance keeps exactly those leaves
            cb = np.where(2 * nur > ni, 1, np.where(2 * nur < ni, 0, blw.astype(np.int64)))
            for r, cbr in zip(rows, cb):
                lf = mesh.find(lev + 1, 2 * c + cbr)
                if lf < 0:
                    raise ValueError(f"unbalanced mesh: no ghost source for block {b} cell {c}")
                out[r, 0] = lf
        out[rows, 1] = KIND_FINE
        out[rows, 2:5] = 2 * (2 * nur - ni * cb)
    return out


# ----------------------------------------------------------------------------- schedule
def substeps(mesh: Mesh) -> int:
    """2^(Delta L) substeps per coarsest step (Sec. 3.6.3)."""
    return 1 << (mesh.lmax - mesh.lmin)


def active_blocks(mesh: Mesh, j: int, mode: str = "lts") -> np.ndarray:
    """B_j (fig. blk_loop): level-lam blocks step at substeps with j mod 2^(lmax-lam) == 0.
    GTS steps every block at every substep."""
    lev = mesh.blocks[:, 2]
    if mode == "gts":
        return np.arange(len(lev))
    r = 1 << (mesh.lmax - lev)
    return np.nonzero(j % r == 0)[0]


def h_level(level, nodes: int = NODES) -> float:
    """Node spacing h_l = 2^(1-l) / (nodes - 1) of a level-l octant of [-1, 1]^3."""
    return 2.0 ** (1 - int(level)) / (nodes - 1)


def dt_level(level, nodes: int = NODES) -> float:
    """dt_l = 0.25 h_l (CFL 0.25, Sec. 3.6): 2^(-l-3) for 5 nodes per side."""
    return 0.25 * h_level(level, nodes)


def speedup_model(mesh: Mesh) -> dict:
    """Sec. 3.7, eqs. w_nuts, w_uts, invS with alpha_l = DG nodes at level lmax - l."""
    Lspan = mesh.lmax - mesh.lmin
    alpha = np.zeros(Lspan + 1, dtype=np.int64)
    for lev in range(mesh.lmin, mesh.lmax + 1):
        alpha[mesh.lmax - lev] = mesh.nodes ** 3 * int((mesh.levels == lev).sum())
    w_lts = int(sum((1 << (Lspan - l)) * int(alpha[l]) for l in range(Lspan + 1)))
    w_gts = int((1 << Lspan) * int(alpha.sum()))
    inv_s = sum(float(alpha[l]) / 2 ** l for l in range(Lspan + 1)) / float(alpha.sum())
    return {"alpha": alpha.tolist(), "w_lts": w_lts, "w_gts": w_gts,
            "s_est": 1.0 / inv_s, "s_max": float(alpha.sum()) / float(alpha[0])}
