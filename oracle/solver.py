"""Plain FP64 LTS / GTS solver on padded blocks (test infrastructure only).

Paper passages:
  * Alg. 1 (GTS, Sec. 3.5): every block takes every stage with the finest step;
    stage values of all blocks are synchronised after each stage.
  * Alg. 2 (LTS, Sec. 3.6.2) with the level-frequency loop of Sec. 3.6.3 and
    fig. blk_loop: at substep j the blocks B_j of every level lam with
    j mod 2^(lmax-lam) == 0 take one step of size dt_lam.
  * eqs. fc_1 / fc_2 (Sec. 3.6.2): stage corrections between levels, applied to
    the values copied into the padding of neighbouring blocks (Sec. 3.6.3, last
    sentences).
  * Sec. 3.3, fig. unzip / fig. overview: unzip (padding), block RHS on the
    uniform block grid, zip (back to octant-local DG nodes).

Readings:
  * The substep loop runs j = 0 .. 2^(Delta L)-1 (Alg. 2 prints "l = l_max to
    l_min"; fig. blk_loop numbers the substeps 0..3).
  * Stages are synchronised across all of B_j: stage s of every active block
    reads only stages 1..s-1 of its neighbours, then the next stage starts.
  * The padding is rebuilt for every stage from the neighbours' step records
    (fig. overview: one unzip per stage).
  * The state is kept as octant-local (DG) nodes, two buffers per octant: a block's
    step writes its new state into the buffer its record does not use, so the
    record (U0, K_1..K_p, start time, step) stays readable by neighbours until the
    block starts its next step.

Layouts (identical to the library's so that arrays compare directly), n = 5 or
7 nodes per octant side:
  U[2][F][N][n][n][n] and K[p][F][N][n][n][n], node index [k][j][i], i fastest.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from typing import Dict, List, Optional

import numpy as np

from . import fd
from .octree import (GHOST, KIND_COARSE, KIND_NONE, KIND_OWN, Mesh, active_blocks, block_octants, dt_level,
                     h_level, substeps, unzip_map)
from .rk import CASES, TABLEAUS, a_f64, b_f64, weight_table_f64


#: Lagrange weights on n = 5 or 7 nodes for the positions xi = 0, 1/2, ..., n-1 (index 2 xi).
LAGRANGE = {n: np.stack([fd.lagrange_weights(v, n) for v in range(2 * n - 1)]) for n in (5, 7)}


class State:
    """DG state, stages and per-block step records."""

    def __init__(self, mesh: Mesh, nfields: int, tableau: str = "rk4", mode: str = "lts"):
        self.mesh = mesh
        self.F = nfields
        self.tab = TABLEAUS[tableau]
        self.p = self.tab.p
        self.mode = mode
        N = mesh.n_oct
        n = self.n = mesh.nodes
        self.U = np.zeros((2, nfields, N, n, n, n))
        self.K = np.zeros((self.p, nfields, N, n, n, n))
        B = len(mesh.blocks)
        lev = mesh.blocks[:, 2]
        # time in ticks of the finest present step; a level-lam step is 2^(lmax-lam) ticks
        self.dt_ticks = np.where(mode == "gts", 1, 1 << (mesh.lmax - lev)).astype(np.int64)
        self.cur_par = np.zeros(B, dtype=np.int64)
        self.cur_t = np.zeros(B, dtype=np.int64)
        self.rec_par = np.full(B, -1, dtype=np.int64)
        self.rec_t0 = np.full(B, -1, dtype=np.int64)
        self.W = weight_table_f64(self.tab)        # [case][stage][i]
        self.b = b_f64(self.tab)
        self._maps: Dict[int, np.ndarray] = {}
        self._plans: Dict[int, dict] = {}

    # ------------------------------------------------------------------ helpers
    def map(self, b: int) -> np.ndarray:
        if b not in self._maps:
            self._maps[b] = unzip_map(self.mesh, b)
        return self._maps[b]

    def dt_phys(self, b: int) -> float:
        lev = self.mesh.lmax if self.mode == "gts" else int(self.mesh.blocks[b, 2])
        return dt_level(lev, self.n)

    def current(self) -> np.ndarray:
        """Current state of every octant, [F][N][n][n][n]."""
        out = np.empty_like(self.U[0])
        for b in range(len(self.mesh.blocks)):
            octs = block_octants(self.mesh, b).ravel()
            out[:, octs] = self.U[self.cur_par[b]][:, octs]
        return out

    def set_initial(self, U0: np.ndarray):
        """U0: [F][N][n][n][n]; all blocks at t = 0, state in buffer 0."""
        self.U[:] = 0.0
        self.U[0] = U0
        self.cur_par[:] = 0
        self.cur_t[:] = 0
        self.rec_par[:] = -1
        self.rec_t0[:] = -1

    # ------------------------------------------------------------------ cases
    def case_of(self, recv: int, src: int) -> int:
        """Time case of a ghost relation from the two blocks' records (Sec. 3.6.2).

        delta = (receiver start - source start) / dt_r, rho = dt_src / dt_r; the
        pair must be one of the four cases a balanced mesh produces."""
        if self.rec_t0[src] < 0:
            raise RuntimeError(f"block {src} has no step record")
        d = Fr(int(self.rec_t0[recv] - self.rec_t0[src]), int(self.dt_ticks[recv]))
        r = Fr(int(self.dt_ticks[src]), int(self.dt_ticks[recv]))
        for ci, (cd, cr) in enumerate(CASES):
            if d == cd and r == cr:
                return ci
        raise RuntimeError(f"illegal time case delta={d} rho={r} for blocks {recv}<-{src}")

    # ------------------------------------------------------------------ unzip
    def plan(self, b: int) -> dict:
        """Static gather description of block b derived from its unzip map."""
        if b in self._plans:
            return self._plans[b]
        mesh = self.mesh
        mp = self.map(b)
        leaf, kind, pos2 = mp[:, 0], mp[:, 1], mp[:, 2:5]
        # points beyond a bounded domain's faces have no source (the block itself
        # stands in for the bookkeeping; their value is never read)
        srcb = np.where(kind == KIND_NONE, b, mesh.block_of_leaf[np.maximum(leaf, 0)])
        ub, inv = np.unique(srcb, return_inverse=True)
        direct = np.nonzero((kind != KIND_COARSE) & (kind != KIND_NONE))[0]
        nd = pos2[direct] // 2
        n = self.n
        flat = leaf[direct] * n ** 3 + nd[:, 2] * n * n + nd[:, 1] * n + nd[:, 0]
        coarse = np.nonzero(kind == KIND_COARSE)[0]
        pl = dict(m=int(mesh.blocks[b, 1]), leaf=leaf, kind=kind, pos2=pos2, srcb=srcb, ub=ub,
                  inv=inv.reshape(-1), direct=direct, flat=flat, coarse=coarse,
                  none=np.nonzero(kind == KIND_NONE)[0],
                  lag=[LAGRANGE[self.n][pos2[coarse, d]] for d in range(3)],
                  octs=block_octants(mesh, b))
        self._plans[b] = pl
        return pl

    def unzip(self, b: int, s: int) -> np.ndarray:
        """Padded stage state Y_s of block b: [F][S][S][S] (Sec. 3.3 and eqs. fc_1/fc_2).

        Every padded point takes, from its source leaf's step record, the value
        Y = U0 + dt_r * sum_i w^_{s,i}(case) K_i; a point that is not a node of a
        coarser source leaf is interpolated from that leaf's n^3 Y values with the
        tensor degree n-1 Lagrange interpolant."""
        mesh = self.mesh
        pl = self.plan(b)
        m = pl["m"]
        n = self.n
        S = (n - 1) * m + 7
        leaf, kind = pl["leaf"], pl["kind"]
        cases = np.array([self.case_of(b, int(x)) for x in pl["ub"]], dtype=np.int64)[pl["inv"]]
        cases[kind == KIND_OWN] = 0
        par = self.rec_par[pl["srcb"]]
        dt = self.dt_phys(b)
        w = self.W[cases, s]                               # [P, p]
        out = np.empty((self.F, S ** 3))
        out[:, pl["none"]] = 0.0
        d = pl["direct"]
        if len(d):
            Uf = self.U.reshape(2, self.F, -1)
            Kf = self.K.reshape(self.p, self.F, -1)
            flat = pl["flat"]
            u0 = np.where(par[d][None, :] == 0, Uf[0][:, flat], Uf[1][:, flat])   # [F, P]
            acc = np.zeros_like(u0)                        # Y = U0 + dt * sum_i w_i K_i
            for i in range(self.p):
                acc += w[d, i][None, :] * Kf[i][:, flat]
            out[:, d] = u0 + dt * acc
        ci = pl["coarse"]
        if len(ci):
            # Y of every distinct (source leaf, case) over the leaf's n^3 nodes
            pairs, pinv = np.unique(np.stack([leaf[ci], cases[ci]], axis=1), axis=0, return_inverse=True)
            pinv = pinv.reshape(-1)
            li, pc = pairs[:, 0], pairs[:, 1]
            pp = self.rec_par[mesh.block_of_leaf[li]]
            wu = self.W[pc, s]                                                # [U, p]
            acc = np.zeros((len(li), self.F, n, n, n))
            for i in range(self.p):
                acc += wu[:, i][:, None, None, None, None] * self.K[i][:, li].transpose(1, 0, 2, 3, 4)
            ysrc = self.U[pp, :, li] + dt * acc                               # [U, F, n,n,n]
            yp = ysrc[pinv]                                                   # [P, F, n,n,n]
            wx, wy, wz = pl["lag"]
            t = (yp * wx[:, None, None, None, :]).sum(axis=4)                 # x
            t = (t * wy[:, None, None, :]).sum(axis=3)                        # y
            t = (t * wz[:, None, :]).sum(axis=2)                              # z
            out[:, ci] = t.T
        return out.reshape(self.F, S, S, S)

    # ------------------------------------------------------------------ zip
    def zip_into(self, b: int, grid: np.ndarray, dest: np.ndarray):
        """Block grid [F][ni m+1]^3 -> every DG node of the block's octants (Sec. 3.3)."""
        m = int(self.mesh.blocks[b, 1])
        octs = self.plan(b)["octs"]
        n = self.n
        ni = n - 1
        for ok in range(m):
            for oj in range(m):
                for oi in range(m):
                    dest[:, octs[ok, oj, oi]] = grid[:, ni * ok:ni * ok + n, ni * oj:ni * oj + n, ni * oi:ni * oi + n]

    # ------------------------------------------------------------------ one substep
    def open_records(self, j: int) -> np.ndarray:
        """Blocks B_j start a step: their record is (current buffer, current time)."""
        act = active_blocks(self.mesh, j, self.mode)
        for b in act:
            self.rec_par[b] = self.cur_par[b]
            self.rec_t0[b] = self.cur_t[b]
        return act

    def close_records(self, act):
        """After the step the state lives in the other buffer, one step later."""
        for b in act:
            self.cur_par[b] = 1 - self.rec_par[b]
            self.cur_t[b] = self.rec_t0[b] + self.dt_ticks[b]

    def geometry(self, b: int) -> dict:
        """Block grid of b in node units: origin X0 (x, y, z), step w, domain side
        Nu, and whether the domain is periodic (for equations that need positions
        or the outer boundary)."""
        mesh = self.mesh
        lev = int(mesh.blocks[b, 2])
        return {"X0": mesh.ni * mesh.blocks[b, 3:6].astype(np.int64), "w": 1 << (mesh.L - lev),
                "Nu": mesh.ni << mesh.L, "periodic": mesh.periodic}

    def stage(self, act, s: int, rhs, sigma: float):
        """Stage s of every block of B_j: unzip, block RHS, zip into K_s."""
        for b in act:
            pad = self.unzip(b, s)
            h = h_level(int(self.mesh.blocks[b, 2]), self.n)     # block grid spacing h_lam
            grid = rhs(pad, h, sigma, self.geometry(b))
            self.zip_into(b, grid, self.K[s])

    def rk_update(self, act):
        """compute_step_partial: U_new = U0 + dt sum_i b_i K_i into the other buffer."""
        for b in act:
            octs = self.plan(b)["octs"].ravel()
            par = self.rec_par[b]
            dt = self.dt_phys(b)
            acc = np.zeros_like(self.U[par][:, octs])
            for i in range(self.p):
                acc += self.b[i] * self.K[i][:, octs]
            self.U[1 - par][:, octs] = self.U[par][:, octs] + dt * acc

    def substep(self, j: int, rhs, sigma: float):
        """Substep j of Alg. 2 (or one step of Alg. 1 in GTS mode)."""
        act = self.open_records(j)
        for s in range(self.p):
            self.stage(act, s, rhs, sigma)
        self.rk_update(act)
        self.close_records(act)


EQ = {"wave": (2, fd.rhs_wave), "maxwell": (6, fd.rhs_maxwell), "nlwave": (2, fd.rhs_nlwave)}


def run(mesh: Mesh, U0: np.ndarray, n_coarse: int, mode: str = "lts", equation: str = "wave",
        tableau: str = "rk4", sigma: float = 0.1, return_state: bool = False, nl_coeff: float = 1.0):
    """Advance U0 ([F][N][n][n][n]) by n_coarse coarsest steps (T = n_coarse dt_lmin).
    nl_coeff: the coefficient c of the non-linear source (equation "nlwave")."""
    F, rhs = EQ[equation]
    if equation == "nlwave":
        def rhs(pad, h, sg, geo, _c=nl_coeff):
            return fd.rhs_nlwave(pad, h, sg, geo, _c)
    st = State(mesh, F, tableau, mode)
    st.set_initial(U0)
    nsub = substeps(mesh)
    for _ in range(n_coarse):
        for j in range(nsub):
            st.substep(j, rhs, sigma)
    assert (st.cur_t == st.cur_t[0]).all()
    return st if return_state else st.current()
