"""MI355X octree local timestepping: thin Python binding of the C ABI (include/lts.h).

Names follow the C entry points (build_mesh, unzip, rhs, rk_stage, zip,
fused_stage, advance).  Arguments are marshalled to raw pointers; PyTorch is used
only for device memory and streams.  Every step of the method runs in the
library's HIP kernels; there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib as _L
from ._lib import (BOUNDARY_OUTER, BOUNDARY_PERIODIC, CRIT_ANNULUS, CRIT_BALL, EQ_MAXWELL, EQ_NLWAVE, EQ_WAVE,
                   FP32_RHS, FP64, MODE_GTS, MODE_LTS, RK4,
                   SSPRK3, LTSError, check, lib)

__all__ = ["Mesh", "Sim", "build_mesh", "unzip", "rhs", "zip", "rk_stage", "fused_stage", "coefficients",
           "norms", "copy_probe", "LTSError", "MODE_LTS", "MODE_GTS", "EQ_WAVE", "EQ_MAXWELL", "EQ_NLWAVE",
           "BOUNDARY_PERIODIC", "BOUNDARY_OUTER", "FP64", "FP32_RHS",
           "RK4", "SSPRK3", "Batch", "batch_advance", "set_launch", "get_launch", "fused_stage_noalloc",
           "remesh_indicators", "remesh", "transfer", "set_batch_launch", "get_batch_launch"]

EQUATIONS = {"wave": EQ_WAVE, "maxwell": EQ_MAXWELL, "nlwave": EQ_NLWAVE}
BOUNDARIES = {"periodic": BOUNDARY_PERIODIC, "outer": BOUNDARY_OUTER}
TABLEAUS = {"rk4": RK4, "ssprk3": SSPRK3}
NFIELDS = {EQ_WAVE: 2, EQ_MAXWELL: 6, EQ_NLWAVE: 2}
NSTAGES = {RK4: 4, SSPRK3: 3}


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return t.data_ptr()
    return int(t)


class Mesh:
    """Octree mesh (leaves, blocks, tiles, ghost tables) built by the library's host code."""

    def __init__(self, spec: Optional[dict] = None, leaves=None, L: Optional[int] = None, block_cap: int = 4,
                 boundary: str = "periodic", nodes: int = 5):
        """spec: a mesh specification dict (l_min, l_max, block_cap, criteria,
        boundary, nodes), or leaves [n][4] with L.  nodes: DG nodes per octant
        side, 5 or 7."""
        cs = _L.MeshSpecC()
        keep = []
        cs.boundary = BOUNDARIES[spec.get("boundary", "periodic") if spec is not None else boundary]
        cs.nodes = int(spec.get("nodes", 5) if spec is not None else nodes)
        if leaves is not None:
            arr = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
            keep.append(arr)
            cs.l_min = int(arr[:, 3].min())
            cs.l_max = int(L if L is not None else arr[:, 3].max())
            cs.block_cap = block_cap
            cs.n_leaves = len(arr)
            cs.leaves = arr.ctypes.data_as(C.POINTER(C.c_int32))
        else:
            cs.l_min = int(spec["l_min"])
            cs.l_max = int(spec["l_max"])
            cs.block_cap = int(spec.get("block_cap", 4))
            crits = spec.get("criteria", [])
            arr = (_L.Criterion * max(1, len(crits)))()
            for i, c in enumerate(crits):
                arr[i].kind = CRIT_BALL if c["kind"] == "ball" else CRIT_ANNULUS
                for d in range(3):
                    arr[i].center[d] = int(c["center"][d])
                for lev in range(_L.MAX_LEVEL):
                    for name in ("r2", "rlo2", "rhi2"):
                        vals = c.get(name, ())
                        getattr(arr[i], name)[lev] = int(vals[lev]) if lev < len(vals) else -1
            keep.append(arr)
            cs.n_criteria = len(crits)
            cs.criteria = arr
        h = C.c_void_p()
        check(lib().lts_build_mesh(C.byref(cs), C.byref(h)), "lts_build_mesh")
        self.h = h

    @classmethod
    def _wrap(cls, h) -> "Mesh":
        """A Mesh owning a handle the library built (lts_remesh)."""
        obj = cls.__new__(cls)
        obj.h = h
        return obj

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                lib().lts_mesh_destroy(h)
            except Exception:
                pass
            self.h = None

    @property
    def _as_parameter_(self):
        return self.h

    def info(self) -> dict:
        inf = _L.MeshInfo()
        check(lib().lts_mesh_query(self.h, C.byref(inf)), "lts_mesh_query")
        d = {k: getattr(inf, k) for k, _ in inf._fields_}
        d["level_count"] = list(inf.level_count)
        return d

    def export(self, kind: int) -> np.ndarray:
        need = C.c_size_t()
        check(lib().lts_mesh_export(self.h, kind, None, 0, C.byref(need)), "lts_mesh_export")
        buf = np.empty(need.value // 4, dtype=np.int32)
        check(lib().lts_mesh_export(self.h, kind, buf.ctypes.data, need.value, C.byref(need)), "lts_mesh_export")
        return buf

    def leaves(self) -> np.ndarray:
        return self.export(_L.EXPORT_LEAVES).reshape(-1, 4)

    def blocks(self) -> np.ndarray:
        return self.export(_L.EXPORT_BLOCKS).reshape(-1, 6)

    def unzip_map(self) -> np.ndarray:
        return self.export(_L.EXPORT_UNZIP_MAP).reshape(-1, 5)

    def schedule(self) -> list:
        raw = self.export(_L.EXPORT_SCHEDULE)
        out, i = [], 0
        while i < len(raw):
            n = int(raw[i])
            out.append(raw[i + 1:i + 1 + n].copy())
            i += 1 + n
        return out

    def tiles(self) -> np.ndarray:
        return self.export(_L.EXPORT_TILES).reshape(-1, 8)

    def ghosts(self) -> np.ndarray:
        """Ghost table [E][8]: coarser source leaf, receiver level, read box
        (x lo, x hi, y lo, y hi, z lo, z hi on the source's half-node grid)."""
        raw = self.export(_L.EXPORT_GHOSTS).reshape(-1, 2)
        out = np.empty((len(raw), 8), np.int64)
        out[:, 0] = raw[:, 0]
        out[:, 1] = raw[:, 1] & 31
        for k in range(6):
            out[:, 2 + k] = (raw[:, 1] >> (5 + 4 * k)) & 15
        return out

    def set_tile(self, t: int):
        check(lib().lts_mesh_set_tile(self.h, int(t)), "lts_mesh_set_tile")


def build_mesh(spec: Optional[dict] = None, leaves=None, L: Optional[int] = None, block_cap: int = 4) -> Mesh:
    return Mesh(spec, leaves=leaves, L=L, block_cap=block_cap)


def coefficients(tableau: int = RK4) -> dict:
    p = NSTAGES[tableau]
    out = np.empty(4 * p * p + p * p + p)
    check(lib().lts_coefficients(tableau, out.ctypes.data_as(C.POINTER(C.c_double)), out.nbytes), "lts_coefficients")
    return {"w": out[:4 * p * p].reshape(4, p, p), "a": out[4 * p * p:5 * p * p].reshape(p, p),
            "b": out[5 * p * p:]}


def _view(U, K, nfields, precision, tableau):
    v = _L.StageView()
    v.U = _ptr(U)
    v.K = _ptr(K)
    v.nfields = nfields
    v.precision = precision
    v.tableau = tableau
    return v


def _pos(substep, mode, coarse_step):
    p = _L.Position()
    p.substep = int(substep)
    p.mode = int(mode)
    p.coarse_step = int(coarse_step)
    return p


def _blocks_arg(blocks):
    if blocks is None:
        return None, 0, None
    arr = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32))
    return arr.ctypes.data_as(C.POINTER(C.c_int32)), len(arr), arr


def unzip(mesh: Mesh, U, K, stage: int, substep: int, mode: int, coarse_step: int, blocks, padded,
          nfields: int = 2, precision: int = FP64, tableau: int = RK4, stream=None):
    b, nb, keep = _blocks_arg(blocks)
    v = _view(U, K, nfields, precision, tableau)
    p = _pos(substep, mode, coarse_step)
    check(lib().lts_unzip(mesh.h, C.byref(v), stage, C.byref(p), b, nb, _ptr(padded), _stream_ptr(stream)),
          "lts_unzip")


def _params(ko_sigma: float, nl_coeff: float = 1.0):
    prm = _L.RhsParams()
    prm.ko_sigma = ko_sigma
    prm.nl_coeff = nl_coeff
    return prm


def rhs(mesh: Mesh, equation: int, ko_sigma: float, padded, precision: int, blocks, k_block, stream=None,
        nl_coeff: float = 1.0):
    b, nb, keep = _blocks_arg(blocks)
    prm = _params(ko_sigma, nl_coeff)
    check(lib().lts_rhs(mesh.h, equation, C.byref(prm), _ptr(padded), precision, b, nb, _ptr(k_block),
                        _stream_ptr(stream)), "lts_rhs")


def zip(mesh: Mesh, nfields: int, precision: int, k_block, blocks, k_octant, stream=None):
    b, nb, keep = _blocks_arg(blocks)
    check(lib().lts_zip(mesh.h, nfields, precision, _ptr(k_block), b, nb, _ptr(k_octant), _stream_ptr(stream)),
          "lts_zip")


def rk_stage(mesh: Mesh, U, K, coef: Sequence[float], substep: int, mode: int, coarse_step: int, blocks, out,
             nfields: int = 2, precision: int = FP64, tableau: int = RK4, stream=None):
    b, nb, keep = _blocks_arg(blocks)
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64))
    v = _view(U, K, nfields, precision, tableau)
    p = _pos(substep, mode, coarse_step)
    check(lib().lts_rk_stage(mesh.h, C.byref(v), c.ctypes.data_as(C.POINTER(C.c_double)), len(c), C.byref(p), b, nb,
                             _ptr(out), _stream_ptr(stream)), "lts_rk_stage")


def fused_stage(mesh: Mesh, U, K, equation: int, ko_sigma: float, stage: int, substep: int, mode: int,
                coarse_step: int, precision: int = FP64, tableau: int = RK4, stream=None, nl_coeff: float = 1.0):
    v = _view(U, K, NFIELDS[equation], precision, tableau)
    prm = _params(ko_sigma, nl_coeff)
    p = _pos(substep, mode, coarse_step)
    check(lib().lts_fused_stage(mesh.h, C.byref(v), equation, C.byref(prm), stage, C.byref(p), _stream_ptr(stream)),
          "lts_fused_stage")


def fused_stage_noalloc(mesh: Mesh, U, K, equation: int, ko_sigma: float, stage: int, substep: int, mode: int,
                        coarse_step: int, precision: int = FP64, tableau: int = RK4, stream=None,
                        nl_coeff: float = 1.0):
    """lts_fused_stage_noalloc: the fused stage with the library's fixed device scratch."""
    v = _view(U, K, NFIELDS[equation], precision, tableau)
    prm = _params(ko_sigma, nl_coeff)
    p = _pos(substep, mode, coarse_step)
    check(lib().lts_fused_stage_noalloc(mesh.h, C.byref(v), equation, C.byref(prm), stage, C.byref(p),
                                        _stream_ptr(stream)), "lts_fused_stage_noalloc")


def remesh_indicators(mesh: Mesh, state, nfields: int = 2, stream=None):
    """lts_remesh_indicators: (leaf indicator [N], family indicator [N], -1 where a
    leaf does not start a complete sibling family) of a device state [F][N][125]."""
    N = mesh.info()["n_oct"]
    lw = np.zeros(N)
    fw = np.zeros(N)
    check(lib().lts_remesh_indicators(mesh.h, nfields, _ptr(state), lw.ctypes.data_as(C.POINTER(C.c_double)),
                                      fw.ctypes.data_as(C.POINTER(C.c_double)), _stream_ptr(stream)),
          "lts_remesh_indicators")
    return lw, fw


def remesh(mesh: Mesh, state, eps: float, l_min: int, l_max: int, nfields: int = 2, stream=None) -> Mesh:
    """lts_remesh: the new octree of a state at a coarse-step boundary."""
    h = C.c_void_p()
    check(lib().lts_remesh(mesh.h, nfields, _ptr(state), float(eps), int(l_min), int(l_max), C.byref(h),
                           _stream_ptr(stream)), "lts_remesh")
    return Mesh._wrap(h)


def transfer(src: Mesh, dst: Mesh, state, nfields: int = 2, stream=None):
    """lts_transfer: the state [F][N_src][125] (device) carried to dst's leaves."""
    import torch
    out = torch.empty((nfields, dst.info()["n_oct"], 125), dtype=torch.float64, device=state.device)
    check(lib().lts_transfer(src.h, dst.h, nfields, _ptr(state), _ptr(out), _stream_ptr(stream)), "lts_transfer")
    return out


def norms(mesh: Mesh, a, b=None, nfields: int = 2, stream=None) -> dict:
    out = np.zeros(2 * nfields + 1)
    st = lib().lts_norms(mesh.h, nfields, _ptr(a), _ptr(b), out.ctypes.data_as(C.POINTER(C.c_double)),
                         _stream_ptr(stream))
    if st not in (_L.OK, _L.ENONFINITE):
        check(st, "lts_norms")
    return {"l2": out[:nfields].copy(), "linf": out[nfields:2 * nfields].copy(), "nonfinite": int(out[-1])}


def set_launch(threads: int, max_workgroups: int, stream_threads: int = 512):
    """Launch shape of every later fused launch: threads of the LDS tile kernels and
    of the streaming kernel (256 or 512 each), grid cap in workgroups."""
    check(lib().lts_set_launch(int(threads), int(max_workgroups), int(stream_threads)), "lts_set_launch")


def set_batch_launch(threads: int, max_workgroups: int):
    check(lib().lts_set_batch_launch(int(threads), int(max_workgroups)), "lts_set_batch_launch")


def get_batch_launch() -> tuple:
    a, b = C.c_int32(), C.c_int32()
    check(lib().lts_get_batch_launch(C.byref(a), C.byref(b)), "lts_get_batch_launch")
    return a.value, b.value


def get_launch() -> tuple:
    """(threads, max_workgroups, stream_threads)"""
    t, w, st = C.c_int32(), C.c_int32(), C.c_int32()
    check(lib().lts_get_launch(C.byref(t), C.byref(w), C.byref(st)), "lts_get_launch")
    return t.value, w.value, st.value


def copy_probe(src, dst, nbytes: int, stream=None):
    check(lib().lts_copy_probe(_ptr(src), _ptr(dst), nbytes, _stream_ptr(stream)), "lts_copy_probe")


class Sim:
    """One simulation: device state U [2][F][N][n^3] (float64) and stages K
    [p][F][N][n^3] (float64, or float32 in FP32-RHS mode) as torch tensors, n the
    mesh's nodes per octant side (5 or 7)."""

    def __init__(self, mesh: Mesh, equation="wave", precision=FP64, tableau="rk4", ko_sigma=0.1, device="cuda",
                 nl_coeff: float = 1.0):
        import torch
        self.mesh = mesh
        self.eq = EQUATIONS[equation] if isinstance(equation, str) else int(equation)
        self.tab = TABLEAUS[tableau] if isinstance(tableau, str) else int(tableau)
        self.prec = int(precision)
        self.F = NFIELDS[self.eq]
        self.p = NSTAGES[self.tab]
        prm = _params(ko_sigma, nl_coeff)
        self.ko_sigma = ko_sigma
        h = C.c_void_p()
        check(lib().lts_sim_create(mesh.h, self.eq, self.prec, self.tab, C.byref(prm), C.byref(h)), "lts_sim_create")
        self.h = h
        inf = mesh.info()
        N = inf["n_oct"]
        self.N = N
        self.nn = inf["nodes"] ** 3
        self.U = torch.zeros((2, self.F, N, self.nn), dtype=torch.float64, device=device)
        kdt = torch.float32 if self.prec == FP32_RHS else torch.float64
        self.K = torch.zeros((self.p, self.F, N, self.nn), dtype=kdt, device=device)
        check(lib().lts_sim_bind(self.h, _ptr(self.U), _ptr(self.K)), "lts_sim_bind")
        self._mode = MODE_LTS

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                lib().lts_sim_destroy(h)
            except Exception:
                pass
            self.h = None

    def set_state(self, U0):
        """U0: [F][N][n][n][n] or [F][N][n^3] (numpy or torch); resets the step counter."""
        import torch
        t = torch.as_tensor(np.asarray(U0) if not hasattr(U0, "device") else U0, dtype=torch.float64)
        self.U.zero_()
        self.K.zero_()
        self.U[0].copy_(t.reshape(self.F, self.N, self.nn).to(self.U.device))
        check(lib().lts_sim_bind(self.h, _ptr(self.U), _ptr(self.K)), "lts_sim_bind")

    def advance(self, n_coarse: int, mode: int = MODE_LTS, graph: bool = True, stream=None, check_finite=False,
                poison: bool = False):
        """n coarse steps; with check_finite the call synchronises and raises
        LTSError (status LTS_ENONFINITE) if an RK update wrote a NaN or Inf.
        poison (race check, debug): every stage's K entries of its active octants
        are set to NaN before the stage runs."""
        flags = ((_L.ADVANCE_GRAPH if graph else 0) | (_L.ADVANCE_CHECK_FINITE if check_finite else 0) |
                 (_L.ADVANCE_POISON if poison else 0))
        check(lib().lts_advance(self.h, int(n_coarse), int(mode), flags, _stream_ptr(stream)), "lts_advance")
        self._mode = int(mode)

    def checkpoint(self, stream=None) -> dict:
        """State at the current coarse-step boundary (host arrays, no pickling)."""
        return {"state": self.current(stream).cpu().numpy(), "coarse_step": self.coarse_step,
                "mode": int(self._mode), "equation": int(self.eq), "tableau": int(self.tab),
                "precision": int(self.prec)}

    def restore(self, ckpt: dict, stream=None):
        """Continue from a checkpoint (bitwise the uninterrupted run)."""
        import torch
        for k in ("equation", "tableau", "precision"):
            if int(ckpt[k]) != int(getattr(self, {"equation": "eq", "tableau": "tab", "precision": "prec"}[k])):
                raise ValueError(f"checkpoint {k} differs from the sim's")
        st = torch.as_tensor(np.asarray(ckpt["state"]), dtype=torch.float64).to(self.U.device).contiguous()
        self.U.zero_()
        self.K.zero_()
        check(lib().lts_sim_bind(self.h, _ptr(self.U), _ptr(self.K)), "lts_sim_bind")
        check(lib().lts_sim_restore(self.h, _ptr(st), int(ckpt["coarse_step"]), int(ckpt["mode"]),
                                    _stream_ptr(stream)), "lts_sim_restore")
        self._mode = int(ckpt["mode"])
        self._keep = st      # the restore kernel reads it asynchronously

    @staticmethod
    def save_checkpoint(ckpt: dict, path: str):
        np.savez(path, **{k: np.asarray(v) for k, v in ckpt.items()})

    @staticmethod
    def load_checkpoint(path: str) -> dict:
        with np.load(path, allow_pickle=False) as z:
            return {k: (z[k] if k == "state" else int(z[k])) for k in z.files}

    def advance_unfused(self, n_coarse: int, mode: int = MODE_LTS, stream=None):
        check(lib().lts_advance_unfused(self.h, int(n_coarse), int(mode), _stream_ptr(stream)), "lts_advance_unfused")
        self._mode = int(mode)

    def current(self, stream=None):
        import torch
        out = torch.empty((self.F, self.N, self.nn), dtype=torch.float64, device=self.U.device)
        check(lib().lts_sim_current(self.h, _ptr(out), _stream_ptr(stream)), "lts_sim_current")
        return out

    @property
    def coarse_step(self) -> int:
        return int(lib().lts_sim_coarse_step(self.h))

    @property
    def rounds_left(self) -> int:
        """Rounds this sim still takes part in while attached to a Batch (else 0)."""
        return int(lib().lts_sim_rounds_left(self.h))


class Batch:
    """Continuous batching of independent sims (one equation, precision, tableau
    and mode): round r runs every attached sim's own substep; each stage of a
    round is one launch per tile side over the union of their active tiles."""

    def __init__(self, equation="wave", precision=FP64, tableau="rk4", mode: int = MODE_LTS, capacity: int = 64):
        self.eq = EQUATIONS[equation] if isinstance(equation, str) else int(equation)
        self.tab = TABLEAUS[tableau] if isinstance(tableau, str) else int(tableau)
        h = C.c_void_p()
        check(lib().lts_batch_create(self.eq, int(precision), self.tab, int(mode), int(capacity), C.byref(h)),
              "lts_batch_create")
        self.h = h
        self._attached = {}   # id(sim) -> sim (keeps attached sims alive)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                lib().lts_batch_destroy(h)
            except Exception:
                pass
            self.h = None

    def attach(self, sim: "Sim", n_coarse: int):
        check(lib().lts_batch_attach(self.h, sim.h, int(n_coarse)), "lts_batch_attach")
        if sim.rounds_left > 0:
            self._attached[id(sim)] = sim

    def detach(self, sim: "Sim", stream=None):
        check(lib().lts_batch_detach(self.h, sim.h, _stream_ptr(stream)), "lts_batch_detach")
        self._attached.pop(id(sim), None)

    def run(self, n_rounds: int, graph: bool = True, stream=None) -> list:
        """Enqueue n rounds (graph-captured rounds by default); returns the sims
        that finished in them."""
        check(lib().lts_batch_run(self.h, int(n_rounds), 1 if graph else 0, _stream_ptr(stream)), "lts_batch_run")
        done = [s for s in self._attached.values() if s.rounds_left == 0]
        for s in done:
            del self._attached[id(s)]
        return done

    def info(self) -> dict:
        i = _L.BatchInfo()
        check(lib().lts_batch_query(self.h, C.byref(i)), "lts_batch_query")
        return {"round": i.round, "rounds_to_drain": i.rounds_to_drain, "attached": i.attached,
                "capacity": i.capacity}

    def drain(self, graph: bool = True, stream=None) -> list:
        return self.run(self.info()["rounds_to_drain"], graph, stream)


def batch_advance(sims: Sequence["Sim"], n_coarse: int, mode: int = MODE_LTS, stream=None):
    """Advance every sim n_coarse coarse steps in one batch."""
    arr = (C.c_void_p * len(sims))(*[s.h.value for s in sims])
    check(lib().lts_batch_advance(arr, len(sims), int(n_coarse), int(mode), _stream_ptr(stream)),
          "lts_batch_advance")
