"""ctypes declarations of include/lts.h and loading of the in-tree libltsmi.so.

Nothing here computes: every step of the method runs in the library's C++/HIP
code.  If the library is missing the import fails loudly (there is no CPU
fallback)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libltsmi.so")

MAX_LEVEL = 16

OK, EINVAL, ENOMEM, EDEVICE, EUNBALANCED, ENONFINITE, EUNSUPPORTED = range(7)
CRIT_BALL, CRIT_ANNULUS = 0, 1
MODE_LTS, MODE_GTS = 0, 1
EQ_WAVE, EQ_MAXWELL, EQ_NLWAVE = 0, 1, 2
BOUNDARY_PERIODIC, BOUNDARY_OUTER = 0, 1
ADVANCE_GRAPH, ADVANCE_CHECK_FINITE, ADVANCE_POISON = 1, 2, 4
FP64, FP32_RHS = 0, 1
RK4, SSPRK3 = 0, 1
EXPORT_LEAVES, EXPORT_BLOCKS, EXPORT_UNZIP_MAP, EXPORT_SCHEDULE, EXPORT_TILES, EXPORT_GHOSTS = range(6)

STATUS_NAMES = {0: "LTS_OK", 1: "LTS_EINVAL", 2: "LTS_ENOMEM", 3: "LTS_EDEVICE", 4: "LTS_EUNBALANCED",
                5: "LTS_ENONFINITE", 6: "LTS_EUNSUPPORTED"}


class Criterion(C.Structure):
    _fields_ = [("kind", C.c_int32), ("center", C.c_int32 * 3), ("r2", C.c_int64 * MAX_LEVEL),
                ("rlo2", C.c_int64 * MAX_LEVEL), ("rhi2", C.c_int64 * MAX_LEVEL)]


class MeshSpecC(C.Structure):
    _fields_ = [("l_min", C.c_int32), ("l_max", C.c_int32), ("block_cap", C.c_int32), ("n_criteria", C.c_int32),
                ("criteria", C.POINTER(Criterion)), ("n_leaves", C.c_int64), ("leaves", C.POINTER(C.c_int32)),
                ("boundary", C.c_int32), ("nodes", C.c_int32)]


class MeshInfo(C.Structure):
    _fields_ = [("n_oct", C.c_int64), ("n_blocks", C.c_int64), ("n_tiles", C.c_int64), ("L", C.c_int32),
                ("lmin", C.c_int32), ("lmax", C.c_int32), ("n_substeps", C.c_int32), ("tile", C.c_int32),
                ("level_count", C.c_int64 * MAX_LEVEL), ("unzip_points", C.c_int64), ("grid_points", C.c_int64),
                ("node_updates_lts", C.c_int64), ("node_updates_gts", C.c_int64), ("s_est", C.c_double),
                ("s_max", C.c_double), ("table_bytes", C.c_int64), ("ghost_entries", C.c_int64),
                ("boundary", C.c_int32), ("nodes", C.c_int32)]


class StageView(C.Structure):
    _fields_ = [("U", C.c_void_p), ("K", C.c_void_p), ("nfields", C.c_int32), ("precision", C.c_int32),
                ("tableau", C.c_int32)]


class Position(C.Structure):
    _fields_ = [("substep", C.c_int32), ("mode", C.c_int32), ("coarse_step", C.c_int64)]


class RhsParams(C.Structure):
    _fields_ = [("ko_sigma", C.c_double), ("nl_coeff", C.c_double)]


class BatchInfo(C.Structure):
    _fields_ = [("round", C.c_int64), ("rounds_to_drain", C.c_int64), ("attached", C.c_int32),
                ("capacity", C.c_int32)]


_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_DP = C.POINTER(C.c_double)

PROTOTYPES = {
    "lts_last_error": (C.c_char_p, []),
    "lts_version": (C.c_char_p, []),
    "lts_build_mesh": (C.c_int, [C.POINTER(MeshSpecC), C.POINTER(_P)]),
    "lts_mesh_destroy": (None, [_P]),
    "lts_mesh_query": (C.c_int, [_P, C.POINTER(MeshInfo)]),
    "lts_mesh_export": (C.c_int, [_P, C.c_int32, _P, C.c_size_t, C.POINTER(C.c_size_t)]),
    "lts_mesh_set_tile": (C.c_int, [_P, C.c_int32]),
    "lts_coefficients": (C.c_int, [C.c_int32, _DP, C.c_size_t]),
    "lts_unzip": (C.c_int, [_P, C.POINTER(StageView), C.c_int32, C.POINTER(Position), _I32P, C.c_int32, _P, _P]),
    "lts_rhs": (C.c_int, [_P, C.c_int32, C.POINTER(RhsParams), _P, C.c_int32, _I32P, C.c_int32, _P, _P]),
    "lts_zip": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _I32P, C.c_int32, _P, _P]),
    "lts_rk_stage": (C.c_int, [_P, C.POINTER(StageView), _DP, C.c_int32, C.POINTER(Position), _I32P, C.c_int32,
                               _P, _P]),
    "lts_fused_stage": (C.c_int, [_P, C.POINTER(StageView), C.c_int32, C.POINTER(RhsParams), C.c_int32,
                                  C.POINTER(Position), _P]),
    "lts_fused_stage_noalloc": (C.c_int, [_P, C.POINTER(StageView), C.c_int32, C.POINTER(RhsParams), C.c_int32,
                                          C.POINTER(Position), _P]),
    "lts_set_launch": (C.c_int, [C.c_int32, C.c_int32, C.c_int32]),
    "lts_get_launch": (C.c_int, [C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lts_set_batch_launch": (C.c_int, [C.c_int32, C.c_int32]),
    "lts_get_batch_launch": (C.c_int, [C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lts_sim_create": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(RhsParams), C.POINTER(_P)]),
    "lts_sim_bind": (C.c_int, [_P, _P, _P]),
    "lts_advance": (C.c_int, [_P, C.c_int64, C.c_int32, C.c_int32, _P]),
    "lts_advance_unfused": (C.c_int, [_P, C.c_int64, C.c_int32, _P]),
    "lts_sim_current": (C.c_int, [_P, _P, _P]),
    "lts_sim_restore": (C.c_int, [_P, _P, C.c_int64, C.c_int32, _P]),
    "lts_sim_coarse_step": (C.c_int64, [_P]),
    "lts_sim_destroy": (None, [_P]),
    "lts_batch_create": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(_P)]),
    "lts_batch_attach": (C.c_int, [_P, _P, C.c_int64]),
    "lts_batch_detach": (C.c_int, [_P, _P, _P]),
    "lts_batch_run": (C.c_int, [_P, C.c_int64, C.c_int32, _P]),
    "lts_batch_query": (C.c_int, [_P, C.POINTER(BatchInfo)]),
    "lts_sim_rounds_left": (C.c_int64, [_P]),
    "lts_batch_destroy": (None, [_P]),
    "lts_batch_advance": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_int64, C.c_int32, _P]),
    "lts_remesh_indicators": (C.c_int, [_P, C.c_int32, _P, _DP, _DP, _P]),
    "lts_remesh": (C.c_int, [_P, C.c_int32, _P, C.c_double, C.c_int32, C.c_int32, C.POINTER(_P), _P]),
    "lts_transfer": (C.c_int, [_P, _P, C.c_int32, _P, _P, _P]),
    "lts_norms": (C.c_int, [_P, C.c_int32, _P, _P, _DP, _P]),
    "lts_copy_probe": (C.c_int, [_P, _P, C.c_size_t, _P]),
}

_lib = None


class LTSError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib() -> C.CDLL:
    """The loaded library (raises if the in-tree build is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2011_10570_amd.build`")
        # torch bundles a HIP runtime with the same soname as the system one this
        # library links: load torch's first, so that the process holds one HIP
        # runtime (loaded the other way round, this library saw no device).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, where: str):
    if status != OK:
        raise LTSError(status, where, lib().lts_last_error().decode())
