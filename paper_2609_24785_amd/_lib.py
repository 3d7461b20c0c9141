"""ctypes declarations of the C ABI in include/lee.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LEE_LIB_PATH selects another build of the same library (e.g. for A/B timing)
LIB_PATH = os.environ.get("LEE_LIB_PATH") or os.path.join(HERE, "liblee.so")

LEE_OK = 0
STATUS = {0: "LEE_OK", -1: "LEE_E_ARG", -2: "LEE_E_GEOMETRY", -3: "LEE_E_CRITICAL_DAMPING",
          -4: "LEE_E_ADE_STIFF", -5: "LEE_E_RANK", -6: "LEE_E_NOMEM", -7: "LEE_E_DEVICE",
          -8: "LEE_E_STATE", -9: "LEE_E_PROBE"}
F32, F64 = 0, 1
WALL = {"none": 0, "line": 1, "circle": 2}
Z_RIGID, Z_MSD, Z_POLES = 0, 1, 2

c_int32, c_int64, c_double, c_void_p, c_size_t = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                   ctypes.c_void_p, ctypes.c_size_t)


class CaseDesc(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("x0", c_double), ("y0", c_double), ("h", c_double),
                ("stencil_half", c_int32), ("cfl", c_double), ("filter_sigma", c_double),
                ("sponge_cells", c_int32), ("sponge_sigma", c_double), ("precision", c_int32),
                ("wall_kind", c_int32), ("wall_cx", c_double), ("wall_cy", c_double),
                ("wall_nx", c_double), ("wall_ny", c_double), ("wall_rc", c_double),
                ("ic_kind", c_int32), ("ic", c_double * 7), ("src_kind", c_int32), ("src", c_double * 5),
                ("radiation", c_int32), ("rad_xc", c_double), ("rad_yc", c_double),
                ("filter_explicit", c_int32)]


ADE_MAX_STATES = 8


class ImpedanceDesc(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("R", c_double), ("M", c_double), ("K", c_double),
                ("n_real", c_int32), ("real_pole", c_double * ADE_MAX_STATES),
                ("real_res", c_double * ADE_MAX_STATES), ("n_pair", c_int32),
                ("pair_alpha", c_double * (ADE_MAX_STATES // 2)), ("pair_beta", c_double * (ADE_MAX_STATES // 2)),
                ("pair_B", c_double * (ADE_MAX_STATES // 2)), ("pair_C", c_double * (ADE_MAX_STATES // 2))]


class GhostSummary(ctypes.Structure):
    _fields_ = [("G", c_int32), ("nnz", c_int64), ("n_degraded", c_int32), ("n_cut", c_int32),
                ("r_min", c_double), ("r_max", c_double), ("w_l1_max", c_double),
                ("fluid_nodes", c_int64), ("ade_kind", c_int32), ("poles", c_double * 4),
                ("ade_states", c_int32)]


SWEEP_TILE, SWEEP_MARCH = 0, 1


class Tiling(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("vec", c_int32), ("cols", c_int32), ("rows", c_int32), ("waves", c_int32),
                ("fused", c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchOpts(ctypes.Structure):
    _fields_ = [("tiling", Tiling), ("persistent_blocks", c_int32), ("graph_steps", c_int32)]


# name -> (restype, argtypes)
SIGNATURES = {
    "lee_last_error": (ctypes.c_char_p, []),
    "lee_setup_grid": (c_int32, [ctypes.POINTER(CaseDesc), ctypes.POINTER(c_void_p)]),
    "lee_build_ghosts": (c_int32, [c_void_p, ctypes.POINTER(ImpedanceDesc), c_int32, ctypes.POINTER(GhostSummary)]),
    "lee_required_bytes": (c_int32, [c_void_p, ctypes.POINTER(c_size_t)]),
    "lee_bind": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "lee_init_fields": (c_int32, [c_void_p]),
    "lee_rk_stage": (c_int32, [c_void_p, c_int32]),
    "lee_step_n": (c_int32, [c_void_p, c_int64]),
    "lee_set_probes": (c_int32, [c_void_p, c_int32, c_void_p, c_int64, c_double, c_int64, c_int64]),
    "lee_probe": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "lee_probe_traces": (c_int32, [c_void_p, c_void_p, c_int64, ctypes.POINTER(c_int64)]),
    "lee_probe_dft": (c_int32, [c_void_p, c_void_p]),
    "lee_get_fields": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "lee_set_fields": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "lee_get_ade_states": (c_int32, [c_void_p, c_void_p]),
    "lee_set_ade_states": (c_int32, [c_void_p, c_void_p]),
    "lee_rhs": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lee_get_step": (c_int32, [c_void_p, ctypes.POINTER(c_int64)]),
    "lee_export_lists": (c_int32, [c_void_p] + [c_void_p] * 7),
    "lee_set_tiling": (c_int32, [c_void_p, ctypes.POINTER(Tiling)]),
    "lee_get_tiling": (c_int32, [c_void_p, ctypes.POINTER(Tiling)]),
    "lee_time_kernels": (c_int32, [c_void_p, c_int64, ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                   ctypes.POINTER(c_double)]),
    "lee_stream_copy": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "lee_synchronize": (c_int32, [c_void_p]),
    "lee_set_watch": (c_int32, [c_void_p, c_double, c_double, c_int64, ctypes.POINTER(c_int32)]),
    "lee_watch_traces": (c_int32, [c_void_p, c_void_p, c_int64, ctypes.POINTER(c_int64)]),
    "lee_set_graph_steps": (c_int32, [c_void_p, c_int32]),
    "lee_set_ghost_wait": (c_int32, [c_void_p, c_int32]),
    "lee_batch_synchronize": (c_int32, [c_void_p]),
    "lee_batch_add": (c_int32, [c_void_p, c_void_p]),
    "lee_batch_remove": (c_int32, [c_void_p, c_void_p]),
    "lee_batch_update": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_int32]),
    "lee_batch_size": (c_int32, [c_void_p, ctypes.POINTER(c_int32)]),
    "lee_batch_graph_captures": (c_int32, [c_void_p, ctypes.POINTER(c_int64)]),
    "lee_batch_set_tiling": (c_int32, [c_void_p, ctypes.POINTER(Tiling)]),
    "lee_batch_get_tiling": (c_int32, [c_void_p, ctypes.POINTER(Tiling)]),
    "lee_batch_set_graph_steps": (c_int32, [c_void_p, c_int32]),
    "lee_destroy": (None, [c_void_p]),
    "lee_batch_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32, ctypes.POINTER(BatchOpts),
                                   ctypes.POINTER(c_void_p)]),
    "lee_batch_set_budget": (c_int32, [c_void_p, c_void_p]),
    "lee_batch_step_n": (c_int32, [c_void_p, c_int64]),
    "lee_batch_time_kernels": (c_int32, [c_void_p, c_int64, ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                         ctypes.POINTER(c_double)]),
    "lee_batch_destroy": (None, [c_void_p]),
    "lee_step_members_noalloc": (c_int32, [ctypes.POINTER(c_void_p), c_int32, ctypes.POINTER(Tiling), c_int64]),
}

_lib = None


class LeeError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


_use_torch = True


def without_torch() -> None:
    """Before the first load: the process binds its instances through hipmem
    and never imports torch, so the library uses the system HIP runtime."""
    global _use_torch
    if _lib is not None:
        raise RuntimeError("liblee.so is already loaded")
    _use_torch = False


def load() -> ctypes.CDLL:
    """Load liblee.so; raises if it has not been built (no fallback path).

    torch is imported first: it ships its own HIP runtime under the same
    soname as the system one the library links, and whichever loads first is
    the one the process uses.  Loading torch's first keeps a single runtime
    for the tensors that hold the library's memory and for its launches
    (unless without_torch() was called)."""
    global _lib
    if _lib is None:
        if _use_torch:
            import torch  # noqa: F401  (selects the process's HIP runtime)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2609_24785_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, where: str) -> None:
    if status != LEE_OK:
        msg = load().lee_last_error()
        raise LeeError(status, where, msg.decode() if msg else "")
