"""ctypes declarations of the C ABI in ``include/dgc.h`` (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libdgc.so"

DGC_TRI, DGC_QUAD, DGC_TET, DGC_MIXED = 0, 1, 2, 3
DGC_COLOR_PAPER, DGC_COLOR_GREEDY_STD = 0x01, 0x02
DGC_LAYOUT_PAPER, DGC_LAYOUT_RENUMBER, DGC_LAYOUT_NONE, DGC_LAYOUT_PAPER_SFC = 0x10, 0x20, 0x40, 0x80
DGC_LAYOUT_PAIRED = 0x100
DGC_MAX_COLORS = 8
DGC_SURF_COLORED, DGC_SURF_ATOMIC, DGC_SURF_GATHER, DGC_SURF_COMPACT = 0, 1, 2, 3
DGC_F64, DGC_F32 = 0, 1
DGC_WS_SURFACE, DGC_WS_RK_STEP = 0, 1
DGC_NOALLOC_MAX_BYTES = 64 << 20
DGC_FORM_DEFAULT, DGC_FORM_TEAM, DGC_FORM_THREAD = 0, 1, 2

STATUS = {
    0: "DGC_OK", -1: "DGC_E_ARG", -2: "DGC_E_MESH", -3: "DGC_E_NOT_COLORED", -4: "DGC_E_COLOR_CAP",
    -5: "DGC_E_COLORING_INVALID", -6: "DGC_E_UNSUPPORTED", -7: "DGC_E_WORKSPACE", -8: "DGC_E_HIP",
    -9: "DGC_E_ALLOC",
}

ARR = {
    "face_elem": (1, "int32"), "face_local": (2, "int8"), "color": (3, "int8"),
    "face_normal": (4, "float64"), "face_measure": (5, "float64"), "elem_detj": (6, "float64"),
    "elem_face": (7, "int32"), "elem_new": (10, "int32"), "face_order": (11, "int32"),
    "color_off": (12, "int64"), "dev_face_lr": (20, "int32"), "dev_face_code": (21, "uint8"),
    "dev_face_geo": (22, "float64"), "dev_elem_geo": (23, "float64"), "dev_elem_slots": (24, "int32"),
    "elem_level": (30, "int8"), "elem_xyz": (31, "float64"), "elem_vert": (32, "int32"),
    "adapt_kind": (33, "int8"), "adapt_src": (34, "int32"), "dev_adapt_kind": (25, "int8"),
    "dev_adapt_src": (26, "int32"), "dev_elem_kind": (27, "int8"),
}


class ColorStats(C.Structure):
    _fields_ = [
        ("conflicts_after_greedy", C.c_int64), ("swaps", C.c_int64), ("loop_breaks", C.c_int64),
        ("deferrals", C.c_int64), ("n_colors", C.c_int32), ("pad_", C.c_int32),
        ("count", C.c_int64 * DGC_MAX_COLORS), ("color_ms", C.c_double), ("layout_ms", C.c_double),
    ]


class MeshInfo(C.Structure):
    _fields_ = [
        ("elem_type", C.c_int32), ("dim", C.c_int32), ("n_vert_per_elem", C.c_int32),
        ("n_face_per_elem", C.c_int32), ("max_slots", C.c_int32), ("n_colors", C.c_int32),
        ("n_elem", C.c_int64), ("n_face", C.c_int64), ("n_boundary", C.c_int64),
        ("color_off", C.c_int64 * (DGC_MAX_COLORS + 1)), ("n_orient", C.c_int32), ("max_level", C.c_int32),
    ]


class TableInfo(C.Structure):
    _fields_ = [
        ("elem_type", C.c_int32), ("p", C.c_int32), ("dim", C.c_int32), ("n_p", C.c_int32),
        ("n_qf", C.c_int32), ("n_qv", C.c_int32), ("n_codes", C.c_int32), ("n_orient", C.c_int32),
        ("off_trace", C.c_int64), ("off_proj", C.c_int64), ("off_vb", C.c_int64), ("off_vd", C.c_int64),
        ("off_prolong", C.c_int64), ("total", C.c_int64),
    ]


class DMesh(C.Structure):
    _fields_ = [
        ("elem_type", C.c_int32), ("p", C.c_int32), ("n_p", C.c_int32), ("n_var", C.c_int32),
        ("n_qf", C.c_int32), ("n_qv", C.c_int32), ("n_codes", C.c_int32), ("n_orient", C.c_int32),
        ("n_colors", C.c_int32), ("max_slots", C.c_int32),
        ("n_elem", C.c_int64), ("n_face", C.c_int64),
        ("color_off", C.c_int64 * (DGC_MAX_COLORS + 1)),
        ("face_lr", C.c_void_p), ("face_code", C.c_void_p), ("face_geo", C.c_void_p),
        ("elem_geo", C.c_void_p), ("elem_slots", C.c_void_p), ("tables", C.c_void_p),
        ("surf_form", C.c_int32), ("block_size", C.c_int32), ("xcd_remap", C.c_int32), ("vol_form", C.c_int32),
        ("rk_form", C.c_int32), ("pad_", C.c_int32), ("elem_kind", C.c_void_p),
    ]


_SIGS = {
    "dgc_mesh_build": (C.c_int, [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "dgc_color_edges": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int64, C.c_uint32, C.POINTER(ColorStats)]),
    "dgc_set_colors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32]),
    "dgc_mesh_refine": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64)]),
    "dgc_mesh_coarsen": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64)]),
    "dgc_adapt_transfer": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "dgc_mesh_info": (C.c_int, [C.c_void_p, C.POINTER(MeshInfo)]),
    "dgc_mesh_export": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "dgc_mesh_free": (None, [C.c_void_p]),
    "dgc_last_error": (C.c_char_p, []),
    "dgc_version": (C.c_char_p, []),
    "dgc_tables": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(TableInfo), C.c_void_p, C.c_size_t,
                             C.POINTER(C.c_size_t)]),
    "dgc_volume_rhs": (C.c_int, [C.POINTER(DMesh), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "dgc_surface_rhs": (C.c_int, [C.POINTER(DMesh), C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                  C.c_size_t, C.c_void_p]),
    "dgc_rk_step": (C.c_int, [C.POINTER(DMesh), C.c_void_p, C.c_double, C.c_int32, C.c_int32, C.c_void_p,
                              C.c_size_t, C.c_void_p]),
    "dgc_rk_step_noalloc": (C.c_int, [C.POINTER(DMesh), C.c_void_p, C.c_double, C.c_int32, C.c_int32, C.c_void_p]),
    "dgc_workspace_bytes": (C.c_int, [C.POINTER(DMesh), C.c_int32, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_size_t)]),
    "dgc_permute_records": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int32,
                                      C.c_void_p]),
    "dgc_child_colors": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "dgc_rk_workspace_layout": (C.c_int, [C.c_int64, C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "dgc_batch_describe": (C.c_int, [C.c_int32, C.POINTER(DMesh), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_double), C.c_int32, C.c_void_p, C.c_size_t,
                                     C.POINTER(C.c_size_t)]),
    "dgc_surface_rhs_batched": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "dgc_volume_rhs_batched": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "dgc_rk_step_batched": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
}


def exported_symbols():
    """Names of the C ABI entry points the binding declares."""
    return list(_SIGS)


_lib = None


def _preload_torch_hip_runtime():
    """Make the HIP runtime that PyTorch ships the one libdgc binds to.

    libdgc.so needs ``libamdhip64.so.7``; when torch's copy (same soname) is
    already mapped, the dynamic loader reuses it, so device pointers and
    streams from torch and the library's launches share one runtime.
    """
    try:
        import torch
    except ImportError:
        return None
    path = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
    if os.path.exists(path):
        C.CDLL(path, mode=C.RTLD_GLOBAL)
        return path
    return None


def hip_runtimes_mapped():
    """Distinct libamdhip64 files mapped into this process."""
    try:
        with open("/proc/self/maps") as fh:
            return sorted({line.split()[-1] for line in fh if "libamdhip64" in line})
    except OSError:
        return []


def load():
    """Load ``libdgc.so`` from the package directory; raise ImportError when it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError("libdgc.so is not built; run `python paper_1601_07613_amd/build.py`")
    _preload_torch_hip_runtime()
    lib = C.CDLL(os.fspath(LIB_PATH))
    rts = hip_runtimes_mapped()
    if len(rts) > 1:
        raise ImportError("two HIP runtimes are mapped (%s); import torch before libdgc" % ", ".join(rts))
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DgcError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__("%s failed with %s: %s" % (where, self.name, msg))


def check(code: int, where: str) -> None:
    if code != 0:
        raise DgcError(code, where, load().dgc_last_error().decode(errors="replace"))
