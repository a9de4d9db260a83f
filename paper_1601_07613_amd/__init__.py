"""MI355X-native edge-colored DG surface integrals (Giuliani & Krivodonova, arXiv:1601.07613).

Thin Python binding over ``libdgc.so`` (C ABI in ``include/dgc.h``).  Every
step of the path runs in the native library: host C++ for the mesh build,
coloring and layout, HIP kernels for the volume and surface terms and the
SSP-RK3 stages.  PyTorch only provides device memory and the stream.  There
is no CPU fallback: if the library is missing the import fails.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (  # noqa: F401
    DGC_COLOR_GREEDY_STD, DGC_COLOR_PAPER, DGC_F32, DGC_F64, DGC_LAYOUT_NONE, DGC_LAYOUT_PAPER,
    DGC_LAYOUT_PAIRED, DGC_LAYOUT_PAPER_SFC, DGC_LAYOUT_RENUMBER, DGC_MIXED, DGC_QUAD, DGC_SURF_ATOMIC, DGC_SURF_COLORED, DGC_SURF_COMPACT,
    DGC_SURF_GATHER, DGC_TET,
    DGC_TRI, DgcError,
)

_L = _lib.load()

VARIANTS = {"colored": DGC_SURF_COLORED, "atomic": DGC_SURF_ATOMIC, "gather": DGC_SURF_GATHER,
            "compact": DGC_SURF_COMPACT}
PRECISIONS = {"f64": DGC_F64, "f32": DGC_F32}
LAYOUTS = {"paper": DGC_LAYOUT_PAPER, "renumber": DGC_LAYOUT_RENUMBER, "none": DGC_LAYOUT_NONE,
           "paper_sfc": DGC_LAYOUT_PAPER_SFC, "paired": DGC_LAYOUT_PAIRED}
ALGORITHMS = {"paper": DGC_COLOR_PAPER, "greedy": DGC_COLOR_GREEDY_STD}


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Mesh:
    """Host mesh owned by the library (face table, geometry, coloring, layout)."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle
        # held by the instance: module globals may already be cleared when
        # the interpreter finalises the last meshes
        self._free = _L.dgc_mesh_free

    @classmethod
    def build(cls, elem_vert, elem_xyz) -> "Mesh":
        ev = np.ascontiguousarray(elem_vert, dtype=np.int32)
        xyz = np.ascontiguousarray(elem_xyz, dtype=np.float64)
        if ev.shape[1] == 3:
            et = DGC_TRI
        elif xyz.shape[2] == 3:
            et = DGC_TET
        else:
            # a -1 fourth vertex marks a triangle of a mixed mesh
            et = DGC_MIXED if (ev[:, 3] < 0).any() else DGC_QUAD
        h = C.c_void_p()
        _lib.check(_L.dgc_mesh_build(et, ev.shape[0], _ptr(ev), _ptr(xyz), C.byref(h)), "dgc_mesh_build")
        return cls(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        free = getattr(self, "_free", None)
        if h is not None and h.value and free is not None:
            free(h)
            self._h = None

    def color(self, seed: int = 0, max_swaps: int = -1, algorithm: str = "paper", layout: str = "paper") -> dict:
        st = _lib.ColorStats()
        flags = ALGORITHMS[algorithm] | LAYOUTS[layout]
        _lib.check(_L.dgc_color_edges(self._h, seed, max_swaps, flags, C.byref(st)), "dgc_color_edges")
        return {
            "conflicts_after_greedy": st.conflicts_after_greedy, "swaps": st.swaps,
            "loop_breaks": st.loop_breaks, "deferrals": st.deferrals, "n_colors": st.n_colors,
            "count": list(st.count[: st.n_colors]), "color_ms": st.color_ms, "layout_ms": st.layout_ms,
        }

    def set_colors(self, colors, layout: str = "paper") -> None:
        c = np.ascontiguousarray(colors, dtype=np.int8)
        _lib.check(_L.dgc_set_colors(self._h, _ptr(c), LAYOUTS[layout]), "dgc_set_colors")

    def refine(self, flags) -> tuple["Mesh", int]:
        f = np.ascontiguousarray(flags, dtype=np.uint8)
        h = C.c_void_p()
        ncl = C.c_int64()
        _lib.check(_L.dgc_mesh_refine(self._h, _ptr(f), C.byref(h), C.byref(ncl)), "dgc_mesh_refine")
        return Mesh(h), int(ncl.value)

    def coarsen(self, flags) -> tuple["Mesh", int]:
        """Merge flagged sibling quadruples back into their parent; returns
        ``(mesh, number of merged families)``."""
        f = np.ascontiguousarray(flags, dtype=np.uint8)
        h = C.c_void_p()
        n = C.c_int64()
        _lib.check(_L.dgc_mesh_coarsen(self._h, _ptr(f), C.byref(h), C.byref(n)), "dgc_mesh_coarsen")
        return Mesh(h), int(n.value)

    def info(self) -> dict:
        i = _lib.MeshInfo()
        _lib.check(_L.dgc_mesh_info(self._h, C.byref(i)), "dgc_mesh_info")
        d = {name: getattr(i, name) for name, _ in _lib.MeshInfo._fields_}
        d["color_off"] = list(i.color_off[: i.n_colors + 1]) if i.n_colors else []
        return d

    def export(self, name: str) -> np.ndarray:
        which, dtype = _lib.ARR[name]
        need = C.c_size_t()
        _lib.check(_L.dgc_mesh_export(self._h, which, None, 0, C.byref(need)), "dgc_mesh_export")
        out = np.empty(need.value // np.dtype(dtype).itemsize, dtype=dtype)
        _lib.check(_L.dgc_mesh_export(self._h, which, _ptr(out), out.nbytes, None), "dgc_mesh_export")
        return out


def tables(elem_type: int, p: int):
    info = _lib.TableInfo()
    need = C.c_size_t()
    _lib.check(_L.dgc_tables(elem_type, p, C.byref(info), None, 0, C.byref(need)), "dgc_tables")
    out = np.empty(need.value // 8, dtype=np.float64)
    _lib.check(_L.dgc_tables(elem_type, p, C.byref(info), _ptr(out), out.nbytes, None), "dgc_tables")
    return {name: getattr(info, name) for name, _ in _lib.TableInfo._fields_}, out


def _stream_ptr(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class DeviceMesh:
    """Device-resident arrays of one laid-out mesh at order ``p`` (torch tensors)."""

    def __init__(self, mesh: Mesh, p: int, device="cuda", with_slots: bool = True):
        import torch

        info = mesh.info()
        if not info["n_colors"]:
            raise DgcError(-3, "DeviceMesh", "mesh is not colored")
        self.mesh = mesh
        self.p = p
        self.info = info
        self.dim = info["dim"]
        tinfo, tab = tables(info["elem_type"], p)
        self.tinfo = tinfo
        self.n_p = tinfo["n_p"]
        self.n_var = self.dim + 2
        self.K = info["n_elem"]
        self.E = info["n_face"]
        dev = torch.device(device)

        def up(a):
            return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

        self.face_lr = up(mesh.export("dev_face_lr"))
        self.face_code = up(mesh.export("dev_face_code"))
        self.face_geo = up(mesh.export("dev_face_geo"))
        self.elem_geo = up(mesh.export("dev_elem_geo"))
        self.elem_slots = up(mesh.export("dev_elem_slots")) if with_slots else None
        self.tables = up(tab)
        self.elem_kind = up(mesh.export("dev_elem_kind")) if info["elem_type"] == DGC_MIXED else None
        self.elem_new = mesh.export("elem_new").astype(np.int64)
        dm = _lib.DMesh()
        dm.elem_type = info["elem_type"]
        dm.p = p
        dm.n_p = tinfo["n_p"]
        dm.n_var = self.n_var
        dm.n_qf = tinfo["n_qf"]
        dm.n_qv = tinfo["n_qv"]
        dm.n_codes = tinfo["n_codes"]
        dm.n_orient = tinfo["n_orient"]
        dm.n_colors = info["n_colors"]
        dm.max_slots = info["max_slots"]
        dm.n_elem = self.K
        dm.n_face = self.E
        for c, v in enumerate(info["color_off"]):
            dm.color_off[c] = v
        dm.face_lr = self.face_lr.data_ptr()
        dm.face_code = self.face_code.data_ptr()
        dm.face_geo = self.face_geo.data_ptr()
        dm.elem_geo = self.elem_geo.data_ptr()
        dm.elem_slots = self.elem_slots.data_ptr() if self.elem_slots is not None else None
        dm.tables = self.tables.data_ptr()
        dm.surf_form = 0
        dm.block_size = 0
        dm.xcd_remap = 0
        dm.vol_form = 0
        dm.rk_form = 0
        dm.elem_kind = self.elem_kind.data_ptr() if self.elem_kind is not None else None
        self.dm = dm

    FORMS = {"default": 0, "team": 1, "thread": 2, "team_prefetch": 3, "mode_team": 4, "team_stream": 5,
             "pair_team": 6}
    VOL_FORMS = {"default": 0, "valu": 1, "mfma": 2, "team": 3}

    RK_FORMS = {"default": 0, "separate": 1, "fused": 2, "block": 3, "fused_volume": 4}

    def set_rk_form(self, form: str = "default") -> None:
        """SSP-RK3 step form: the stage combination fused into the last
        color's face kernel where exact ("fused"); in addition the volume term
        fused into the first color's face kernel ("fused_volume"); the
        combination as a separate kernel ("separate"); or the whole step in
        one work-group ("block", an alternative for small meshes, measured
        slower).  "default" is "fused_volume" for triangles at p <= 3,
        quadrilaterals (f32 only at p = 3) and f64 tetrahedra at p = 1 (with
        the default volume form), else "fused" (tetrahedra at p = 2:
        "separate")."""
        self.dm.rk_form = self.RK_FORMS[form]

    def set_volume_form(self, form: str = "default") -> None:
        """Volume-kernel form: one work-item per element ("valu"), a team of
        lanes per element ("team"), or the two basis contractions on the
        matrix cores ("mfma": 2D, f64, p <= 3); "default" picks the form
        measured fastest for the element type, order and precision."""
        self.dm.vol_form = self.VOL_FORMS[form]

    def set_launch(self, form: str = "default", block: int = 0, xcd_remap: bool = False) -> None:
        """Choose the face-kernel form ("team" of lanes per face, with the
        right-hand-side reads issued early "team_prefetch", visiting the
        quadrature points one at a time "team_stream", lane = mode
        "mode_team" for tetrahedra at p = 1, or one work-item per face
        "thread"), the work-group size (0 = library default) and whether
        work-groups are remapped to contiguous face ranges per XCD."""
        self.dm.surf_form = self.FORMS[form]
        self.dm.block_size = int(block)
        self.dm.xcd_remap = int(bool(xcd_remap))

    # -- DOF permutation between original element ids and layout ids --------
    def to_layout(self, U: np.ndarray) -> np.ndarray:
        out = np.empty_like(U)
        out[self.elem_new] = U
        return out

    def from_layout(self, Ul: np.ndarray) -> np.ndarray:
        return Ul[self.elem_new]

    def _perm_dev(self):
        import torch

        if getattr(self, "_perm", None) is None:
            self._perm = torch.from_numpy(self.elem_new.astype(np.int32)).to(self.face_lr.device)
        return self._perm

    def to_layout_device(self, U, stream=None):
        """Device gather of element records (caller's order) into the layout order."""
        import torch

        out = torch.empty_like(U)
        rb = U[0].numel() * U.element_size()
        _lib.check(_L.dgc_permute_records(U.data_ptr(), out.data_ptr(), self._perm_dev().data_ptr(), U.shape[0], rb, 1,
                                          _stream_ptr(stream)), "dgc_permute_records")
        return out

    def from_layout_device(self, Ul, stream=None):
        """Device gather of element records from the layout order back to the caller's order."""
        import torch

        out = torch.empty_like(Ul)
        rb = Ul[0].numel() * Ul.element_size()
        _lib.check(_L.dgc_permute_records(Ul.data_ptr(), out.data_ptr(), self._perm_dev().data_ptr(), Ul.shape[0], rb,
                                          0, _stream_ptr(stream)), "dgc_permute_records")
        return out

    def alloc(self, precision: str = "f64", zero: bool = True):
        import torch

        dt = torch.float64 if precision == "f64" else torch.float32
        shape = (self.K, self.n_var, self.n_p)
        return torch.zeros(shape, dtype=dt, device=self.face_lr.device) if zero else torch.empty(
            shape, dtype=dt, device=self.face_lr.device)

    def workspace_bytes(self, what: str = "surface", variant: str = "colored", precision: str = "f64") -> int:
        b = C.c_size_t()
        w = _lib.DGC_WS_SURFACE if what == "surface" else _lib.DGC_WS_RK_STEP
        _lib.check(_L.dgc_workspace_bytes(C.byref(self.dm), w, VARIANTS[variant], PRECISIONS[precision], C.byref(b)),
                   "dgc_workspace_bytes")
        return int(b.value)

    def workspace(self, what: str = "surface", variant: str = "colored", precision: str = "f64"):
        import torch

        n = self.workspace_bytes(what, variant, precision)
        return torch.empty(max(n, 1), dtype=torch.uint8, device=self.face_lr.device)

    def volume_rhs(self, U, rhs, precision: str = "f64", stream=None):
        _lib.check(_L.dgc_volume_rhs(C.byref(self.dm), U.data_ptr(), rhs.data_ptr(), PRECISIONS[precision],
                                     _stream_ptr(stream)), "dgc_volume_rhs")

    def surface_rhs(self, U, rhs, variant: str = "colored", precision: str = "f64", ws=None, stream=None):
        wp = ws.data_ptr() if ws is not None else None
        wb = ws.numel() * ws.element_size() if ws is not None else 0
        _lib.check(_L.dgc_surface_rhs(C.byref(self.dm), U.data_ptr(), rhs.data_ptr(), VARIANTS[variant],
                                      PRECISIONS[precision], wp, wb, _stream_ptr(stream)), "dgc_surface_rhs")

    def adapt_arrays(self):
        """Device copies (made once) of this mesh's origin arrays: kind
        ``[K]`` int8 and sources ``[4, K]`` int32, both in layout order."""
        if getattr(self, "_adapt", None) is None:
            dev = self.face_lr.device
            import torch

            self._adapt = (torch.from_numpy(self.mesh.export("dev_adapt_kind")).to(dev),
                           torch.from_numpy(self.mesh.export("dev_adapt_src")).to(dev))
        return self._adapt

    def transfer_from(self, U_old, stream=None):
        """Solution on this mesh (made by ``Mesh.refine`` / ``Mesh.coarsen``)
        from ``U_old`` (f64 device tensor ``[K_old, M, N_p]``, layout order of
        the mesh it was made from), by L2 projection on the device."""
        import torch

        if U_old.dtype != torch.float64 or not U_old.is_contiguous() or U_old.dim() != 3:
            raise ValueError("U_old must be a contiguous float64 [K, M, N_p] tensor")
        dev = U_old.device
        kind, src = self.adapt_arrays()
        U_new = torch.empty((self.K, self.n_var, self.n_p), dtype=torch.float64, device=dev)
        _lib.check(_L.dgc_adapt_transfer(C.byref(self.dm), U_old.data_ptr(), U_old.shape[0], U_new.data_ptr(),
                                         kind.data_ptr(), src.data_ptr(), _stream_ptr(stream)), "dgc_adapt_transfer")
        return U_new

    def rk_step(self, U, dt: float, variant: str = "colored", precision: str = "f64", ws=None, stream=None):
        if ws is None:
            ws = self.workspace("rk", variant, precision)
        _lib.check(_L.dgc_rk_step(C.byref(self.dm), U.data_ptr(), float(dt), VARIANTS[variant],
                                  PRECISIONS[precision], ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
                   "dgc_rk_step")

    def rk_step_noalloc(self, U, dt: float, variant: str = "colored", precision: str = "f64", stream=None):
        """``rk_step`` with the stage storage held by the library (no
        workspace, no allocation; at most ``DGC_NOALLOC_MAX_BYTES`` of stage
        storage; calls that overlap on one GPU race)."""
        _lib.check(_L.dgc_rk_step_noalloc(C.byref(self.dm), U.data_ptr(), float(dt), VARIANTS[variant],
                                          PRECISIONS[precision], _stream_ptr(stream)), "dgc_rk_step_noalloc")


def child_colors(parent_colors, stream=None):
    """Child-edge colors of split elements computed on the device: parent
    colors ``[n, 3]`` (int8 tensor on the GPU) -> ``[n, 9]``."""
    import torch

    out = torch.empty((parent_colors.shape[0], 9), dtype=torch.int8, device=parent_colors.device)
    _lib.check(_L.dgc_child_colors(parent_colors.data_ptr(), parent_colors.shape[0], out.data_ptr(),
                                   _stream_ptr(stream)), "dgc_child_colors")
    return out


def rk_workspace_layout(n: int, precision: str = "f64"):
    """Byte offsets (U1, U2, rhs, shadow) and size of the RK-stage workspace of ``n`` values."""
    off = (C.c_size_t * 4)()
    tot = C.c_size_t()
    _lib.check(_L.dgc_rk_workspace_layout(n, PRECISIONS[precision], off, C.byref(tot)), "dgc_rk_workspace_layout")
    return [int(x) for x in off], int(tot.value)


def device_footprint(mesh: Mesh, p: int, precision: str = "f64", variant: str = "colored") -> int:
    """Device bytes that ``DeviceMesh(mesh, p)``, one f64 state and its SSP-RK3
    workspace (``precision``, ``variant``) occupy: the sizes the library
    reports for every device array (face and element arrays, tables) and for
    the stage storage, each rounded up to 512 bytes as device allocations are."""
    info = mesh.info()
    tinfo, _ = tables(info["elem_type"], p)

    def rnd(b):
        return (int(b) + 511) // 512 * 512

    total = 0
    names = ["dev_face_lr", "dev_face_code", "dev_face_geo", "dev_elem_geo", "dev_elem_slots"]
    if info["elem_type"] == DGC_MIXED:
        names.append("dev_elem_kind")
    need = C.c_size_t()
    for name in names:
        _lib.check(_L.dgc_mesh_export(mesh._h, _lib.ARR[name][0], None, 0, C.byref(need)), "dgc_mesh_export")
        total += rnd(need.value)
    total += rnd(tinfo["total"] * 8)
    n = info["n_elem"] * (info["dim"] + 2) * tinfo["n_p"]
    total += rnd(n * 8)
    _, ws = rk_workspace_layout(n, precision)
    elt = 8 if precision == "f64" else 4
    if variant == "gather":
        ws += 2 * info["n_face"] * (info["dim"] + 2) * tinfo["n_p"] * elt
    elif variant == "compact":
        ws += info["n_face"] * (tinfo["n_qf"] * (info["dim"] + 2) + 1) * elt
    return total + rnd(ws)


class Batch:
    """Many meshes of one element type and order advanced together.

    ``members`` is a list of ``(DeviceMesh, U, ws, dt)``: the f64 state, the
    RK workspace (``DeviceMesh.workspace("rk", ..., precision)``) and the time
    step of each mesh.  The descriptor is built by the library on the host and
    copied to the device once; every batched call launches a fixed number of
    kernels whatever the number of meshes.
    """

    def __init__(self, members, precision: str = "f64", device="cuda"):
        import torch

        self.members = list(members)
        self.precision = precision
        n = len(self.members)
        self._dms = (_lib.DMesh * n)(*[m[0].dm for m in self.members])
        self._U = (C.c_void_p * n)(*[m[1].data_ptr() for m in self.members])
        self._ws = (C.c_void_p * n)(*[m[2].data_ptr() for m in self.members])
        self._dt = (C.c_double * n)(*[float(m[3]) for m in self.members])
        need = C.c_size_t()
        _lib.check(_L.dgc_batch_describe(n, self._dms, self._U, self._ws, self._dt, PRECISIONS[precision], None, 0,
                                         C.byref(need)), "dgc_batch_describe")
        self.host = np.zeros(need.value, dtype=np.uint8)
        _lib.check(_L.dgc_batch_describe(n, self._dms, self._U, self._ws, self._dt, PRECISIONS[precision],
                                         _ptr(self.host), self.host.nbytes, None), "dgc_batch_describe")
        self.dev = torch.from_numpy(self.host).to(device)

    def set_dt(self, dts) -> None:
        """Change the time steps in place (same descriptor size; safe between graph replays)."""
        for i, v in enumerate(dts):
            self._dt[i] = float(v)
        n = len(self.members)
        _lib.check(_L.dgc_batch_describe(n, self._dms, self._U, self._ws, self._dt, PRECISIONS[self.precision],
                                         _ptr(self.host), self.host.nbytes, None), "dgc_batch_describe")
        self.dev.copy_(torch_from(self.host), non_blocking=False)

    def surface(self, stage: int = 0, stream=None):
        _lib.check(_L.dgc_surface_rhs_batched(_ptr(self.host), self.dev.data_ptr(), stage, _stream_ptr(stream)),
                   "dgc_surface_rhs_batched")

    def volume(self, stage: int = 0, stream=None):
        _lib.check(_L.dgc_volume_rhs_batched(_ptr(self.host), self.dev.data_ptr(), stage, _stream_ptr(stream)),
                   "dgc_volume_rhs_batched")

    def rk_step(self, stream=None):
        _lib.check(_L.dgc_rk_step_batched(_ptr(self.host), self.dev.data_ptr(), _stream_ptr(stream)),
                   "dgc_rk_step_batched")

    def stage_rhs(self, i: int):
        """View of member ``i``'s stage right-hand side inside its workspace."""
        D, U, ws, _ = self.members[i]
        n = D.K * D.n_var * D.n_p
        off, _ = rk_workspace_layout(n, self.precision)
        import torch

        dt = torch.float64 if self.precision == "f64" else torch.float32
        elt = 8 if self.precision == "f64" else 4
        return ws[off[2]:off[2] + n * elt].view(dt).view(D.K, D.n_var, D.n_p)

    def capture(self, steps: int = 1, warm: bool = True):
        """Capture ``steps`` batched RK3 steps in a graph; returns the graph
        (replay with ``.replay()``).  ``warm`` first runs a stage-0 volume +
        surface evaluation, which loads the kernels before the capture (it
        writes only the stage right-hand side in the workspaces, never a
        state); a caller that has already stepped this batch may skip it."""
        import torch

        if warm:
            self.volume(0)
            self.surface(0)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(steps):
                self.rk_step()
        return g


def torch_from(a: np.ndarray):
    import torch

    return torch.from_numpy(a)
