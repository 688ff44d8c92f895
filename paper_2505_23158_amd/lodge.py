"""ctypes binding of liblodge.so (include/lodge.h), names kept one-to-one.

Argument marshalling only: every step of a frame runs in the HIP kernels of
liblodge.so.  PyTorch supplies device memory (tensors) and streams.  If the
library is missing or cannot be loaded this module raises; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblodge.so")

LODGE_OK, LODGE_ERR_INVALID_ARG, LODGE_ERR_CAPACITY, LODGE_ERR_HIP, LODGE_ERR_UNSUPPORTED = range(5)
SELECT_ALL, SELECT_LOD_CAMERA, SELECT_CHUNKED = 0, 1, 2
MAX_LEVELS = 8
MAX_CHUNKS = 128
TILE = 16


class LodgeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lodge status {status}: {msg}")
        self.status = status


# --------------------------------------------------------------------------- structs

class lodge_level(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p), ("sh_degree", C.c_int32), ("filter3d_var", C.c_float)]


class lodge_chunks(C.Structure):
    _fields_ = [("k", C.c_int32), ("center", C.c_void_p), ("offset", C.c_void_p), ("band", C.c_float)]


class lodge_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("pos", C.c_float * 3), ("znear", C.c_float), ("lim_x", C.c_float), ("lim_y", C.c_float),
                ("bg", C.c_float * 3)]


class lodge_workspace(C.Structure):
    _fields_ = [("base", C.c_void_p), ("bytes", C.c_size_t), ("width", C.c_int32), ("height", C.c_int32),
                ("max_active", C.c_uint32), ("max_instances", C.c_uint64)]


class lodge_selection(C.Structure):
    _fields_ = [("ids", C.c_void_p), ("w", C.c_void_p), ("count", C.c_void_p), ("cap", C.c_uint32)]


class lodge_render_opts(C.Structure):
    _fields_ = [("s2d", C.c_float), ("compensate", C.c_int32), ("stage_events", C.c_void_p)]


STAGE_EVENTS = 5


class lodge_frame_info(C.Structure):
    _fields_ = [("n_selected", C.c_uint32), ("n_front", C.c_uint32), ("n_visible", C.c_uint32),
                ("max_tile_len", C.c_uint32), ("n_instances", C.c_uint64), ("pairs_evaluated", C.c_uint64),
                ("pairs_blended", C.c_uint64), ("overflow", C.c_uint32), ("f", C.c_int32), ("o", C.c_int32),
                ("t", C.c_float), ("n_long", C.c_uint32), ("n_merge", C.c_uint32),
                ("pixels_stopped", C.c_uint64)]


class lodge_grads(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p), ("opacity", C.c_void_p),
                ("sh", C.c_void_p)]


# --------------------------------------------------------------------------- library

_lib = None


def lib():
    """The loaded liblodge.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        # torch first: liblodge.so then binds to the HIP runtime torch already
        # loaded (same soname), so streams and memory are shared.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_23158_amd.build`")
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        vp = C.c_void_p
        sig = {
            "lodge_status_string": (C.c_char_p, [st]),
            "lodge_last_error": (C.c_char_p, []),
            "lodge_version": (C.c_char_p, []),
            "lodge_scene_create": (st, [C.POINTER(lodge_level), C.c_int32, vp, C.POINTER(lodge_chunks),
                                        C.POINTER(vp)]),
            "lodge_scene_destroy": (None, [vp]),
            "lodge_scene_total": (C.c_int64, [vp]),
            "lodge_workspace_size": (st, [vp, C.c_int32, C.c_int32, C.c_uint32, C.c_uint64, C.POINTER(C.c_size_t)]),
            "lodge_pack_size": (st, [vp, C.POINTER(C.c_size_t)]),
            "lodge_scene_pack": (st, [vp, vp, C.c_size_t, vp]),
            "lodge_set_camera": (st, [C.POINTER(lodge_workspace), vp, vp]),
            "lodge_select": (st, [vp, vp, C.c_int32, C.POINTER(lodge_workspace), C.POINTER(lodge_selection), vp]),
            "lodge_chunk_sets_size": (st, [vp, C.POINTER(C.c_size_t)]),
            "lodge_chunk_sets_build": (st, [vp, vp, C.c_size_t, vp]),
            "lodge_select_chunk_sets": (st, [vp, vp, vp, C.POINTER(lodge_workspace), C.POINTER(lodge_selection),
                                             vp]),
            "lodge_select_chunk": (st, [vp, vp, C.c_int32, C.POINTER(lodge_workspace), C.POINTER(lodge_selection),
                                        vp]),
            "lodge_importance": (st, [vp, C.POINTER(lodge_selection), vp, C.POINTER(lodge_render_opts),
                                      C.POINTER(lodge_workspace), vp, vp]),
            "lodge_chunk_sets_prune": (st, [vp, vp, C.c_size_t, C.c_int32, vp, C.c_float, vp]),
            "lodge_render": (st, [vp, C.POINTER(lodge_selection), vp, C.POINTER(lodge_render_opts),
                                  C.POINTER(lodge_workspace), vp, vp, vp, vp]),
            "lodge_frame_info_read": (st, [C.POINTER(lodge_workspace), C.POINTER(lodge_frame_info), vp]),
            "lodge_check": (st, [C.POINTER(lodge_workspace), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), vp]),
            "lodge_debug_views": (st, [C.POINTER(lodge_workspace), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                       C.POINTER(vp), C.POINTER(vp)]),
            "lodge_render_backward": (st, [vp, C.POINTER(lodge_selection), vp, C.POINTER(lodge_render_opts),
                                           C.POINTER(lodge_workspace), vp, vp, vp, C.c_int32,
                                           C.POINTER(lodge_grads), vp]),
            "lodge_render_static": (st, [vp, C.POINTER(lodge_selection), vp, C.POINTER(lodge_render_opts), vp, vp,
                                         vp, vp, vp]),
            "lodge_l1_grad": (st, [C.c_int64, vp, vp, C.c_float, vp, vp, vp]),
            "lodge_adam": (st, [C.c_int64, vp, vp, vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32,
                                vp]),
            "lodge_keep_scratch_size": (st, [C.c_int64, C.POINTER(C.c_size_t)]),
            "lodge_dssim_scratch_size": (st, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
            "lodge_dssim_grad": (st, [C.c_int32, C.c_int32, C.c_int32, vp, vp, C.c_float, vp, vp, vp, C.c_size_t,
                                      vp]),
            "lodge_keep_indices": (st, [C.c_int64, vp, C.c_float, vp, vp, vp, C.c_size_t, vp]),
            "lodge_gather_planes": (st, [C.c_int32, C.c_int64, C.c_int64, vp, vp, vp, vp, vp]),
            "lodge_microbench_copy": (st, [vp, vp, C.c_size_t, vp]),
            "lodge_microbench_read_blocks": (st, [C.c_size_t, C.POINTER(C.c_uint32)]),
            "lodge_microbench_read": (st, [vp, C.c_size_t, vp, C.c_uint32, vp]),
            "lodge_microbench_fma": (st, [vp, C.c_uint32, C.c_uint32, C.c_float, C.c_float, vp]),
            "lodge_fp32_div_sqrt": (st, [vp, vp, vp, vp, C.c_size_t, vp]),
            "lodge_activate": (st, [C.c_int64, vp, vp, vp, vp, vp, vp, vp]),
            "lodge_activate_backward": (st, [C.c_int64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != LODGE_OK:
        raise LodgeError(status, lib().lodge_last_error().decode())


EXPORTED = ["lodge_status_string", "lodge_last_error", "lodge_version", "lodge_scene_create", "lodge_scene_destroy",
            "lodge_scene_total", "lodge_workspace_size", "lodge_set_camera", "lodge_select", "lodge_chunk_sets_size",
            "lodge_chunk_sets_build", "lodge_select_chunk_sets", "lodge_render", "lodge_frame_info_read",
            "lodge_check", "lodge_debug_views", "lodge_render_backward", "lodge_activate", "lodge_activate_backward",
            "lodge_render_static", "lodge_select_chunk", "lodge_importance", "lodge_chunk_sets_prune",
            "lodge_l1_grad", "lodge_adam", "lodge_keep_scratch_size", "lodge_keep_indices", "lodge_gather_planes",
            "lodge_pack_size", "lodge_scene_pack", "lodge_dssim_scratch_size", "lodge_dssim_grad",
            "lodge_microbench_copy", "lodge_microbench_read_blocks", "lodge_microbench_read", "lodge_microbench_fma",
            "lodge_fp32_div_sqrt"]
STATIC_SCRATCH_BYTES = 256 << 20


# --------------------------------------------------------------------------- helpers

def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_ptr(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _event_array(stage_events, n: int):
    """hipEvent_t array of torch.cuda.Event objects.  torch creates an event's HIP handle at its first record(), so
    each must have been recorded once."""
    if stage_events is None:
        return None
    if len(stage_events) < n:
        raise ValueError(f"stage_events: {n} events needed, {len(stage_events)} given")
    handles = [e.cuda_event for e in stage_events]
    if any(h == 0 for h in handles):
        raise ValueError("stage_events: record() each event once before passing it (its HIP event is created then)")
    return (C.c_void_p * len(handles))(*handles)


def make_camera(cam) -> lodge_camera:
    """lodge_camera from any object with the synth.Camera fields."""
    c = lodge_camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    for i, v in enumerate(np.asarray(cam.R, np.float32).ravel()):
        c.R[i] = float(v)
    for i in range(3):
        c.t[i] = float(cam.t[i])
        c.pos[i] = float(cam.pos[i])
        c.bg[i] = float(cam.bg[i])
    c.znear, c.lim_x, c.lim_y = float(cam.znear), float(cam.lim_x), float(cam.lim_y)
    return c


# --------------------------------------------------------------------------- objects

class Scene:
    """A lodge_scene over device tensors (levels stay owned by this object)."""

    def __init__(self, levels: Sequence[dict], d: Sequence[float], chunks=None):
        torch = _torch()
        self.levels = []
        arr = (lodge_level * len(levels))()
        for i, lv in enumerate(levels):
            keep = {k: lv[k] for k in ("mean", "scale", "quat", "opacity", "sh")}
            for k, t in keep.items():
                if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                    raise ValueError(f"level {i} {k}: need a contiguous float32 CUDA tensor")
            n = int(keep["mean"].shape[-1])
            deg = int(lv.get("sh_degree", 3))
            nsh = (deg + 1) ** 2
            shapes = {"mean": (3, n), "scale": (3, n), "quat": (4, n), "opacity": (n,)}
            for k, shp in shapes.items():
                if tuple(keep[k].shape) != shp:
                    raise ValueError(f"level {i} {k}: shape {tuple(keep[k].shape)} != {shp}")
            if keep["sh"].shape[-1] != n or keep["sh"].numel() < nsh * 3 * n:
                raise ValueError(f"level {i} sh: need at least [{nsh}][3][{n}]")
            arr[i].n = n
            arr[i].mean, arr[i].scale, arr[i].quat = _ptr(keep["mean"]), _ptr(keep["scale"]), _ptr(keep["quat"])
            arr[i].opacity, arr[i].sh = _ptr(keep["opacity"]), _ptr(keep["sh"])
            arr[i].sh_degree = deg
            arr[i].filter3d_var = float(lv.get("filter3d_var", 0.0))
            self.levels.append(dict(keep, n=n, sh_degree=deg, filter3d_var=arr[i].filter3d_var))
        self._arr = arr
        self.d = np.asarray(list(d) if d is not None else [], np.float32)
        ch = None
        if chunks is not None:
            self.centers = np.ascontiguousarray(chunks.centers, np.float32)
            self.offsets = np.ascontiguousarray(chunks.offsets, np.float32)
            ch = lodge_chunks(k=len(self.centers), center=self.centers.ctypes.data, offset=self.offsets.ctypes.data,
                              band=float(chunks.band))
        h = C.c_void_p()
        _check(lib().lodge_scene_create(arr, len(levels), self.d.ctypes.data if len(self.d) else None,
                                        C.byref(ch) if ch is not None else None, C.byref(h)))
        self.handle = h
        self.total = int(lib().lodge_scene_total(h))

    def pack(self, stream=None):
        """Fills a packed copy of the levels (lodge_scene_pack) that the projection then reads; the copy is
        owned by this object.  Call again after changing the level parameters."""
        torch = _torch()
        nb = C.c_size_t()
        _check(lib().lodge_pack_size(self.handle, C.byref(nb)))
        if getattr(self, "_pack", None) is None or self._pack.numel() < int(nb.value) + 256:
            self._pack = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device="cuda")
        base = self._pack.data_ptr()
        off = (-base) % 256
        _check(lib().lodge_scene_pack(self.handle, C.c_void_p(base + off), C.c_size_t(nb.value), _stream_ptr(stream)))
        return int(nb.value)

    def unpack(self):
        _check(lib().lodge_scene_pack(self.handle, None, 0, None))
        self._pack = None

    @classmethod
    def from_synth(cls, sc, device="cuda"):
        torch = _torch()
        levels = []
        for lv in sc.levels:
            nsh = (lv.sh_degree + 1) ** 2
            levels.append(dict(mean=torch.from_numpy(lv.mean).to(device), scale=torch.from_numpy(lv.scale).to(device),
                               quat=torch.from_numpy(lv.quat).to(device),
                               opacity=torch.from_numpy(lv.opacity).to(device),
                               sh=torch.from_numpy(np.ascontiguousarray(lv.sh[:nsh])).to(device),
                               sh_degree=lv.sh_degree, filter3d_var=lv.filter3d_var))
        return cls(levels, sc.d, sc.chunks)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.lodge_scene_destroy(h)
            self.handle = None


class Workspace:
    """Caller-owned device scratch for one frame in flight (a torch uint8 tensor)."""

    def __init__(self, scene: Scene, width: int, height: int, max_active: int, max_instances: int, device="cuda"):
        torch = _torch()
        nb = C.c_size_t()
        _check(lib().lodge_workspace_size(scene.handle, width, height, max_active, max_instances, C.byref(nb)))
        self.tensor = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=device)
        base = self.tensor.data_ptr()
        self.offset = (-base) % 256
        self.desc = lodge_workspace(base=base + self.offset, bytes=int(nb.value), width=width, height=height,
                                    max_active=max_active, max_instances=max_instances)
        self.width, self.height = width, height
        self.max_active, self.max_instances = max_active, max_instances

    def view(self, ptr: int, nbytes: int, dtype):
        torch = _torch()
        off = ptr - self.tensor.data_ptr()
        return self.tensor[off:off + nbytes].view(dtype)


class Selection:
    def __init__(self, cap: int, device="cuda"):
        torch = _torch()
        self.ids = torch.empty(max(cap, 1), dtype=torch.int32, device=device)
        self.w = torch.empty(max(cap, 1), dtype=torch.float32, device=device)
        self.count = torch.zeros(1, dtype=torch.int32, device=device)
        self.desc = lodge_selection(ids=_ptr(self.ids), w=_ptr(self.w), count=_ptr(self.count), cap=cap)
        self.cap = cap


# --------------------------------------------------------------------------- calls

def _cam_arg(cam):
    """(pointer, keep-alive) for a camera argument; None = the camera stored on the workspace."""
    if cam is None:
        return None, None
    c = cam if isinstance(cam, lodge_camera) else make_camera(cam)
    return C.c_void_p(C.addressof(c)), c


def lodge_set_camera(ws: "Workspace", cam, stream=None):
    cp, keep = _cam_arg(cam)
    _check(lib().lodge_set_camera(C.byref(ws.desc), cp, _stream_ptr(stream)))


def lodge_select(scene: Scene, cam, mode: int, ws: Workspace, sel: Selection, stream=None):
    cp, keep = _cam_arg(cam)
    _check(lib().lodge_select(scene.handle, cp, mode, C.byref(ws.desc), C.byref(sel.desc), _stream_ptr(stream)))


class ChunkSets:
    """Device buffer of a scene's precomputed per-chunk active sets (lodge_chunk_sets_build)."""

    def __init__(self, scene: Scene, stream=None, device="cuda"):
        torch = _torch()
        nb = C.c_size_t()
        _check(lib().lodge_chunk_sets_size(scene.handle, C.byref(nb)))
        self.bytes = int(nb.value)
        self.buf = torch.empty(max(4, self.bytes), dtype=torch.uint8, device=device)
        self.scene = scene
        _check(lib().lodge_chunk_sets_build(scene.handle, _ptr(self.buf), C.c_size_t(self.bytes),
                                            _stream_ptr(stream)))


def lodge_select_chunk_sets(scene: Scene, sets: ChunkSets, cam, ws: Workspace, sel: Selection, stream=None):
    cp, keep = _cam_arg(cam)
    _check(lib().lodge_select_chunk_sets(scene.handle, _ptr(sets.buf), cp, C.byref(ws.desc), C.byref(sel.desc),
                                         _stream_ptr(stream)))


def lodge_select_chunk(scene: Scene, sets: Optional[ChunkSets], k: int, ws: Workspace, sel: Selection, stream=None):
    _check(lib().lodge_select_chunk(scene.handle, _ptr(sets.buf) if sets is not None else None, int(k),
                                    C.byref(ws.desc), C.byref(sel.desc), _stream_ptr(stream)))


def lodge_importance(scene: Scene, sel: Selection, cam, ws: Workspace, score, s2d: float = 0.3,
                     compensate: bool = True, stream=None, stage_events=None):
    """score: float32 CUDA tensor of scene.total elements, max-accumulated by global id.
    stage_events: None or STAGE_EVENTS torch.cuda.Event objects (the last two bracket the importance walk)."""
    if score.numel() != scene.total or score.dtype != _torch().float32 or not score.is_contiguous():
        raise ValueError("score must be a contiguous float32 tensor of scene.total elements")
    cp, keep = _cam_arg(cam)
    evs = _event_array(stage_events, STAGE_EVENTS)
    opts = lodge_render_opts(s2d=s2d, compensate=int(compensate), stage_events=C.cast(evs, C.c_void_p) if evs else None)
    _check(lib().lodge_importance(scene.handle, C.byref(sel.desc), cp, C.byref(opts), C.byref(ws.desc),
                                  _ptr(score), _stream_ptr(stream)))


def lodge_chunk_sets_prune(scene: Scene, sets: ChunkSets, k: int, score, threshold: float, stream=None):
    _check(lib().lodge_chunk_sets_prune(scene.handle, _ptr(sets.buf), C.c_size_t(sets.bytes), int(k), _ptr(score),
                                        float(threshold), _stream_ptr(stream)))


def lodge_render(scene: Scene, sel: Selection, cam, ws: Workspace, image, final_T, n_contrib, s2d: float = 0.3,
                 compensate: bool = True, stream=None, stage_events=None):
    """stage_events: None or STAGE_EVENTS torch.cuda.Event objects recorded at the stage boundaries."""
    cp, keep = _cam_arg(cam)
    evs = _event_array(stage_events, STAGE_EVENTS)
    opts = lodge_render_opts(s2d=s2d, compensate=int(compensate), stage_events=C.cast(evs, C.c_void_p) if evs else None)
    _check(lib().lodge_render(scene.handle, C.byref(sel.desc), cp, C.byref(opts), C.byref(ws.desc), _ptr(image),
                              _ptr(final_T), _ptr(n_contrib), _stream_ptr(stream)))


def lodge_render_static(scene: Scene, sel: Selection, cam, image, final_T, n_contrib, overflow=None, s2d: float = 0.3,
                        compensate: bool = True, stream=None):
    """lodge_render with the library's static scratch in place of a workspace (allocates nothing);
    overflow: None or a device int32 tensor of one element that receives the overflow bits."""
    if cam is None:
        raise ValueError("lodge_render_static needs a camera")
    cp, keep = _cam_arg(cam)
    opts = lodge_render_opts(s2d=s2d, compensate=int(compensate))
    _check(lib().lodge_render_static(scene.handle, C.byref(sel.desc), cp, C.byref(opts), _ptr(image), _ptr(final_T),
                                     _ptr(n_contrib), _ptr(overflow), _stream_ptr(stream)))


def lodge_frame_info_read(ws: Workspace, stream=None) -> dict:
    fi = lodge_frame_info()
    _check(lib().lodge_frame_info_read(C.byref(ws.desc), C.byref(fi), _stream_ptr(stream)))
    return {k: getattr(fi, k) for k, _ in lodge_frame_info._fields_}


def lodge_check(ws: Workspace, stream=None):
    na, ni = C.c_uint32(), C.c_uint64()
    st = lib().lodge_check(C.byref(ws.desc), C.byref(na), C.byref(ni), _stream_ptr(stream))
    return st, int(na.value), int(ni.value)


def lodge_debug_views(ws: Workspace, n_instances: int):
    """Views into ws: sorted_ids [M] int32, tile_ranges [T, 2] int32, proj [max_active, 12] float32
    (u, v, -A/2, -B, -C/2, o_eff, thr, r, g, b, ex, ey: the conic (A, B, C) pre-scaled as the
    compositor reads it), depth [max_active] float32, rect [max_active, 2] int32."""
    torch = _torch()
    s, r, p, d, rc = C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_void_p()
    _check(lib().lodge_debug_views(C.byref(ws.desc), C.byref(s), C.byref(r), C.byref(p), C.byref(d), C.byref(rc)))
    T = ((ws.width + TILE - 1) // TILE) * ((ws.height + TILE - 1) // TILE)
    sorted_ids = ws.view(s.value, 4 * n_instances, torch.int32)
    ranges = ws.view(r.value, 8 * T, torch.int32).view(T, 2)
    proj = ws.view(p.value, 48 * ws.max_active, torch.float32).view(ws.max_active, 12)
    depth = ws.view(d.value, 4 * ws.max_active, torch.float32)
    rect = ws.view(rc.value, 8 * ws.max_active, torch.int32).view(ws.max_active, 2)
    return sorted_ids, ranges, proj, depth, rect


def lodge_render_backward(scene: Scene, sel: Selection, cam, ws: Workspace, final_T, n_contrib, dL_dimage,
                          grads: Sequence[dict], grad_level: int = -1, s2d: float = 0.3, compensate: bool = True,
                          stream=None, stage_events=None):
    """stage_events: None or three torch.cuda.Event objects, recorded before the compositing adjoint, between it
    and the projection adjoint, and after."""
    cp, keep = _cam_arg(cam)
    evs = _event_array(stage_events, 3)
    opts = lodge_render_opts(s2d=s2d, compensate=int(compensate),
                             stage_events=C.cast(evs, C.c_void_p) if evs else None)
    arr = (lodge_grads * len(scene.levels))()
    for i, g in enumerate(grads):
        for k in ("mean", "scale", "quat", "opacity", "sh"):
            setattr(arr[i], k, _ptr(g.get(k)))
    _check(lib().lodge_render_backward(scene.handle, C.byref(sel.desc), cp, C.byref(opts), C.byref(ws.desc),
                                       _ptr(final_T), _ptr(n_contrib), _ptr(dL_dimage), grad_level, arr,
                                       _stream_ptr(stream)))


def lodge_activate(log_scale, quat_raw, opacity_logit, scale, quat, opacity, stream=None):
    n = int(opacity_logit.numel())
    _check(lib().lodge_activate(n, _ptr(log_scale), _ptr(quat_raw), _ptr(opacity_logit), _ptr(scale), _ptr(quat),
                                _ptr(opacity), _stream_ptr(stream)))


def lodge_activate_backward(quat_raw, scale, opacity, g_scale, g_quat, g_opacity, g_log_scale, g_quat_raw,
                            g_opacity_logit, stream=None):
    n = int(opacity.numel())
    _check(lib().lodge_activate_backward(n, _ptr(quat_raw), _ptr(scale), _ptr(opacity), _ptr(g_scale), _ptr(g_quat),
                                         _ptr(g_opacity), _ptr(g_log_scale), _ptr(g_quat_raw),
                                         _ptr(g_opacity_logit), _stream_ptr(stream)))


def lodge_l1_grad(image, target, grad, scale: float, loss=None, stream=None):
    n = int(image.numel())
    if target.numel() != n or grad.numel() != n:
        raise ValueError("image, target and grad must have the same size")
    _check(lib().lodge_l1_grad(n, _ptr(image), _ptr(target), float(scale), _ptr(grad), _ptr(loss),
                               _stream_ptr(stream)))


def lodge_adam(param, grad, m, v, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999,
               eps: float = 1e-15, stream=None):
    n = int(param.numel())
    if not (grad.numel() == m.numel() == v.numel() == n):
        raise ValueError("param, grad, m and v must have the same size")
    _check(lib().lodge_adam(n, _ptr(param), _ptr(grad), _ptr(m), _ptr(v), float(lr), float(beta1), float(beta2),
                            float(eps), int(step), _stream_ptr(stream)))


def lodge_dssim_grad(image, target, grad, weight: float, loss=None, scratch=None, stream=None):
    """image, target, grad: [C, H, W] float32 CUDA tensors; grad += weight * d(1 - mean SSIM)/d image.
    Returns the scratch tensor used (pass it back to reuse it)."""
    torch = _torch()
    Cc, H, W = image.shape
    nb = C.c_size_t()
    _check(lib().lodge_dssim_scratch_size(int(W), int(H), int(Cc), C.byref(nb)))
    if scratch is None or scratch.numel() * scratch.element_size() < nb.value:
        scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=image.device)
    _check(lib().lodge_dssim_grad(int(W), int(H), int(Cc), _ptr(image), _ptr(target), float(weight), _ptr(grad),
                                  _ptr(loss), _ptr(scratch), C.c_size_t(scratch.numel()), _stream_ptr(stream)))
    return scratch


def lodge_keep_indices(score, threshold: float, idx, count, scratch=None, stream=None):
    """idx: int32 tensor (>= score.numel()), count: int32 tensor [1]; returns the scratch used."""
    torch = _torch()
    n = int(score.numel())
    nb = C.c_size_t()
    _check(lib().lodge_keep_scratch_size(n, C.byref(nb)))
    if scratch is None or scratch.numel() * scratch.element_size() < nb.value:
        scratch = torch.empty(max(4, int(nb.value)), dtype=torch.uint8, device=score.device)
    _check(lib().lodge_keep_indices(n, _ptr(score), float(threshold), _ptr(idx), _ptr(count), _ptr(scratch),
                                    C.c_size_t(scratch.numel()), _stream_ptr(stream)))
    return scratch


def lodge_gather_planes(inp, idx, count, out, stream=None):
    """inp [P, n_in] -> out [P, n_out] (float32, contiguous)."""
    P, n_in = inp.shape
    P2, n_out = out.shape
    if P != P2:
        raise ValueError("plane counts differ")
    _check(lib().lodge_gather_planes(int(P), int(n_in), int(n_out), _ptr(inp), _ptr(idx), _ptr(count), _ptr(out),
                                     _stream_ptr(stream)))


# --------------------------------------------------------------------------- one frame

@dataclass
class Frame:
    image: object
    final_T: object
    n_contrib: object


class Renderer:
    """Convenience owner of a workspace, a selection and output buffers for one image size."""

    def __init__(self, scene: Scene, width: int, height: int, max_active: Optional[int] = None,
                 max_instances: Optional[int] = None, device="cuda"):
        torch = _torch()
        self.scene = scene
        if max_active is None:
            max_active = max(1, scene.total)
        if max_instances is None:
            max_instances = max(1 << 20, 8 * max_active)
        self.ws = Workspace(scene, width, height, max_active, min(max_instances, (1 << 32) - 1), device)
        self.sel = Selection(max_active, device)
        self.image = torch.empty((3, height, width), dtype=torch.float32, device=device)
        self.final_T = torch.empty((height, width), dtype=torch.float32, device=device)
        self.n_contrib = torch.empty((height, width), dtype=torch.int32, device=device)
        self.width, self.height = width, height

    def frame(self, cam, mode: int, s2d: float = 0.3, compensate: bool = True, stream=None,
              stage_events=None, sets: Optional["ChunkSets"] = None) -> Frame:
        """One select + render; with sets (chunked mode only) the selection reads the stored chunk sets."""
        if sets is not None:
            if mode != SELECT_CHUNKED:
                raise ValueError("chunk sets serve the chunked selection only")
            lodge_select_chunk_sets(self.scene, sets, cam, self.ws, self.sel, stream)
        else:
            lodge_select(self.scene, cam, mode, self.ws, self.sel, stream)
        lodge_render(self.scene, self.sel, cam, self.ws, self.image, self.final_T, self.n_contrib, s2d, compensate,
                     stream, stage_events)
        return Frame(self.image, self.final_T, self.n_contrib)

    def info(self, stream=None) -> dict:
        return lodge_frame_info_read(self.ws, stream)


# --------------------------------------------------------------------------- measurement helpers

def lodge_microbench_copy(src, dst, stream=None):
    """Streaming device copy src -> dst (same-size contiguous CUDA tensors, 16-byte multiple)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst must have the same size in bytes")
    _check(lib().lodge_microbench_copy(_ptr(src), _ptr(dst), C.c_size_t(nbytes), _stream_ptr(stream)))


def lodge_microbench_read(src, out=None, stream=None):
    """Streaming read of src (a contiguous CUDA tensor, 16-byte multiple); returns the per-thread sums tensor."""
    torch = _torch()
    nbytes = src.numel() * src.element_size()
    blocks = C.c_uint32()
    _check(lib().lodge_microbench_read_blocks(C.c_size_t(nbytes), C.byref(blocks)))
    if out is None or out.numel() < blocks.value * 256:
        out = torch.empty((blocks.value * 256,), dtype=torch.float32, device=src.device)
    _check(lib().lodge_microbench_read(_ptr(src), C.c_size_t(nbytes), _ptr(out), blocks.value, _stream_ptr(stream)))
    return out


def lodge_microbench_fma(out, iters: int, a: float = 1.0, b: float = 1.0, stream=None):
    """Chains of dependent FMAs: out is a float32 CUDA tensor of blocks x 256 elements; returns the lane-ops."""
    n = int(out.numel())
    if n == 0 or n % 256:
        raise ValueError("out must hold a positive multiple of 256 floats")
    _check(lib().lodge_microbench_fma(_ptr(out), n // 256, int(iters), float(a), float(b), _stream_ptr(stream)))
    return 8 * int(iters) * n


def lodge_fp32_div_sqrt(a, b, q, r, stream=None):
    """q = a / b and r = sqrt(a) elementwise on the device (float32 CUDA tensors of one size)."""
    n = int(a.numel())
    if any(t.numel() != n or t.dtype != _torch().float32 for t in (b, q, r)):
        raise ValueError("a, b, q, r: float32 tensors of one size")
    _check(lib().lodge_fp32_div_sqrt(_ptr(a), _ptr(b), _ptr(q), _ptr(r), C.c_size_t(n), _stream_ptr(stream)))
