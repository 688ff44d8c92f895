"""The C ABI without a GPU: the library loads, exports every entry point of
include/lodge.h, and its host-side validation rejects bad arguments before
any HIP call (none of these tests touches device memory)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2505_23158_amd import lodge as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "lodge.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const char\*|lodge_status|void|int64_t)\s+(lodge_\w+)\s*\(", src, re.M)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(L.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    for name in header_functions():
        assert getattr(lib, name) is not None
        assert re.search(rf"\bT {name}$", out, re.M), name


def test_status_strings_and_version():
    lib = L.lib()
    assert lib.lodge_status_string(0) == b"ok"
    assert lib.lodge_status_string(2) == b"capacity exceeded"
    assert lib.lodge_version().startswith(b"lodge-gfx950")


def _fake_level(n=10, deg=3, var=0.0, null=False):
    fake = 0 if null else 0x1000
    return L.lodge_level(n=n, mean=fake, scale=fake, quat=fake, opacity=fake, sh=fake, sh_degree=deg, filter3d_var=var)


def _create(levels, d=None, chunks=None):
    arr = (L.lodge_level * len(levels))(*levels)
    h = C.c_void_p()
    dd = np.asarray(d if d is not None else [], np.float32)
    st = L.lib().lodge_scene_create(arr, len(levels), dd.ctypes.data if len(dd) else None,
                                    C.byref(chunks) if chunks is not None else None, C.byref(h))
    return st, h


def test_scene_validation():
    lib = L.lib()
    st, h = _create([_fake_level()])
    assert st == L.LODGE_OK and lib.lodge_scene_total(h) == 10
    lib.lodge_scene_destroy(h)
    assert _create([_fake_level(deg=4)])[0] == L.LODGE_ERR_INVALID_ARG
    assert _create([_fake_level(var=-1.0)])[0] == L.LODGE_ERR_INVALID_ARG
    assert _create([_fake_level(null=True)])[0] == L.LODGE_ERR_INVALID_ARG
    assert _create([_fake_level(n=0, null=True)])[0] == L.LODGE_OK
    assert _create([_fake_level(), _fake_level()], d=[0.0])[0] == L.LODGE_ERR_INVALID_ARG
    assert _create([_fake_level(), _fake_level(), _fake_level()], d=[5.0, 3.0])[0] == L.LODGE_ERR_INVALID_ARG
    st, h = _create([_fake_level(), _fake_level(), _fake_level()], d=[5.0, 30.0])
    assert st == L.LODGE_OK and lib.lodge_scene_total(h) == 30
    lib.lodge_scene_destroy(h)
    assert _create([_fake_level()] * 9, d=list(range(1, 9)))[0] == L.LODGE_ERR_INVALID_ARG
    c = np.zeros((200, 3), np.float32)
    r = np.zeros(200, np.float32)
    ch = L.lodge_chunks(k=200, center=c.ctypes.data, offset=r.ctypes.data, band=0.0)
    assert _create([_fake_level()], chunks=ch)[0] == L.LODGE_ERR_INVALID_ARG
    # 64 coincident centres: Eq. 4 would divide by |m_f - m_o|^2 = 0
    ch = L.lodge_chunks(k=64, center=c.ctypes.data, offset=r.ctypes.data, band=10.0)
    assert _create([_fake_level()], chunks=ch)[0] == L.LODGE_ERR_INVALID_ARG
    c[:64, 0] = np.arange(64, dtype=np.float32) * 5.0
    st, h = _create([_fake_level()], chunks=ch)
    assert st == L.LODGE_OK
    lib.lodge_scene_destroy(h)
    c[7] = c[40]                       # one coincident pair among distinct centres
    assert _create([_fake_level()], chunks=ch)[0] == L.LODGE_ERR_INVALID_ARG
    c[7] = (35.0, 0.0, 0.0)
    c[9, 2] = np.inf
    assert _create([_fake_level()], chunks=ch)[0] == L.LODGE_ERR_INVALID_ARG
    c[9, 2] = 0.0
    for band in (np.nan, np.inf):
        chb = L.lodge_chunks(k=64, center=c.ctypes.data, offset=r.ctypes.data, band=band)
        assert _create([_fake_level()], chunks=chb)[0] == L.LODGE_ERR_INVALID_ARG
    r[3] = -1.0
    assert _create([_fake_level()], chunks=ch)[0] == L.LODGE_ERR_INVALID_ARG


def test_workspace_size_and_argument_checks():
    lib = L.lib()
    st, h = _create([_fake_level(n=1000)])
    assert st == 0
    nb = C.c_size_t()
    assert lib.lodge_workspace_size(h, 1920, 1080, 4_000_000, 16_000_000, C.byref(nb)) == 0
    # per-active records, per-instance ids + merge scratch, per-tile tables
    assert nb.value >= 4_000_000 * (48 + 4 + 4 + 48) + 16_000_000 * 12 + 8160 * 24
    assert lib.lodge_workspace_size(h, 0, 1080, 10, 10, C.byref(nb)) == L.LODGE_ERR_INVALID_ARG
    assert lib.lodge_workspace_size(h, 64, 64, 10, 1 << 32, C.byref(nb)) == L.LODGE_ERR_INVALID_ARG
    # the largest frame: 3840 x 2160 is 32400 16x16 tiles (the limit is 32768); one more tile column is too many
    assert lib.lodge_workspace_size(h, 3840, 2160, 10, 100, C.byref(nb)) == 0
    assert lib.lodge_workspace_size(h, 4096, 2048, 10, 100, C.byref(nb)) == 0
    assert lib.lodge_workspace_size(h, 4097, 2048, 10, 100, C.byref(nb)) == L.LODGE_ERR_UNSUPPORTED
    assert lib.lodge_workspace_size(h, 64, 64, 10, 100, C.byref(nb)) == 0
    ws = L.lodge_workspace(base=0x10000, bytes=nb.value, width=64, height=64, max_active=10, max_instances=100)
    sel = L.lodge_selection(ids=0x2000, w=0x3000, count=0x4000, cap=10)
    cam = L.lodge_camera(width=64, height=64, fx=50, fy=50, cx=32, cy=32, znear=0.2, lim_x=1, lim_y=1)
    # invalid mode / chunked without chunks / cap mismatch / small workspace / misaligned: all before any HIP call
    assert lib.lodge_select(h, C.byref(cam), 7, C.byref(ws), C.byref(sel), None) == L.LODGE_ERR_INVALID_ARG
    assert lib.lodge_select(h, C.byref(cam), L.SELECT_CHUNKED, C.byref(ws), C.byref(sel), None) == L.LODGE_ERR_INVALID_ARG
    assert b"chunks" in lib.lodge_last_error()
    sel.cap = 9
    assert lib.lodge_select(h, C.byref(cam), 0, C.byref(ws), C.byref(sel), None) == L.LODGE_ERR_INVALID_ARG
    sel.cap = 10
    ws.bytes = nb.value - 1
    assert lib.lodge_select(h, C.byref(cam), 0, C.byref(ws), C.byref(sel), None) == L.LODGE_ERR_INVALID_ARG
    ws.bytes = nb.value
    ws.base = 0x10010
    assert lib.lodge_select(h, C.byref(cam), 0, C.byref(ws), C.byref(sel), None) == L.LODGE_ERR_INVALID_ARG
    ws.base = 0x10000
    cam.fx = -1.0
    assert lib.lodge_select(h, C.byref(cam), 0, C.byref(ws), C.byref(sel), None) == L.LODGE_ERR_INVALID_ARG
    cam.fx = 50.0
    cam.width = 65
    out = 0x5000
    assert lib.lodge_render(h, C.byref(sel), C.byref(cam), None, C.byref(ws), out, out, out, None) \
        == L.LODGE_ERR_INVALID_ARG
    cam.width = 64
    assert lib.lodge_render(h, C.byref(sel), C.byref(cam), None, C.byref(ws), None, out, out, None) \
        == L.LODGE_ERR_INVALID_ARG
    opts = L.lodge_render_opts(s2d=-1.0, compensate=1)
    assert lib.lodge_render(h, C.byref(sel), C.byref(cam), C.byref(opts), C.byref(ws), out, out, out, None) \
        == L.LODGE_ERR_INVALID_ARG
    lib.lodge_scene_destroy(h)
