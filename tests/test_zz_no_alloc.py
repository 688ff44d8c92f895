"""lodge_render_static (the entry point that allocates nothing: its
workspace is the library's static scratch array) against lodge_render on a
caller workspace, through the C ABI: two calls in a row, the second with a
smaller input, bit for bit (both run the same kernels)."""
import ctypes as C

import numpy as np
import pytest

import synth

from parity_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_23158_amd import lodge
    lodge.lib()
    return lodge


def _static_frame(L, dev, R, cam):
    import torch
    H, W = cam.height, cam.width
    img = torch.full((3, H, W), -1.0, device="cuda")
    T = torch.full((H, W), -1.0, device="cuda")
    nc = torch.full((H, W), -1, dtype=torch.int32, device="cuda")
    ovf = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    L.lodge_render_static(dev, R.sel, cam, img, T, nc, overflow=ovf)
    torch.cuda.synchronize()
    return img, T, nc, int(ovf.item())


def test_static_scratch_render_equals_workspace_render(L):
    import torch
    cases = [
        ("lod3-frac0.02-320x180-chunked", synth.config2_scene(frac=0.02, width=320, height=180), L.SELECT_CHUNKED),
        ("plain-3000-128x96-all", synth.plain_scene(n=3000, seed=81, width=128, height=96), L.SELECT_ALL),
    ]
    for label, sc, mode in cases:
        cam = sc.cameras[0]
        log(f"[no-alloc] {label}")
        dev = L.Scene.from_synth(sc)
        R = L.Renderer(dev, cam.width, cam.height)
        R.frame(cam, mode)
        torch.cuda.synchronize()
        assert L.lodge_check(R.ws)[0] == L.LODGE_OK
        img, T, nc, ovf = _static_frame(L, dev, R, cam)
        assert ovf == 0
        assert torch.equal(img, R.image), label
        assert torch.equal(T, R.final_T), label
        assert torch.equal(nc, R.n_contrib), label
        assert float(R.image.abs().sum()) > 0


def test_static_scratch_rejects_what_does_not_fit(L):
    import torch
    sc = synth.plain_scene(n=1000, seed=82, width=64, height=64)
    dev = L.Scene.from_synth(sc)
    R = L.Renderer(dev, 64, 64)
    big = L.lodge_selection(ids=R.sel.desc.ids, w=R.sel.desc.w, count=R.sel.desc.count, cap=50_000_000)
    cam = synth.look_at((0, 0, -15), (0, 0, 0), (0, -1, 0), 1920, 1080)
    img = torch.empty((3, 1080, 1920), device="cuda")
    T = torch.empty((1080, 1920), device="cuda")
    nc = torch.empty((1080, 1920), dtype=torch.int32, device="cuda")
    c = L.make_camera(cam)
    st = L.lib().lodge_render_static(dev.handle, C.byref(big), C.c_void_p(C.addressof(c)), None, img.data_ptr(),
                                     T.data_ptr(), nc.data_ptr(), None, None)
    assert st == L.LODGE_ERR_INVALID_ARG
    assert b"static scratch" in L.lib().lodge_last_error()
