"""The packed copy of the levels (lodge_scene_pack): a layout change only,
so every frame of a packed scene equals the same frame of the unpacked one
bit for bit (selection, projection records, depths, rectangles, sorted
lists, image, final T, n_contrib), for every SH degree (each a different
packed stride), and the packed frame matches the oracle."""
import numpy as np
import pytest

import oracle
import synth

from parity_util import full_parity, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_23158_amd import lodge
    lodge.lib()
    return lodge


def frame(L, dev, cam, mode):
    import torch
    R = L.Renderer(dev, cam.width, cam.height)
    R.frame(cam, mode)
    torch.cuda.synchronize()
    info = R.info()
    assert L.lodge_check(R.ws)[0] == L.LODGE_OK
    n = info["n_selected"]
    s, r, p, d, rc = L.lodge_debug_views(R.ws, int(info["n_instances"]))
    return {"image": R.image.cpu().numpy(), "T": R.final_T.cpu().numpy(), "nc": R.n_contrib.cpu().numpy(),
            "sorted": s.cpu().numpy(), "ranges": r.cpu().numpy(), "proj": p[:n].cpu().numpy(),
            "depth": d[:n].cpu().numpy(), "rect": rc[:n].cpu().numpy(), "ids": R.sel.ids[:n].cpu().numpy()}


def same(a, b, label):
    vis = (a["rect"][:, 0] != 0) | (a["rect"][:, 1] != 0)
    for k in ("image", "T", "nc", "sorted", "ranges", "depth", "rect", "ids"):
        assert np.array_equal(a[k].view(np.uint32) if a[k].dtype == np.float32 else a[k],
                              b[k].view(np.uint32) if b[k].dtype == np.float32 else b[k]), (label, k)
    assert np.array_equal(a["proj"][vis].view(np.uint32), b["proj"][vis].view(np.uint32)), (label, "proj")


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_packed_equals_planes_every_sh_degree(L, deg):
    lv = synth.gaussians(5000, (91, deg), synth._cube(5.0), -3.0, 0.5, sh_degree=deg)
    sc = synth.Scene(levels=[lv], d=[], chunks=None)
    cam = synth.look_at((2, -1, -14), (0, 0, 0), (0, -1, 0), 200, 120)
    dev = L.Scene.from_synth(sc)
    a = frame(L, dev, cam, L.SELECT_ALL)
    nb = dev.pack()
    assert nb >= 5000 * (32 + 16 * ((3 * (deg + 1) ** 2 + 3) // 4))
    b = frame(L, dev, cam, L.SELECT_ALL)
    same(a, b, f"deg {deg}")
    dev.unpack()
    c = frame(L, dev, cam, L.SELECT_ALL)
    same(a, c, f"deg {deg} detached")
    log(f"[pack] SH degree {deg}: packed frame identical ({nb} bytes)")


def test_packed_lod_scene_matches_oracle(L, oracle32):
    sc = synth.config2_scene(frac=0.02, width=320, height=180)
    dev = L.Scene.from_synth(sc)
    a = frame(L, dev, sc.cameras[0], L.SELECT_CHUNKED)
    dev.pack()
    b = frame(L, dev, sc.cameras[0], L.SELECT_CHUNKED)
    same(a, b, "lod3 chunked")
    full_parity(oracle32, sc, dev, sc.cameras[0], L.SELECT_CHUNKED, "lod3-frac0.02 packed 320x180")


def test_pack_errors(L):
    import ctypes as C
    import torch
    sc = synth.plain_scene(n=300, seed=92, width=32, height=32)
    dev = L.Scene.from_synth(sc)
    nb = C.c_size_t()
    assert L.lib().lodge_pack_size(dev.handle, C.byref(nb)) == L.LODGE_OK
    buf = torch.empty(int(nb.value) + 512, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr() + ((-buf.data_ptr()) % 256)
    assert L.lib().lodge_scene_pack(dev.handle, C.c_void_p(base), C.c_size_t(nb.value - 1), None) == \
        L.LODGE_ERR_INVALID_ARG
    assert L.lib().lodge_scene_pack(dev.handle, C.c_void_p(base + 16), C.c_size_t(nb.value), None) == \
        L.LODGE_ERR_INVALID_ARG
