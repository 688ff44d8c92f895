"""Selection from the precomputed per-chunk sets (Sec. 3 "chunk-based
rendering") against the per-frame selection and the oracle: chunk pair,
ids, weights and count bit for bit, and the rendered frame identical."""
import numpy as np
import pytest

import oracle
import synth
from synth import Chunks, Scene

from parity_util import compare_selection, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_23158_amd import lodge
    lodge.lib()
    return lodge


def sets_frame(L, d, sets, cam, R=None):
    import torch
    R = R or L.Renderer(d, cam.width, cam.height)
    R.frame(cam, L.SELECT_CHUNKED, sets=sets)
    torch.cuda.synchronize()
    info = R.info()
    n = min(info["n_selected"], R.sel.cap)
    return dict(info=info, ids=R.sel.ids[:n].cpu().numpy().astype(np.uint32), w=R.sel.w[:n].cpu().numpy(),
                image=R.image.cpu().numpy(), final_T=R.final_T.cpu().numpy(),
                n_contrib=R.n_contrib.cpu().numpy()), R


def check(L, oracle32, sc, d, sets, cam, tag):
    import torch
    log(f"[chunk-sets] {tag}")
    g, R = sets_frame(L, d, sets, cam)
    ids, w, (f, o, t) = oracle32.select(sc, oracle.CHUNKED, cam.pos)
    compare_selection(g, ids, w)
    assert (g["info"]["f"], g["info"]["o"]) == (f, o)
    assert np.float32(g["info"]["t"]) == np.float32(t)
    # the per-frame selection on a second renderer gives the identical frame
    R2 = L.Renderer(d, cam.width, cam.height)
    R2.frame(cam, L.SELECT_CHUNKED)
    torch.cuda.synchronize()
    assert np.array_equal(R2.image.cpu().numpy(), g["image"])
    assert np.array_equal(R2.n_contrib.cpu().numpy(), g["n_contrib"])
    return g


def test_chunk_sets_lod_city(L, oracle32):
    sc = synth.config2_scene(frac=0.05, width=500, height=270)
    d = L.Scene.from_synth(sc)
    sets = L.ChunkSets(d)
    check(L, oracle32, sc, d, sets, sc.cameras[0], "lod3-frac0.05")
    rng = np.random.default_rng(5)
    for k in range(4):
        eye = np.array([rng.uniform(-90, 90), rng.uniform(-90, 90), 1.7])
        cam = synth.look_at(eye, eye + np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), -0.05]), (0, 0, 1), 320, 180)
        check(L, oracle32, sc, d, sets, cam, f"lod3-frac0.05-random{k}")


def test_chunk_sets_large_path_and_band_edges(L, oracle32):
    sc = synth.config3_scene(frac=0.01, n_frames=300, width=496, height=280)
    d = L.Scene.from_synth(sc)
    sets = L.ChunkSets(d)
    for k in (0, 37, 150, 299):
        check(L, oracle32, sc, d, sets, sc.cameras[k], f"lod4-frac0.01-frame{k}")
    sc2 = synth.lod_city_scene(counts=(40000, 10000), half_xy=30.0, d=(8.0,), grid=2, spacing=20.0, chunk_z=1.0,
                               band=6.0, seed=46)
    d2 = L.Scene.from_synth(sc2)
    sets2 = L.ChunkSets(d2)
    for x in (-12.0, -1.0, 0.0, 2.9, 11.0):
        cam = synth.look_at((x, -10.0, 1.2), (x + 5.0, 20.0, 0.0), (0, 0, 1), 160, 96)
        check(L, oracle32, sc2, d2, sets2, cam, f"band-x{x}")


def test_chunk_sets_single_chunk_and_errors(L, oracle32):
    """One chunk: o = -1 and t = 1, every member weight 1; a scene without
    chunks has no chunk sets."""
    sc = synth.lod_city_scene(counts=(8000, 2000), half_xy=20.0, d=(6.0,), grid=2, spacing=8.0, chunk_z=1.0,
                              band=0.0, seed=11)
    one = Scene(levels=sc.levels, d=sc.d, chunks=Chunks(centers=sc.chunks.centers[:1], offsets=sc.chunks.offsets[:1]))
    d = L.Scene.from_synth(one)
    sets = L.ChunkSets(d)
    cam = synth.look_at((3.0, -12.0, 1.5), (3.0, 10.0, 0.0), (0, 0, 1), 128, 72)
    g = check(L, oracle32, one, d, sets, cam, "single-chunk")
    assert g["info"]["o"] == -1 and np.all(g["w"] == 1.0)
    plain = synth.plain_scene(n=500)
    dp = L.Scene.from_synth(plain)
    with pytest.raises(L.LodgeError):
        L.ChunkSets(dp)
