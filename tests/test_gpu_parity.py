"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact: chunk pair, selected ids and weights, visibility, tile
rectangles, depth keys, tile ranges and the sorted per-tile lists.
Tolerance: FP32 images, final transmittance within 1e-4 per channel, with
threshold flips accepted only where the oracle shows the ambiguity.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import Chunks, Scene

from parity_util import compare_binning, compare_image, compare_projection, compare_selection, full_parity, \
    gpu_frame, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_23158_amd import lodge
    lodge.lib()
    return lodge


def dev(L, sc):
    return L.Scene.from_synth(sc)


def test_plain_config(L, oracle32):
    """Plain render, no LOD: 10k Gaussians, 256 x 256."""
    sc = synth.plain_scene()
    full_parity(oracle32, sc, dev(L, sc), sc.cameras[0], oracle.ALL, "plain-10k")


@pytest.mark.parametrize("s2d,compensate", [(0.0, True), (0.0, False), (1.0, True)])
def test_screen_filter_variance(L, oracle32, s2d, compensate):
    """The renderer's 2-D filter is an option of the boundary: off (the plain
    EWA projection, where thin splats come close to a singular covariance and
    some are culled by det <= 0), and wider than the default, with and without
    the opacity compensation."""
    sc = synth.plain_scene(n=8000, seed=43, width=192, height=144)
    full_parity(oracle32, sc, dev(L, sc), sc.cameras[0], oracle.ALL, f"plain-s2d{s2d}-comp{int(compensate)}",
                s2d=s2d, compensate=compensate)


def test_background_behind_partly_transparent_pixels(L, oracle32):
    """A non-zero background shows through each pixel in proportion to the
    transmittance left after its last blended splat (C + T_final bg)."""
    import dataclasses
    sc = synth.plain_scene(n=3000, seed=44, width=160, height=96)
    cam = dataclasses.replace(sc.cameras[0], bg=(0.2, 0.4, 0.6))
    g, r = full_parity(oracle32, sc, dev(L, sc), cam, oracle.ALL, "plain-bg")
    T = g["final_T"]
    assert (T > 0.5).any() and (T < 0.5).any()   # both mostly-background and mostly-covered pixels


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_sh_degrees_below_three(L, oracle32, deg):
    """Colour from fewer SH bands: only the level's (d + 1)^2 coefficients
    enter the sum."""
    lv = synth.gaussians(4000, (45, deg), synth._cube(5.0), -3.0, 0.5, sh_degree=deg)
    sc = Scene(levels=[lv], d=[])
    cam = synth.look_at((3, -2, -14), (0, 0, 0), (0, -1, 0), 176, 112)
    full_parity(oracle32, sc, dev(L, sc), cam, oracle.ALL, f"plain-sh{deg}")


def test_levels_of_different_sh_degrees(L, oracle32):
    """Three LOD levels with SH degrees 3, 1 and 0 in one frame: the colour
    pass takes each queued Gaussian's coefficients from its own level."""
    lvs = [synth.gaussians(6000, (46, 0), synth._cube(12.0), -3.0, 0.5, sh_degree=3),
           synth.gaussians(3000, (46, 1), synth._cube(12.0), -3.0 + np.log(2.0), 0.5, sh_degree=1),
           synth.gaussians(1500, (46, 2), synth._cube(12.0), -3.0 + 2 * np.log(2.0), 0.5, sh_degree=0)]
    sc = Scene(levels=lvs, d=[12.0, 18.0])
    cam = synth.look_at((0, 0, -14), (0, 0, 0), (0, -1, 0), 208, 128)
    g, r = full_parity(oracle32, sc, dev(L, sc), cam, oracle.LOD_CAMERA, "lod-mixed-sh")
    # every level contributes to the frame
    bases = np.cumsum([0] + [lv.n for lv in lvs])
    for l in range(3):
        assert ((r["ids"] >= bases[l]) & (r["ids"] < bases[l + 1])).any(), f"level {l} selects nothing"


def test_gaussians_at_the_near_plane(L, oracle32):
    """Gaussians from 0.1 to 0.7 m in front of the camera (near plane 0.2 m):
    those behind it are culled, those just past it project to large splats,
    and many sit outside the Jacobian clamp (|x/z| above lim_x)."""
    def near_means(rng, m):
        return np.stack([rng.uniform(-0.35, 0.35, m), rng.uniform(-0.25, 0.25, m), rng.uniform(0.1, 0.7, m)])
    sc = Scene(levels=[synth.gaussians(1500, (47, 0), near_means, -5.0, 0.5),
                       synth.gaussians(40, (47, 1), near_means, -3.0, 0.3)], d=[1000.0])
    cam = synth.look_at((0, 0, 0), (0, 0, 1), (0, -1, 0), 256, 192)
    g, r = full_parity(oracle32, sc, dev(L, sc), cam, oracle.ALL, "near-plane", max_instances=1_000_000)
    z = np.concatenate([lv.mean[2] for lv in sc.levels])
    x = np.concatenate([lv.mean[0] for lv in sc.levels])
    assert (z <= cam.znear).sum() > 100 and (np.abs(x / z) > cam.lim_x).sum() > 100


def test_opaque_stack_stops_most_pixels(L, oracle32):
    """6000 wide Gaussians of opacity 0.97: most pixels reach T < 1e-4 on the
    next splat and stop there, so the stop decision, the last contributor and
    the quadrant waves' early exit carry the image."""
    lv = synth.gaussians(6000, (48, 0), synth._cube(4.0), -1.5, 0.3)
    lv.opacity[:] = np.float32(0.97)
    sc = Scene(levels=[lv], d=[])
    cam = synth.look_at((0, 0, -12), (0, 0, 0), (0, -1, 0), 160, 128)
    g, r = full_parity(oracle32, sc, dev(L, sc), cam, oracle.ALL, "opaque-stack")
    assert (r["final_T"] < 1e-3).mean() > 0.5
    assert g["final_T"].min() >= np.float32(1e-4)   # a pixel stops before T falls below the threshold


def test_plain_ragged_edges(L, oracle32):
    sc = synth.plain_scene(n=6000, seed=41, width=200, height=120)
    full_parity(oracle32, sc, dev(L, sc), sc.cameras[0], oracle.ALL, "plain-ragged-200x120")


@pytest.mark.parametrize("mode", [oracle.CHUNKED, oracle.LOD_CAMERA, oracle.ALL])
def test_lod_city_reduced(L, oracle32, mode):
    """The 3-level ground-plane scene at 5% density, 500 x 270 (ragged)."""
    sc = synth.config2_scene(frac=0.05, width=500, height=270)
    full_parity(oracle32, sc, dev(L, sc), sc.cameras[0], mode, f"lod3-frac0.05-mode{mode}")


def test_large_path_frames_reduced(L, oracle32):
    """The 4-level 1 km scene at 1% density along its camera path."""
    sc = synth.config3_scene(frac=0.01, n_frames=300, width=496, height=280)
    d = dev(L, sc)
    for k in (0, 37, 150, 299):
        full_parity(oracle32, sc, d, sc.cameras[k], oracle.CHUNKED, f"lod4-frac0.01-frame{k}")


def test_tiny_images(L, oracle32):
    sc = synth.plain_scene(n=3000, seed=43, width=17, height=9)
    d = dev(L, sc)
    full_parity(oracle32, sc, d, sc.cameras[0], oracle.ALL, "17x9")
    cam1 = synth.look_at((0, 0, -15), (0, 0, 0), (0, -1, 0), 1, 1)
    full_parity(oracle32, sc, d, cam1, oracle.ALL, "1x1")


def test_largest_frame_4k(L, oracle32):
    """3840 x 2160: 32400 tiles, near the 32768-tile limit of the packed
    16-bit tile histograms (the binning LDS is then over 64 KB)."""
    sc = synth.plain_scene(n=20000, seed=48, width=3840, height=2160)
    full_parity(oracle32, sc, dev(L, sc), sc.cameras[0], oracle.ALL, "plain-20k-3840x2160", max_instances=4_000_000)


def test_nothing_selected_or_visible(L, oracle32):
    far = synth.gaussians(2000, (44, 0), synth._cube(1.0), -3.0, 0.5)
    far.mean[0] += 50.0                       # all 50 m away
    empty = synth.gaussians(0, (44, 1), synth._cube(1.0), -3.0, 0.5)
    sc = Scene(levels=[far, empty], d=[10.0])
    cam = synth.look_at((0, 0, -5), (0, 0, 0), (0, -1, 0), 64, 48, bg=(0.2, 0.4, 0.6))
    g, r = full_parity(oracle32, sc, dev(L, sc), cam, oracle.LOD_CAMERA, "empty-selection")
    assert len(r["ids"]) == 0 and np.all(g["image"][1] == np.float32(0.4))
    # selected but all behind the camera
    cam2 = synth.look_at((50, 0, -5), (50, 0, -10), (0, -1, 0), 64, 48)
    g, r = full_parity(oracle32, sc, dev(L, sc), cam2, oracle.ALL, "nothing-visible")
    assert g["info"]["n_visible"] == 0 and np.all(g["final_T"] == 1.0)


@pytest.mark.parametrize("n", [200, 1500, 3000, 6000, 9000, 40000])
def test_long_tile_lists(L, oracle32, n):
    """Many small Gaussians in front of one tile: per-tile runs in every sort
    band (one wave up to 256, 2048, 4096, 8192, 16384, and the merge fallback
    beyond)."""
    lv = synth.gaussians(n, (45, n), synth._cube(0.05), -6.0, 0.3, morton=False)
    lv.mean[2] += 10.0
    sc = Scene(levels=[lv], d=[])
    cam = synth.look_at((0, 0, 0), (0, 0, 1), (0, -1, 0), 64, 64)
    g, r = full_parity(oracle32, sc, dev(L, sc), cam, oracle.ALL, f"long-lists-{n}", compensate=False)
    assert g["info"]["max_tile_len"] == int((r["binned"].ranges[:, 1] - r["binned"].ranges[:, 0]).max())
    if n > 16384:
        assert g["info"]["n_merge"] > 0
    elif n > 2048:
        assert g["info"]["n_long"] > 0


@pytest.mark.parametrize("n", [64, 65, 128, 129, 256, 257, 512, 513, 2048, 2049, 4096, 4097, 8192, 8193, 16384, 16385])
def test_sort_band_edges(L, oracle32, n):
    """Exactly n instances in one tile, at the edges of the sort's length
    bands: one wave with 1, 2 or 4 keys per lane up to 64, 128 and 256; four
    waves and their merge rounds up to 2048; eight up to 4096; 4097 (two
    halves, the second of one key, and the LDS merge); 8192 (two full
    halves); 8193 (an 8192-key chunk, a one-key chunk and a merge pass in
    global memory); past 16384 the queue of the longest runs."""
    lv = synth.gaussians(n, (47, n), synth._cube(0.05), -6.0, 0.3, morton=False)
    cam = synth.look_at((0, 0, 0), (0, 0, 1), (0, -1, 0), 64, 64)
    z = 10.0
    # all projected within 2.5 px of the centre of tile (1, 1): one tile each
    lv.mean[2] += z
    lv.mean[0] += (24.0 - cam.cx) * z / cam.fx
    lv.mean[1] += (24.0 - cam.cy) * z / cam.fy
    sc = Scene(levels=[lv], d=[])
    g, r = full_parity(oracle32, sc, dev(L, sc), cam, oracle.ALL, f"sort-band-{n}", compensate=False)
    lens = r["binned"].ranges[:, 1] - r["binned"].ranges[:, 0]
    assert int(lens.max()) == n and int((lens > 0).sum()) == 1
    assert g["info"]["max_tile_len"] == n
    assert g["info"]["n_merge"] == (1 if n > 16384 else 0)
    assert g["info"]["n_long"] == (1 if 2048 < n <= 16384 else 0)


def test_chunk_weights_at_band_edges(L, oracle32):
    """Cameras across the blend band of two chunks (t from 0 ... 1)."""
    sc = synth.lod_city_scene(counts=(40000, 10000), half_xy=30.0, d=(8.0,), grid=2, spacing=20.0, chunk_z=1.0,
                              band=6.0, seed=46)
    d = dev(L, sc)
    for x in (-12.0, -2.5, -1.0, 0.0, 0.7, 2.9, 11.0):
        cam = synth.look_at((x, -10.0, 1.2), (x + 5.0, 20.0, 0.0), (0, 0, 1), 160, 96)
        g, r = full_parity(oracle32, sc, d, cam, oracle.CHUNKED, f"band-x{x}")
        f, o, t = r["fot"]
        assert (g["info"]["f"], g["info"]["o"]) == (f, o)
        assert np.float32(g["info"]["t"]) == np.float32(t)


def test_capacity_overflow_is_reported(L, oracle32):
    sc = synth.plain_scene(n=5000, seed=47, width=128, height=128)
    d = dev(L, sc)
    g = gpu_frame(d, sc.cameras[0], oracle.ALL, max_instances=1000)
    st, na, ni = L.lodge_check(g["renderer"].ws)
    assert st == L.LODGE_ERR_CAPACITY and ni > 1000
    assert np.all(g["final_T"] == 1.0)            # an overflowed frame renders background only
    g2 = gpu_frame(d, sc.cameras[0], oracle.ALL, max_active=100)
    st, na, ni = L.lodge_check(g2["renderer"].ws)
    assert st == L.LODGE_ERR_CAPACITY and na == 5000
    # the retry protocol: grow to what lodge_check reports until the frame fits (after a selection
    # overflow the instance count covers only the truncated set, so it can take two rounds)
    ma, mi = na, 1000
    for _ in range(3):
        g3 = gpu_frame(d, sc.cameras[0], oracle.ALL, max_active=ma, max_instances=mi)
        st, na, ni = L.lodge_check(g3["renderer"].ws)
        if st == L.LODGE_OK:
            break
        ma, mi = max(ma, na), max(mi, ni)
    assert st == L.LODGE_OK
    r = oracle32.render(sc, sc.cameras[0], oracle.ALL)
    compare_binning(g3, r["binned"])
    compare_image(oracle32, g3, r, sc.cameras[0])


def test_repeat_is_bit_identical(L):
    sc = synth.config2_scene(frac=0.02, width=320, height=180)
    d = dev(L, sc)
    import torch
    R = L.Renderer(d, 320, 180)
    R.frame(sc.cameras[0], oracle.CHUNKED)
    a = R.image.clone()
    for _ in range(3):
        R.frame(sc.cameras[0], oracle.CHUNKED)
        torch.cuda.synchronize()
        assert torch.equal(a, R.image)


def test_storage_order_does_not_change_the_image(L):
    import torch
    sc = synth.config2_scene(frac=0.01, width=320, height=180)
    rng = np.random.default_rng(1)
    sp = Scene(levels=[synth.permuted(l, rng.permutation(l.n)) for l in sc.levels], d=sc.d, chunks=sc.chunks)
    a = gpu_frame(dev(L, sc), sc.cameras[0], oracle.CHUNKED)
    b = gpu_frame(dev(L, sp), sc.cameras[0], oracle.CHUNKED)
    assert a["info"]["n_selected"] == b["info"]["n_selected"]
    assert np.abs(a["image"] - b["image"]).max() <= 1e-6


def test_full_size_large_lod_frame(L, oracle32):
    """The 20M/5M/1.25M/300k scene at 1920 x 1080 (frame 10 of the path), in
    the launch configuration the benchmark times: selection, projection,
    binning and the whole image against the oracle."""
    log("[parity] generating the 26.55M-Gaussian scene")
    sc = synth.config3_scene(n_frames=300)
    d = dev(L, sc)
    cam = sc.cameras[10]
    full_parity(oracle32, sc, d, cam, oracle.CHUNKED, "lod4-26.55M-frame10", max_active=6_000_000,
                max_instances=24_000_000)


def _copies(lv, k):
    return [lv] * k


@pytest.mark.parametrize("mode", [oracle.ALL, oracle.LOD_CAMERA])
def test_identical_levels_exact_depth_ties(L, oracle32, mode):
    """Three identical copies of one level: in ALL mode every Gaussian is
    selected three times with the same depth, so every sort key ties three
    ways and the active index alone orders them; in LOD_CAMERA mode the
    copies partition the Gaussians by distance (Gaussians placed exactly on
    the switch distances included)."""
    base = synth.gaussians(3000, (901, 0), synth._cube(4.0), -3.0, 0.5, morton=False)
    base.mean[:, 0] = [2.0, 0.0, 0.0]
    base.mean[:, 1] = [0.0, 4.0, 0.0]
    base.mean[:, 2] = [0.0, 0.0, 2.0]
    sc = Scene(levels=_copies(base, 3), d=[2.0, 4.0])
    cam = synth.look_at((0.0, 0.5, -6.0), (0.0, 0.0, 0.0), (0, -1, 0), 96, 80)
    if mode == oracle.LOD_CAMERA:
        cam = synth.look_at((0.0, 0.0, 0.0), (0.0, 0.3, 1.0), (0, -1, 0), 96, 80)
    g, r = full_parity(oracle32, sc, dev(L, sc), cam, mode, f"identical-levels-mode{mode}")
    if mode == oracle.ALL:
        bn = r["binned"]
        same = (bn.dkey[1:] == bn.dkey[:-1]) & (bn.tile[1:] == bn.tile[:-1])
        assert same.sum() >= bn.M // 2, "most sort keys tie"


@pytest.mark.parametrize("n", [64, 65, 256, 257, 2048, 2049, 4096, 4097, 8192, 8193, 16385])
def test_tied_depths_at_sort_band_edges(L, oracle32, n):
    """Exactly n instances in one tile, built from duplicated Gaussians (two
    identical levels, plus a third of one Gaussian for odd n): every depth
    occurs twice, in every length band of the sort."""
    h = n // 2
    cam = synth.look_at((0, 0, 0), (0, 0, 1), (0, -1, 0), 64, 64)
    z = 10.0

    def level(m, key):
        lv = synth.gaussians(m, (49, key), synth._cube(0.05), -6.0, 0.3, morton=False)
        lv.mean[2] += z
        lv.mean[0] += (24.0 - cam.cx) * z / cam.fx
        lv.mean[1] += (24.0 - cam.cy) * z / cam.fy
        return lv

    base = level(h, n)
    levels = [base, base] + ([level(1, n + 1)] if n % 2 else [])
    sc = Scene(levels=levels, d=[1e3, 2e3][:len(levels) - 1])
    g, r = full_parity(oracle32, sc, dev(L, sc), cam, oracle.ALL, f"tied-sort-band-{n}", compensate=False)
    lens = r["binned"].ranges[:, 1] - r["binned"].ranges[:, 0]
    assert int(lens.max()) == n and int((lens > 0).sum()) == 1
    dk = r["binned"].dkey
    assert int((dk[1:] == dk[:-1]).sum()) >= h


def _signed_perms(v):
    import itertools
    out = set()
    for p in itertools.permutations(v):
        for s in itertools.product((1, -1), repeat=3):
            out.add(tuple(a * b for a, b in zip(p, s)))
    return sorted(out)


def test_gaussians_on_switch_distances_camera_mode(L, oracle32):
    """Gaussians at exactly d_1 = 7 and d_2 = 9 from the camera centre (integer
    offsets of those norms, exact in FP32) among random ones, in three
    identical levels: each boundary Gaussian belongs to the level whose
    interval starts at its distance (inclusive lower bound of Eq. 2)."""
    p = np.array([0.5, -0.25, 1.0])
    offs = _signed_perms((2, 3, 6)) + _signed_perms((1, 4, 8)) + _signed_perms((4, 4, 7))
    rng = np.random.default_rng(71)
    fill = rng.uniform(-12, 12, (4000, 3))
    pts = np.concatenate([p + np.asarray(offs, np.float64), p + fill])
    lv = synth.gaussians(len(pts), (71, 0), synth._cube(1.0), -2.5, 0.4, morton=False)
    lv.mean[:] = pts.T.astype(np.float32)
    sc = Scene(levels=_copies(lv, 3), d=[7.0, 9.0])
    cam = synth.look_at(p, p + np.array([0.2, 0.1, 1.0]), (0, -1, 0), 160, 120)
    assert np.array_equal(cam.pos, p.astype(np.float32))
    g, r = full_parity(oracle32, sc, dev(L, sc), cam, oracle.LOD_CAMERA, "switch-distances-camera")
    n = lv.n
    lvl = dict(zip((r["ids"] % n).tolist(), (r["ids"] // n).tolist()))
    nb = len(offs)
    for i, o in enumerate(offs):
        dist = int(round(np.linalg.norm(o)))
        assert lvl[i] == (1 if dist == 7 else 2), (o, lvl[i])


def test_gaussians_on_switch_distances_chunked(L, oracle32):
    """2 x 2 chunks 20 m apart (offset r = 20) and d_1 = 6: Gaussians at exactly
    d_1 + r = 26 from each chunk centre (offsets (6, 8, 24), (0, 10, 24) and
    their signed permutations), in two identical levels, for cameras on
    either side of the bisectors."""
    ch = synth.chunk_grid(2, 20.0, 1.0, band=4.0)
    assert np.all(ch.offsets == 20.0)
    offs = np.asarray(_signed_perms((6, 8, 24)) + _signed_perms((0, 10, 24)), np.float64)
    rng = np.random.default_rng(72)
    pts = [c + offs for c in ch.centers.astype(np.float64)] + [rng.uniform(-40, 40, (6000, 3)) * [1, 1, 0.1]]
    pts = np.concatenate(pts)
    lv = synth.gaussians(len(pts), (72, 0), synth._cube(1.0), -2.0, 0.4, morton=False)
    lv.mean[:] = pts.T.astype(np.float32)
    sc = Scene(levels=_copies(lv, 2), d=[6.0], chunks=ch)
    d = dev(L, sc)
    for eye in ((-3.0, -12.0, 1.5), (1.0, 4.0, 1.2), (14.0, 9.0, 2.0)):
        cam = synth.look_at(eye, (eye[0] + 5.0, eye[1] + 20.0, 0.0), (0, 0, 1), 160, 96)
        g, r = full_parity(oracle32, sc, d, cam, oracle.CHUNKED, f"switch-distances-chunked-{eye}")
        f, o, t = r["fot"]
        n = lv.n
        ids = set(r["ids"].tolist())
        # a boundary Gaussian of chunk f sits in level 1 about f (inclusive), not in level 0 about f
        for j in range(len(offs)):
            i = f * len(offs) + j
            assert (n + i) in ids
