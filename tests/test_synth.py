"""Seeded input generators: reproducible, with the stated shapes and distributions."""
import math

import numpy as np

import synth


def test_reproducible_and_shapes():
    a = synth.plain_scene(n=5000, seed=3)
    b = synth.plain_scene(n=5000, seed=3)
    la, lb = a.levels[0], b.levels[0]
    for f in ("mean", "scale", "quat", "opacity", "sh"):
        assert np.array_equal(getattr(la, f), getattr(lb, f))
    assert la.mean.shape == (3, 5000) and la.sh.shape == (16, 3, 5000) and la.quat.shape == (4, 5000)
    assert la.mean.dtype == np.float32
    assert np.allclose(np.linalg.norm(la.quat.astype(np.float64), axis=0), 1.0, atol=1e-6)
    assert np.all((la.opacity > 0) & (la.opacity < 1))
    assert np.abs(la.mean).max() <= 5.0


def test_distributions_roughly_as_stated():
    lv = synth.gaussians(200_000, (77, 0), synth._cube(5.0), -3.0, 0.5)
    ls = np.log(lv.scale.astype(np.float64))
    assert abs(ls.mean() + 3.0) < 0.01 and abs(ls.std() - 0.5) < 0.01
    assert abs(lv.sh[0].mean() - 0.5) < 0.01 and abs(lv.sh[0].std() - 0.2) < 0.01
    assert abs(lv.sh[1:].std() - 0.1) < 0.005
    logit = np.log(lv.opacity / (1 - lv.opacity))
    assert abs(logit.mean()) < 0.01 and abs(logit.std() - 1.0) < 0.01


def test_morton_order_is_a_permutation_of_the_draws():
    a = synth.gaussians(30_000, (5, 1), synth._ground(50.0), -3.0, 0.5, morton=True)
    b = synth.gaussians(30_000, (5, 1), synth._ground(50.0), -3.0, 0.5, morton=False)
    ka = np.lexsort(a.mean)
    kb = np.lexsort(b.mean)
    assert np.array_equal(a.mean[:, ka], b.mean[:, kb])
    # neighbours in storage are close in space
    step = np.linalg.norm(np.diff(a.mean.astype(np.float64), axis=1), axis=0)
    step_b = np.linalg.norm(np.diff(b.mean.astype(np.float64), axis=1), axis=0)
    assert np.median(step) < 0.1 * np.median(step_b)


def test_look_at_camera():
    cam = synth.look_at((-3.0, 12.0, 1.7), (97.0, 12.0, 0.0), (0, 0, 1), 1920, 1080)
    R = cam.R.astype(np.float64)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-6)
    assert np.allclose(-R.T @ cam.t, cam.pos, atol=1e-5)
    assert abs(cam.fx - 1662.77) < 0.01 and cam.cx == 960 and cam.cy == 540
    # the target projects to the principal point
    p = R @ np.array([97.0, 12.0, 0.0]) + cam.t
    assert abs(p[0] / p[2]) < 1e-6 and abs(p[1] / p[2]) < 1e-6 and p[2] > 0
    c1 = synth.plain_scene().cameras[0]
    assert np.allclose(c1.R, np.eye(3)) and np.allclose(c1.t, [0, 0, 15])


def test_chunk_grid_offsets_are_nearest_centre_distance():
    ch = synth.chunk_grid(8, 125.0, 2.0, 15.0)
    assert ch.centers.shape == (64, 3) and np.allclose(ch.offsets, 125.0)
    assert sorted(set(ch.centers[:, 0].tolist())) == [-437.5, -312.5, -187.5, -62.5, 62.5, 187.5, 312.5, 437.5]


def test_config_paths_and_requests():
    cams = synth.config3_path(300)
    assert len(cams) == 300
    for c in cams[::37]:
        assert abs(np.linalg.norm(c.pos[:2]) - 300.0) < 1e-3 and abs(c.pos[2] - 2.0) < 1e-6
        fwd = c.R[2].astype(np.float64)
        assert abs(math.degrees(math.asin(-fwd[2])) - 5.0) < 1e-4
    req = synth.serving_requests(256)
    t = np.array([r[0] for r in req])
    assert len(req) == 256 and t[0] == 0 and np.all(np.diff(t) >= 0)
    assert 90.0 < 255 / t[-1] < 150.0   # mean rate ~120/s
    assert {(c.width, c.height) for _, c in req} == set(synth.SERVE_RESOLUTIONS)
