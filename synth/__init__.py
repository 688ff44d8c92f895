"""Seeded synthetic inputs for the LOD Gaussian-splatting renderer.

This module only *draws* inputs: Gaussian parameters, LOD levels, chunk grids
and pinhole cameras.  It holds none of the renderer's arithmetic (no
selection, projection, binning or compositing), so both the CPU oracle and
the HIP path can consume what it makes without sharing any computation.

Recipe (one numpy ``PCG64`` stream per (config, level, attribute, block) key,
blocks of 2**20 Gaussians, drawn in parallel threads):

* means: per workload (uniform cube, or uniform ground plane with a clipped
  normal height); each level is then stored in 3-D Morton order of its means,
  so spatially close Gaussians sit close in memory.  The other attributes are
  i.i.d. and are drawn directly in storage order.
* log-scales ~ N(mu_l, sd) per axis, quaternions ~ N(0, 1)^4, opacity logits
  ~ N(0, 1), SH DC ~ N(0.5, 0.2), higher SH bands ~ N(0, 0.1).
* activation (the form the renderer consumes) is done in float64 and rounded
  once to float32: scale = exp(log-scale), q = q / |q|, opacity = sigmoid.

The paper evaluates on captured city-scale datasets that are not available
here; these scenes keep their workload shape (Gaussian counts, LOD level
counts, level switch distances, chunk grids, ~1 MP frames) instead.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

BLOCK = 1 << 20
SH_COEFFS = 16

# attribute stream ids inside a seed key
_A_MEAN, _A_LOGSCALE, _A_QUAT, _A_OPAC, _A_SHDC, _A_SHREST = range(6)


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _rng(key) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


@dataclass
class Level:
    """One LOD level, structure of arrays, float32 (activated parameters)."""
    mean: np.ndarray          # (3, n)
    scale: np.ndarray         # (3, n) linear scale
    quat: np.ndarray          # (4, n) unit quaternion (w, x, y, z)
    opacity: np.ndarray       # (n,) in (0, 1)
    sh: np.ndarray            # (16, 3, n) SH coefficients [basis][channel][n]
    sh_degree: int = 3
    filter3d_var: float = 0.0
    raw: Optional[dict] = None  # pre-activation params (log_scale, quat_raw, opacity_logit)

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])


@dataclass
class Chunks:
    centers: np.ndarray       # (K, 3) float32
    offsets: np.ndarray       # (K,) float32, threshold offset r_k per chunk
    band: float = 0.0         # <= 0: the plain linear ramp between the two centres


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray             # (3, 3) float32, world -> camera, row-major
    t: np.ndarray             # (3,) float32
    pos: np.ndarray           # (3,) float32 camera centre
    znear: float = 0.2
    lim_x: float = 0.0
    lim_y: float = 0.0
    bg: tuple = (0.0, 0.0, 0.0)


@dataclass
class Scene:
    levels: list
    d: list                   # switch distances d_1 .. d_{L-1} (metres)
    chunks: Optional[Chunks] = None
    name: str = ""
    cameras: list = field(default_factory=list)

    @property
    def n_total(self) -> int:
        return sum(l.n for l in self.levels)


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------

def look_at(eye, target, up, width: int, height: int, hfov_deg: float = 60.0,
            znear: float = 0.2, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Pinhole camera with OpenCV axes (x right, y down, z forward).

    forward = normalize(target - eye), right = normalize(forward x up),
    down = forward x right; world->camera rotation rows are (right, down,
    forward) and t = -R eye.  Square pixels, principal point at the image
    centre, Jacobian clamp at 1.3x the half field of view.
    """
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ eye
    fx = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    fy = fx
    return Camera(width=width, height=height, fx=float(np.float32(fx)), fy=float(np.float32(fy)),
                  cx=width / 2.0, cy=height / 2.0,
                  R=R.astype(np.float32), t=t.astype(np.float32), pos=eye.astype(np.float32),
                  znear=znear, lim_x=float(np.float32(1.3 * (width / 2.0) / fx)),
                  lim_y=float(np.float32(1.3 * (height / 2.0) / fy)), bg=tuple(float(b) for b in bg))


# ----------------------------------------------------------------------------
# Gaussians
# ----------------------------------------------------------------------------

def _morton3(mean: np.ndarray) -> np.ndarray:
    """3-D Morton code of each column of ``mean`` over its bounding box (21 bits/axis)."""
    lo = mean.min(axis=1, keepdims=True).astype(np.float64)
    hi = mean.max(axis=1, keepdims=True).astype(np.float64)
    span = np.where(hi > lo, hi - lo, 1.0)
    q = ((mean - lo) / span * ((1 << 21) - 1)).astype(np.uint64)

    def spread(v):
        v = v & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
        return v

    return spread(q[0]) | (spread(q[1]) << np.uint64(1)) | (spread(q[2]) << np.uint64(2))


def _blocks(n: int):
    return [(b, b * BLOCK, min(n, (b + 1) * BLOCK)) for b in range((n + BLOCK - 1) // BLOCK)]


def gaussians(n: int, key: tuple, mean_fn: Callable, log_scale_mu: float, log_scale_sd: float,
              sh_degree: int = 3, filter3d_var: float = 0.0, morton: bool = True,
              keep_raw: bool = False) -> Level:
    """Draw one level of ``n`` Gaussians (see the module docstring for the recipe).

    ``mean_fn(rng, m) -> (3, m) float64`` draws the means of one block.
    """
    blocks = _blocks(n)
    mean = np.empty((3, n), np.float32)
    scale = np.empty((3, n), np.float32)
    quat = np.empty((4, n), np.float32)
    opacity = np.empty((n,), np.float32)
    nsh = (sh_degree + 1) ** 2
    sh = np.zeros((SH_COEFFS, 3, n), np.float32)
    raw = None
    if keep_raw:
        raw = {"log_scale": np.empty((3, n), np.float32), "quat": np.empty((4, n), np.float32),
               "opacity_logit": np.empty((n,), np.float32)}

    def draw_means(blk):
        b, s, e = blk
        mean[:, s:e] = mean_fn(_rng(key + (_A_MEAN, b)), e - s).astype(np.float32)

    def draw_rest(blk):
        b, s, e = blk
        m = e - s
        ls = _rng(key + (_A_LOGSCALE, b)).normal(log_scale_mu, log_scale_sd, (3, m))
        q = _rng(key + (_A_QUAT, b)).standard_normal((4, m))
        lo = _rng(key + (_A_OPAC, b)).standard_normal(m)
        # activation in float64, one rounding to float32
        scale[:, s:e] = np.exp(ls).astype(np.float32)
        qn = np.linalg.norm(q, axis=0)
        qn = np.where(qn > 0, qn, 1.0)
        quat[:, s:e] = (q / qn).astype(np.float32)
        opacity[s:e] = (1.0 / (1.0 + np.exp(-lo))).astype(np.float32)
        if raw is not None:
            raw["log_scale"][:, s:e] = ls.astype(np.float32)
            raw["quat"][:, s:e] = q.astype(np.float32)
            raw["opacity_logit"][s:e] = lo.astype(np.float32)
        sh[0, :, s:e] = 0.5 + 0.2 * _rng(key + (_A_SHDC, b)).standard_normal((3, m), dtype=np.float32)
        if nsh > 1:
            sh[1:nsh, :, s:e] = 0.1 * _rng(key + (_A_SHREST, b)).standard_normal((nsh - 1, 3, m),
                                                                                dtype=np.float32)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(draw_means, blocks))
        if morton and n > 1:
            order = np.argsort(_morton3(mean), kind="stable")
            mean = np.ascontiguousarray(mean[:, order])
            del order
        list(ex.map(draw_rest, blocks))
    return Level(mean=mean, scale=scale, quat=quat, opacity=opacity, sh=sh, sh_degree=sh_degree,
                 filter3d_var=float(np.float32(filter3d_var)), raw=raw)


def _cube(half: float):
    def fn(rng, m):
        return rng.uniform(-half, half, (3, m))
    return fn


def _ground(half_xy: float, z_sd: float = 2.0, z_clip: float = 10.0):
    def fn(rng, m):
        xy = rng.uniform(-half_xy, half_xy, (2, m))
        z = np.clip(rng.normal(0.0, z_sd, m), -z_clip, z_clip)
        return np.vstack([xy, z[None]])
    return fn


def chunk_grid(per_axis: int, spacing: float, z: float, band: float, offset: Optional[float] = None) -> Chunks:
    """Regular chunk grid centred on the origin.  The threshold offset of each
    chunk defaults to the distance to its nearest other centre."""
    c = (np.arange(per_axis) - (per_axis - 1) / 2.0) * spacing
    xs, ys = np.meshgrid(c, c, indexing="xy")
    centers = np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, z)], axis=1).astype(np.float32)
    if offset is None:
        d = np.linalg.norm(centers[:, None, :].astype(np.float64) - centers[None, :, :], axis=2)
        np.fill_diagonal(d, np.inf)
        offs = d.min(axis=1) if len(centers) > 1 else np.zeros(1)
    else:
        offs = np.full(len(centers), offset)
    return Chunks(centers=centers, offsets=offs.astype(np.float32), band=float(band))


F_REF = 1662.77  # focal length (px) of a 1920-wide, 60 degree camera


def filter_var(d_l: float, s: float = 0.2, f_ref: float = F_REF) -> float:
    """Per-level 3-D smoothing variance s * (d_l / f)^2 (m^2)."""
    return float(np.float32(s * (d_l / f_ref) ** 2))


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def plain_scene(n: int = 10_000, seed: int = 1, width: int = 256, height: int = 256,
                sh_degree: int = 3) -> Scene:
    """Plain render, no LOD: cube [-5,5]^3, one camera at (0,0,-15) looking at the origin."""
    lv = gaussians(n, (seed, 0), _cube(5.0), -3.0, 0.5, sh_degree=sh_degree)
    cam = look_at((0, 0, -15), (0, 0, 0), (0, -1, 0), width, height)
    return Scene(levels=[lv], d=[], chunks=None, name=f"plain-{n}", cameras=[cam])


def lod_city_scene(counts=(2_000_000, 500_000, 125_000), half_xy: float = 100.0, d=(20.0, 60.0),
                   grid: int = 4, spacing: float = 50.0, chunk_z: float = 1.7, band: float = 10.0,
                   seed: int = 2, sh_degree: int = 3, frac: float = 1.0) -> Scene:
    """Ground-plane LOD scene: level l has counts[l]*frac Gaussians on
    [-half,half]^2 x N(0,2), log-scale mean -3 + l ln 2, and a 3-D filter for d_l."""
    dd = [0.0] + list(d)
    levels = []
    for l, n in enumerate(counts):
        m = max(1, int(round(n * frac)))
        levels.append(gaussians(m, (seed, l), _ground(half_xy), -3.0 + l * math.log(2.0), 0.5,
                                sh_degree=sh_degree, filter3d_var=filter_var(dd[l])))
    ch = chunk_grid(grid, spacing, chunk_z, band)
    return Scene(levels=levels, d=list(d), chunks=ch, name=f"lod-{len(counts)}L")


def config2_scene(frac: float = 1.0, width: int = 1920, height: int = 1080) -> Scene:
    """3 levels 2M/500k/125k on 200x200 m, d = (20, 60), 4x4 chunks, 10 m bands."""
    sc = lod_city_scene(frac=frac, seed=2)
    sc.name = "lod3-2.625M" if frac == 1.0 else f"lod3-frac{frac}"
    sc.cameras = [look_at((-3.0, 12.0, 1.7), (97.0, 12.0, 0.0), (0, 0, 1), width, height)]
    return sc


def config3_path(n_frames: int = 300, width: int = 1920, height: int = 1080, radius: float = 300.0,
                 height_m: float = 2.0, pitch_deg: float = 5.0):
    """Circular camera path: eye on a circle of ``radius`` at ``height_m``,
    looking along the tangent pitched down by ``pitch_deg``."""
    cams = []
    p = math.radians(pitch_deg)
    for k in range(n_frames):
        th = 2.0 * math.pi * k / n_frames
        eye = np.array([radius * math.cos(th), radius * math.sin(th), height_m])
        fwd = np.array([-math.sin(th) * math.cos(p), math.cos(th) * math.cos(p), -math.sin(p)])
        cams.append(look_at(eye, eye + fwd, (0, 0, 1), width, height))
    return cams


def config3_scene(frac: float = 1.0, n_frames: int = 300, width: int = 1920, height: int = 1080) -> Scene:
    """4 levels 20M/5M/1.25M/300k on 1x1 km, d = (20, 60, 180), 8x8 chunks, 15 m bands."""
    sc = lod_city_scene(counts=(20_000_000, 5_000_000, 1_250_000, 300_000), half_xy=500.0,
                        d=(20.0, 60.0, 180.0), grid=8, spacing=125.0, chunk_z=2.0, band=15.0,
                        seed=3, frac=frac)
    sc.name = "lod4-26.55M" if frac == 1.0 else f"lod4-frac{frac}"
    sc.cameras = config3_path(n_frames, width, height)
    return sc


SERVE_RESOLUTIONS = ((640, 360), (1280, 720), (1920, 1080))


def serving_requests(n: int = 256, rate: float = 120.0, half_xy: float = 500.0, seed: int = 4):
    """Poisson arrivals (exponential gaps at ``rate``/s), resolution uniform over
    SERVE_RESOLUTIONS, eye uniform over the ground at 1.5-50 m, random yaw and a
    pitch in [-45, 0] degrees.  Returns a list of (arrival_s, Camera)."""
    rng = _rng((seed, 0, 99, 0))
    gaps = rng.exponential(1.0 / rate, n)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        w, h = SERVE_RESOLUTIONS[int(rng.integers(0, len(SERVE_RESOLUTIONS)))]
        eye = np.array([rng.uniform(-half_xy, half_xy), rng.uniform(-half_xy, half_xy),
                        rng.uniform(1.5, 50.0)])
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        pitch = math.radians(rng.uniform(-45.0, 0.0))
        fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
        out.append((float(arrivals[i]), look_at(eye, eye + fwd, (0, 0, 1), w, h)))
    return out


def diff_scene(n: int = 1_000_000, n_views: int = 8, width: int = 1280, height: int = 720,
               seed: int = 5) -> Scene:
    """One level (cube distributions), 3-D filter 2.89e-5 m^2, views on a circle of
    radius 15 in the xz-plane every 360/n_views degrees, looking at the origin."""
    lv = gaussians(n, (seed, 0), _cube(5.0), -3.0, 0.5, filter3d_var=filter_var(20.0), keep_raw=True)
    cams = []
    for k in range(n_views):
        th = 2.0 * math.pi * k / n_views
        cams.append(look_at((15.0 * math.sin(th), 0.0, -15.0 * math.cos(th)), (0, 0, 0), (0, -1, 0),
                            width, height))
    return Scene(levels=[lv], d=[], chunks=None, name=f"diff-{n}", cameras=cams)


def check_scene(n: int = 64, width: int = 32, height: int = 32, seed: int = 55,
                filter3d_var: float = 0.0) -> Scene:
    """Tiny differentiation check scene: cube [-1,1]^3, log-scale N(-2, 0.3), eye (0,0,-4)."""
    lv = gaussians(n, (seed, 0), _cube(1.0), -2.0, 0.3, filter3d_var=filter3d_var, keep_raw=True,
                   morton=False)
    cam = look_at((0, 0, -4), (0, 0, 0), (0, -1, 0), width, height)
    return Scene(levels=[lv], d=[], chunks=None, name=f"check-{n}", cameras=[cam])


def target_images(n_views: int, width: int, height: int, seed: int = 5) -> np.ndarray:
    """Seeded U[0,1] target images, (n_views, 3, H, W) float32."""
    return _rng((seed, 0, 98, 0)).random((n_views, 3, height, width), dtype=np.float32)


def permuted(level: Level, perm: np.ndarray) -> Level:
    """The same level stored in another order (for storage-permutation invariance)."""
    return Level(mean=np.ascontiguousarray(level.mean[:, perm]), scale=np.ascontiguousarray(level.scale[:, perm]),
                 quat=np.ascontiguousarray(level.quat[:, perm]), opacity=np.ascontiguousarray(level.opacity[perm]),
                 sh=np.ascontiguousarray(level.sh[:, :, perm]), sh_degree=level.sh_degree,
                 filter3d_var=level.filter3d_var)


def chunk_views(chunks: Chunks, k: int, n_positions: int = 4, n_orientations: int = 3, width: int = 320,
                height: int = 180, spread: float = 0.5, height_range=(1.5, 3.0), seed: int = 7):
    """Views of chunk k for its visibility filtering: camera positions drawn
    around the chunk centre (uniform in a disc of radius spread * r_k in the
    ground plane, heights uniform in height_range), standing in for the
    training cameras the chunk was clustered from, each seen under
    n_orientations random orientations (yaw uniform, pitch uniform in
    [-30, 10] degrees).  Returns a list of Cameras."""
    rng = _rng((seed, k, 98, 0))
    c = np.asarray(chunks.centers[k], np.float64)
    r = float(chunks.offsets[k]) * spread
    cams = []
    for _ in range(n_positions):
        rho = r * math.sqrt(rng.uniform(0.0, 1.0))
        phi = rng.uniform(0.0, 2.0 * math.pi)
        eye = np.array([c[0] + rho * math.cos(phi), c[1] + rho * math.sin(phi), rng.uniform(*height_range)])
        for _ in range(n_orientations):
            yaw = rng.uniform(0.0, 2.0 * math.pi)
            pitch = math.radians(rng.uniform(-30.0, 10.0))
            fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
            cams.append(look_at(eye, eye + fwd, (0, 0, 1), width, height))
    return cams


def threshold_views(n: int = 4, half_xy: float = 100.0, width: int = 320, height: int = 180, seed: int = 8):
    """Views for the depth-threshold search, standing in for a subset of
    training views: eyes uniform over the ground at 1.5-10 m, random yaw,
    pitch uniform in [-20, 0] degrees."""
    rng = _rng((seed, 0, 97, 0))
    cams = []
    for _ in range(n):
        eye = np.array([rng.uniform(-half_xy, half_xy), rng.uniform(-half_xy, half_xy), rng.uniform(1.5, 10.0)])
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        pitch = math.radians(rng.uniform(-20.0, 0.0))
        fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
        cams.append(look_at(eye, eye + fwd, (0, 0, 1), width, height))
    return cams


def lod_build_workload(n: int = 400, n_views: int = 6, width: int = 48, height: int = 32, d=(4.0,),
                       seed: int = 61, steps_per_round: int = 4, rounds: int = 3):
    """Inputs of the LOD-level construction loop: the finest level G^(0) as raw
    parameters (cube [-2,2]^3, log-scale N(-2.5, 0.3)), training views at 3-9 m
    from the centre looking at it, and the random draws of every fine-tuning
    step: for level l and round r, a list of (training view index, factor u
    ~ U(0.7, 1.3) of d_l).  Returns (base raw dict with mean/log_scale/
    quat_raw/opacity_logit/sh [16*3][n] as float32, cams, d, schedule)."""
    lv = gaussians(n, (seed, 0), _cube(2.0), -2.5, 0.3, keep_raw=True, morton=False)
    base = {"mean": lv.mean, "log_scale": lv.raw["log_scale"], "quat_raw": lv.raw["quat"],
            "opacity_logit": lv.raw["opacity_logit"], "sh": np.ascontiguousarray(lv.sh.reshape(-1, n))}
    rng = _rng((seed, 1, 96, 0))
    cams = []
    for _ in range(n_views):
        r = rng.uniform(3.0, 9.0)
        th = rng.uniform(0.0, 2.0 * math.pi)
        el = rng.uniform(-0.4, 0.4)
        eye = (r * math.cos(el) * math.sin(th), r * math.sin(el), -r * math.cos(el) * math.cos(th))
        cams.append(look_at(eye, (0, 0, 0), (0, -1, 0), width, height))
    schedule = [[[(int(rng.integers(0, n_views)), float(rng.uniform(0.7, 1.3))) for _ in range(steps_per_round)]
                 for _ in range(rounds)] for _ in d]
    return base, cams, list(d), schedule
