"""CPU oracle for the LOD Gaussian-splatting renderer -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never loads it, and it never loads
the product library: the two share only the seeded input generators in
``synth``.

The arithmetic lives in ``lodge_oracle.c`` (plain C, built twice: FP32 and
FP64, ``-O2 -ffp-contract=off``).  This module only marshals numpy arrays
into it and builds it with gcc on first use.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lodge_oracle.c")
BUILD = os.path.join(HERE, "_build")

ALL, LOD_CAMERA, CHUNKED = 0, 1, 2
TILE = 16


# tag -> (REAL, extra flags).  "f32omp" is the benchmark's timing build: the same source and
# arithmetic as "f32", with the per-Gaussian and per-pixel loops spread over the host cores.
VARIANTS = {"f32": ("float", []), "f64": ("double", []), "f32omp": ("float", ["-fopenmp"])}


def build(force: bool = False) -> None:
    """Compile liblodge_oracle_{f32,f64,f32omp}.so with gcc (no FMA contraction, no fast-math)."""
    os.makedirs(BUILD, exist_ok=True)
    for tag, (real, extra) in VARIANTS.items():
        out = os.path.join(BUILD, f"liblodge_oracle_{tag}.so")
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall",
                               "-fPIC", "-shared", f"-DREAL={real}", *extra, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)


_LIBS = {}


def _lib(tag: str):
    if tag not in _LIBS:
        build()
        lib = C.CDLL(os.path.join(BUILD, f"liblodge_oracle_{tag}.so"))
        _LIBS[tag] = lib
    return _LIBS[tag]


def _structs(real):
    class Level(C.Structure):
        _fields_ = [("n", C.c_int64), ("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p),
                    ("opacity", C.c_void_p), ("sh", C.c_void_p), ("sh_degree", C.c_int32),
                    ("filter3d_var", real)]

    class Camera(C.Structure):
        _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", real), ("fy", real), ("cx", real),
                    ("cy", real), ("R", real * 9), ("t", real * 3), ("pos", real * 3), ("znear", real),
                    ("lim_x", real), ("lim_y", real), ("bg", real * 3)]

    class Grads(C.Structure):
        _fields_ = [("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p), ("opacity", C.c_void_p),
                    ("sh", C.c_void_p)]

    return Level, Camera, Grads


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


@dataclass
class Projection:
    depth: np.ndarray
    uv: np.ndarray
    conic: np.ndarray
    o_eff: np.ndarray
    rgb: np.ndarray
    rect: np.ndarray
    tiles: np.ndarray
    radius: np.ndarray


@dataclass
class Binned:
    tile: np.ndarray
    dkey: np.ndarray
    val: np.ndarray
    ranges: np.ndarray
    M: int


class Oracle:
    """The oracle in one precision ('f32' decides like the FP32 renderer; 'f64' for the adjoint)."""

    def __init__(self, precision: str = "f32"):
        assert precision in VARIANTS
        self.tag = precision
        self.dt = np.float64 if precision == "f64" else np.float32
        self.real = C.c_double if precision == "f64" else C.c_float
        self.L, self.Cam, self.G = _structs(self.real)
        self.lib = _lib(precision)
        self._keep = []

    # -- marshalling ---------------------------------------------------------
    def _arr(self, a):
        a = np.ascontiguousarray(a, dtype=self.dt)
        self._keep.append(a)
        return a

    def levels(self, levels):
        arr = (self.L * len(levels))()
        for i, lv in enumerate(levels):
            arr[i].n = lv.n
            for f in ("mean", "scale", "quat", "opacity", "sh"):
                setattr(arr[i], f, _p(self._arr(getattr(lv, f))))
            arr[i].sh_degree = lv.sh_degree
            arr[i].filter3d_var = lv.filter3d_var
        return arr

    def camera(self, cam):
        c = self.Cam()
        c.width, c.height = cam.width, cam.height
        c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
        for i, v in enumerate(np.asarray(cam.R, np.float64).ravel()):
            c.R[i] = v
        for i in range(3):
            c.t[i] = float(cam.t[i]); c.pos[i] = float(cam.pos[i]); c.bg[i] = float(cam.bg[i])
        c.znear, c.lim_x, c.lim_y = cam.znear, cam.lim_x, cam.lim_y
        return c

    # -- steps ---------------------------------------------------------------
    def chunk_pair(self, centers, band, pos):
        centers = self._arr(centers)
        f, o, t = C.c_int32(), C.c_int32(), self.real()
        rc = self.lib.orc_chunk_pair(_p(centers), C.c_int32(len(centers)), self.real(band), _p(self._arr(pos)),
                                     C.byref(f), C.byref(o), C.byref(t))
        if rc != 0:
            raise ValueError("chunk_pair: no chunks")
        return f.value, o.value, t.value

    def select(self, scene, mode: int, pos, cap: int | None = None):
        lv = self.levels(scene.levels)
        d = self._arr(np.asarray(scene.d if scene.d else [0.0]))
        ch = scene.chunks
        K = 0 if ch is None else len(ch.centers)
        centers = self._arr(ch.centers if K else np.zeros((1, 3)))
        offs = self._arr(ch.offsets if K else np.zeros(1))
        band = ch.band if K else 0.0
        if cap is None:
            cap = scene.n_total
        ids = np.empty(max(cap, 1), np.uint32)
        w = np.empty(max(cap, 1), self.dt)
        f, o, t = C.c_int32(), C.c_int32(), self.real()
        fn = self.lib.orc_select
        fn.restype = C.c_int64
        n = fn(lv, C.c_int32(len(scene.levels)), _p(d), C.c_int32(mode), _p(centers), _p(offs), C.c_int32(K),
               self.real(band), _p(self._arr(pos)), _p(ids), _p(w), C.c_int64(cap), C.byref(f), C.byref(o),
               C.byref(t))
        if n < 0:
            raise ValueError("select: bad arguments")
        return ids[:n].copy(), w[:n].copy(), (f.value, o.value, t.value)

    def select_chunk(self, scene, k: int):
        """The stored active set of chunk k alone (Eq. 2 at the chunk centre, offsets r_k), weight 1."""
        lv = self.levels(scene.levels)
        d = self._arr(np.asarray(scene.d if scene.d else [0.0]))
        ch = scene.chunks
        centers, offs = self._arr(ch.centers), self._arr(ch.offsets)
        cap = max(scene.n_total, 1)
        ids = np.empty(cap, np.uint32)
        w = np.empty(cap, self.dt)
        fn = self.lib.orc_select_chunk
        fn.restype = C.c_int64
        n = fn(lv, C.c_int32(len(scene.levels)), _p(d), _p(centers), _p(offs), C.c_int32(len(ch.centers)),
               C.c_int32(k), _p(ids), _p(w), C.c_int64(cap))
        if n < 0:
            raise ValueError("select_chunk: bad chunk index")
        return ids[:n].copy(), w[:n].copy()

    def project(self, scene, ids, w, cam, s2d=0.3, compensate=True) -> Projection:
        lv = self.levels(scene.levels)
        n = len(ids)
        ids = np.ascontiguousarray(ids, np.uint32)
        w = self._arr(w)
        out = Projection(depth=np.empty(n, self.dt), uv=np.empty((n, 2), self.dt), conic=np.empty((n, 3), self.dt),
                         o_eff=np.empty(n, self.dt), rgb=np.empty((n, 3), self.dt), rect=np.empty((n, 4), np.int32),
                         tiles=np.empty(n, np.uint32), radius=np.empty(n, self.dt))
        c = self.camera(cam)
        self.lib.orc_project(lv, C.c_int32(len(scene.levels)), _p(ids), _p(w), C.c_int64(n), C.byref(c),
                             self.real(s2d), C.c_int32(int(compensate)), _p(out.depth), _p(out.uv), _p(out.conic),
                             _p(out.o_eff), _p(out.rgb), _p(out.rect), _p(out.tiles), _p(out.radius))
        return out

    def bin_sort(self, proj: Projection, cam) -> Binned:
        TX = (cam.width + TILE - 1) // TILE
        TY = (cam.height + TILE - 1) // TILE
        M = int(proj.tiles.astype(np.int64).sum())
        tile = np.empty(max(M, 1), np.uint32)
        dkey = np.empty(max(M, 1), np.uint64)
        val = np.empty(max(M, 1), np.uint32)
        ranges = np.empty((TX * TY, 2), np.uint32)
        fn = self.lib.orc_bin_sort
        fn.restype = C.c_int64
        m = fn(C.c_int64(len(proj.depth)), _p(proj.depth), _p(proj.rect), _p(proj.tiles), C.c_int32(TX),
               C.c_int32(TY), _p(tile), _p(dkey), _p(val), C.c_int64(M), _p(ranges))
        assert m == M
        return Binned(tile=tile[:M], dkey=dkey[:M], val=val[:M], ranges=ranges, M=M)

    def composite(self, proj: Projection, binned: Binned, cam):
        H, W = cam.height, cam.width
        img = np.empty((3, H, W), self.dt)
        T = np.empty((H, W), self.dt)
        nc = np.empty((H, W), np.uint32)
        nb = np.empty((H, W), np.uint32)
        ne = np.empty((H, W), np.uint32)
        near = np.empty((H, W), np.uint8)
        c = self.camera(cam)
        val = binned.val if binned.M else np.zeros(1, np.uint32)
        self.lib.orc_composite(C.byref(c), _p(proj.uv), _p(proj.conic), _p(proj.o_eff), _p(proj.rgb),
                               _p(binned.ranges), _p(val), _p(img), _p(T), _p(nc), _p(nb), _p(ne), _p(near))
        return {"image": img, "final_T": T, "n_contrib": nc, "n_blend": nb, "n_eval": ne, "near": near}

    def composite_brute(self, proj: Projection, cam):
        H, W = cam.height, cam.width
        img = np.empty((3, H, W), self.dt)
        T = np.empty((H, W), self.dt)
        nc = np.empty((H, W), np.uint32)
        c = self.camera(cam)
        self.lib.orc_composite_brute(C.byref(c), C.c_int64(len(proj.depth)), _p(proj.depth), _p(proj.rect),
                                     _p(proj.tiles), _p(proj.uv), _p(proj.conic), _p(proj.o_eff), _p(proj.rgb),
                                     _p(img), _p(T), _p(nc))
        return {"image": img, "final_T": T, "n_contrib": nc}

    def composite_pixels(self, proj: Projection, binned: Binned, cam, xs, ys):
        """The per-pixel walk at the listed pixels only: colour [n, 3], final_T, n_contrib, near."""
        xs = np.ascontiguousarray(xs, np.int32)
        ys = np.ascontiguousarray(ys, np.int32)
        n = len(xs)
        col = np.empty((max(n, 1), 3), self.dt)
        T = np.empty(max(n, 1), self.dt)
        nc = np.empty(max(n, 1), np.uint32)
        near = np.empty(max(n, 1), np.uint8)
        c = self.camera(cam)
        val = binned.val if binned.M else np.zeros(1, np.uint32)
        self.lib.orc_composite_pixels(C.byref(c), _p(proj.uv), _p(proj.conic), _p(proj.o_eff), _p(proj.rgb),
                                      _p(binned.ranges), _p(val), C.c_int64(n), _p(xs), _p(ys), _p(col), _p(T),
                                      _p(nc), _p(near))
        return {"color": col[:n], "final_T": T[:n], "n_contrib": nc[:n], "near": near[:n]}

    def pixel_accept(self, proj: Projection, binned: Binned, cam, x: int, y: int, probe, tol: float) -> bool:
        c = self.camera(cam)
        probe = self._arr(np.asarray(probe))
        val = binned.val if binned.M else np.zeros(1, np.uint32)
        return bool(self.lib.orc_pixel_accept(C.byref(c), _p(proj.uv), _p(proj.conic), _p(proj.o_eff), _p(proj.rgb),
                                              _p(binned.ranges), _p(val), C.c_int32(x), C.c_int32(y), _p(probe),
                                              self.real(tol)))

    def importance(self, proj: Projection, binned: Binned, cam, ids, n_total: int, score=None, amb=None):
        """Max-accumulates each Gaussian's largest blending weight alpha T over the view's pixels into
        score[global id] (Sec. 3 "Preliminaries: Importance pruning"); amb[global id] marks weights
        that a near-threshold decision leaves open.  Returns (score, amb)."""
        if score is None:
            score = np.zeros(n_total, self.dt)
        if amb is None:
            amb = np.zeros(n_total, np.uint8)
        assert score.dtype == self.dt and score.flags.c_contiguous and len(score) == n_total
        assert amb.dtype == np.uint8 and amb.flags.c_contiguous and len(amb) == n_total
        c = self.camera(cam)
        ids = np.ascontiguousarray(ids, np.uint32)
        val = binned.val if binned.M else np.zeros(1, np.uint32)
        self.lib.orc_importance(C.byref(c), _p(proj.uv), _p(proj.conic), _p(proj.o_eff), _p(proj.rgb),
                                _p(binned.ranges), _p(val), _p(ids), _p(score), _p(amb))
        return score, amb

    def pixel_weights(self, proj: Projection, binned: Binned, cam, x: int, y: int):
        """Blending weights of pixel (x, y): (active indices, alpha T, list positions) of its blended entries
        in blend order, and the list position of its first near-threshold decision."""
        cap = max(1, int(binned.M))
        act = np.empty(cap, np.uint32)
        wt = np.empty(cap, self.dt)
        pos = np.empty(cap, np.int64)
        near = C.c_int64()
        c = self.camera(cam)
        val = binned.val if binned.M else np.zeros(1, np.uint32)
        fn = self.lib.orc_pixel_weights
        fn.restype = C.c_int64
        m = fn(C.byref(c), _p(proj.uv), _p(proj.conic), _p(proj.o_eff), _p(proj.rgb), _p(binned.ranges), _p(val),
               C.c_int32(x), C.c_int32(y), _p(act), _p(wt), _p(pos), C.c_int64(cap), C.byref(near))
        assert m >= 0
        return act[:m].copy(), wt[:m].copy(), pos[:m].copy(), int(near.value)

    def sh_basis(self, x, y, z):
        Y = np.empty(16, self.dt)
        self.lib.orc_sh_basis(self.real(x), self.real(y), self.real(z), _p(Y))
        return Y

    # -- adjoint ---------------------------------------------------------------
    def grad2d(self, proj: Projection, binned: Binned, cam, dL_dimage):
        g2 = np.zeros((len(proj.depth), 9), self.dt)
        c = self.camera(cam)
        dl = self._arr(dL_dimage)
        val = binned.val if binned.M else np.zeros(1, np.uint32)
        self.lib.orc_composite_grad2d(C.byref(c), _p(proj.uv), _p(proj.conic), _p(proj.o_eff), _p(proj.rgb),
                                      _p(binned.ranges), _p(val), _p(dl), _p(g2))
        return g2

    def project_grad(self, scene, ids, w, cam, g2, s2d=0.3, compensate=True, grad_level=-1, grads=None):
        lv = self.levels(scene.levels)
        if grads is None:
            grads = [{"mean": np.zeros((3, l.n), self.dt), "scale": np.zeros((3, l.n), self.dt),
                      "quat": np.zeros((4, l.n), self.dt), "opacity": np.zeros(l.n, self.dt),
                      "sh": np.zeros((16, 3, l.n), self.dt)} for l in scene.levels]
        garr = (self.G * len(grads))()
        for i, g in enumerate(grads):
            for f in ("mean", "scale", "quat", "opacity", "sh"):
                setattr(garr[i], f, _p(g[f]))
        c = self.camera(cam)
        ids = np.ascontiguousarray(ids, np.uint32)
        self.lib.orc_project_grad(lv, C.c_int32(len(scene.levels)), _p(ids), _p(self._arr(w)), C.c_int64(len(ids)),
                                  C.byref(c), self.real(s2d), C.c_int32(int(compensate)), _p(self._arr(g2)),
                                  C.c_int32(grad_level), garr)
        return grads

    # -- whole frame -------------------------------------------------------------
    def lists(self, scene, cam, mode: int, s2d=0.3, compensate=True):
        """select -> project -> bin/sort, without compositing (for sampled-pixel checks)."""
        ids, w, fot = self.select(scene, mode, cam.pos)
        proj = self.project(scene, ids, w, cam, s2d, compensate)
        binned = self.bin_sort(proj, cam)
        self._keep.clear()
        return dict(ids=ids, w=w, fot=fot, proj=proj, binned=binned)

    def render(self, scene, cam, mode: int, s2d=0.3, compensate=True, brute=False):
        """select -> project -> bin/sort -> composite, all intermediates returned."""
        ids, w, fot = self.select(scene, mode, cam.pos)
        proj = self.project(scene, ids, w, cam, s2d, compensate)
        binned = self.bin_sort(proj, cam)
        out = self.composite(proj, binned, cam)
        out.update(ids=ids, w=w, fot=fot, proj=proj, binned=binned)
        if brute:
            out["brute"] = self.composite_brute(proj, cam)
        self._keep.clear()
        return out

    def view_lists(self, scene, ids, w, cam, s2d=0.3, compensate=True):
        """project -> bin/sort for a given selection (ids, w) seen from cam."""
        proj = self.project(scene, ids, w, cam, s2d, compensate)
        binned = self.bin_sort(proj, cam)
        self._keep.clear()
        return proj, binned

    def view_importance(self, scene, ids, w, cam, score=None, amb=None, s2d=0.3, compensate=True):
        """project -> bin/sort -> importance for a given selection (ids, w) seen from cam."""
        proj = self.project(scene, ids, w, cam, s2d, compensate)
        binned = self.bin_sort(proj, cam)
        out = self.importance(proj, binned, cam, ids, scene.n_total, score, amb)
        self._keep.clear()
        return out

    def render_grad(self, scene, cam, mode: int, dL_dimage, s2d=0.3, compensate=True, grad_level=-1,
                    composite=True):
        """Forward, then the adjoint of L = sum(dL_dimage * image) w.r.t. activated params.
        composite=False skips the forward image (the adjoint recomputes each pixel's trace; pixels
        with a zero loss gradient are skipped), for large frames with sparse dL_dimage."""
        fwd = self.render(scene, cam, mode, s2d, compensate) if composite else self.lists(scene, cam, mode, s2d,
                                                                                            compensate)
        g2 = self.grad2d(fwd["proj"], fwd["binned"], cam, dL_dimage)
        grads = self.project_grad(scene, fwd["ids"], fwd["w"], cam, g2, s2d, compensate, grad_level)
        self._keep.clear()
        return fwd, g2, grads


# -- visibility filtering of the stored chunk sets (Sec. 3 "Visibility filtering") -------------------------


def prune_chunk_set(ids, score, threshold):
    """Chunk set after visibility filtering: the members whose importance score reaches the threshold
    (Gaussians scoring below it are removed).  ids ascending global ids, score by global id."""
    ids = np.asarray(ids, np.uint32)
    return ids[np.asarray(score)[ids] >= threshold]


def union_select(n_total, set_f, set_o, t):
    """The two-chunk selection from stored sets A_f, A_o (ascending global ids): their union in ascending
    id, weight 1 in both, t in A_f only and 1 - t (one FP32 rounding) in A_o only (Eq. 4 and its text:
    only the symmetric difference is re-weighted).  set_o None: A_f alone, weight 1."""
    in_f = np.zeros(n_total, bool)
    in_f[np.asarray(set_f, np.int64)] = True
    in_o = np.zeros(n_total, bool)
    if set_o is not None:
        in_o[np.asarray(set_o, np.int64)] = True
    ids = np.nonzero(in_f | in_o)[0].astype(np.uint32)
    t32 = np.float32(t)
    w = np.where(in_f[ids] & in_o[ids], np.float32(1.0),
                 np.where(in_f[ids], t32, np.float32(1.0) - t32)).astype(np.float32)
    if set_o is None:
        w[:] = 1.0
    return ids, w


# -- depth-threshold selection (Sec. 3 "Selecting depth thresholds") ---------------------------------------


def lod_instances(O: "Oracle", scene, d, n_levels: int, cam, s2d=0.3, compensate=True) -> int:
    """Tile instances of one LOD frame: levels 0..n_levels-1 of the scene with switch distances d
    (n_levels - 1 values), Eq. 2 about the camera, every selected Gaussian counted once per 16 x 16
    tile its projected rectangle covers (the Gaussians each tile processes)."""
    from synth import Scene
    sub = Scene(levels=list(scene.levels[:n_levels]), d=[float(x) for x in d], chunks=None)
    ids, w, _ = O.select(sub, LOD_CAMERA, cam.pos)
    proj = O.project(sub, ids, w, cam, s2d, compensate)
    O._keep.clear()
    return int(proj.tiles.astype(np.int64).sum())


def tiles_of(cam) -> int:
    return ((cam.width + TILE - 1) // TILE) * ((cam.height + TILE - 1) // TILE)


def threshold_cost(O: "Oracle", scene, d, n_levels: int, cams, s2d=0.3, compensate=True) -> float:
    """The cost the search minimises: the average number of Gaussians per tile over the views."""
    return float(np.mean([lod_instances(O, scene, d, n_levels, c, s2d, compensate) / tiles_of(c) for c in cams]))


def greedy_thresholds(cost, candidates, n_levels: int):
    """Greedy 1-D search: d_1 is the candidate minimising cost((d_1,)) over two levels; with d_1..d_{l-1}
    fixed, d_l is the candidate above d_{l-1} minimising cost((d_1, ..., d_l)) over levels 0..l.  Ties go
    to the smaller candidate.  cost(d) takes the tuple of thresholds (its length fixes the level count).
    Returns (thresholds, per-step list of (candidate, cost) pairs)."""
    cands = sorted(float(c) for c in candidates)
    chosen, curves = [], []
    for l in range(1, n_levels):
        lo = chosen[-1] if chosen else -np.inf
        curve = [(c, cost(tuple(chosen) + (c,))) for c in cands if c > lo]
        if not curve:
            raise ValueError("no candidate above the previous threshold")
        best = min(curve, key=lambda p: (p[1], p[0]))
        chosen.append(best[0])
        curves.append(curve)
    return chosen, curves


# -- LOD-level construction (supplementary "LOD structure optimization steps") --------------------------------
# float64 throughout; the parameters of a level are raw (pre-activation): mean [3][n], log_scale [3][n],
# quat_raw [4][n], opacity_logit [n], sh [16][3][n].

RAW_KEYS = ("mean", "log_scale", "quat_raw", "opacity_logit", "sh")


def activate(raw):
    """3DGS parameterisation: scale = exp(log_scale), q = q_raw / |q_raw|, opacity = 1 / (1 + exp(-logit))."""
    q = np.asarray(raw["quat_raw"], np.float64)
    return {"mean": np.asarray(raw["mean"], np.float64), "scale": np.exp(np.asarray(raw["log_scale"], np.float64)),
            "quat": q / np.linalg.norm(q, axis=0), "opacity": 1.0 / (1.0 + np.exp(-np.asarray(raw["opacity_logit"],
                                                                                              np.float64))),
            "sh": np.asarray(raw["sh"], np.float64)}


def activate_adjoint(raw, g):
    """Gradients w.r.t. the raw parameters from gradients w.r.t. the activated ones (chain rule of
    activate): d/dlog_scale = g_scale * scale; d/dq_raw = (g_q - u (u . g_q)) / |q_raw| with u = q_raw/|q_raw|;
    d/dlogit = g_opacity * o (1 - o)."""
    act = activate(raw)
    q = np.asarray(raw["quat_raw"], np.float64)
    qn = np.linalg.norm(q, axis=0)
    u = q / qn
    return {"mean": g["mean"], "log_scale": g["scale"] * act["scale"],
            "quat_raw": (g["quat"] - u * np.sum(u * g["quat"], axis=0)) / qn,
            "opacity_logit": g["opacity"] * act["opacity"] * (1.0 - act["opacity"]), "sh": g["sh"]}


def l1_loss_grad(image, target):
    """Mean L1 loss over all values and its gradient sign(image - target) / N (0 where equal)."""
    d = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    return float(np.mean(np.abs(d))), np.sign(d) / d.size


def adam_update(p, g, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (Kingma and Ba, Algorithm 1) at step t >= 1: returns the new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def lod_level_scene(levels_raw, sh_degrees, filter_vars, d):
    """A Scene (float64, activated) of the given raw levels and switch distances."""
    from synth import Level, Scene
    lv = []
    for raw, deg, var in zip(levels_raw, sh_degrees, filter_vars):
        a = activate(raw)
        sh = np.zeros((16, 3, a["mean"].shape[1]))
        nsh = (deg + 1) ** 2
        sh[:nsh] = np.asarray(raw["sh"], np.float64).reshape(nsh, 3, -1)
        lv.append(Level(mean=a["mean"], scale=a["scale"], quat=a["quat"], opacity=a["opacity"], sh=sh,
                        sh_degree=deg, filter3d_var=var))
    return Scene(levels=lv, d=[float(x) for x in d], chunks=None)


def finetune_grad(O64: "Oracle", levels_raw, sh_degrees, filter_vars, d, l, cam, target, d_factor, dL=None,
                  lam=0.0):
    """The gradient of one fine-tuning step of level l w.r.t. level l's raw parameters: render levels
    0..l with Eq. 2 about the camera and d_l replaced by d_factor * d_l (both rounded to FP32 like the
    switch distances a scene stores), loss (1 - lam) mean L1 + lam (1 - mean SSIM) against target,
    adjoint restricted to level l.
    dL: use this dL/dimage instead of the loss's (to follow another renderer's sign decisions).
    Returns (loss, dL/dimage, raw gradient of level l, rendered image)."""
    dd = [float(np.float32(x)) for x in d[:l]]
    dd[l - 1] = float(np.float32(np.float32(dd[l - 1]) * np.float32(d_factor)))
    sc = lod_level_scene(levels_raw[:l + 1], sh_degrees[:l + 1], filter_vars[:l + 1], dd)
    fwd = O64.render(sc, cam, LOD_CAMERA)
    loss, g_img = l1_loss_grad(fwd["image"], target)
    loss, g_img = (1.0 - lam) * loss, (1.0 - lam) * g_img
    if lam:
        ls, gs = dssim_grad(fwd["image"], target)
        loss, g_img = loss + lam * ls, g_img + lam * gs
    if dL is not None:
        g_img = dL
    g2 = O64.grad2d(fwd["proj"], fwd["binned"], cam, g_img)
    grads = O64.project_grad(sc, fwd["ids"], fwd["w"], cam, g2, grad_level=l)
    O64._keep.clear()
    nsh = (sh_degrees[l] + 1) ** 2
    g = dict(grads[l])
    g["sh"] = g["sh"][:nsh].reshape(nsh * 3, -1)
    return loss, g_img, activate_adjoint(levels_raw[l], g), fwd["image"]


def keep_indices(score, threshold):
    """Importance pruning: indices (ascending) of the items whose score reaches the threshold."""
    return np.flatnonzero(np.asarray(score) >= threshold).astype(np.uint32)


# -- the D-SSIM term of the construction loss (3DGS's L = (1 - lambda) L1 + lambda (1 - SSIM)) -----------------

SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window(size=11, sigma=1.5):
    """Normalised 1-D Gaussian window (the separable factor of SSIM's 11 x 11 window)."""
    x = np.arange(size, dtype=np.float64) - size // 2
    w = np.exp(-(x * x) / (2.0 * sigma * sigma))
    return w / w.sum()


def _blur(img):
    """Separable window filter of each channel with zero padding outside the image ('same' size)."""
    w = ssim_window()
    h = len(w) // 2

    def same(r):   # the centred part of the full convolution: also for lines shorter than the window
        return np.convolve(r, w, mode="full")[h:h + len(r)]
    out = np.empty_like(img, dtype=np.float64)
    for c in range(img.shape[0]):
        rows = np.apply_along_axis(same, 1, img[c].astype(np.float64))
        out[c] = np.apply_along_axis(same, 0, rows)
    return out


def ssim_map(x, y):
    """Per-pixel SSIM of two images [C][H][W] (Wang et al. 2004 with the 11 x 11 Gaussian window of
    sigma 1.5, C1 = 0.01^2, C2 = 0.03^2, local statistics by zero-padded filtering)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = _blur(x), _blur(y)
    sxx = _blur(x * x) - mx * mx
    syy = _blur(y * y) - my * my
    sxy = _blur(x * y) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def dssim_grad(x, y):
    """(1 - mean SSIM) and its gradient w.r.t. x.  With m the SSIM map, mu_x = w * x, E_xx = w * x^2,
    E_xy = w * (x y) (w the window, * zero-padded filtering), the chain rule through the three filtered
    maps and the window's symmetry give
        d(mean m)/dx = w * (g dm/dmu_x) + 2 x (w * (g dm/dE_xx)) + y (w * (g dm/dE_xy)),  g = 1 / N."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = _blur(x), _blur(y)
    exx, eyy, exy = _blur(x * x), _blur(y * y), _blur(x * y)
    a1 = 2 * mx * my + SSIM_C1
    a2 = 2 * (exy - mx * my) + SSIM_C2
    b1 = mx * mx + my * my + SSIM_C1
    b2 = (exx - mx * mx) + (eyy - my * my) + SSIM_C2
    m = (a1 * a2) / (b1 * b2)
    g = 1.0 / m.size
    d_mx = (2 * my * a2 - 2 * my * a1) / (b1 * b2) - m * (2 * mx) / b1 + m * (2 * mx) / b2
    d_exx = -m / b2
    d_exy = 2 * a1 / (b1 * b2)
    grad = _blur(g * d_mx) + 2 * x * _blur(g * d_exx) + y * _blur(g * d_exy)
    return float(1.0 - m.mean()), -grad
