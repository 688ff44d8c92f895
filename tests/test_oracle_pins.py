"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these retypes the oracle's own formulas: each checks a closed form
of a special case, an invariant, hand-worked values, a library routine or a
brute-force alternative, chosen so that a dropped term, a wrong sign or
index, or a transposed operand in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from synth import Camera, Chunks, Level, Scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# helpers: hand-built scenes
# ---------------------------------------------------------------------------

def axis_camera(W=64, H=64, f=80.0, bg=(0.0, 0.0, 0.0), pos=(0.0, 0.0, 0.0)):
    """Camera at `pos` looking down +z with identity rotation."""
    pos = np.asarray(pos, np.float32)
    return Camera(width=W, height=H, fx=f, fy=f, cx=W / 2.0, cy=H / 2.0, R=np.eye(3, dtype=np.float32),
                  t=(-pos).astype(np.float32), pos=pos, znear=0.2, lim_x=1.3 * (W / 2.0) / f,
                  lim_y=1.3 * (H / 2.0) / f, bg=bg)


def make_level(means, scales, quats=None, opac=None, dc=None, var=0.0, sh=None):
    means = np.asarray(means, np.float64).reshape(-1, 3)
    n = len(means)
    scales = np.broadcast_to(np.asarray(scales, np.float64), (n, 3)) if np.ndim(scales) else np.full((n, 3), scales)
    if quats is None:
        quats = np.tile([1.0, 0, 0, 0], (n, 1))
    if opac is None:
        opac = np.full(n, 0.5)
    if sh is None:
        sh = np.zeros((16, 3, n))
        sh[0] = np.broadcast_to(np.asarray(dc if dc is not None else 0.5, np.float64).reshape(-1, 1), (3, n)) \
            if np.ndim(dc) <= 1 else np.asarray(dc).T
    return Level(mean=np.ascontiguousarray(means.T, np.float32), scale=np.ascontiguousarray(np.asarray(scales).T, np.float32),
                 quat=np.ascontiguousarray(np.asarray(quats, np.float64).T, np.float32),
                 opacity=np.asarray(opac, np.float32), sh=np.asarray(sh, np.float32), sh_degree=3,
                 filter3d_var=float(np.float32(var)))


def one_level_scene(level):
    return Scene(levels=[level], d=[], chunks=None)


C0 = 1.0 / (2.0 * math.sqrt(math.pi))


# ---------------------------------------------------------------------------
# Eq. 4: chunk pair and t
# ---------------------------------------------------------------------------

def test_chunk_pair_hand_worked_cases(oracle32, oracle64):
    g = json.load(open(os.path.join(GOLDEN, "chunk_pair_cases.json")))
    centers = np.asarray(g["centers"], np.float64)
    for O in (oracle32, oracle64):
        for case in g["cases"]:
            f, o, t = O.chunk_pair(centers, case["band"], np.asarray(case["c"], np.float64))
            assert (f, o) == (case["f"], case["o"]), case
            assert t == case["t"], case


def test_chunk_pair_nearest_two_by_enumeration(oracle32):
    rng = np.random.default_rng(7)
    for trial in range(200):
        K = int(rng.integers(2, 20))
        centers = rng.uniform(-50, 50, (K, 3)).astype(np.float32)
        c = rng.uniform(-60, 60, 3).astype(np.float32)
        f, o, t = oracle32.chunk_pair(centers, 0.0, c)
        d = np.linalg.norm(centers.astype(np.float64) - c, axis=1)
        order = np.argsort(d, kind="stable")
        assert f == order[0] and o == order[1]
        # the nearest chunk never weighs less than one half (its weights are "close to 1")
        assert t >= 0.5
        # t is the projection of c - m_o on the centre line, clamped (float64 reference within FP32 rounding)
        g_ = centers[f].astype(np.float64) - centers[o]
        tb = np.dot(c - centers[o].astype(np.float64), g_) / np.dot(g_, g_)
        assert abs(t - min(1.0, max(0.0, tb))) <= 1e-5


def test_chunk_pair_single_chunk_and_none(oracle32):
    f, o, t = oracle32.chunk_pair(np.zeros((1, 3)), 0.0, np.ones(3))
    assert (f, o, t) == (0, -1, 1.0)
    with pytest.raises(ValueError):
        oracle32.chunk_pair(np.zeros((0, 3)), 0.0, np.ones(3))


# ---------------------------------------------------------------------------
# Eq. 2: active set; chunk offsets
# ---------------------------------------------------------------------------

def test_lod_partition_identical_levels_select_each_gaussian_once(oracle32):
    """L identical copies of one level, camera mode: [d_l, d_{l+1}) partitions
    [0, inf), so each Gaussian is selected from exactly one copy, and the LOD
    render equals the plain render of the single level bit for bit."""
    base = synth.gaussians(3000, (901, 0), synth._cube(4.0), -3.0, 0.5, morton=False)
    # three Gaussians exactly on the switch distances 2 and 4 (inclusive lower bound)
    base.mean[:, 0] = [2.0, 0.0, 0.0]
    base.mean[:, 1] = [0.0, 4.0, 0.0]
    base.mean[:, 2] = [0.0, 0.0, 2.0]
    lod = Scene(levels=[base, base, base], d=[2.0, 4.0])
    cam = synth.look_at((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0, -1, 0), 96, 80)
    cam.pos = np.zeros(3, np.float32)
    ids, w, _ = oracle32.select(lod, oracle.LOD_CAMERA, cam.pos)
    n = base.n
    local = ids % n
    lvl = ids // n
    assert np.array_equal(np.sort(local), np.arange(n)), "each Gaussian exactly once"
    assert np.all(w == 1.0)
    sel_level = dict(zip(local.tolist(), lvl.tolist()))
    assert sel_level[0] == 1 and sel_level[2] == 1 and sel_level[1] == 2
    dist = np.linalg.norm(base.mean.T.astype(np.float64), axis=1)
    expect = np.where(dist < 2.0, 0, np.where(dist < 4.0, 1, 2))
    assert np.array_equal(np.array([sel_level[i] for i in range(n)]), expect)
    # image equality with the plain render
    cam2 = synth.look_at((0.0, 0.5, -6.0), (0.0, 0.0, 0.0), (0, -1, 0), 96, 80)
    r_lod = oracle32.render(lod, cam2, oracle.LOD_CAMERA)
    r_one = oracle32.render(one_level_scene(base), cam2, oracle.ALL)
    assert np.array_equal(r_lod["image"], r_one["image"])
    assert np.array_equal(r_lod["final_T"], r_one["final_T"])


def test_chunk_offsets_and_union_weights(oracle32):
    """Two chunks 10 m apart with offset r = 10; level thresholds d = (3,):
    level 0 about chunk k covers [0, 13), level 1 covers [13, inf)."""
    rng = np.random.default_rng(3)
    m = rng.uniform(-30, 30, (4000, 3))
    m[0] = [13.0, 0.0, 0.0]   # exactly d_1 + r from chunk 0
    lv0 = make_level(m, 0.05)
    lv1 = make_level(m, 0.05)
    ch = Chunks(centers=np.array([[0, 0, 0], [10, 0, 0]], np.float32), offsets=np.array([10, 10], np.float32))
    sc = Scene(levels=[lv0, lv1], d=[3.0], chunks=ch)
    pos = np.array([2.0, 1.0, 0.0], np.float32)   # tau = 1/5 -> t = 0.8
    ids, w, (f, o, t) = oracle32.select(sc, oracle.CHUNKED, pos)
    assert (f, o) == (0, 1) and t == np.float32(0.8)
    n = len(m)
    md = m.astype(np.float32).astype(np.float64)
    dF = np.linalg.norm(md - [0, 0, 0], axis=1)
    dO = np.linalg.norm(md - [10, 0, 0], axis=1)
    inF = [dF < 13.0, dF >= 13.0]
    inO = [dO < 13.0, dO >= 13.0]
    exp_ids, exp_w = [], []
    for l in range(2):
        for i in range(n):
            a, b = inF[l][i], inO[l][i]
            if a or b:
                exp_ids.append(l * n + i)
                exp_w.append(1.0 if (a and b) else (np.float32(0.8) if a else np.float32(1) - np.float32(0.8)))
    assert np.array_equal(ids, np.asarray(exp_ids, np.uint32))
    assert np.array_equal(w, np.asarray(exp_w, np.float32))
    # the Gaussian exactly at distance d_1 + r_0 from chunk 0 belongs to level 1 about chunk 0
    assert n + 0 in set(ids.tolist())


def test_camera_at_chunk_centre_renders_nearest_set_alone(oracle32):
    """Camera at m_f: t = 1, so every Gaussian only in the other chunk's set
    gets weight 0 and the image equals the render of A_f alone."""
    sc = synth.lod_city_scene(counts=(6000, 1500), half_xy=20.0, d=(6.0,), grid=2, spacing=8.0, chunk_z=1.0,
                              band=0.0, seed=11)
    pos = sc.chunks.centers[0].astype(np.float64)
    cam = synth.look_at(pos, pos + np.array([1.0, 0.2, -0.1]), (0, 0, 1), 128, 72)
    cam.pos = sc.chunks.centers[0].copy()
    r = oracle32.render(sc, cam, oracle.CHUNKED)
    f, o, t = r["fot"]
    assert f == 0 and t == 1.0
    assert set(np.unique(r["w"]).tolist()) <= {0.0, 1.0}
    # A_f alone: a scene whose only chunk is f
    only_f = Scene(levels=sc.levels, d=sc.d, chunks=Chunks(centers=sc.chunks.centers[:1], offsets=sc.chunks.offsets[:1]))
    r_f = oracle32.render(only_f, cam, oracle.CHUNKED)
    assert set(r_f["ids"].tolist()) == set(r["ids"][r["w"] == 1.0].tolist())
    assert np.array_equal(r["image"], r_f["image"])


def test_storage_permutation_invariance(oracle32):
    sc = synth.lod_city_scene(counts=(5000, 1200), half_xy=15.0, d=(5.0,), grid=2, spacing=6.0, chunk_z=1.0,
                              band=3.0, seed=12)
    cam = synth.look_at((-1.0, 0.5, 1.2), (10.0, 0.0, 0.0), (0, 0, 1), 112, 64)
    r = oracle32.render(sc, cam, oracle.CHUNKED)
    rng = np.random.default_rng(0)
    perms = [rng.permutation(l.n) for l in sc.levels]
    sp = Scene(levels=[synth.permuted(l, p) for l, p in zip(sc.levels, perms)], d=sc.d, chunks=sc.chunks)
    rp = oracle32.render(sp, cam, oracle.CHUNKED)
    # same selected set (mapped back to original storage) with the same weights
    def keyed(res, perm_list):
        out = {}
        base = 0
        bases = [0]
        for l in sc.levels:
            bases.append(bases[-1] + l.n)
        for g, w in zip(res["ids"].tolist(), res["w"].tolist()):
            l = max(i for i in range(len(sc.levels)) if bases[i] <= g)
            i = g - bases[l]
            orig = i if perm_list is None else int(perm_list[l][i])
            out[(l, orig)] = w
        return out
    assert keyed(r, None) == keyed(rp, perms)
    assert np.array_equal(r["image"], rp["image"])


# ---------------------------------------------------------------------------
# projection closed forms (EWA, Eq. 3, 2-D filter, SH)
# ---------------------------------------------------------------------------

def isotropic_expected(W, H, f, z, sigma, o, k_dc, s2d=0.3, var=0.0, X=0.0):
    """Closed form of one isotropic Gaussian at (X, 0, z) seen by axis_camera:
    J = [[f/z, 0, -f X / z^2], [0, f/z, 0]], Sigma' = (sigma^2 + var) J J^T + s2d I."""
    v = sigma * sigma + var
    a0 = v * ((f / z) ** 2 + (f * X / z ** 2) ** 2)
    c0 = v * (f / z) ** 2
    a, c = a0 + s2d, c0 + s2d
    comp2 = math.sqrt(a0 * c0 / (a * c))
    comp3 = (sigma * sigma / v) ** 1.5
    u, vv = f * X / z + W / 2.0, H / 2.0
    r = math.ceil(3.0 * math.sqrt(max(a, c)))
    rgb = C0 * k_dc + 0.5
    img = np.zeros((3, H, W))
    T = np.ones((H, W))
    TX, TY = (W + 15) // 16, (H + 15) // 16
    x0, x1 = max(0, math.floor((u - r) / 16)), min(TX, math.floor((u + r) / 16) + 1)
    y0, y1 = max(0, math.floor((vv - r) / 16)), min(TY, math.floor((vv + r) / 16) + 1)
    for py in range(H):
        for px in range(W):
            if not (x0 <= px // 16 < x1 and y0 <= py // 16 < y1):
                continue
            dx, dy = u - (px + 0.5), vv - (py + 0.5)
            alpha = min(0.99, o * comp3 * comp2 * math.exp(-0.5 * (dx * dx / a + dy * dy / c)))
            if alpha < 1.0 / 255.0:
                continue
            img[:, py, px] = rgb * alpha
            T[py, px] = 1.0 - alpha
    return dict(a=a, c=c, u=u, v=vv, r=r, rect=(x0, y0, x1, y1), comp2=comp2, comp3=comp3, img=img, T=T, rgb=rgb)


@pytest.mark.parametrize("X,var", [(0.0, 0.0), (0.0, 0.004), (1.5, 0.0), (-2.0, 0.002)])
def test_isotropic_gaussian_closed_form(oracle64, oracle32, X, var):
    W = H = 64
    f, z, sigma, o, k = 80.0, 5.0, 0.1, 0.8, 0.7
    lv = make_level([[X, 0.0, z]], sigma, opac=[o], dc=k, var=var)
    # float32 inputs: use the values they round to in the closed form
    X32, z32, s32 = float(np.float32(X)), float(np.float32(z)), float(np.float32(sigma))
    e = isotropic_expected(W, H, f, z32, s32, float(np.float32(o)), float(np.float32(k)), var=float(np.float32(var)), X=X32)
    cam = axis_camera(W, H, f)
    for O, tol in ((oracle64, 1e-12), (oracle32, 2e-6)):
        r = O.render(one_level_scene(lv), cam, oracle.ALL)
        p = r["proj"]
        assert tuple(p.rect[0]) == e["rect"]
        assert p.radius[0] == e["r"]
        assert abs(p.uv[0, 0] - e["u"]) <= tol * 100 and abs(p.uv[0, 1] - e["v"]) <= tol * 100
        assert np.allclose(p.conic[0], [1 / e["a"], 0.0, 1 / e["c"]], rtol=tol * 10, atol=tol)
        assert abs(p.o_eff[0] - float(np.float32(o)) * e["comp2"] * e["comp3"]) <= tol
        assert np.allclose(p.rgb[0], e["rgb"], atol=tol)
        assert np.abs(r["image"] - e["img"]).max() <= tol * 10
        assert np.abs(r["final_T"] - e["T"]).max() <= tol * 10


def test_quaternion_quarter_turn_swaps_axes(oracle64):
    """q = (cos 45, 0, 0, sin 45) turns x into y: Sigma = diag(sy^2, sx^2, sz^2)."""
    f, z, sx, sy = 80.0, 5.0, 0.2, 0.05
    h = math.sqrt(0.5)
    lv = make_level([[0.0, 0.0, z]], [[sx, sy, 0.1]], quats=[[h, 0.0, 0.0, h]], opac=[0.5])
    cam = axis_camera(64, 64, f)
    p = oracle64.render(one_level_scene(lv), cam, oracle.ALL)["proj"]
    sx32, sy32 = float(np.float32(sx)), float(np.float32(sy))
    a = (f / z) ** 2 * sy32 ** 2 + 0.3
    c = (f / z) ** 2 * sx32 ** 2 + 0.3
    assert np.allclose(p.conic[0], [1 / a, 0.0, 1 / c], rtol=1e-6, atol=1e-6)  # q rounded to float32
    # an unrotated copy has the axes the other way round
    lv2 = make_level([[0.0, 0.0, z]], [[sx, sy, 0.1]], opac=[0.5])
    p2 = oracle64.render(one_level_scene(lv2), cam, oracle.ALL)["proj"]
    assert np.allclose(p2.conic[0], [1 / c, 0.0, 1 / a], rtol=1e-6, atol=1e-6)


def test_anisotropic_general_matches_matrix_product(oracle64):
    """A random rotated anisotropic Gaussian: Sigma' from numpy's matrix
    products of (J W) R S^2 R^T (J W)^T (library routine, not the oracle's sums)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        mu = rng.uniform(-1, 1, 3) + [0, 0, 6]
        s = np.exp(rng.normal(-2, 0.4, 3))
        q = rng.normal(size=4); q /= np.linalg.norm(q)
        lv = make_level([mu], [s], quats=[q], opac=[0.6], var=0.001)
        cam = synth.look_at((0.3, -0.2, -1.0), (0.1, 0.0, 6.0), (0, -1, 0), 96, 64)
        p = oracle64.render(one_level_scene(lv), cam, oracle.ALL)["proj"]
        mu32 = lv.mean[:, 0].astype(np.float64); s32 = lv.scale[:, 0].astype(np.float64)
        w, x, y, z = lv.quat[:, 0].astype(np.float64)
        # rotation of a unit quaternion via scipy (independent formula)
        from scipy.spatial.transform import Rotation
        Rq = Rotation.from_quat([x, y, z, w]).as_matrix()
        Sig = Rq @ np.diag(s32 ** 2 + np.float32(0.001)) @ Rq.T
        Wc = cam.R.astype(np.float64)
        tc = Wc @ mu32 + cam.t.astype(np.float64)
        J = np.array([[cam.fx / tc[2], 0, -cam.fx * tc[0] / tc[2] ** 2], [0, cam.fy / tc[2], -cam.fy * tc[1] / tc[2] ** 2]])
        Sp = J @ Wc @ Sig @ Wc.T @ J.T + 0.3 * np.eye(2)
        inv = np.linalg.inv(Sp)
        if p.tiles[0] == 0:
            continue
        assert np.allclose(p.conic[0], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-5)
        assert abs(p.depth[0] - tc[2]) < 1e-9


def test_sh_basis_orthonormal_by_quadrature(oracle64):
    """Integral of Y_i Y_j over the sphere is delta_ij (Gauss-Legendre in
    cos(theta) x uniform phi; exact for these polynomial degrees)."""
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 24
    G = np.zeros((16, 16))
    for ct, wt in zip(xg, wg):
        st = math.sqrt(1 - ct * ct)
        for k in range(nphi):
            ph = 2 * math.pi * k / nphi
            Y = oracle64.sh_basis(st * math.cos(ph), st * math.sin(ph), ct)
            G += wt * (2 * math.pi / nphi) * np.outer(Y, Y)
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_sh_addition_theorem(oracle64):
    """sum_m Y_lm(u) Y_lm(v) = (2l+1)/(4 pi) P_l(u.v): fixes each band's span and scale."""
    rng = np.random.default_rng(1)
    for _ in range(50):
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        v = rng.normal(size=3); v /= np.linalg.norm(v)
        Yu, Yv = oracle64.sh_basis(*u), oracle64.sh_basis(*v)
        for l in range(4):
            sl = slice(l * l, (l + 1) * (l + 1))
            lhs = float(np.dot(Yu[sl], Yv[sl]))
            Pl = np.polynomial.legendre.Legendre.basis(l)(float(np.dot(u, v)))
            assert abs(lhs - (2 * l + 1) / (4 * math.pi) * Pl) < 1e-12


# ---------------------------------------------------------------------------
# compositing (Eq. 1, front-to-back blending)
# ---------------------------------------------------------------------------

def test_blend_weights_plus_transmittance_is_one(oracle32, oracle64):
    """With every colour 1 and bg 0, image = sum_k alpha_k T_k = 1 - T_final."""
    sc = synth.plain_scene(n=3000, seed=21, width=96, height=80)
    lv = sc.levels[0]
    lv.sh[:] = 0.0
    lv.sh[0] = 0.5 / C0
    for O, tol in ((oracle32, 1e-5), (oracle64, 1e-12)):
        r = O.render(sc, sc.cameras[0], oracle.ALL)
        for ch in range(3):
            c = r["proj"].rgb[0, ch]          # the float32-stored DC gives c = 1 up to rounding
            assert np.all(r["proj"].rgb[:, ch] == c) and abs(c - 1.0) < 1e-6
            assert np.abs(r["image"][ch] / c + r["final_T"] - 1.0).max() <= tol


def test_tiled_equals_brute_force(oracle32):
    sc = synth.plain_scene(n=2500, seed=22, width=80, height=72)
    r = oracle32.render(sc, sc.cameras[0], oracle.ALL, brute=True)
    b = r["brute"]
    assert np.array_equal(r["image"], b["image"])
    assert np.array_equal(r["final_T"], b["final_T"])
    assert np.array_equal(r["n_contrib"], b["n_contrib"])


def test_sort_order_and_ranges(oracle32):
    sc = synth.plain_scene(n=2000, seed=23, width=96, height=64)
    r = oracle32.render(sc, sc.cameras[0], oracle.ALL)
    bn, p = r["binned"], r["proj"]
    key = np.lexsort((bn.val, bn.dkey, bn.tile))      # numpy's sort of the same triples
    assert np.array_equal(key, np.arange(bn.M))
    assert np.array_equal(bn.dkey, p.depth[bn.val].view(np.uint32).astype(np.uint64))
    for t in range(len(bn.ranges)):
        s, e = bn.ranges[t]
        assert np.all(bn.tile[s:e] == t)
    assert int(bn.ranges[:, 1].max()) == bn.M
    # instance count per Gaussian = rectangle area
    cnt = np.bincount(bn.val, minlength=len(p.tiles))
    assert np.array_equal(cnt, p.tiles)


def test_special_cases_opaque_empty_two_layers(oracle64):
    W = H = 64
    f = 80.0
    bg = (0.1, 0.2, 0.3)
    cam = axis_camera(W, H, f, bg=bg)
    # one near-opaque wide Gaussian at the centre: alpha clamps at 0.99
    lv = make_level([[0.0, 0.0, 5.0]], 0.6, opac=[1.0], dc=0.5 / C0)
    r = oracle64.render(one_level_scene(lv), cam, oracle.ALL, compensate=False)
    assert abs(r["final_T"][32, 32] - 0.01) < 1e-12
    # an empty frame is pure background
    far = make_level([[0.0, 0.0, -5.0]], 0.1)     # behind the camera: culled
    r2 = oracle64.render(one_level_scene(far), cam, oracle.ALL)
    for ch in range(3):
        assert np.all(r2["image"][ch] == bg[ch])
    assert np.all(r2["final_T"] == 1.0) and np.all(r2["n_contrib"] == 0)
    # two layers: C = c1 a1 + c2 a2 (1 - a1) (+ T bg); storage order back-to-front
    s = 0.3
    lv2 = make_level([[0.0, 0.0, 8.0], [0.0, 0.0, 4.0]], s, opac=[0.7, 0.6], dc=[[0.2, 0.2, 0.2], [0.9, 0.9, 0.9]])
    r3 = oracle64.render(one_level_scene(lv2), cam, oracle.ALL, compensate=False)
    px = py = 34
    def alpha(z, o):
        a = (f * float(np.float32(s)) / z) ** 2 + 0.3
        d = 32 - (px + 0.5)
        return min(0.99, float(np.float32(o)) * math.exp(-0.5 * (d * d / a + d * d / a)))
    a1, a2 = alpha(4.0, 0.6), alpha(8.0, 0.7)
    c1, c2 = C0 * float(np.float32(0.9)) + 0.5, C0 * float(np.float32(0.2)) + 0.5
    T = (1 - a1) * (1 - a2)
    assert a1 > 1 / 255 and a2 > 1 / 255
    for ch in range(3):
        assert abs(r3["image"][ch, py, px] - (c1 * a1 + c2 * a2 * (1 - a1) + T * bg[ch])) < 1e-12
    assert r3["n_contrib"][py, px] == 2


def test_early_termination(oracle64):
    """Stacked wide opaque layers: T = prod (1 - alpha_k); the layer that would
    push T below 1e-4 is not blended and ends the pixel."""
    W = H = 32
    cam = axis_camera(W, H, 40.0)
    zs = [3.0 + 0.5 * k for k in range(10)]
    lv = make_level([[0.0, 0.0, z] for z in zs[::-1]], 0.5, opac=[0.9] * 10, dc=0.5 / C0)
    r = oracle64.render(one_level_scene(lv), cam, oracle.ALL, compensate=False)
    px = py = 16
    T, k_last = 1.0, 0
    for k, z in enumerate(zs):
        a = (40.0 * 0.5 / z) ** 2 + 0.3
        d = 16 - (px + 0.5)
        al = min(0.99, float(np.float32(0.9)) * math.exp(-0.5 * (2 * d * d / a)))
        if T * (1 - al) < 1e-4:
            break
        T *= (1 - al)
        k_last = k + 1
    assert r["n_contrib"][py, px] == k_last < 10
    assert abs(r["final_T"][py, px] - T) < 1e-12


def test_f32_and_f64_oracles_agree(oracle32, oracle64):
    sc = synth.plain_scene(n=1500, seed=24, width=64, height=64)
    r32 = oracle32.render(sc, sc.cameras[0], oracle.ALL)
    r64 = oracle64.render(sc, sc.cameras[0], oracle.ALL)
    assert np.array_equal(r32["binned"].val, r64["binned"].val)
    ok = (r32["near"] == 0)
    assert np.abs(r32["image"] - r64["image"]).max(axis=0)[ok].max() < 1e-5


# ---------------------------------------------------------------------------
# adjoint vs central finite differences (FP64)
# ---------------------------------------------------------------------------

def _fd_check(O, sc, cam, params, rng, n_coords, mode=oracle.ALL, grad_level=-1):
    H, W = cam.height, cam.width
    dL = rng.normal(size=(3, H, W))
    fwd, g2, grads = O.render_grad(sc, cam, mode, dL, grad_level=grad_level)
    base_sig = (fwd["n_contrib"].copy(), fwd["n_blend"].copy(), fwd["proj"].tiles.copy(), fwd["proj"].rect.copy())

    def loss_and_sig():
        r = O.render(sc, cam, mode)
        return float(np.sum(dL * r["image"])), (r["n_contrib"], r["n_blend"], r["proj"].tiles, r["proj"].rect)

    report = {}
    for name in params:
        for l, lv in enumerate(sc.levels):
            arr = getattr(lv, name)
            flat = arr.reshape(-1)
            idx = rng.choice(flat.size, size=min(n_coords, flat.size), replace=False)
            fd, an = [], []
            skipped = 0
            for j in idx:
                th = flat[j]
                h = 1e-6 * max(1.0, abs(th))
                flat[j] = th + h
                lp, sp = loss_and_sig()
                flat[j] = th - h
                lm, sm = loss_and_sig()
                flat[j] = th
                if not all(np.array_equal(x, y) for x, y in zip(sp, base_sig)) or \
                        not all(np.array_equal(x, y) for x, y in zip(sm, base_sig)):
                    skipped += 1
                    continue
                fd.append((lp - lm) / (2 * h))
                an.append(grads[l][name].reshape(-1)[j])
            fd, an = np.asarray(fd), np.asarray(an)
            report[(name, l)] = (fd, an, skipped)
    return report


@pytest.mark.parametrize("var", [0.0, 0.003])
def test_adjoint_matches_central_differences(oracle64, var):
    sc = synth.check_scene(n=64, width=32, height=32, filter3d_var=var)
    lv = sc.levels[0]
    for f in ("mean", "scale", "quat", "opacity", "sh"):
        setattr(lv, f, getattr(lv, f).astype(np.float64))
    cam = sc.cameras[0]
    rng = np.random.default_rng(17)
    rep = _fd_check(oracle64, sc, cam, ["mean", "scale", "quat", "opacity", "sh"], rng, n_coords=60)
    for key, (fd, an, skipped) in rep.items():
        assert len(fd) >= 20, (key, skipped)
        nrm = np.linalg.norm(fd)
        assert nrm > 0, key
        rel = np.linalg.norm(fd - an) / nrm
        assert rel <= 1e-3, (key, rel)
        assert np.all(np.abs(fd - an) <= 1e-3 * (np.abs(fd) + np.sqrt(np.mean(fd ** 2)))), key


def test_adjoint_level_mask(oracle64):
    """grad_level restricts the update to one level's Gaussians."""
    sc = synth.lod_city_scene(counts=(800, 200), half_xy=6.0, d=(3.0,), grid=1, spacing=1.0, chunk_z=1.0,
                              band=0.0, seed=31)
    for lv in sc.levels:
        for f in ("mean", "scale", "quat", "opacity", "sh"):
            setattr(lv, f, getattr(lv, f).astype(np.float64))
    cam = synth.look_at((0.0, -8.0, 1.5), (0.0, 0.0, 0.0), (0, 0, 1), 48, 32)
    dL = np.random.default_rng(2).normal(size=(3, 32, 48))
    _, _, g_all = oracle64.render_grad(sc, cam, oracle.LOD_CAMERA, dL)
    _, _, g_1 = oracle64.render_grad(sc, cam, oracle.LOD_CAMERA, dL, grad_level=1)
    assert np.all(g_1[0]["mean"] == 0) and np.abs(g_all[0]["mean"]).max() > 0
    assert np.array_equal(g_1[1]["mean"], g_all[1]["mean"])


def test_sh_colour_uses_direction_from_camera_to_gaussian(oracle64):
    """Colour is evaluated in the unit direction from the camera centre to the
    mean: a Gaussian straight ahead (+z) with only the z-linear band set shows
    0.5 + c1 k, one seen from behind (camera on the other side) 0.5 - c1 k."""
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    k = 0.25
    sh = np.zeros((16, 3, 1)); sh[2, :, 0] = k
    lv = make_level([[0.0, 0.0, 5.0]], 0.1, sh=sh)
    p = oracle64.render(one_level_scene(lv), axis_camera(), oracle.ALL)["proj"]
    assert np.allclose(p.rgb[0], 0.5 + c1 * float(np.float32(k)), atol=1e-12)
    cam_back = synth.look_at((0.0, 0.0, 10.0), (0.0, 0.0, 0.0), (0, -1, 0), 64, 64)
    p2 = oracle64.render(one_level_scene(lv), cam_back, oracle.ALL)["proj"]
    assert np.allclose(p2.rgb[0], 0.5 - c1 * float(np.float32(k)), atol=1e-6)


def test_chunked_selection_is_union_of_stored_chunk_sets(oracle32):
    """Per-chunk storage (Sec. 3 "chunk-based rendering"): the set chunk k keeps
    is the selection about its centre alone; a frame's chunked selection is the
    union of the two nearest chunks' sets, weighted 1 / t / 1 - t by membership
    (Eq. 4).  Checked for several camera positions on a 4 x 4 chunk grid."""
    sc = synth.lod_city_scene(counts=(20000, 5000, 1250), half_xy=40.0, d=(6.0, 18.0), grid=4, spacing=20.0,
                              chunk_z=1.7, band=5.0, seed=21)
    K = len(sc.chunks.centers)
    stored = []
    for k in range(K):
        only_k = Scene(levels=sc.levels, d=sc.d,
                       chunks=Chunks(centers=sc.chunks.centers[k:k + 1], offsets=sc.chunks.offsets[k:k + 1]))
        ids_k, w_k, (f1, o1, t1) = oracle32.select(only_k, oracle.CHUNKED, np.zeros(3, np.float32))
        assert (f1, o1, t1) == (0, -1, 1.0) and np.all(w_k == 1.0)
        stored.append(set(ids_k.tolist()))
    rng = np.random.default_rng(22)
    for _ in range(6):
        pos = np.array([rng.uniform(-40, 40), rng.uniform(-40, 40), 1.7], np.float32)
        ids, w, (f, o, t) = oracle32.select(sc, oracle.CHUNKED, pos)
        union = sorted(stored[f] | stored[o])
        assert ids.tolist() == union
        t32 = np.float32(t)
        expect = [1.0 if (g in stored[f] and g in stored[o]) else (t32 if g in stored[f] else np.float32(1) - t32)
                  for g in union]
        assert np.array_equal(w, np.asarray(expect, np.float32))


# ---------------------------------------------------------------------------
# the threshold-flip acceptance rule of the image comparison
# ---------------------------------------------------------------------------

def _bisect_flip(decides, lo, hi, iters=80):
    """Largest / smallest float32 opacity on either side of the oracle's own
    decision boundary: decides(lo) is False, decides(hi) is True."""
    lo, hi = float(np.float32(lo)), float(np.float32(hi))
    assert not decides(lo) and decides(hi)
    for _ in range(iters):
        mid = float(np.float32(0.5 * (lo + hi)))
        if mid in (lo, hi):
            break
        if decides(mid):
            hi = mid
        else:
            lo = mid
    return lo, hi


def _accept(O, r, cam, x, y, probe, tol=1e-4):
    return O.pixel_accept(r["proj"], r["binned"], cam, x, y, np.asarray(probe, np.float64), tol)


def _iso_alpha(o, sigma, z, f, dx, dy, s2d=0.3):
    """alpha of an isotropic on-axis Gaussian at pixel offset (dx, dy), float64 closed form."""
    a = (f * float(np.float32(sigma)) / z) ** 2 + s2d
    return min(0.99, float(np.float32(o)) * math.exp(-0.5 * (dx * dx + dy * dy) / a))


def test_pixel_accept_alpha_threshold_flip(oracle32):
    """One Gaussian whose alpha at a pixel is within a few ulp of 1/255 (its
    opacity bisected onto the oracle's own decision boundary): the rule
    accepts the colour with the splat blended and the colour with it skipped,
    and rejects either one moved by 2e-4."""
    W = H = 64
    f, z, sigma, k = 80.0, 5.0, 0.3, 0.7
    cam = axis_camera(W, H, f)
    px, py = 36, 32

    def frame(o):
        lv = make_level([[0.0, 0.0, z]], sigma, opac=[o], dc=k)
        return oracle32.render(one_level_scene(lv), cam, oracle.ALL, compensate=False)

    lo, hi = _bisect_flip(lambda o: frame(o)["n_contrib"][py, px] > 0, 1e-3, 1.0)
    rgb = C0 * float(np.float32(k)) + 0.5
    dx, dy = 32.0 - (px + 0.5), 32.0 - (py + 0.5)
    for o in (lo, hi):
        r = frame(o)
        assert r["near"][py, px] == 1, "the boundary pixel must carry a near-threshold decision"
        a = _iso_alpha(o, sigma, z, f, dx, dy)
        assert abs(a - 1.0 / 255.0) < 1e-6
        blended, skipped = np.full(3, rgb * a), np.zeros(3)
        for probe in (blended, skipped):
            assert _accept(oracle32, r, cam, px, py, probe)
            assert not _accept(oracle32, r, cam, px, py, probe + 2e-4)
            assert not _accept(oracle32, r, cam, px, py, probe - 2e-4)
        # half-way between the two outcomes is neither
        assert not _accept(oracle32, r, cam, px, py, 0.5 * (blended + skipped))


def test_pixel_accept_stop_threshold_flip(oracle32):
    """Three wide layers on the axis (alpha 0.99 clamped, 0.9, ~0.9): the
    third's opacity is bisected onto the oracle's T (1 - alpha) < 1e-4 stop
    boundary.  The rule accepts the colour with the third layer blended and
    the colour with the pixel stopped before it, rejects either moved by
    2e-4, and rejects the colour without the second layer (a decision far
    from every threshold: flipping it is not a legitimate difference)."""
    W = H = 64
    f, sigma = 80.0, 0.6
    cam = axis_camera(W, H, f)
    px, py = 32, 32
    dx = dy = 32.0 - 32.5
    zs = (5.0, 6.0, 7.0)
    cols = (0.2, 0.5, 0.9)
    dcs = [(c - 0.5) / C0 for c in cols]
    a_of = lambda z: (f * float(np.float32(sigma)) / z) ** 2 + 0.3
    G = [math.exp(-0.5 * (dx * dx + dy * dy) / a_of(z)) for z in zs]
    o2 = float(np.float32(0.9 / G[1]))

    def frame(o3):
        # storage order back to front: the sort, not the storage, orders them
        lv = make_level([[0.0, 0.0, zs[2]], [0.0, 0.0, zs[1]], [0.0, 0.0, zs[0]]], sigma, opac=[o3, o2, 1.0],
                        dc=[[dcs[2]] * 3, [dcs[1]] * 3, [dcs[0]] * 3])
        return oracle32.render(one_level_scene(lv), cam, oracle.ALL, compensate=False)

    def stops(o3):
        r = frame(o3)
        assert r["n_contrib"][py, px] >= 2
        return r["n_contrib"][py, px] == 2

    lo, hi = _bisect_flip(stops, 0.5, 0.99)
    c = [float(np.float32(d)) * C0 + 0.5 for d in dcs]
    a1 = 0.99
    a2 = _iso_alpha(o2, sigma, zs[1], f, dx, dy)
    T1 = 1.0 - a1
    T2 = T1 * (1.0 - a2)
    for o3 in (lo, hi):
        r = frame(o3)
        assert r["near"][py, px] == 1
        a3 = _iso_alpha(o3, sigma, zs[2], f, dx, dy)
        assert abs(T2 * (1.0 - a3) - 1e-4) < 1e-8
        stopped = np.full(3, c[0] * a1 + c[1] * a2 * T1)
        blended = stopped + c[2] * a3 * T2
        assert float(blended[0] - stopped[0]) > 5e-4
        for probe in (blended, stopped):
            assert _accept(oracle32, r, cam, px, py, probe)
            assert not _accept(oracle32, r, cam, px, py, probe + 2e-4)
            assert not _accept(oracle32, r, cam, px, py, probe - 2e-4)
        without_second = np.full(3, c[0] * a1 + c[2] * a3 * T1)
        assert not _accept(oracle32, r, cam, px, py, without_second)


def test_pixel_accept_rejects_off_values_without_near_decisions(oracle32):
    """Pixels of a random scene with no near-threshold decision: a probe
    within tol of the oracle's value is accepted, one off by more than tol
    in any channel is rejected."""
    sc = synth.plain_scene(n=1500, seed=25, width=64, height=48)
    cam = sc.cameras[0]
    r = oracle32.render(sc, cam, oracle.ALL)
    img = r["image"].astype(np.float64)
    cand = np.argwhere((r["near"] == 0) & (r["n_contrib"] > 0))
    assert len(cand) > 100
    rng = np.random.default_rng(3)
    for y, x in cand[rng.choice(len(cand), 40, replace=False)]:
        v = img[:, y, x]
        assert _accept(oracle32, r, cam, int(x), int(y), v + 0.5e-4)
        for ch in range(3):
            for s in (1.5e-4, -1.5e-4, 3e-3):
                p = v.copy()
                p[ch] += s
                assert not _accept(oracle32, r, cam, int(x), int(y), p), (x, y, ch, s)


# ---------------------------------------------------------------------------
# the Jacobian clamp of the EWA projection (off-screen means)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("axis", ["x", "y"])
def test_jacobian_clamp_closed_form(oracle64, oracle32, axis):
    """An isotropic Gaussian whose mean sits at twice the clamp limit
    (|x/z| = 2 lim): the Jacobian is evaluated at the limit, J02 = -f lim / z
    (not -f x / z^2), so Sigma' = v [[(f/z)^2 + (f lim / z)^2, 0], [0, (f/z)^2]]
    + s2d I.  The projected centre itself is not clamped.  Conic, radius,
    tile rectangle and the alpha at a pixel of the visible edge follow."""
    W = H = 64
    f, z, sigma, o = 80.0, 5.0, 1.4, 0.9
    cam = axis_camera(W, H, f)
    lim = 1.3 * 32.0 / f          # as the camera carries it
    X = 2.0 * lim * z
    pos = [X, 0.0, z] if axis == "x" else [0.0, X, z]
    lv = make_level([pos], sigma, opac=[o], dc=0.3)
    X32, z32 = float(np.float32(X)), float(np.float32(z))
    v = float(np.float32(sigma)) ** 2
    big = v * ((f / z32) ** 2 + (f * lim / z32) ** 2) + 0.3
    small = v * (f / z32) ** 2 + 0.3
    a, c = (big, small) if axis == "x" else (small, big)
    uc = f * X32 / z32 + 32.0
    u, vv = (uc, 32.0) if axis == "x" else (32.0, uc)
    r = math.ceil(3.0 * math.sqrt(max(a, c)))
    x0, x1 = max(0, math.floor((u - r) / 16)), min(4, math.floor((u + r) / 16) + 1)
    y0, y1 = max(0, math.floor((vv - r) / 16)), min(4, math.floor((vv + r) / 16) + 1)
    assert x0 < x1 and y0 < y1, "the clamped Gaussian reaches the image"
    # the unclamped form would be wider along the clamped axis
    assert v * ((f / z32) ** 2 + (f * X32 / z32 ** 2) ** 2) + 0.3 > 1.5 * max(a, c)
    for O, tol in ((oracle64, 1e-12), (oracle32, 3e-6)):
        res = O.render(one_level_scene(lv), cam, oracle.ALL, compensate=False)
        p = res["proj"]
        assert p.radius[0] == r
        assert tuple(p.rect[0]) == (x0, y0, x1, y1)
        assert abs(p.uv[0, 0] - u) <= 1e-4 and abs(p.uv[0, 1] - vv) <= 1e-4
        assert np.allclose(p.conic[0], [1 / a, 0.0, 1 / c], rtol=tol * 10, atol=tol)
        # a pixel on the image edge nearest the centre
        px, py = (63, 32) if axis == "x" else (32, 63)
        dx, dy = u - (px + 0.5), vv - (py + 0.5)
        al = float(np.float32(o)) * math.exp(-0.5 * (dx * dx / a + dy * dy / c))
        assert al > 1 / 255
        rgb = C0 * float(np.float32(0.3)) + 0.5
        assert abs(res["image"][0, py, px] - rgb * al) <= 10 * tol


def test_jacobian_clamp_adjoint_matches_central_differences(oracle64):
    """Central differences of the FP64 forward on two clamped Gaussians (one
    past the x limit, one past the y limit) and one unclamped: the adjoint's
    clamped branches (the clamped Jacobian entry depends on depth only)."""
    W = H = 64
    f = 80.0
    cam = axis_camera(W, H, f)
    lim = 1.3 * 32.0 / f
    rng = np.random.default_rng(41)
    means = [[2.0 * lim * 5.0, 0.3, 5.0], [-0.2, -2.2 * lim * 5.5, 5.5], [0.4, 0.2, 6.0]]
    q = rng.normal(size=(3, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    lv = make_level(means, [[1.5, 1.2, 1.3], [1.4, 1.6, 1.2], [0.3, 0.2, 0.25]], quats=q, opac=[0.8, 0.7, 0.6],
                    dc=[[0.4, 0.6, 0.2], [0.1, 0.3, 0.8], [0.5, 0.5, 0.5]], var=0.002)
    for fld in ("mean", "scale", "quat", "opacity", "sh"):
        setattr(lv, fld, getattr(lv, fld).astype(np.float64))
    sc = one_level_scene(lv)
    r = oracle64.render(sc, cam, oracle.ALL)
    assert np.all(r["proj"].tiles > 0)
    rep = _fd_check(oracle64, sc, cam, ["mean", "scale", "quat", "opacity"], rng, n_coords=12)
    for key, (fd, an, skipped) in rep.items():
        assert len(fd) >= min(6, getattr(lv, key[0]).size), (key, skipped)
        nrm = np.linalg.norm(fd)
        assert nrm > 0, key
        rel = np.linalg.norm(fd - an) / nrm
        assert rel <= 1e-3, (key, rel)
        assert np.all(np.abs(fd - an) <= 1e-3 * (np.abs(fd) + np.sqrt(np.mean(fd ** 2)))), key


# ---------------------------------------------------------------------------
# importance scores and per-chunk visibility filtering
# (Sec. 3 "Preliminaries: Importance pruning", "Visibility filtering")
# ---------------------------------------------------------------------------

def _importance(O, sc, cam, compensate=False):
    ids, w, _ = O.select(sc, oracle.ALL, cam.pos)
    return O.view_importance(sc, ids, w, cam, compensate=compensate)


@pytest.mark.parametrize("o", [0.7, 1.0])
def test_importance_lone_gaussian_at_a_pixel_centre(oracle64, oracle32, o):
    """One Gaussian whose mean projects exactly onto a pixel centre: nothing
    lies in front of it, so its weight there is its alpha at G = 1, i.e.
    min(0.99, o), and no pixel gives more."""
    cam = axis_camera(32, 32, 40.0)
    # u = f X / z + c = 40 * 0.0625 / 5 + 16 = 16.5, a pixel centre (exact in binary)
    lv = make_level([[0.0625, 0.0625, 5.0]], 0.05, opac=[o])
    for O in (oracle64, oracle32):
        score, amb = _importance(O, one_level_scene(lv), cam)
        assert score[0] == O.dt(min(0.99, float(np.float32(o)))), (O.tag, score)
        # power = 0 exactly at the centre pixel sits on the skip test (power > 0):
        # a near decision, so this Gaussian's weight is marked as open to rounding
        assert amb[0] == 1


def test_importance_single_pixel_stack_with_termination(oracle64):
    """A 1 x 1 view of wide Gaussians centred on the optical axis (G = 1 at
    the only pixel), stored back to front: the k-th nearest weighs
    alpha_k prod_{j<k} (1 - alpha_j); the one that would take T below 1e-4
    stops the pixel and, like every Gaussian behind it, weighs nothing."""
    cam = axis_camera(1, 1, 2.0)
    zs = [3.0, 4.0, 5.0, 6.0, 7.0]
    ops = [0.95, 0.6, 0.95, 0.95, 0.5]
    lv = make_level([[0.0, 0.0, z] for z in zs[::-1]], 0.5, opac=ops[::-1])
    score, amb = _importance(oracle64, one_level_scene(lv), cam)
    score = score[::-1]                       # nearest first
    a = [float(np.float32(x)) for x in ops]
    T, expect = 1.0, []
    for k in range(len(zs)):
        if T * (1 - a[k]) < 1e-4 or (expect and expect[-1] == 0.0):
            expect.append(0.0)
            continue
        expect.append(a[k] * T)
        T *= 1 - a[k]
    # 0.95, 0.6*0.05, 0.95*0.02, then T = 0.001 * 0.05 < 1e-4 stops at the fourth
    assert expect[3] == 0.0 and expect[4] == 0.0 and expect[2] > 0
    assert np.allclose(score, expect, rtol=0, atol=1e-12), (score, expect)
    # the first entry's power is exactly 0 (a near decision at list position 0): all are marked
    assert amb.all()


def test_importance_of_a_gaussian_behind_an_opaque_one(oracle64):
    """A wide front Gaussian of opacity 1 clamps to alpha 0.99 over the whole
    footprint of a small one behind it: the back one weighs 0.01 times its
    own alpha at its centre pixel, the front one 0.99."""
    cam = axis_camera(16, 16, 40.0)
    front = [0.0, 0.0, 3.0]
    back = [0.125, 0.125, 10.0]   # u = 40 * 0.125 / 10 + 8 = 8.5: a pixel centre
    lv = make_level([back, front], [[0.03] * 3, [5.0] * 3], opac=[0.8, 1.0])
    score, _ = _importance(oracle64, one_level_scene(lv), cam)
    assert score[1] == 0.99
    assert abs(score[0] - 0.01 * float(np.float32(0.8))) < 1e-9, score
    # and with the front one removed the back one weighs its full alpha
    lv1 = make_level([back], [0.03], opac=[0.8])
    s1, _ = _importance(oracle64, one_level_scene(lv1), cam)
    assert abs(s1[0] - float(np.float32(0.8))) < 1e-12


def test_importance_invariant_to_storage_order_and_bounded(oracle32):
    sc = synth.plain_scene(n=1500, seed=25, width=64, height=48)
    cam = sc.cameras[0]
    score, amb = _importance(oracle32, sc, cam, compensate=True)
    perm = np.random.default_rng(26).permutation(sc.n_total)
    lv = sc.levels[0]
    pl = Level(mean=lv.mean[:, perm].copy(), scale=lv.scale[:, perm].copy(), quat=lv.quat[:, perm].copy(),
               opacity=lv.opacity[perm].copy(), sh=lv.sh[:, :, perm].copy(), sh_degree=lv.sh_degree,
               filter3d_var=lv.filter3d_var)
    sp, ap = _importance(oracle32, one_level_scene(pl), cam, compensate=True)
    assert np.array_equal(sp, score[perm]) and np.array_equal(ap, amb[perm])
    # a weight is alpha T <= alpha <= min(0.99, o); most Gaussians of this view are seen
    assert np.all(score <= np.minimum(0.99, lv.opacity) + 1e-7)
    assert (score > 0).mean() > 0.3
    # max over views: scores of two views accumulate to their elementwise maximum
    cam2 = synth.look_at((3.0, -2.0, -14.0), (0, 0, 0), (0, -1, 0), 64, 48)
    s2, _ = _importance(oracle32, sc, cam2, compensate=True)
    ids, w, _ = oracle32.select(sc, oracle.ALL, cam.pos)
    acc = score.copy()
    oracle32.view_importance(sc, ids, w, cam2, score=acc)
    assert np.array_equal(acc, np.maximum(score, s2))


def test_single_chunk_set_and_union_of_stored_sets(oracle32):
    """A chunk's stored set (Eq. 2 at its centre with offset thresholds) and
    the two-chunk selection rebuilt from stored sets (Eq. 4 weights) equal the
    per-frame chunked selection bit for bit."""
    sc = synth.lod_city_scene(counts=(20000, 5000, 1250), half_xy=40.0, d=(6.0, 18.0), grid=4, spacing=20.0,
                              chunk_z=1.7, band=5.0, seed=21)
    K = len(sc.chunks.centers)
    sets = [oracle32.select_chunk(sc, k) for k in range(K)]
    for k in (0, 5, K - 1):
        only_k = Scene(levels=sc.levels, d=sc.d,
                       chunks=Chunks(centers=sc.chunks.centers[k:k + 1], offsets=sc.chunks.offsets[k:k + 1]))
        ids_k, w_k, _ = oracle32.select(only_k, oracle.CHUNKED, np.zeros(3, np.float32))
        assert np.array_equal(sets[k][0], ids_k) and np.all(sets[k][1] == 1.0)
    rng = np.random.default_rng(27)
    for _ in range(6):
        pos = np.array([rng.uniform(-40, 40), rng.uniform(-40, 40), 1.7], np.float32)
        ids, w, (f, o, t) = oracle32.select(sc, oracle.CHUNKED, pos)
        uid, uw = oracle.union_select(sc.n_total, sets[f][0], sets[o][0], t)
        assert np.array_equal(uid, ids) and np.array_equal(uw, w)
    with pytest.raises(ValueError):
        oracle32.select_chunk(sc, K)


def test_pruned_chunk_sets(oracle32):
    """Visibility filtering removes exactly the members scoring below the
    threshold; the union of pruned sets keeps Eq. 4's weights by membership
    of the pruned sets."""
    ids = np.array([2, 3, 5, 8, 13], np.uint32)
    score = np.zeros(16, np.float32)
    score[[2, 5, 13]] = [0.5, 0.02, 0.019999]
    assert oracle.prune_chunk_set(ids, score, 0.02).tolist() == [2, 5]
    uid, uw = oracle.union_select(16, [2, 5], [5, 7], 0.75)
    assert uid.tolist() == [2, 5, 7]
    assert uw.tolist() == [np.float32(0.75), 1.0, np.float32(1.0) - np.float32(0.75)]


# ---------------------------------------------------------------------------
# depth-threshold selection (Sec. 3 "Selecting depth thresholds")
# ---------------------------------------------------------------------------

def _small_city():
    return synth.lod_city_scene(counts=(20000, 5000, 1250), half_xy=40.0, d=(6.0, 18.0), grid=2, spacing=20.0,
                                chunk_z=1.7, band=5.0, seed=41)


def test_lod_instances_sum_per_gaussian_tiles_over_distance_bands(oracle32):
    """The instance count of an LOD frame is the sum, over levels, of the tile
    counts of the Gaussians whose camera distance falls in that level's band
    [d_l, d_{l+1}): each level is projected whole once and banded by float64
    distances (an independent route to the same number)."""
    sc = _small_city()
    cams = synth.threshold_views(3, half_xy=40.0, width=160, height=96, seed=42)
    for cam in cams:
        per_level = []
        for lv in sc.levels:
            one = one_level_scene(lv)
            ids, w, _ = oracle32.select(one, oracle.ALL, cam.pos)
            p = oracle32.project(one, ids, w, cam)
            dist = np.linalg.norm(lv.mean.T.astype(np.float64) - np.asarray(cam.pos, np.float64), axis=1)
            per_level.append((p.tiles.astype(np.int64), dist))
        for d in ((5.0, 12.0), (3.0, 30.0), (10.0, 11.0)):
            bounds = [0.0, *d, np.inf]
            expect = sum(int(t[(dist >= bounds[l]) & (dist < bounds[l + 1])].sum())
                         for l, (t, dist) in enumerate(per_level))
            assert oracle.lod_instances(oracle32, sc, d, 3, cam) == expect, d
        # limits: every Gaussian nearer than d_1 -> level 0 alone; none nearer -> level 1 alone
        assert oracle.lod_instances(oracle32, sc, (1e6,), 2, cam) == int(per_level[0][0].sum())
        assert oracle.lod_instances(oracle32, sc, (1e-3,), 2, cam) == int(per_level[1][0][per_level[1][1] >= 1e-3].sum())


def test_greedy_threshold_search_on_known_costs():
    """The greedy search finds d_1 from the two-level cost, then d_2 above it
    from the three-level cost; ties go to the smaller candidate."""
    cands = [5.0 * k for k in range(1, 21)]

    def separable(d):
        return (d[0] - 30.0) ** 2 + (0.0 if len(d) < 2 else (d[1] - 70.0) ** 2)
    chosen, curves = oracle.greedy_thresholds(separable, cands, 3)
    assert chosen == [30.0, 70.0]
    assert [c for c, _ in curves[1]] == [c for c in cands if c > 30.0]

    # the second step only looks above the first threshold, even when lower would be cheaper
    def below(d):
        return abs(d[0] - 50.0) if len(d) == 1 else abs(d[1] - 10.0)
    chosen, _ = oracle.greedy_thresholds(below, cands, 3)
    assert chosen == [50.0, 55.0]

    def flat(d):
        return 1.0
    assert oracle.greedy_thresholds(flat, cands, 4)[0] == [5.0, 10.0, 15.0]
    with pytest.raises(ValueError):
        oracle.greedy_thresholds(flat, [5.0], 3)


def test_threshold_cost_is_mean_gaussians_per_tile(oracle32):
    sc = _small_city()
    cams = synth.threshold_views(2, half_xy=40.0, width=100, height=50, seed=43)   # 7 x 4 tiles, ragged
    c = oracle.threshold_cost(oracle32, sc, (6.0, 18.0), 3, cams)
    m = [oracle.lod_instances(oracle32, sc, (6.0, 18.0), 3, cam) for cam in cams]
    assert c == pytest.approx(np.mean(m) / 28.0, rel=0, abs=1e-12)


# ---------------------------------------------------------------------------
# LOD-level construction (supplementary "LOD structure optimization steps")
# ---------------------------------------------------------------------------

def test_adam_update_matches_torch_optimizer():
    """Kingma and Ba's Adam, checked against torch.optim.Adam in float64 over
    several steps with varying gradients (including zeros and sign changes)."""
    import torch
    rng = np.random.default_rng(51)
    p0 = rng.normal(size=40)
    grads = [rng.normal(size=40) * 10.0 ** rng.uniform(-6, 1, 40) for _ in range(6)]
    grads[2][:5] = 0.0
    p, m, v = p0.copy(), np.zeros(40), np.zeros(40)
    tp = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=2e-3, betas=(0.9, 0.999), eps=1e-15)
    for t, g in enumerate(grads, start=1):
        p, m, v = oracle.adam_update(p, g, m, v, 2e-3, t)
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        assert np.allclose(p, tp.detach().numpy(), rtol=0, atol=1e-14), t
    # the first step moves every coordinate with a non-zero gradient by lr against its sign
    p1, _, _ = oracle.adam_update(p0, grads[0], np.zeros(40), np.zeros(40), 2e-3, 1)
    assert np.allclose(p1 - p0, -2e-3 * np.sign(grads[0]), rtol=1e-5, atol=0)


def test_l1_loss_gradient_matches_torch_autograd():
    import torch
    rng = np.random.default_rng(52)
    img, tgt = rng.random((3, 8, 10)), rng.random((3, 8, 10))
    img[0, 0, :3] = tgt[0, 0, :3]     # equal values: gradient 0
    loss, g = oracle.l1_loss_grad(img, tgt)
    ti = torch.tensor(img, requires_grad=True)
    tl = torch.nn.functional.l1_loss(ti, torch.tensor(tgt))
    tl.backward()
    assert loss == pytest.approx(float(tl.detach()), rel=1e-15)
    assert np.array_equal(g, ti.grad.numpy())


def test_activation_adjoint_by_central_differences():
    rng = np.random.default_rng(53)
    raw = {"mean": rng.normal(size=(3, 5)), "log_scale": rng.normal(-2, 0.3, (3, 5)),
           "quat_raw": rng.normal(size=(4, 5)), "opacity_logit": rng.normal(size=5), "sh": rng.normal(size=(48, 5))}
    w = {k: rng.normal(size=np.shape(v)) for k, v in oracle.activate(raw).items()}

    def f(r):
        a = oracle.activate(r)
        return sum(float(np.sum(w[k] * a[k])) for k in a)
    g = oracle.activate_adjoint(raw, {"mean": w["mean"], "scale": w["scale"], "quat": w["quat"],
                                      "opacity": w["opacity"], "sh": w["sh"]})
    for k in oracle.RAW_KEYS:
        flat = raw[k].reshape(-1)
        for j in range(0, flat.size, 3):
            th = flat[j]
            flat[j] = th + 1e-6
            fp = f(raw)
            flat[j] = th - 1e-6
            fm = f(raw)
            flat[j] = th
            assert abs((fp - fm) / 2e-6 - g[k].reshape(-1)[j]) <= 1e-6 * max(1.0, abs(g[k].reshape(-1)[j])), (k, j)


def test_finetune_gradient_of_level_l_by_central_differences(oracle64):
    """The gradient of a fine-tuning step (levels 0..l rendered with Eq. 2
    about the camera, d_l scaled by the step's draw, 0.8 mean L1 + 0.2 D-SSIM) w.r.t.
    level l's raw parameters, against central differences of that loss; the
    scaled switch distance is the one the render uses."""
    base, cams, d, sched = synth.lod_build_workload(n=48, n_views=3, width=24, height=16, d=(5.0,), seed=62)
    base = {k: np.asarray(v, np.float64) for k, v in base.items()}
    lvl1 = {k: v.copy() for k, v in base.items()}
    rng = np.random.default_rng(54)
    lvl1["mean"] = lvl1["mean"] + rng.normal(0, 0.05, lvl1["mean"].shape)
    levels = [base, lvl1]
    degs, vars_ = [3, 3], [0.0, synth.filter_var(5.0)]
    cam = cams[0]
    tgt = synth.target_images(1, 24, 16, seed=63)[0].astype(np.float64)
    u = 0.83
    lam = 0.2
    loss, dL, g, _ = oracle.finetune_grad(oracle64, levels, degs, vars_, d, 1, cam, tgt, u, lam=lam)
    dd = [float(np.float32(np.float32(5.0) * np.float32(u)))]
    sc0 = oracle.lod_level_scene(levels, degs, vars_, dd)
    sel_ids, _, _ = oracle64.select(sc0, oracle.LOD_CAMERA, cam.pos)
    base_sig = None

    def loss_sig():
        sc = oracle.lod_level_scene(levels, degs, vars_, dd)
        r = oracle64.render(sc, cam, oracle.LOD_CAMERA)
        lv = (1 - lam) * oracle.l1_loss_grad(r["image"], tgt)[0] + lam * (1 - oracle.ssim_map(r["image"], tgt).mean())
        return lv, (r["n_contrib"], r["n_blend"], r["proj"].tiles, r["ids"], np.sign(r["image"] - tgt))
    l0, base_sig = loss_sig()
    assert l0 == pytest.approx(loss, rel=1e-14)
    assert np.any(sel_ids >= 48) and np.any(sel_ids < 48)   # both levels take part
    checked = 0
    for k in ("mean", "log_scale", "quat_raw", "opacity_logit", "sh"):
        flat = lvl1[k].reshape(-1)
        fd, an = [], []
        for j in rng.choice(flat.size, size=min(25, flat.size), replace=False):
            th = flat[j]
            h = 1e-6 * max(1.0, abs(th))
            flat[j] = th + h
            lp, sp = loss_sig()
            flat[j] = th - h
            lm, sm = loss_sig()
            flat[j] = th
            if any(not np.array_equal(a, b) for s in (sp, sm) for a, b in zip(s, base_sig)):
                continue
            fd.append((lp - lm) / (2 * h))
            an.append(g[k].reshape(-1)[j])
        fd, an = np.asarray(fd), np.asarray(an)
        assert len(fd) >= 8, k
        if np.linalg.norm(fd) > 0:
            assert np.linalg.norm(fd - an) <= 1e-3 * np.linalg.norm(fd), k
            checked += 1
    assert checked >= 4


def test_keep_indices_and_workload_draws():
    s = np.array([0.5, 0.01, 0.02, 0.0, 0.3], np.float32)
    assert oracle.keep_indices(s, 0.02).tolist() == [0, 2, 4]
    base, cams, d, sched = synth.lod_build_workload(d=(4.0, 9.0), steps_per_round=50)
    assert len(sched) == 2 and all(len(r) == 3 and len(r[0]) == 50 for r in sched)
    us = np.array([u for lv in sched for r in lv for _, u in r])
    assert us.min() >= 0.7 and us.max() < 1.3 and abs(us.mean() - 1.0) < 0.05


def test_ssim_identity_symmetry_and_constant_patches():
    """SSIM(x, x) = 1 everywhere; SSIM is symmetric; on constant images a, b the
    pixels at least 5 away from the border (where the window sees only the image)
    take the closed form (2ab + C1) / (a^2 + b^2 + C1)."""
    rng = np.random.default_rng(81)
    x = rng.random((3, 20, 24))
    y = rng.random((3, 20, 24))
    assert np.allclose(oracle.ssim_map(x, x), 1.0, atol=1e-12)
    assert np.allclose(oracle.ssim_map(x, y), oracle.ssim_map(y, x), atol=1e-14)
    a, b = 0.3, 0.7
    m = oracle.ssim_map(np.full((1, 16, 16), a), np.full((1, 16, 16), b))
    expect = (2 * a * b + 0.01 ** 2) / (a * a + b * b + 0.01 ** 2)
    assert np.allclose(m[0, 5:11, 5:11], expect, rtol=1e-12)
    assert oracle.ssim_window().sum() == pytest.approx(1.0, abs=1e-15)
    assert oracle.ssim_window()[5] == oracle.ssim_window().max()


def test_dssim_gradient_by_central_differences():
    rng = np.random.default_rng(82)
    x = rng.random((3, 13, 17))
    y = rng.random((3, 13, 17))
    loss, g = oracle.dssim_grad(x, y)
    assert loss == pytest.approx(1.0 - oracle.ssim_map(x, y).mean(), abs=1e-14)
    for idx in [(0, 0, 0), (1, 6, 8), (2, 12, 16), (0, 3, 15), (1, 12, 0), (2, 7, 2)]:
        h = 1e-6
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = ((1 - oracle.ssim_map(xp, y).mean()) - (1 - oracle.ssim_map(xm, y).mean())) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-12), idx


def test_ssim_window_filter_by_brute_force_including_images_smaller_than_the_window():
    """The zero-padded window filter behind SSIM, against a direct double sum
    over the 11 x 11 window, on images narrower and lower than the window."""
    rng = np.random.default_rng(83)
    w = oracle.ssim_window()
    for H, W in ((3, 5), (13, 4), (12, 17)):
        img = rng.random((2, H, W))
        got = oracle._blur(img)
        ref = np.zeros_like(img)
        for c in range(2):
            for i in range(H):
                for j in range(W):
                    for a in range(11):
                        for b in range(11):
                            ii, jj = i + a - 5, j + b - 5
                            if 0 <= ii < H and 0 <= jj < W:
                                ref[c, i, j] += w[a] * w[b] * img[c, ii, jj]
        assert np.allclose(got, ref, rtol=0, atol=1e-14), (H, W)


def test_pixel_weights_sum_with_transmittance_to_one_and_bound_the_scores(oracle64, oracle32):
    """A pixel's blending weights and its final transmittance sum to 1 (the
    compositing identity); the importance score of every Gaussian is the
    largest of its weights over the pixels."""
    sc = synth.plain_scene(n=800, seed=27, width=40, height=24)
    cam = sc.cameras[0]
    for O, tol in ((oracle64, 1e-12), (oracle32, 2e-6)):
        r = O.render(sc, cam, oracle.ALL)
        best = np.zeros(sc.n_total)
        for y in range(cam.height):
            for x in range(cam.width):
                act, wt, pos, near = O.pixel_weights(r["proj"], r["binned"], cam, x, y)
                assert abs(float(np.sum(wt.astype(np.float64))) + float(r["final_T"][y, x]) - 1.0) <= tol
                assert np.all(np.diff(pos) > 0)
                np.maximum.at(best, r["ids"][act].astype(np.int64), wt.astype(np.float64))
        score, _ = O.view_importance(sc, r["ids"], r["w"], cam)
        assert np.array_equal(best.astype(O.dt), score)
