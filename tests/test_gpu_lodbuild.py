"""LOD-level construction on the GPU (supplementary "LOD structure
optimization steps") against the oracle:

* lodge_adam against the float64 Adam update from the same float32 state;
* lodge_l1_grad bit-exact (scale * sign), its loss within rounding;
* lodge_keep_indices / lodge_gather_planes bit-exact (ties at the threshold,
  ragged sizes, nothing and everything kept);
* fine-tuning steps one at a time from the GPU's own state: the level-l raw
  gradient against the float64 oracle gradient of the same step (levels 0..l,
  Eq. 2 about the camera, d_l scaled by the step's draw; relative error per
  tensor <= 1e-3), the Adam update against the oracle's, the other levels
  untouched;
* a pruning round: importance scores of the LOD render against the oracle's,
  the kept set and the compacted parameters and moments bit-exact."""
import numpy as np
import pytest

import oracle
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


def test_adam_kernel(L):
    import torch
    rng = np.random.default_rng(71)
    n = 10007
    p = rng.normal(size=n).astype(np.float32)
    g = (rng.normal(size=n) * 10.0 ** rng.uniform(-5, 1, n)).astype(np.float32)
    g[:7] = 0.0
    m = (rng.normal(size=n) * 1e-2).astype(np.float32)
    v = (rng.random(n) * 1e-3).astype(np.float32)
    tp, tg, tm, tv = (torch.from_numpy(x.copy()).cuda() for x in (p, g, m, v))
    L.lodge_adam(tp, tg, tm, tv, 5e-3, 3)
    torch.cuda.synchronize()
    p64, g64, m64, v64 = (x.astype(np.float64) for x in (p, g, m, v))
    # the hyperparameters as the kernel receives them (FP32: 1 - beta2 is 0.00099998713, not 0.001)
    b1, b2, lr = float(np.float32(0.9)), float(np.float32(0.999)), float(np.float32(5e-3))
    pe, me, ve = oracle.adam_update(p64, g64, m64, v64, lr, 3, beta1=b1, beta2=b2, eps=float(np.float32(1e-15)))
    mg, vg, pg = (t.cpu().numpy().astype(np.float64) for t in (tm, tv, tp))
    # the moments: FP32 rounding relative to the size of their two terms (they may cancel)
    assert np.all(np.abs(mg - me) <= 1e-6 * (b1 * np.abs(m64) + (1 - b1) * np.abs(g64)) + 1e-30)
    assert np.all(np.abs(vg - ve) <= 1e-6 * (b2 * v64 + (1 - b2) * g64 * g64) + 1e-30)
    # the step, from the kernel's own moments: rounding relative to |p| and the update
    upd = lr * (mg / (1 - b1 ** 3)) / (np.sqrt(vg / (1 - b2 ** 3)) + 1e-15)
    assert np.all(np.abs(pg - (p64 - upd)) <= 1e-6 * (np.abs(p64) + np.abs(upd)))
    # coordinates whose first moment does not cancel land on the float64 step
    ok = np.abs(me) > 1e-3 * (b1 * np.abs(m64) + (1 - b1) * np.abs(g64))
    assert np.all(np.abs(pg - pe)[ok] <= 1e-5 * (np.abs(p64) + 5e-3)[ok])
    with pytest.raises(L.LodgeError):
        L.lodge_adam(tp, tg, tm, tv, 5e-3, 0)


def test_l1_grad_kernel(L):
    import torch
    rng = np.random.default_rng(72)
    img = rng.random((3, 37, 53)).astype(np.float32)
    tgt = rng.random((3, 37, 53)).astype(np.float32)
    tgt[1, 3, :9] = img[1, 3, :9]
    ti, tt = torch.from_numpy(img).cuda(), torch.from_numpy(tgt).cuda()
    grad = torch.empty_like(ti)
    loss = torch.zeros(1, device="cuda")
    s = 1.0 / img.size
    L.lodge_l1_grad(ti, tt, grad, s, loss)
    torch.cuda.synchronize()
    l_o, g_o = oracle.l1_loss_grad(img, tgt)
    assert np.array_equal(grad.cpu().numpy(), (np.sign(img - tgt) * np.float32(s)).astype(np.float32))
    assert np.allclose(grad.cpu().numpy(), g_o, rtol=1e-6, atol=0)
    assert float(loss.item()) == pytest.approx(l_o, rel=1e-5)


@pytest.mark.parametrize("W,H", [(48, 32), (37, 23), (5, 3)])
def test_dssim_kernel(L, W, H):
    """lodge_dssim_grad against the oracle's SSIM map and adjoint: loss and gradient within FP32 rounding
    of the float64 definition, added onto what grad already holds."""
    import torch
    rng = np.random.default_rng(74 + W)
    x = rng.random((3, H, W)).astype(np.float32)
    y = rng.random((3, H, W)).astype(np.float32)
    base = (1e-3 * rng.normal(size=(3, H, W))).astype(np.float32)   # small: its FP32 rounding stays below 1e-10
    tx, ty = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    grad = torch.from_numpy(base.copy()).cuda()
    loss = torch.full((1,), 0.5, device="cuda")
    L.lodge_dssim_grad(tx, ty, grad, 0.2, loss)
    torch.cuda.synchronize()
    l_o, g_o = oracle.dssim_grad(x, y)
    assert float(loss.item()) == pytest.approx(0.5 + 0.2 * l_o, abs=2e-6)
    got = grad.cpu().numpy().astype(np.float64) - base
    ref = 0.2 * g_o
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max() + 1e-9, np.abs(got - ref).max()


@pytest.mark.parametrize("n", [0, 1, 4095, 4096, 4097, 100003])
def test_keep_and_gather(L, n):
    import torch
    rng = np.random.default_rng(73 + n)
    s = rng.choice(np.array([0.0, 0.01, 0.02, 0.03, 0.5], np.float32), size=n)
    P = 7
    planes = rng.normal(size=(P, n)).astype(np.float32)
    for thr in (0.02, 0.0, 1.0):
        ts = torch.from_numpy(s).cuda()
        idx = torch.full((max(1, n),), -1, dtype=torch.int32, device="cuda")
        cnt = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        L.lodge_keep_indices(ts, thr, idx, cnt)
        torch.cuda.synchronize()
        k_o = oracle.keep_indices(s, thr)
        m = int(cnt.item())
        assert m == len(k_o), (n, thr)
        assert np.array_equal(idx[:m].cpu().numpy().astype(np.uint32), k_o)
        out = torch.full((P, max(1, m)), np.nan, dtype=torch.float32, device="cuda")
        if n > 0:
            L.lodge_gather_planes(torch.from_numpy(planes).cuda(), idx, cnt, out)
            torch.cuda.synchronize()
            assert np.array_equal(out[:, :m].cpu().numpy(), planes[:, k_o])


def _builder(L, n=400, d=(4.0,), steps=4, seed=61):
    import torch
    from paper_2505_23158_amd import lodbuild as LB
    base_raw, cams, d, sched = synth.lod_build_workload(n=n, d=d, seed=seed, steps_per_round=steps)
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in base_raw.items()}
    base = LB.level_from_raw(t["mean"], t["log_scale"], t["quat_raw"], t["opacity_logit"], t["sh"], 3, 0.0)
    # training images: renders of G^(0) alone
    sc0 = L.Scene([base.scene_level()], [], None)
    R0 = L.Renderer(sc0, cams[0].width, cams[0].height)
    targets = torch.empty((len(cams), 3, cams[0].height, cams[0].width), device="cuda")
    for v, cam in enumerate(cams):
        R0.frame(cam, L.SELECT_ALL)
        targets[v].copy_(R0.image)
    B = LB.LodBuilder([base], d, cams, targets)
    return B, base_raw, cams, d, sched, targets.cpu().numpy()


def _raw_np(lv):
    r = lv.raw.detach().cpu().numpy().astype(np.float64)
    return {"mean": r[0:3], "log_scale": r[3:6], "quat_raw": r[6:10], "opacity_logit": r[10], "sh": r[11:]}


def test_finetune_steps_vs_oracle(L, oracle64):
    import torch
    from paper_2505_23158_amd import lodbuild as LB
    B, base_raw, cams, d, sched, targets = _builder(L)
    fv = [0.0, synth.filter_var(d[0])]
    B.levels.append(LB.copy_with_filter(B.levels[0], fv[1]))
    lv0_before = B.levels[0].raw.clone()
    for step, (view, u) in enumerate(sched[0][0] + sched[0][1]):
        pre = [_raw_np(lv) for lv in B.levels]
        m_pre = B.levels[1].m.cpu().numpy().astype(np.float64)
        v_pre = B.levels[1].v.cpu().numpy().astype(np.float64)
        graw = B.finetune_step(1, view, u).cpu().numpy().astype(np.float64)
        torch.cuda.synchronize()
        dL = B.dL.cpu().numpy().astype(np.float64)
        loss, dL_o, g_o, img = oracle.finetune_grad(oracle64, pre, [3, 3], fv, d, 1, cams[view], targets[view], u,
                                                    dL=dL, lam=B.lam)
        # the GPU's dL/dimage ((1 - lambda) sign / n + lambda D-SSIM gradient) is the oracle's wherever the
        # image is not within rounding of the target (where level 0 alone covers a pixel the GPU render
        # equals its target exactly, and the L1 sign is 0)
        _, dL_own, _, _ = oracle.finetune_grad(oracle64, pre, [3, 3], fv, d, 1, cams[view], targets[view], u,
                                               lam=B.lam)
        far = np.abs(img - targets[view]) > 1e-5
        dd = np.abs(dL - dL_own)[far]
        assert np.mean(dd > 1e-3 * np.abs(dL_own).max()) < 1e-3
        row = 0
        for k, p in (("mean", 3), ("log_scale", 3), ("quat_raw", 4), ("opacity_logit", 1), ("sh", 48)):
            ref = np.asarray(g_o[k], np.float64).reshape(p, -1)
            got = graw[row:row + p]
            nrm = np.linalg.norm(ref)
            rel = np.linalg.norm(got - ref) / nrm if nrm > 0 else np.abs(got).max()
            assert rel <= 1e-3, (step, k, rel)
            row += p
        # Adam from the GPU's state and gradient, group by group
        post = B.levels[1].raw.cpu().numpy().astype(np.float64)
        p_pre = np.concatenate([pre[1][k].reshape(-1, pre[1]["mean"].shape[1]) for k in oracle.RAW_KEYS])
        groups = [("mean", 0, 3), ("log_scale", 3, 3), ("quat_raw", 6, 4), ("opacity_logit", 10, 1),
                  ("sh_dc", 11, 3), ("sh_rest", 14, 45)]
        for gname, o, p in groups:
            pe, _, _ = oracle.adam_update(p_pre[o:o + p], graw[o:o + p], m_pre[o:o + p], v_pre[o:o + p],
                                          float(np.float32(LB.LRS[gname])), step + 1,
                                          beta1=float(np.float32(0.9)), beta2=float(np.float32(0.999)))
            assert np.abs(post[o:o + p] - pe).max() <= 1e-6, (step, gname)
        log(f"[lodbuild] step {step}: view {view}, d_1 x {u:.3f}, loss {loss:.5f}, grads and Adam match")
    assert torch.equal(B.levels[0].raw, lv0_before)


def test_pruning_round_vs_oracle(L, oracle32):
    import torch
    from paper_2505_23158_amd import lodbuild as LB
    B, base_raw, cams, d, sched, targets = _builder(L)
    fv = [0.0, synth.filter_var(d[0])]
    B.levels.append(LB.copy_with_filter(B.levels[0], fv[1]))
    for view, u in sched[0][0]:
        B.finetune_step(1, view, u)
    before = {k: v.clone() for k, v in (("raw", B.levels[1].raw), ("m", B.levels[1].m), ("v", B.levels[1].v))}
    # the FP32 planes the GPU renders from (activated on the GPU), before the pruning
    host = []
    for lv in B.levels:
        n = lv.n
        host.append(synth.Level(mean=lv.view("mean").cpu().numpy(), scale=lv.act["scale"].cpu().numpy(),
                                quat=lv.act["quat"].cpu().numpy(), opacity=lv.act["opacity"].cpu().numpy(),
                                sh=lv.view("sh").cpu().numpy().reshape(16, 3, n), sh_degree=3,
                                filter3d_var=lv.filter3d_var))
    # a threshold that keeps about 60% (the scores are deterministic: maxima taken with atomics)
    thr = float(np.float32(np.quantile(B.importance(1).cpu().numpy(), 0.4)))
    s_gpu = B.prune(1, thr).cpu().numpy()
    torch.cuda.synchronize()
    # the oracle's scores of level 1 over the training views (levels 0..1, nominal switch distance)
    sc32 = synth.Scene(levels=host, d=[float(np.float32(d[0]))], chunks=None)
    n0 = host[0].n
    score = np.zeros(sc32.n_total, np.float32)
    amb = np.zeros(sc32.n_total, np.uint8)
    for cam in cams:
        ids, w, _ = oracle32.select(sc32, oracle.LOD_CAMERA, cam.pos)
        oracle32.view_importance(sc32, ids, w, cam, score=score, amb=amb)
    s_o, a_o = score[n0:], amb[n0:]
    dd = np.abs(s_gpu.astype(np.float64) - s_o)
    assert np.all((dd <= 1e-4) | (a_o != 0)), dd.max()
    keep = oracle.keep_indices(s_gpu, np.float32(thr))
    assert B.levels[1].n == len(keep) and 0 < len(keep) < len(s_gpu)
    for name, buf in (("raw", B.levels[1].raw), ("m", B.levels[1].m), ("v", B.levels[1].v)):
        assert torch.equal(buf, before[name][:, torch.from_numpy(keep.astype(np.int64)).cuda()]), name
    log(f"[lodbuild] prune at {thr}: {len(s_gpu)} -> {len(keep)} Gaussians")


def test_build_levels_end_to_end(L):
    """Two coarser levels, three rounds of (prune, fine-tune) each: every
    round keeps a subset, the filter variance follows d_l, parameters stay
    finite, and the built hierarchy renders with LOD selection."""
    import torch
    from paper_2505_23158_amd import lodbuild as LB
    base_raw, cams, d, sched = synth.lod_build_workload(n=400, d=(4.0, 7.0), seed=64, steps_per_round=3)
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in base_raw.items()}
    base = LB.level_from_raw(t["mean"], t["log_scale"], t["quat_raw"], t["opacity_logit"], t["sh"], 3, 0.0)
    sc0 = L.Scene([base.scene_level()], [], None)
    R0 = L.Renderer(sc0, cams[0].width, cams[0].height)
    targets = torch.empty((len(cams), 3, cams[0].height, cams[0].width), device="cuda")
    for v, cam in enumerate(cams):
        R0.frame(cam, L.SELECT_ALL)
        targets[v].copy_(R0.image)
    fv = [synth.filter_var(x) for x in d]
    B = LB.build_levels(base, d, fv, cams, targets, gamma=0.05, schedule=sched, steps_per_round=3)
    assert len(B.levels) == 3
    for l in (1, 2):
        lv = B.levels[l]
        assert lv.filter3d_var == pytest.approx(fv[l - 1])
        assert 0 < lv.n <= base.n
        assert torch.isfinite(lv.raw).all()
    sc = B.scene(2, d)
    R = L.Renderer(sc, cams[0].width, cams[0].height)
    R.frame(cams[0], L.SELECT_LOD_CAMERA)
    torch.cuda.synchronize()
    assert L.lodge_check(R.ws)[0] == L.LODGE_OK
    assert torch.isfinite(R.image).all()
    log(f"[lodbuild] built levels of {[lv.n for lv in B.levels]} Gaussians")


def test_full_size_finetune_touches_only_rendered_level_l_gaussians(L):
    """The construction workload the benchmark times (1M-Gaussian G^(0), level 1
    at d_1 = 15 m, 1280x720): after a pruning round and two fine-tuning steps,
    level 0 is unchanged bit for bit, every parameter is finite, and a level-1
    Gaussian that neither step selected (nearer than that step's scaled d_1 to
    its camera) keeps its parameters and zero Adam moments exactly."""
    import torch
    from paper_2505_23158_amd import lodbuild as LB
    n, views, W, H, d = 1_000_000, 8, 1280, 720, (15.0,)
    sc = synth.diff_scene(n=n, n_views=views, width=W, height=H)
    lv = sc.levels[0]
    t = {"mean": lv.mean, "log_scale": lv.raw["log_scale"], "quat_raw": lv.raw["quat"],
         "opacity_logit": lv.raw["opacity_logit"], "sh": lv.sh.reshape(-1, n)}
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in t.items()}
    base = LB.level_from_raw(t["mean"], t["log_scale"], t["quat_raw"], t["opacity_logit"], t["sh"], 3, 0.0)
    sc0 = L.Scene([base.scene_level()], [], None)
    R0 = L.Renderer(sc0, W, H, max_active=n, max_instances=24_000_000)
    targets = torch.empty((views, 3, H, W), device="cuda")
    for v, cam in enumerate(sc.cameras):
        R0.frame(cam, L.SELECT_ALL)
        targets[v].copy_(R0.image)
    del R0, sc0
    B = LB.LodBuilder([base], d, sc.cameras, targets, max_active=2 * n, max_instances=48_000_000)
    B.levels.append(LB.copy_with_filter(base, synth.filter_var(d[0])))
    lv0 = base.raw.clone()
    B.prune(1, 0.2 * 0.02)
    before = B.levels[1].raw.clone()
    draws = [(2, 0.8), (5, 1.2)]
    for view, u in draws:
        B.finetune_step(1, view, u)
    torch.cuda.synchronize()
    assert L.lodge_check(B.R.ws)[0] == L.LODGE_OK
    assert torch.equal(B.levels[0].raw, lv0)
    raw = B.levels[1].raw
    assert torch.isfinite(raw).all()
    mean = before[0:3].cpu().numpy().astype(np.float64)
    never = np.ones(B.levels[1].n, bool)
    for view, u in draws:
        pos = np.asarray(sc.cameras[view].pos, np.float64)
        dd = float(np.float32(np.float32(d[0]) * np.float32(u)))
        never &= np.linalg.norm(mean.T - pos, axis=1) < dd * (1 - 1e-5)
    assert never.sum() > 0 and (~never).sum() > 0
    idx = torch.from_numpy(np.flatnonzero(never)).cuda()
    assert torch.equal(raw[:, idx], before[:, idx])
    assert not B.levels[1].m[:, idx].any() and not B.levels[1].v[:, idx].any()
    log(f"[lodbuild] full size: level 1 kept {B.levels[1].n} of {n}; {int(never.sum())} never selected, unchanged")


def test_finetuning_lowers_the_loss_of_a_pruned_level(L):
    """The construction loop optimises: a level pruned hard renders the training views worse than G^(0)
    does, and its fine-tuning steps (random view and d_l draw each, L1 + D-SSIM, adjoint of that level only,
    Adam) bring the loss at the nominal switch distance down."""
    import torch
    from paper_2505_23158_amd import lodbuild as LB
    base_raw, cams, d, _ = synth.lod_build_workload(n=2000, n_views=6, width=64, height=48, d=(4.0,), seed=66)
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in base_raw.items()}
    base = LB.level_from_raw(t["mean"], t["log_scale"], t["quat_raw"], t["opacity_logit"], t["sh"], 3, 0.0)
    sc0 = L.Scene([base.scene_level()], [], None)
    R0 = L.Renderer(sc0, cams[0].width, cams[0].height)
    targets = torch.empty((len(cams), 3, cams[0].height, cams[0].width), device="cuda")
    for v, cam in enumerate(cams):
        R0.frame(cam, L.SELECT_ALL)
        targets[v].copy_(R0.image)
    B = LB.LodBuilder([base], d, cams, targets)
    B.levels.append(LB.copy_with_filter(base, synth.filter_var(d[0])))
    s = B.importance(1)
    B.prune(1, float(torch.quantile(s, 0.7)))
    before = B.eval_loss(1)
    rng = np.random.default_rng(5)
    for _ in range(150):
        B.finetune_step(1, int(rng.integers(0, len(cams))), float(rng.uniform(0.7, 1.3)))
    after = B.eval_loss(1)
    log(f"[lodbuild] pruned to {B.levels[1].n} of {base.n}; loss {before:.5f} -> {after:.5f}")
    assert np.isfinite(after) and after < 0.9 * before, (before, after)
