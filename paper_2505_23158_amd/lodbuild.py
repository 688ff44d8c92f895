"""Construction of the LOD levels (LODGE supplementary "LOD structure
optimization steps"; Sec. 3 "Building LOD representation", Eq. 3).

Given the finest level G^(0) and switch distances d_1 < ... < d_{L-1}, the
levels are built from the finest to the coarsest.  Level l starts as a copy
of G^(0) whose Gaussians carry the 3-D smoothing filter of depth d_l (the
filter is part of the Gaussian function; the parameters are unchanged, so
no Gaussian can become smaller than the filter).  Then, three times: the
level is pruned by importance score (thresholds 0.2, 0.6 and 1.0 times
gamma) and fine-tuned for a number of steps (the paper uses 1000).  A
fine-tuning step renders levels 0..l with Eq. 2 about the camera of a
training view, d_l replaced by a draw from U(0.7 d_l, 1.3 d_l), and updates
only level l's parameters.

Every step runs in liblodge.so's kernels: activation, selection, rendering,
the L1 loss gradient, the adjoint restricted to level l, the activation's
adjoint, Adam, importance scores, and the compaction after pruning.  This
module holds the host loop and the parameter buffers (torch tensors).

Readings (the paper is silent on them): the loss is 3DGS's
(1 - lambda) L1 + lambda D-SSIM with lambda = 0.2 (the paper's "DSSIM + L1");
importance scores for pruning come from LOD renders of
levels 0..l at the nominal switch distances over the training views; Adam
(beta 0.9 / 0.999, eps 1e-15) uses the 3DGS learning rates per parameter
group and its moments follow the kept Gaussians through a pruning; the
random draws (training view and d_l factor of every step) are inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence

from . import lodge as L

# raw parameter groups: name -> number of planes (sh: (d+1)^2 * 3)
GROUPS = ("mean", "log_scale", "quat_raw", "opacity_logit", "sh")
LRS = {"mean": 1.6e-4, "log_scale": 5e-3, "quat_raw": 1e-3, "opacity_logit": 0.05, "sh_dc": 2.5e-3,
       "sh_rest": 2.5e-3 / 20.0}


def _planes(sh_degree: int) -> Dict[str, int]:
    return {"mean": 3, "log_scale": 3, "quat_raw": 4, "opacity_logit": 1, "sh": 3 * (sh_degree + 1) ** 2}


@dataclass
class LevelState:
    """One level's raw parameters as one [P][n] buffer (attribute-major planes), its Adam moments, the
    activated planes the renderer reads, and its 3-D filter variance."""
    raw: object
    m: object
    v: object
    sh_degree: int
    filter3d_var: float
    act: Dict[str, object] = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.raw.shape[1])

    def view(self, name: str):
        off = 0
        for g, p in _planes(self.sh_degree).items():
            if g == name:
                return self.raw[off:off + p]
            off += p
        raise KeyError(name)

    def rows(self):
        off = 0
        for g, p in _planes(self.sh_degree).items():
            yield g, off, p
            off += p

    def activate(self):
        torch = L._torch()
        n = self.n
        if not self.act or int(self.act["scale"].shape[1]) != n:
            self.act = {"scale": torch.empty((3, n), dtype=torch.float32, device="cuda"),
                        "quat": torch.empty((4, n), dtype=torch.float32, device="cuda"),
                        "opacity": torch.empty((n,), dtype=torch.float32, device="cuda")}
        L.lodge_activate(self.view("log_scale"), self.view("quat_raw"), self.view("opacity_logit")[0],
                         self.act["scale"], self.act["quat"], self.act["opacity"])

    def scene_level(self) -> dict:
        return dict(mean=self.view("mean"), scale=self.act["scale"], quat=self.act["quat"],
                    opacity=self.act["opacity"], sh=self.view("sh").reshape(-1, 3, self.n),
                    sh_degree=self.sh_degree, filter3d_var=self.filter3d_var)


def level_from_raw(mean, log_scale, quat_raw, opacity_logit, sh, sh_degree: int, filter3d_var: float) -> LevelState:
    torch = L._torch()
    n = int(mean.shape[-1])
    raw = torch.cat([mean.reshape(3, n), log_scale.reshape(3, n), quat_raw.reshape(4, n),
                     opacity_logit.reshape(1, n), sh.reshape(-1, n)], dim=0).contiguous()
    st = LevelState(raw=raw, m=torch.zeros_like(raw), v=torch.zeros_like(raw), sh_degree=sh_degree,
                    filter3d_var=float(filter3d_var))
    st.activate()
    return st


def copy_with_filter(base: LevelState, filter3d_var: float) -> LevelState:
    """Level l's starting point: G^(0)'s parameters with the 3-D filter of depth d_l, fresh moments."""
    torch = L._torch()
    st = LevelState(raw=base.raw.clone(), m=torch.zeros_like(base.raw), v=torch.zeros_like(base.raw),
                    sh_degree=base.sh_degree, filter3d_var=float(filter3d_var))
    st.activate()
    return st


class LodBuilder:
    """Renders, losses and updates for building level l on top of levels 0..l-1."""

    def __init__(self, levels: List[LevelState], d: Sequence[float], cams: Sequence, targets, max_active=None,
                 max_instances=None, lambda_dssim: float = 0.2):
        torch = L._torch()
        self.levels = levels
        self.d = [float(x) for x in d]
        self.cams = list(cams)
        self.targets = targets                      # [V, 3, H, W] float32, cuda
        W, H = self.cams[0].width, self.cams[0].height
        total = sum(lv.n for lv in levels)
        self.W, self.H = W, H
        self.max_active = max_active or max(1, total)
        self.max_instances = max_instances
        self.R = None
        self.dL = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.step = {}
        self.lam = float(lambda_dssim)
        self.ssim_scratch = None

    def _renderer(self, scene: L.Scene) -> L.Renderer:
        if self.R is None or self.R.scene.total < scene.total:
            self.R = L.Renderer(scene, self.W, self.H, max_active=max(self.max_active, scene.total),
                                max_instances=self.max_instances)
        return self.R

    def scene(self, l: int, d: Sequence[float]) -> L.Scene:
        return L.Scene([lv.scene_level() for lv in self.levels[:l + 1]], list(d)[:l], None)

    def render(self, l: int, d: Sequence[float], cam):
        sc = self.scene(l, d)
        R = self._renderer(sc)
        L.lodge_select(sc, cam, L.SELECT_LOD_CAMERA, R.ws, R.sel)
        L.lodge_render(sc, R.sel, cam, R.ws, R.image, R.final_T, R.n_contrib)
        return sc, R

    def finetune_step(self, l: int, view: int, d_factor: float):
        """One fine-tuning step of level l: d_l scaled by d_factor (a draw from U(0.7, 1.3)), the given
        training view, loss (1 - lambda) mean L1 + lambda D-SSIM, gradients of level l only, one Adam step
        per parameter group."""
        import numpy as np
        torch = L._torch()
        lv = self.levels[l]
        d = list(self.d)
        d[l - 1] = float(np.float32(np.float32(d[l - 1]) * np.float32(d_factor)))
        cam = self.cams[view]
        sc, R = self.render(l, d, cam)
        n_px = 3 * self.W * self.H
        self.loss.zero_()
        L.lodge_l1_grad(R.image, self.targets[view], self.dL, (1.0 - self.lam) / n_px, self.loss)
        if self.lam:
            self.ssim_scratch = L.lodge_dssim_grad(R.image, self.targets[view], self.dL, self.lam, self.loss,
                                                   self.ssim_scratch)
        g = {"mean": torch.zeros((3, lv.n), dtype=torch.float32, device="cuda"),
             "scale": torch.zeros((3, lv.n), dtype=torch.float32, device="cuda"),
             "quat": torch.zeros((4, lv.n), dtype=torch.float32, device="cuda"),
             "opacity": torch.zeros((lv.n,), dtype=torch.float32, device="cuda"),
             "sh": torch.zeros((3 * (lv.sh_degree + 1) ** 2, lv.n), dtype=torch.float32, device="cuda")}
        grads = [{} for _ in range(l)] + [g]
        L.lodge_render_backward(sc, R.sel, cam, R.ws, R.final_T, R.n_contrib, self.dL, grads, grad_level=l)
        graw = torch.zeros_like(lv.raw)
        rows = {name: (off, p) for name, off, p in lv.rows()}
        o, p = rows["mean"]
        graw[o:o + p].copy_(g["mean"])
        o, p = rows["sh"]
        graw[o:o + p].copy_(g["sh"])
        ls, qr, ol = rows["log_scale"], rows["quat_raw"], rows["opacity_logit"]
        L.lodge_activate_backward(lv.view("quat_raw"), lv.act["scale"], lv.act["opacity"], g["scale"], g["quat"],
                                  g["opacity"], graw[ls[0]:ls[0] + 3], graw[qr[0]:qr[0] + 4], graw[ol[0]])
        t = self.step.get(l, 0) + 1
        self.step[l] = t
        for name, off, p in lv.rows():
            if name == "sh":
                groups = [("sh_dc", off, 3), ("sh_rest", off + 3, p - 3)]
            else:
                groups = [(name, off, p)]
            for gname, go, gp in groups:
                if gp <= 0:
                    continue
                L.lodge_adam(lv.raw[go:go + gp], graw[go:go + gp], lv.m[go:go + gp], lv.v[go:go + gp], LRS[gname], t)
        lv.activate()
        return graw

    def eval_loss(self, l: int) -> float:
        """The training loss of levels 0..l, (1 - lambda) mean L1 + lambda D-SSIM, averaged over the training
        views rendered at the nominal switch distances (no parameter changes)."""
        torch = L._torch()
        n_px = 3 * self.W * self.H
        total = torch.zeros(1, dtype=torch.float32, device="cuda")
        for v, cam in enumerate(self.cams):
            _, R = self.render(l, self.d, cam)
            self.loss.zero_()
            L.lodge_l1_grad(R.image, self.targets[v], self.dL, (1.0 - self.lam) / n_px, self.loss)
            if self.lam:
                self.ssim_scratch = L.lodge_dssim_grad(R.image, self.targets[v], self.dL, self.lam, self.loss,
                                                       self.ssim_scratch)
            total += self.loss
        return float(total.item()) / len(self.cams)

    def importance(self, l: int):
        """Importance of every Gaussian of levels 0..l over the training views (LOD renders at the nominal
        switch distances); returns level l's slice of the score array."""
        torch = L._torch()
        sc = self.scene(l, self.d)
        R = self._renderer(sc)
        score = torch.zeros(sc.total, dtype=torch.float32, device="cuda")
        for cam in self.cams:
            L.lodge_select(sc, cam, L.SELECT_LOD_CAMERA, R.ws, R.sel)
            L.lodge_importance(sc, R.sel, cam, R.ws, score)
        base = sum(lv.n for lv in self.levels[:l])
        return score[base:base + self.levels[l].n]

    def prune(self, l: int, threshold: float):
        """Removes level l's Gaussians whose importance is below threshold (parameters and moments)."""
        torch = L._torch()
        lv = self.levels[l]
        s = self.importance(l).contiguous()
        idx = torch.empty(max(1, lv.n), dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        L.lodge_keep_indices(s, threshold, idx, cnt)
        m = int(cnt.item())
        out = []
        for buf in (lv.raw, lv.m, lv.v):
            o = torch.empty((buf.shape[0], max(1, m)), dtype=torch.float32, device="cuda")
            L.lodge_gather_planes(buf, idx, cnt, o)
            out.append(o[:, :m].contiguous())
        lv.raw, lv.m, lv.v = out
        lv.activate()
        return s


def build_levels(base: LevelState, d: Sequence[float], filter_vars: Sequence[float], cams, targets, gamma: float,
                 schedule, steps_per_round: int, rounds=(0.2, 0.6, 1.0), max_instances=None,
                 lambda_dssim: float = 0.2) -> LodBuilder:
    """Builds levels 1..len(d) on top of base (level 0).  schedule[l-1][r] is the list of (view, d factor)
    draws of round r of level l (steps_per_round of them)."""
    levels = [base]
    B = LodBuilder(levels, d, cams, targets, max_instances=max_instances, lambda_dssim=lambda_dssim)
    for l in range(1, len(d) + 1):
        levels.append(copy_with_filter(base, filter_vars[l - 1]))
        for r, frac in enumerate(rounds):
            B.prune(l, frac * gamma)
            for view, u in schedule[l - 1][r][:steps_per_round]:
                B.finetune_step(l, int(view), float(u))
    return B
