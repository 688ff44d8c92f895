"""Differentiable LOD rendering for per-level fine-tuning.

The paper's supplementary "LOD structure optimization steps" fine-tunes level
G_l with LOD rendering of levels up to l and updates only G_l's parameters.
``DiffRenderer`` holds the raw (pre-activation) parameters of every level as
leaf tensors; ``render`` returns an image that is differentiable with
respect to them through ``LodgeRender`` (a torch.autograd.Function):

  forward:  lodge_activate (exp / normalise / sigmoid, in place into fixed
            buffers the scene points at) -> lodge_select -> lodge_render
  backward: lodge_render_backward (grad_level restricts to one level)
            -> lodge_activate_backward

Every step runs in the HIP kernels of liblodge.so; this module only
marshals tensors.  A workspace holds one frame's intermediates until its
backward, so each view in flight uses its own slot.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import lodge as L

PARAMS = ("mean", "log_scale", "quat_raw", "opacity_logit", "sh")


class DiffRenderer:
    def __init__(self, raw_levels: Sequence[dict], d: Sequence[float] = (), chunks=None, width: int = 64,
                 height: int = 64, n_slots: int = 1, max_active: Optional[int] = None,
                 max_instances: Optional[int] = None):
        self.raw = []
        self.act = []
        levels = []
        for lv in raw_levels:
            r = {k: lv[k] for k in PARAMS}
            for k, t in r.items():
                if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                    raise ValueError(f"{k}: need a contiguous float32 CUDA tensor")
            a = {"scale": torch.empty_like(r["log_scale"]), "quat": torch.empty_like(r["quat_raw"]),
                 "opacity": torch.empty_like(r["opacity_logit"])}
            self.raw.append(r)
            self.act.append(a)
            levels.append(dict(mean=r["mean"], scale=a["scale"], quat=a["quat"], opacity=a["opacity"], sh=r["sh"],
                               sh_degree=int(lv.get("sh_degree", 3)), filter3d_var=float(lv.get("filter3d_var", 0.0))))
        self.scene = L.Scene(levels, d, chunks)
        self.slots = [L.Renderer(self.scene, width, height, max_active=max_active, max_instances=max_instances)
                      for _ in range(n_slots)]
        self.width, self.height = width, height

    @classmethod
    def from_synth(cls, sc, width=None, height=None, n_slots=1, **kw):
        levels = []
        for lv in sc.levels:
            assert lv.raw is not None, "the synthetic scene must keep its raw parameters"
            nsh = (lv.sh_degree + 1) ** 2
            levels.append(dict(mean=torch.from_numpy(lv.mean).cuda(),
                               log_scale=torch.from_numpy(lv.raw["log_scale"]).cuda(),
                               quat_raw=torch.from_numpy(lv.raw["quat"]).cuda(),
                               opacity_logit=torch.from_numpy(lv.raw["opacity_logit"]).cuda(),
                               sh=torch.from_numpy(lv.sh[:nsh].copy()).cuda(), sh_degree=lv.sh_degree,
                               filter3d_var=lv.filter3d_var))
        cam = sc.cameras[0]
        return cls(levels, sc.d, sc.chunks, width or cam.width, height or cam.height, n_slots, **kw)

    def parameters(self, level: Optional[int] = None):
        lv = self.raw if level is None else [self.raw[level]]
        return [t for r in lv for t in r.values()]

    def activate(self):
        for r, a in zip(self.raw, self.act):
            L.lodge_activate(r["log_scale"], r["quat_raw"], r["opacity_logit"], a["scale"], a["quat"], a["opacity"])

    def render(self, cam, mode: int = L.SELECT_ALL, slot: int = 0, grad_level: int = -1, s2d: float = 0.3,
               compensate: bool = True):
        flat = [t for r in self.raw for t in (r[k] for k in PARAMS)]
        return LodgeRender.apply(self, cam, mode, slot, grad_level, s2d, compensate, *flat)


class LodgeRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, dr: DiffRenderer, cam, mode, slot, grad_level, s2d, compensate, *flat):
        R = dr.slots[slot]
        dr.activate()
        R.frame(cam, mode, s2d=s2d, compensate=compensate)
        ctx.dr, ctx.cam, ctx.slot, ctx.grad_level = dr, cam, slot, grad_level
        ctx.s2d, ctx.compensate = s2d, compensate
        ctx.final_T = R.final_T.clone()
        ctx.n_contrib = R.n_contrib.clone()
        return R.image.clone()

    @staticmethod
    def backward(ctx, dL_dimage):
        dr: DiffRenderer = ctx.dr
        R = dr.slots[ctx.slot]
        g_act = []
        for r in dr.raw:
            g_act.append({"mean": torch.zeros_like(r["mean"]), "scale": torch.zeros_like(r["log_scale"]),
                          "quat": torch.zeros_like(r["quat_raw"]), "opacity": torch.zeros_like(r["opacity_logit"]),
                          "sh": torch.zeros_like(r["sh"])})
        L.lodge_render_backward(dr.scene, R.sel, ctx.cam, R.ws, ctx.final_T, ctx.n_contrib,
                                dL_dimage.contiguous(), g_act, grad_level=ctx.grad_level, s2d=ctx.s2d,
                                compensate=ctx.compensate)
        out = []
        for r, a, g in zip(dr.raw, dr.act, g_act):
            g_ls = torch.zeros_like(r["log_scale"])
            g_qr = torch.zeros_like(r["quat_raw"])
            g_ol = torch.zeros_like(r["opacity_logit"])
            L.lodge_activate_backward(r["quat_raw"], a["scale"], a["opacity"], g["scale"], g["quat"], g["opacity"],
                                      g_ls, g_qr, g_ol)
            out += [g["mean"], g_ls, g_qr, g_ol, g["sh"]]
        return (None, None, None, None, None, None, None, *out)
