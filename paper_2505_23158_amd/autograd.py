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

``render_views`` renders a batch of views through one Function
(``LodgeRenderViews``): its backward runs every view's adjoint into one set
of activated-parameter gradient planes (zeroed once per batch) and chains
them through the activation once, instead of once per view.  Activation in
the forward runs only when a raw parameter has changed since the last one
(torch's in-place version counters), so the views of a batch share it.

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
        self._act_version = None
        # gradients w.r.t. the activated parameters: one set, reused by every backward
        self.g_act = [{"mean": torch.empty_like(r["mean"]), "scale": torch.empty_like(r["log_scale"]),
                       "quat": torch.empty_like(r["quat_raw"]), "opacity": torch.empty_like(r["opacity_logit"]),
                       "sh": torch.empty_like(r["sh"])} for r in self.raw]

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

    def _version(self):
        return tuple((t.data_ptr(), t._version) for r in self.raw for t in
                     (r["log_scale"], r["quat_raw"], r["opacity_logit"]))

    def activate(self, force: bool = False):
        """exp / normalise / sigmoid into the planes the scene reads, unless no raw parameter has changed."""
        v = self._version()
        if not force and v == self._act_version:
            return
        for r, a in zip(self.raw, self.act):
            L.lodge_activate(r["log_scale"], r["quat_raw"], r["opacity_logit"], a["scale"], a["quat"], a["opacity"])
        self._act_version = v

    def render(self, cam, mode: int = L.SELECT_ALL, slot: int = 0, grad_level: int = -1, s2d: float = 0.3,
               compensate: bool = True):
        flat = [t for r in self.raw for t in (r[k] for k in PARAMS)]
        return LodgeRender.apply(self, cam, mode, slot, grad_level, s2d, compensate, *flat)

    def render_views(self, cams, mode: int = L.SELECT_ALL, grad_level: int = -1, s2d: float = 0.3,
                     compensate: bool = True):
        """Images [V, 3, H, W] of V <= n_slots views (view v on slot v), differentiable as one batch."""
        if len(cams) > len(self.slots):
            raise ValueError(f"{len(cams)} views need as many slots (have {len(self.slots)})")
        flat = [t for r in self.raw for t in (r[k] for k in PARAMS)]
        return LodgeRenderViews.apply(self, tuple(cams), mode, grad_level, s2d, compensate, *flat)

    def _zero_grads(self):
        for g in self.g_act:
            for t in g.values():
                t.zero_()

    def _raw_grads(self):
        """Chain the accumulated activated-parameter gradients through the activation: new tensors per call
        (autograd may keep a returned gradient while the next backward runs)."""
        out = []
        for r, a, g in zip(self.raw, self.act, self.g_act):
            g_ls = torch.zeros_like(r["log_scale"])
            g_qr = torch.zeros_like(r["quat_raw"])
            g_ol = torch.zeros_like(r["opacity_logit"])
            L.lodge_activate_backward(r["quat_raw"], a["scale"], a["opacity"], g["scale"], g["quat"], g["opacity"],
                                      g_ls, g_qr, g_ol)
            out += [g["mean"].clone(), g_ls, g_qr, g_ol, g["sh"].clone()]
        return out


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
        dr._zero_grads()
        L.lodge_render_backward(dr.scene, R.sel, ctx.cam, R.ws, ctx.final_T, ctx.n_contrib,
                                dL_dimage.contiguous(), dr.g_act, grad_level=ctx.grad_level, s2d=ctx.s2d,
                                compensate=ctx.compensate)
        return (None, None, None, None, None, None, None, *dr._raw_grads())


class LodgeRenderViews(torch.autograd.Function):
    @staticmethod
    def forward(ctx, dr: DiffRenderer, cams, mode, grad_level, s2d, compensate, *flat):
        dr.activate()
        out = torch.empty((len(cams), 3, dr.height, dr.width), dtype=torch.float32, device=flat[0].device)
        Ts, ncs = [], []
        for v, cam in enumerate(cams):
            R = dr.slots[v]
            R.frame(cam, mode, s2d=s2d, compensate=compensate)
            out[v].copy_(R.image)
            Ts.append(R.final_T.clone())
            ncs.append(R.n_contrib.clone())
        ctx.dr, ctx.cams, ctx.grad_level, ctx.s2d, ctx.compensate = dr, cams, grad_level, s2d, compensate
        ctx.final_T, ctx.n_contrib = Ts, ncs
        return out

    @staticmethod
    def backward(ctx, dL_dimages):
        dr: DiffRenderer = ctx.dr
        dr._zero_grads()
        dL = dL_dimages.contiguous()
        # the views' adjoints run one after another on one stream into the same planes (a plain add per
        # Gaussian: they must not overlap)
        for v, cam in enumerate(ctx.cams):
            R = dr.slots[v]
            L.lodge_render_backward(dr.scene, R.sel, cam, R.ws, ctx.final_T[v], ctx.n_contrib[v], dL[v], dr.g_act,
                                    grad_level=ctx.grad_level, s2d=ctx.s2d, compensate=ctx.compensate)
        return (None, None, None, None, None, None, *dr._raw_grads())
