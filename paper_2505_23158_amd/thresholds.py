"""Automatic depth-threshold selection (LODGE Sec. 3 "Selecting depth
thresholds").

The cost of a set of switch distances d_1 < ... < d_l is the average number
of Gaussians each 16 x 16 tile processes -- tile instances per tile -- over
a set of views, rendered with levels 0..l and Eq. 2 about each camera.  The
search is greedy and one-dimensional: d_1 is the candidate of least cost
with two levels; then, with d_1..d_{l-1} fixed, d_l is the candidate above
d_{l-1} of least cost with levels 0..l.  Ties go to the smaller candidate.

Every cost evaluation is a GPU frame (lodge_select + lodge_render on a scene
created for those thresholds: scenes borrow the level planes, so that is
host bookkeeping only); the instance count is read from the frame counters.
"""
from __future__ import annotations

from typing import Sequence

from . import lodge as L


class CostEvaluator:
    """Per-view tile-instance counts of LOD frames for candidate thresholds."""

    def __init__(self, dev: L.Scene, cams: Sequence, max_instances: int | None = None):
        self.levels = dev.levels
        self.cams = list(cams)
        sizes = {(c.width, c.height) for c in self.cams}
        self.renderers = {}
        for (w, h) in sizes:
            self.renderers[(w, h)] = L.Renderer(dev, w, h, max_active=max(1, dev.total), max_instances=max_instances)
        self.cache = {}

    def instances(self, d: Sequence[float]) -> list:
        """Tile instances per view with levels 0..len(d) and switch distances d."""
        key = tuple(float(x) for x in d)
        if key not in self.cache:
            sub = L.Scene(self.levels[:len(key) + 1], list(key), None)
            out = []
            for cam in self.cams:
                R = self.renderers[(cam.width, cam.height)]
                L.lodge_select(sub, cam, L.SELECT_LOD_CAMERA, R.ws, R.sel)
                L.lodge_render(sub, R.sel, cam, R.ws, R.image, R.final_T, R.n_contrib)
                st, na, ni = L.lodge_check(R.ws)
                # an instance overflow still counts every instance (the count is taken before emission)
                if st != L.LODGE_OK and na > R.sel.cap:
                    raise L.LodgeError(st, "threshold search: selection capacity exceeded")
                out.append(int(R.info()["n_instances"]))
            self.cache[key] = out
        return self.cache[key]

    def cost(self, d: Sequence[float]) -> float:
        """Average number of Gaussians per tile over the views."""
        m = self.instances(d)
        return sum(mi / (((c.width + L.TILE - 1) // L.TILE) * ((c.height + L.TILE - 1) // L.TILE))
                   for mi, c in zip(m, self.cams)) / len(self.cams)


def greedy_search(ev: CostEvaluator, candidates: Sequence[float], n_levels: int):
    """Returns (thresholds, per-step [(candidate, cost)] curves)."""
    cands = sorted(float(c) for c in candidates)
    chosen, curves = [], []
    for l in range(1, n_levels):
        lo = chosen[-1] if chosen else float("-inf")
        curve = [(c, ev.cost(tuple(chosen) + (c,))) for c in cands if c > lo]
        if not curve:
            raise ValueError("no candidate above the previous threshold")
        best = min(curve, key=lambda p: (p[1], p[0]))
        chosen.append(best[0])
        curves.append(curve)
    return chosen, curves


def cost_table(ev: CostEvaluator, grid1: Sequence[float], grid2: Sequence[float]):
    """Three-level cost over (d_1, d_2) pairs with d_1 < d_2 (None elsewhere)."""
    return [[ev.cost((a, b)) if a < b else None for b in grid2] for a in grid1]
