"""Per-chunk visibility filtering (LODGE Sec. 3 "Visibility filtering", with
the importance score of "Preliminaries: Importance pruning").

For each chunk k: its stored active set is rendered from the chunk's views
(camera positions of the chunk under random orientations), every Gaussian's
importance is the largest blending weight alpha T it receives in any pixel
of those views, and the members scoring below a fixed threshold leave the
chunk's set.  Frames then load the filtered sets through
lodge_select_chunk_sets exactly as before.

Host orchestration only: the selection, the importance walk and the pruning
are the library's kernels (lodge_select_chunk, lodge_importance,
lodge_chunk_sets_prune).
"""
from __future__ import annotations

from typing import Sequence

from . import lodge as L


def chunk_scores(scene: L.Scene, sets: L.ChunkSets, k: int, views: Sequence, ws: L.Workspace, sel: L.Selection,
                 score, s2d: float = 0.3, compensate: bool = True, stream=None):
    """Importance of every Gaussian of chunk k's stored set over its views, into score (by global id,
    zeroed here).  Raises LodgeError if a view overflowed the workspace."""
    score.zero_()
    L.lodge_select_chunk(scene, sets, k, ws, sel, stream)
    for cam in views:
        L.lodge_importance(scene, sel, cam, ws, score, s2d, compensate, stream)
        st, na, ni = L.lodge_check(ws, stream)
        if st != L.LODGE_OK:
            raise L.LodgeError(st, f"chunk {k}: the workspace needs {na} actives and {ni} instances")
    return score


def filter_chunk_sets(scene: L.Scene, sets: L.ChunkSets, views_per_chunk: Sequence[Sequence], threshold: float,
                      ws: L.Workspace, sel: L.Selection, s2d: float = 0.3, compensate: bool = True,
                      stream=None) -> list:
    """Filters every chunk's stored set in place; returns each chunk's member count before and after."""
    torch = L._torch()
    score = torch.zeros(scene.total, dtype=torch.float32, device="cuda")
    counts = []
    for k, views in enumerate(views_per_chunk):
        chunk_scores(scene, sets, k, views, ws, sel, score, s2d, compensate, stream)
        before = int(sel.count.item())
        L.lodge_chunk_sets_prune(scene, sets, k, score, threshold, stream)
        L.lodge_select_chunk(scene, sets, k, ws, sel, stream)
        counts.append((before, int(sel.count.item())))
    return counts
