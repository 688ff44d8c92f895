"""Depth-threshold search on the GPU (Sec. 3 "Selecting depth thresholds")
against the oracle: the tile-instance count of every evaluated LOD frame is
bit-exact (an integer fixed by the selection and the tile rectangles), so the
costs, the greedy choice and a two-threshold cost table are identical."""
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


def test_greedy_search_and_cost_table_match_oracle(L, oracle32):
    from paper_2505_23158_amd import thresholds as TH
    sc = synth.lod_city_scene(counts=(200000, 50000, 12500), half_xy=100.0, d=(20.0, 60.0), grid=4,
                              spacing=50.0, chunk_z=1.7, band=10.0, seed=32)
    cams = synth.threshold_views(3, half_xy=100.0, width=320, height=180, seed=44)
    cams.append(synth.threshold_views(1, half_xy=60.0, width=100, height=37, seed=45)[0])   # ragged tiles
    dev = L.Scene.from_synth(sc)
    ev = TH.CostEvaluator(dev, cams)
    cands = [5.0, 10.0, 15.0, 20.0, 30.0, 40.0, 60.0, 80.0]
    chosen, curves = TH.greedy_search(ev, cands, 3)
    grid = [10.0, 20.0, 40.0, 80.0]
    table = TH.cost_table(ev, grid, grid)
    # every count the GPU produced, against the oracle's
    for d, counts in ev.cache.items():
        ref = [oracle.lod_instances(oracle32, sc, d, len(d) + 1, c) for c in cams]
        assert counts == ref, (d, counts, ref)
    o_chosen, o_curves = oracle.greedy_thresholds(lambda d: oracle.threshold_cost(oracle32, sc, d, len(d) + 1, cams),
                                                  cands, 3)
    assert chosen == o_chosen
    for g, o in zip(curves, o_curves):
        assert [c for c, _ in g] == [c for c, _ in o]
        assert np.allclose([v for _, v in g], [v for _, v in o], rtol=1e-12, atol=0)
    for i, a in enumerate(grid):
        for j, b in enumerate(grid):
            if a < b:
                assert table[i][j] == pytest.approx(oracle.threshold_cost(oracle32, sc, (a, b), 3, cams), rel=1e-12)
            else:
                assert table[i][j] is None
    log(f"[thresholds] greedy choice {chosen}; {len(ev.cache)} threshold sets evaluated, all counts bit-exact")


def test_full_size_instance_counts(L, oracle32):
    """The lod3 scene at full size (2.625M Gaussians) and 1080p views: the tile
    instances of LOD frames at two sets of switch distances, bit-exact against
    the oracle (the integers the search compares)."""
    from paper_2505_23158_amd import thresholds as TH
    sc = synth.config2_scene()
    cams = synth.threshold_views(2, half_xy=100.0, width=1920, height=1080, seed=47)
    dev = L.Scene.from_synth(sc)
    ev = TH.CostEvaluator(dev, cams, max_instances=32_000_000)
    for d in ((20.0, 60.0), (10.0, 40.0)):
        got = ev.instances(d)
        ref = [oracle.lod_instances(oracle32, sc, d, 3, c) for c in cams]
        assert got == ref, (d, got, ref)
        log(f"[thresholds] full size d={d}: {got} instances per view")
