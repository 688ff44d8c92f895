"""The served form on the GPU: captured-graph replays re-read the pinned
camera and equal eager renders; requests served concurrently in a mix of
resolutions equal the same requests rendered alone; frames in flight on
several streams equal the same frames rendered one at a time."""
import numpy as np
import pytest

import synth

from parity_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_23158_amd import lodge as L
    sc = synth.config3_scene(frac=0.01, n_frames=8)
    dev = L.Scene.from_synth(sc)
    return L, sc, dev


CAPS = {(640, 360): (400_000, 2_000_000), (1280, 720): (400_000, 4_000_000), (1920, 1080): (400_000, 8_000_000)}


def alone(L, dev, cam):
    import torch
    R = L.Renderer(dev, cam.width, cam.height, *CAPS[(cam.width, cam.height)])
    R.frame(cam, L.SELECT_CHUNKED)
    torch.cuda.synchronize()
    assert L.lodge_check(R.ws)[0] == L.LODGE_OK
    return R.image.clone()


def test_graph_replays_follow_the_pinned_camera(env):
    import torch
    from paper_2505_23158_amd.serve import GpuBackend, Request
    L, sc, dev = env
    be = GpuBackend(dev, L.SELECT_CHUNKED, CAPS, use_graphs=True, keep_images=True)
    sid = be.new_slot((640, 360))
    cams = synth.config3_path(6, 640, 360)
    for k, cam in enumerate(cams):
        log(f"[serve] replay {k}")
        be.launch(sid, Request(k, 0.0, cam))
        while be.poll(sid) is None:
            pass
        ref = alone(L, dev, cam)              # eager work and syncs between replays
        assert torch.equal(be.images[k], ref), k


def test_mixed_concurrent_requests_equal_alone(env):
    import torch
    from paper_2505_23158_amd.serve import Request, serve
    L, sc, dev = env
    reqs = synth.serving_requests(24, rate=2000.0, half_xy=40.0, seed=12)   # arrivals ~0.5 ms apart: overlap
    requests = [Request(i, t, cam) for i, (t, cam) in enumerate(reqs)]
    log(f"[serve] {len(requests)} requests, resolutions {sorted({r.resolution for r in requests})}")
    rep, be = serve(dev, requests, L.SELECT_CHUNKED, CAPS, max_slots_per_class=4, prewarm=2, keep_images=True)
    torch.cuda.synchronize()
    s = rep.summary()
    log(f"[serve] summary {s}")
    assert s["requests"] == len(requests) and s["peak_in_flight"] >= 2
    for r in requests:
        ref = alone(L, dev, r.cam)
        got = be.images[r.rid]
        assert float((got - ref).abs().max()) <= 1e-4, r.rid
        assert torch.equal(got, ref), r.rid       # deterministic kernels: bit-identical in fact


def test_capacity_overflow_is_retried_outside_the_graph(env):
    import torch
    from paper_2505_23158_amd.serve import Request, serve
    L, sc, dev = env
    tiny = {(640, 360): (400_000, 2_000)}
    cam = synth.config3_path(3, 640, 360)[1]
    rep, be = serve(dev, [Request(0, 0.0, cam)], L.SELECT_CHUNKED, tiny, prewarm=1, keep_images=True)
    assert rep.results[0].retried
    assert torch.equal(be.images[0], alone(L, dev, cam))


def test_frames_in_flight_equal_frames_one_at_a_time(env):
    """Consecutive frames of a camera path on three renderers and three
    streams, handed out round robin (the throughput form of the benchmark),
    give the same images, final T and n_contrib as the same frames rendered
    one after another."""
    import torch
    L, sc, dev = env
    cams = sc.cameras
    W, H = cams[0].width, cams[0].height
    F = 3
    rens = [L.Renderer(dev, W, H, *CAPS[(W, H)]) for _ in range(F)]
    streams = [torch.cuda.Stream() for _ in range(F)]
    serial = L.Renderer(dev, W, H, *CAPS[(W, H)])
    n = len(cams)
    got = []
    for k in range(n):
        rens[k % F].frame(cams[k], L.SELECT_CHUNKED, stream=streams[k % F])
        if k % F == F - 1 or k == n - 1:
            # the slots are reused from the next round on: copy this round's outputs first
            torch.cuda.synchronize()
            for j in range(k - k % F, k + 1):
                r = rens[j % F]
                assert L.lodge_check(r.ws)[0] == L.LODGE_OK
                got.append((r.image.clone(), r.final_T.clone(), r.n_contrib.clone()))
    for k in range(n):
        serial.frame(cams[k], L.SELECT_CHUNKED)
        torch.cuda.synchronize()
        img, T, nc = got[k]
        assert torch.equal(img, serial.image) and torch.equal(T, serial.final_T), f"frame {k}"
        assert torch.equal(nc, serial.n_contrib), f"frame {k}"
    log(f"[in-flight] {n} frames on {F} streams equal the serial renders")
