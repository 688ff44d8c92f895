"""The served form on the GPU: captured-graph replays re-read the pinned
camera and equal eager renders; requests served concurrently in a mix of
resolutions equal the same requests rendered alone; frames in flight on
several streams equal the same frames rendered one at a time."""
import numpy as np
import pytest

import oracle
import synth

from parity_util import compare_image, log

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


def test_replies_copied_to_pinned_host_memory(env):
    """copy_to_host: a request completes once its image is in its slot's pinned host buffer, which then holds
    the image of that request (graph replays, the copy ordered after them on the slot's stream)."""
    import torch
    from paper_2505_23158_amd.serve import GpuBackend, Request
    L, sc, dev = env
    be = GpuBackend(dev, L.SELECT_CHUNKED, CAPS, use_graphs=True, copy_to_host=True)
    sid = be.new_slot((640, 360))
    assert be.slots[sid]["host"].is_pinned()
    for k, cam in enumerate(synth.config3_path(3, 640, 360)):
        be.launch(sid, Request(k, 0.0, cam))
        while be.poll(sid) is None:
            pass
        assert torch.equal(be.slots[sid]["host"], alone(L, dev, cam).cpu()), k


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
    assert be.caps[(640, 360)][1] > 2_000


def test_selection_overflow_grows_the_slot_until_the_frame_fits(env, oracle32):
    """Both capacities far too small: the selection overflows first (so the
    first instance count covers only the truncated set), the slot grows until
    lodge_check passes, later requests of the class reuse the grown slot, and
    every served result equals the oracle."""
    import torch
    from paper_2505_23158_amd.serve import Request, serve
    L, sc, dev = env
    tiny = {(640, 360): (1_000, 1_000)}
    cams = synth.config3_path(5, 640, 360)[1:4]
    reqs = [Request(i, 0.004 * i, c) for i, c in enumerate(cams)]
    rep, be = serve(dev, reqs, L.SELECT_CHUNKED, tiny, prewarm=1, keep_images=True, max_slots_per_class=1)
    assert rep.results[0].retried
    ma, mi = be.caps[(640, 360)]
    assert ma > 1_000 and mi > 1_000
    assert rep.mem_bytes > be._bytes((640, 360), (1_000, 1_000))
    for r in reqs:
        out = be.outputs[r.rid]
        ref = oracle32.render(sc, r.cam, oracle.CHUNKED)
        assert np.array_equal(out["ids"].cpu().numpy().astype(np.uint32), ref["ids"])
        g = {k: out[k].cpu().numpy() for k in ("image", "final_T", "n_contrib")}
        g["n_contrib"] = g["n_contrib"].astype(np.uint32)
        compare_image(oracle32, g, ref, r.cam)


@pytest.fixture(scope="module")
def env5():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_23158_amd import lodge as L
    sc = synth.config3_scene(frac=0.05, n_frames=4)
    return L, sc, L.Scene.from_synth(sc)


def test_served_requests_match_the_oracle(env5, oracle32):
    """Requests at the serving poses (1.5-50 m up, pitch 0 to -45 degrees,
    mixed resolutions) served concurrently through captured graphs on a
    1.33M-Gaussian scene: each served selection equals the oracle's bit for
    bit and each served image, final T and n_contrib the oracle's within the
    image tolerance."""
    import torch
    from paper_2505_23158_amd.serve import Request, serve
    L, sc, dev = env5
    reqs = synth.serving_requests(24, rate=3000.0, half_xy=60.0, seed=13)
    requests = [Request(i, t, cam) for i, (t, cam) in enumerate(reqs)]
    caps = {(640, 360): (600_000, 4_000_000), (1280, 720): (600_000, 8_000_000),
            (1920, 1080): (600_000, 12_000_000)}
    rep, be = serve(dev, requests, L.SELECT_CHUNKED, caps, max_slots_per_class=3, prewarm=2, keep_images=True)
    torch.cuda.synchronize()
    assert rep.peak_in_flight >= 2
    chosen, seen = [], {}
    for r in requests:
        if seen.get(r.resolution, 0) < 3:
            chosen.append(r)
            seen[r.resolution] = seen.get(r.resolution, 0) + 1
    assert len(seen) == 3 and len(chosen) >= 6
    for r in chosen:
        out = be.outputs[r.rid]
        ref = oracle32.render(sc, r.cam, oracle.CHUNKED)
        assert np.array_equal(out["ids"].cpu().numpy().astype(np.uint32), ref["ids"]), r.rid
        assert np.array_equal(out["w"].cpu().numpy().view(np.uint32), ref["w"].astype(np.float32).view(np.uint32))
        g = {k: out[k].cpu().numpy() for k in ("image", "final_T", "n_contrib")}
        g["n_contrib"] = g["n_contrib"].astype(np.uint32)
        flips, err = compare_image(oracle32, g, ref, r.cam)
        log(f"[serve-oracle] request {r.rid} {r.resolution} eye_z={r.cam.pos[2]:.1f}: active={len(ref['ids'])} "
            f"M={ref['binned'].M} flips={flips} max_err={err:.2e}")


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
