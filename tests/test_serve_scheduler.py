"""The serving scheduler on the CPU, against a simulated device backend:
admission by free slot and memory budget, slot reuse, FIFO order within a
resolution class, retries, and the latency bookkeeping."""
import numpy as np
import pytest

from paper_2505_23158_amd.serve import Request, Scheduler, SimulatedBackend

R360, R720, R1080 = (640, 360), (1280, 720), (1920, 1080)


class Cam:
    def __init__(self, w, h):
        self.width, self.height = w, h


def reqs(arrivals, res):
    return [Request(i, float(t), Cam(*r)) for i, (t, r) in enumerate(zip(arrivals, res))]


def test_single_slot_serialises_and_latency_is_queueing_plus_service():
    be = SimulatedBackend({R720: 0.010}, {R720: 100}, parallel=4)
    rep = Scheduler(be, mem_budget=100, max_slots_per_class=8).run(reqs([0.0, 0.001, 0.002], [R720] * 3))
    lat = [r.latency for r in rep.results]
    assert np.allclose(lat, [0.010, 0.019, 0.028])
    assert rep.slots_created == {R720: 1} and rep.peak_in_flight == 1
    assert [s for _, s in be.order] == [0, 0, 0]      # the one slot is reused


def test_memory_budget_bounds_slots_and_overlap():
    be = SimulatedBackend({R720: 0.010}, {R720: 100}, parallel=8)
    rep = Scheduler(be, mem_budget=300, max_slots_per_class=8).run(reqs([0.0] * 6, [R720] * 6))
    assert rep.slots_created == {R720: 3} and rep.peak_in_flight == 3 and rep.mem_bytes == 300
    assert np.allclose(sorted(r.latency for r in rep.results), [0.01] * 3 + [0.02] * 3)


def test_classes_run_concurrently_and_fifo_within_class():
    be = SimulatedBackend({R360: 0.002, R1080: 0.008}, {R360: 10, R1080: 40}, parallel=4)
    arr = [0.0, 0.0, 0.0005, 0.001, 0.001]
    res = [R1080, R360, R360, R1080, R360]
    rep = Scheduler(be, mem_budget=100, max_slots_per_class=1).run(reqs(arr, res))
    # one slot per class: within a class requests complete in arrival order
    by_class = {}
    for r in sorted(rep.results, key=lambda r: r.done):
        by_class.setdefault(r.resolution, []).append(r.rid)
    assert by_class[R360] == [1, 2, 4] and by_class[R1080] == [0, 3]
    assert rep.peak_in_flight == 2


def test_device_parallelism_limit_shares_time():
    # 4 requests on 4 slots but the device runs 2 at a time
    be = SimulatedBackend({R360: 0.004}, {R360: 1}, parallel=2)
    rep = Scheduler(be, mem_budget=10, max_slots_per_class=4).run(reqs([0.0] * 4, [R360] * 4))
    assert np.allclose(sorted(r.latency for r in rep.results), [0.004, 0.004, 0.008, 0.008])


def test_retry_after_capacity_overflow_is_counted():
    be = SimulatedBackend({R360: 0.003}, {R360: 1}, parallel=4, fail_first={1})
    rep = Scheduler(be, mem_budget=10).run(reqs([0.0, 0.0], [R360] * 2))
    assert [r.retried for r in rep.results] == [False, True]
    assert rep.results[1].latency == pytest.approx(0.006)
    assert rep.summary()["retries"] == 1


def test_grown_slot_counts_against_the_memory_budget():
    # request 0 overflows and its slot grows by 2 units (reported when it completes, at 6 ms): with a
    # budget of 3, request 2 (arriving while request 1 holds slot 0) cannot get a slot of its own
    be = SimulatedBackend({R360: 0.003}, {R360: 1}, parallel=4, fail_first={0}, grow_bytes=2)
    rep = Scheduler(be, mem_budget=3, max_slots_per_class=4).run(reqs([0.0, 0.007, 0.0071], [R360] * 3))
    assert rep.results[0].retried and rep.mem_bytes == 3
    assert rep.slots_created[R360] == 1
    assert be.order == [(0, 0), (1, 0), (2, 0)]
    # without the growth the same arrivals open a second slot
    be2 = SimulatedBackend({R360: 0.003}, {R360: 1}, parallel=4, fail_first={0}, grow_bytes=0)
    rep2 = Scheduler(be2, mem_budget=3, max_slots_per_class=4).run(reqs([0.0, 0.007, 0.0071], [R360] * 3))
    assert rep2.slots_created[R360] == 2


def test_budget_below_one_slot_is_an_error():
    be = SimulatedBackend({R1080: 0.01}, {R1080: 1000}, parallel=4)
    with pytest.raises(RuntimeError):
        Scheduler(be, mem_budget=10).run(reqs([0.0], [R1080]))


def test_poisson_load_summary_percentiles():
    rng = np.random.default_rng(0)
    n = 256
    arr = np.cumsum(rng.exponential(1 / 120.0, n))
    arr -= arr[0]
    res = [(R360, R720, R1080)[i] for i in rng.integers(0, 3, n)]
    be = SimulatedBackend({R360: 0.0005, R720: 0.001, R1080: 0.002}, {R360: 1, R720: 2, R1080: 4}, parallel=4)
    rep = Scheduler(be, mem_budget=64).run(reqs(arr, res))
    s = rep.summary()
    assert s["requests"] == n
    lat = rep.latencies_ms()
    assert s["p50_ms"] == pytest.approx(np.percentile(lat, 50)) and s["p99_ms"] >= s["p50_ms"]
    # light load: every request is served at its own service time
    svc = {R360: 0.5, R720: 1.0, R1080: 2.0}
    assert np.allclose(lat, [svc[r.resolution] for r in rep.results], atol=1e-6) or s["p99_ms"] < 10
    assert s["frames_per_s"] == pytest.approx(n / rep.makespan)
