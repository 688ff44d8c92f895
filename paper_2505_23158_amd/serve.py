"""Continuous-batching render server over one resident LOD scene.

Requests (camera + resolution) arrive over time.  Each resolution class owns
render slots; a slot is a workspace, a selection, output buffers, a HIP
stream and a captured HIP graph of one frame (lodge_select + lodge_render
with the camera taken from the workspace).  The scheduler admits a waiting
request as soon as a slot of its class is free, or creates a new slot when
the memory budget allows; it stores the request's camera in the slot's
workspace (lodge_set_camera) and replays the slot's graph on the slot's
stream, so requests of different resolutions that arrive while others are on
the GPU run concurrently.
Completion is detected by polling the slot's event; latency is completion
minus arrival (the device-to-host copy of the image is not included, as in
the paper's timing protocol).  A frame whose capacities overflowed is
rendered again on its slot, which is rebuilt with capacities grown to what
the frame needed: the slot stays busy meanwhile (other slots keep being
admitted and polled), the grown slot renders eagerly from then on, the
class's capacities grow for slots created later, and the extra device bytes
count against the memory budget.  A request that still overflows after a
few growths fails loudly.

The scheduler talks to a backend with four calls (slot_bytes, new_slot,
launch, poll), so its admission and bookkeeping are tested on the CPU with
``SimulatedBackend``.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    cam: object             # synth.Camera-like
    resolution: Tuple[int, int] = (0, 0)

    def __post_init__(self):
        if self.resolution == (0, 0):
            self.resolution = (int(self.cam.width), int(self.cam.height))


@dataclass
class Result:
    rid: int
    arrival: float
    start: float
    done: float
    slot: int
    resolution: Tuple[int, int]
    retried: bool = False

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class Report:
    results: List[Result]
    makespan: float
    slots_created: Dict[Tuple[int, int], int]
    peak_in_flight: int
    mem_bytes: int

    def latencies_ms(self) -> np.ndarray:
        return np.array([r.latency for r in self.results]) * 1e3

    def summary(self) -> dict:
        lat = self.latencies_ms()
        return {"requests": len(self.results), "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
                "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
                "mean_ms": float(lat.mean()) if len(lat) else None,
                "frames_per_s": len(self.results) / self.makespan if self.makespan > 0 else None,
                "makespan_s": self.makespan, "peak_in_flight": self.peak_in_flight,
                "slots": {f"{w}x{h}": n for (w, h), n in self.slots_created.items()},
                "retries": sum(r.retried for r in self.results), "slot_memory_bytes": self.mem_bytes}


class Scheduler:
    """Admission by free slot and memory budget; FIFO within a resolution class."""

    def __init__(self, backend, mem_budget: int, max_slots_per_class: int = 16, spin_sleep: float = 0.0,
                 prewarmed: Optional[Dict[Tuple[int, int], List[int]]] = None):
        self.backend = backend
        self.mem_budget = mem_budget
        self.max_slots = max_slots_per_class
        self.spin_sleep = spin_sleep
        self.prewarmed = prewarmed or {}

    def run(self, requests: Sequence[Request]) -> Report:
        be = self.backend
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting: Dict[Tuple[int, int], deque] = {}
        free: Dict[Tuple[int, int], List[int]] = {r: list(s) for r, s in self.prewarmed.items()}
        n_slots: Dict[Tuple[int, int], int] = {r: len(s) for r, s in self.prewarmed.items()}
        busy: Dict[int, Tuple[Request, float]] = {}
        results: List[Result] = []
        mem = sum(be.slot_bytes(r) * len(s) for r, s in self.prewarmed.items())
        peak = 0
        t0 = be.now()
        n = len(pending)
        while len(results) < n:
            now = be.now() - t0
            progressed = False
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                waiting.setdefault(r.resolution, deque()).append(r)
                progressed = True
            for sid in list(busy):
                fin = be.poll(sid)
                if fin is not None:
                    req, start = busy.pop(sid)
                    done_t, retried, grown = fin
                    mem += grown
                    results.append(Result(req.rid, req.arrival, start, done_t - t0, sid, req.resolution, retried))
                    free.setdefault(req.resolution, []).append(sid)
                    progressed = True
            for res, q in waiting.items():
                while q:
                    slots = free.setdefault(res, [])
                    if not slots:
                        need = be.slot_bytes(res)
                        if n_slots.get(res, 0) >= self.max_slots or mem + need > self.mem_budget:
                            break
                        slots.append(be.new_slot(res))
                        n_slots[res] = n_slots.get(res, 0) + 1
                        mem += need
                    sid = slots.pop()
                    req = q.popleft()
                    be.launch(sid, req)
                    busy[sid] = (req, be.now() - t0)
                    peak = max(peak, len(busy))
                    progressed = True
            if not progressed:
                nxt = pending[0].arrival if pending else None
                be.idle(t0, nxt, bool(busy))
                if self.spin_sleep:
                    time.sleep(self.spin_sleep)
            if not busy and not pending and any(waiting.values()) and not progressed:
                raise RuntimeError("requests cannot be admitted: memory budget below one slot of their resolution")
        makespan = max(r.done for r in results) - min(r.arrival for r in results) if results else 0.0
        results.sort(key=lambda r: r.rid)
        return Report(results, makespan, n_slots, peak, mem)


class SimulatedBackend:
    """Virtual-time backend: a slot serves one request in `service[res]`
    seconds; up to `parallel` launches make progress at once (the rest wait
    in a device queue), which is how overlapping streams behave."""

    def __init__(self, service: Dict[Tuple[int, int], float], slot_mem: Dict[Tuple[int, int], int], parallel: int = 4,
                 fail_first: Optional[set] = None, grow_bytes: int = 0):
        self.service = service
        self.mem = slot_mem
        self.parallel = parallel
        self.t = 0.0
        self.slots: Dict[int, Tuple[int, int]] = {}
        self.running: Dict[int, float] = {}      # sid -> remaining service
        self.done_at: Dict[int, float] = {}
        self.order: List[Tuple[int, int]] = []    # (rid, sid) launch order
        self.fail_first = set(fail_first or ())
        self.grow_bytes = grow_bytes          # device bytes a retried request's slot grows by
        self.retried: Dict[int, bool] = {}

    def now(self):
        return self.t

    def slot_bytes(self, res):
        return self.mem[res]

    def new_slot(self, res):
        sid = len(self.slots)
        self.slots[sid] = res
        return sid

    def launch(self, sid, req):
        extra = 0.0
        retried = req.rid in self.fail_first
        if retried:        # capacity overflow: the frame is rendered again outside the graph
            extra = self.service[req.resolution]
        self.running[sid] = self.service[req.resolution] + extra
        self.retried[sid] = retried
        self.order.append((req.rid, sid))

    def poll(self, sid):
        if sid in self.done_at:
            t = self.done_at.pop(sid)
            r = self.retried.pop(sid)
            return t, r, self.grow_bytes if r else 0
        return None

    def idle(self, t0, next_arrival, any_busy):
        # advance virtual time to the next event: an arrival or a completion
        active = sorted(self.running.items())[: self.parallel]
        t_next = [next_arrival] if next_arrival is not None else []
        if active:
            t_next.append(self.t + min(rem for _, rem in active))
        if not t_next:
            return
        dt = max(0.0, min(t_next) - self.t)
        for sid, rem in active:
            self.running[sid] = rem - dt
        self.t += dt
        for sid in [s for s, rem in self.running.items() if rem <= 1e-12]:
            del self.running[sid]
            self.done_at[sid] = self.t


class GpuBackend:
    """Slots on the GPU: per-slot workspace, pinned camera, stream and graph.  copy_to_host: each frame's
    image also goes to a pinned host buffer of its slot, and a request completes when that copy has."""

    MAX_GROWTHS = 4

    def __init__(self, scene, mode: int, caps: Dict[Tuple[int, int], Tuple[int, int]], use_graphs: bool = True,
                 keep_images: bool = False, copy_to_host: bool = False):
        import torch
        from . import lodge as L
        self.torch, self.L = torch, L
        self.scene, self.mode = scene, mode
        self.caps = dict(caps)
        self.use_graphs = use_graphs
        self.keep_images = keep_images
        self.copy_to_host = copy_to_host
        self.slots = []
        self.images: Dict[int, object] = {}
        self.outputs: Dict[int, dict] = {}

    def now(self):
        return time.perf_counter()

    def _bytes(self, res, caps):
        import ctypes as C
        w, h = res
        ma, mi = caps
        L = self.L
        nb = C.c_size_t()
        L._check(L.lib().lodge_workspace_size(self.scene.handle, w, h, ma, mi, C.byref(nb)))
        return int(nb.value) + 8 * ma + 4 * 5 * w * h

    def slot_bytes(self, res):
        return self._bytes(res, self.caps[res])

    def _make(self, res, caps):
        torch, L = self.torch, self.L
        w, h = res
        return L.Renderer(self.scene, w, h, max_active=caps[0], max_instances=caps[1])

    def prewarm(self, res, k: int):
        """Creates k slots of a class ahead of the run (returned to the scheduler's free lists)."""
        return [self.new_slot(res) for _ in range(k)]

    def new_slot(self, res):
        torch, L = self.torch, self.L
        caps = self.caps[res]
        R = self._make(res, caps)
        stream = torch.cuda.Stream()
        graph = None
        if self.use_graphs:
            # any valid camera of this size; the graph reads whatever camera is set before a replay
            c = L.lodge_camera(width=res[0], height=res[1], fx=float(res[0]), fy=float(res[0]), cx=res[0] / 2.0,
                               cy=res[1] / 2.0, znear=0.2, lim_x=1.0, lim_y=1.0)
            c.R[0] = c.R[4] = c.R[8] = 1.0
            with torch.cuda.stream(stream):
                R.frame(c, self.mode)            # warm-up outside the capture
            stream.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                R.frame(None, self.mode)
        done = torch.cuda.Event()
        host = None
        if self.copy_to_host:
            host = torch.empty((3, res[1], res[0]), dtype=torch.float32, pin_memory=True)
            # the first copy into a fresh pinned buffer pays a one-time cost: take it here, not in a request
            with torch.cuda.stream(stream):
                host.copy_(R.image, non_blocking=True)
            stream.synchronize()
        sid = len(self.slots)
        self.slots.append({"res": res, "R": R, "caps": caps, "stream": stream, "graph": graph, "done": done,
                           "req": None, "growths": 0, "grown_bytes": 0, "host": host})
        return sid

    def _render(self, s, cam):
        with self.torch.cuda.stream(s["stream"]):
            if s["graph"] is not None:
                self.L.lodge_set_camera(s["R"].ws, cam, s["stream"])
                s["graph"].replay()
            else:
                s["R"].frame(cam, self.mode, stream=s["stream"])
            if s["host"] is not None:
                s["host"].copy_(s["R"].image, non_blocking=True)
            s["done"].record()

    def launch(self, sid, req):
        s = self.slots[sid]
        s["req"] = req
        s["growths"] = 0
        self._render(s, req.cam)

    def _grow(self, s, na, ni):
        """Replaces the slot's renderer by one with the capacities the frame needed (a selection overflow
        truncates the projected set, so its instance count is only a lower bound: the instance capacity at
        least doubles then).  The grown slot renders eagerly from now on."""
        res = s["res"]
        ma, mi = s["caps"]
        sel_ovf = na > ma
        new_ma = max(ma, na)
        new_mi = max(mi, int(ni * 1.25) + 1)
        if sel_ovf:
            new_mi = max(new_mi, 2 * mi)
        new_mi = min(new_mi, (1 << 32) - 1)
        caps = (new_ma, new_mi)
        grown = self._bytes(res, caps) - self._bytes(res, s["caps"])
        s["R"] = self._make(res, caps)
        s["graph"] = None
        s["caps"] = caps
        s["grown_bytes"] += grown
        cur = self.caps[res]
        self.caps[res] = (max(cur[0], caps[0]), max(cur[1], caps[1]))

    def poll(self, sid):
        s = self.slots[sid]
        if not s["done"].query():
            return None
        t = time.perf_counter()
        L = self.L
        st, na, ni = L.lodge_check(s["R"].ws, stream=s["stream"])
        if st == L.LODGE_ERR_CAPACITY:
            if s["growths"] >= self.MAX_GROWTHS:
                raise RuntimeError(f"request {s['req'].rid}: capacity still exceeded after {s['growths']} growths "
                                   f"(needs {na} active, {ni} instances)")
            s["growths"] += 1
            self._grow(s, na, ni)
            self._render(s, s["req"].cam)     # the slot stays busy until the re-render completes
            return None
        if st != L.LODGE_OK:
            L._check(st)
        if self.keep_images:
            # copies ordered on the slot's stream, before its next launch overwrites the outputs
            R = s["R"]
            with self.torch.cuda.stream(s["stream"]):
                n = min(int(R.sel.count[0].item()), R.sel.cap)
                self.images[s["req"].rid] = R.image.clone()
                self.outputs[s["req"].rid] = {"image": R.image.clone(), "final_T": R.final_T.clone(),
                                              "n_contrib": R.n_contrib.clone(), "ids": R.sel.ids[:n].clone(),
                                              "w": R.sel.w[:n].clone(), "caps": s["caps"]}
        grown, s["grown_bytes"] = s["grown_bytes"], 0
        return t, s["growths"] > 0, grown

    def idle(self, t0, next_arrival, any_busy):
        if not any_busy and next_arrival is not None:
            wait = next_arrival - (time.perf_counter() - t0)
            if wait > 2e-4:
                time.sleep(wait - 1e-4)


def serve(scene, requests: Sequence[Request], mode: int, caps, mem_budget: int = 64 << 30,
          max_slots_per_class: int = 8, prewarm: int = 2, use_graphs: bool = True, keep_images: bool = False):
    """Serves `requests` (arrival times relative to the start) and returns (Report, backend)."""
    be = GpuBackend(scene, mode, caps, use_graphs=use_graphs, keep_images=keep_images)
    classes = sorted({r.resolution for r in requests})
    pre = {res: be.prewarm(res, prewarm) for res in classes}
    be.torch.cuda.synchronize()
    rep = Scheduler(be, mem_budget, max_slots_per_class, prewarmed=pre).run(requests)
    return rep, be
