"""Continuous-batching serving loop over the rc C ABI.

Many sensors emit radar frames (each one synthetic aperture) at their own
times; the server admits frames into the plan's frame slots as slots free up,
copies each admitted frame's beat cube from pinned host memory to its device
slot (the paper's pinned-memory "Load", Sec. IV), enqueues the admitted frames
as one batch on one of several HIP streams, so batches overlap on the GPU, and
harvests completed frames (detections on the host) as they finish.

Admission is bounded by HBM: the number of frame slots is the HBM budget
divided by the device bytes of one slot (``rc_plan_slot_bytes``) plus the
device input buffer of one frame.  A frame that arrives while every slot is
busy waits in a FIFO queue; its latency counts from its arrival.

All compute runs in librc's kernels; this module only moves buffers, keeps
the clock and does the bookkeeping.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import rc as _rc


@dataclasses.dataclass
class SensorStream:
    """One sensor: its frame (beat cube in pinned host memory, geometry, grid)."""

    sensor_id: int
    frame: object          # synth.Frame
    raw_pinned: object     # torch pinned CPU tensor, complex64 [M, CH, N_s]
    pix_dev: object        # torch device tensor, float32 [n_pix, 2]


@dataclasses.dataclass
class Completed:
    frame_id: int
    sensor_id: int
    arrival: float
    admitted: float
    done: float
    detections: np.ndarray


class Server:
    """Admits frames into the plan's slots and keeps several batches in flight."""

    def __init__(self, plan_cfg: "_rc.PlanConfig", n_streams: int = 2, keep_images: bool = False):
        import torch

        self.torch = torch
        self.cfg = plan_cfg
        self.plan = _rc.Plan(plan_cfg)
        self.n_slots = plan_cfg.max_frames_in_flight
        dev = torch.device("cuda")
        n_in = plan_cfg.n_chirps_max * plan_cfg.n_channels_max * plan_cfg.n_samples_max
        # device input buffer per slot (the raw cube is copied in from pinned memory)
        self.inputs = [torch.empty(n_in, dtype=torch.complex64, device=dev) for _ in range(self.n_slots)]
        self.images = [torch.empty((plan_cfg.n_pix_max, 2), dtype=torch.float32, device=dev)
                       for _ in range(self.n_slots)] if keep_images else None
        self.free = list(range(self.n_slots))
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.next_stream = 0
        self.inflight: Dict[int, tuple] = {}   # frame_id -> (slot, sensor_id, arrival, admitted)
        self.results: List[Completed] = []
        self.image_of: Dict[int, np.ndarray] = {}

    def close(self):
        self.torch.cuda.synchronize()
        self.plan.close()

    def submit(self, items):
        """items: list of (frame_id, SensorStream, arrival_time); all admitted
        at once (the caller guarantees len(items) <= free slots)."""
        torch = self.torch
        if not items:
            return
        stream = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        descs = []
        now = time.perf_counter()
        with torch.cuda.stream(stream):
            for fid, sens, arrival in items:
                slot = self.free.pop()
                fr = sens.frame
                n = fr.raw.size
                dst = self.inputs[slot][:n]
                dst.copy_(sens.raw_pinned.reshape(-1), non_blocking=True)
                img = self.images[slot] if self.images is not None else None
                descs.append(_rc.Plan.make_frame(
                    fid, data=dst, q_tx=fr.q_tx, q_rx=fr.q_rx, vel=fr.vel, pixels=sens.pix_dev,
                    n_rows=fr.n_rows, n_cols=fr.n_cols, n_bins=fr.n_bins, n_fft=fr.n_fft, fs=fr.fs,
                    n_samples=fr.cfg.n_samples, image_out=img, sensor_id=sens.sensor_id,
                    height=fr.cfg.height))
                self.inflight[fid] = (slot, sens.sensor_id, arrival, now)
        self.plan.process(descs, stream)

    def _complete(self, fid: int) -> None:
        slot, sid, arrival, admitted = self.inflight.pop(fid)
        dets = self.plan.detections(fid)
        done = time.perf_counter()
        if self.images is not None:
            self.torch.cuda.synchronize()
            self.image_of[fid] = self.images[slot].cpu().numpy().copy()
        self.plan.release(fid)
        self.free.append(slot)
        self.results.append(Completed(fid, sid, arrival, admitted, done, dets))

    def harvest(self, block: bool = False) -> int:
        """Collects every completed frame (all in flight if block); returns how many."""
        n = 0
        for fid in list(self.inflight):
            if not block and not self.plan.poll(fid):
                continue
            self._complete(fid)
            n += 1
        return n

    def harvest_until(self, max_inflight: int) -> int:
        """Waits for the oldest frames in flight until at most max_inflight remain."""
        n = 0
        while len(self.inflight) > max_inflight:
            self._complete(next(iter(self.inflight)))
            n += 1
        return n


def run_poisson(server: Server, sensors: List[SensorStream], rate_hz: float, duration_s: float,
                seed: int = 4000, max_batch: Optional[int] = None) -> dict:
    """Open-loop Poisson arrivals at rate_hz (sensors chosen uniformly) for
    duration_s; returns throughput and latency statistics."""
    rng = np.random.default_rng(seed)
    n_expected = int(rate_hz * duration_s * 1.2) + 16
    gaps = rng.exponential(1.0 / rate_hz, n_expected)
    arrivals = np.cumsum(gaps)
    arrivals = arrivals[arrivals < duration_s]
    who = rng.integers(0, len(sensors), len(arrivals))
    queue = collections.deque()
    t0 = time.perf_counter()
    i = 0
    fid = 1
    max_batch = max_batch or server.n_slots
    while i < len(arrivals) or queue or server.inflight:
        now = time.perf_counter() - t0
        while i < len(arrivals) and arrivals[i] <= now:
            queue.append((fid, sensors[who[i]], t0 + arrivals[i]))
            fid += 1
            i += 1
        server.harvest()
        if queue and server.free:
            k = min(len(queue), len(server.free), max_batch)
            server.submit([queue.popleft() for _ in range(k)])
        elif not queue and i < len(arrivals) and not server.inflight:
            time.sleep(max(0.0, min(arrivals[i] - (time.perf_counter() - t0), 1e-3)))
    wall = time.perf_counter() - t0
    lat = np.array([r.done - r.arrival for r in server.results])
    per_sensor = collections.defaultdict(list)
    for r in server.results:
        per_sensor[r.sensor_id].append(r.done - r.arrival)
    return {
        "frames": len(server.results),
        "wall_s": wall,
        "frames_per_s": len(server.results) / wall,
        "offered_rate_hz": rate_hz,
        "p50_ms": 1e3 * float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": 1e3 * float(np.percentile(lat, 99)) if len(lat) else None,
        "max_ms": 1e3 * float(lat.max()) if len(lat) else None,
        "worst_sensor_p99_ms": 1e3 * max(float(np.percentile(v, 99)) for v in per_sensor.values())
        if per_sensor else None,
    }
