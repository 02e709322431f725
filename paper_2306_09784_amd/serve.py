"""Continuous-batching serving loop over the rc C ABI.

Many sensors emit radar frames (each one synthetic aperture) at their own
times; the server admits frames into the plan's frame slots as slots free up,
copies each admitted frame's beat cube from pinned host memory to its device
slot (the paper's pinned-memory "Load", Sec. IV), enqueues the admitted frames
as one batch on one of several HIP streams, so batches overlap on the GPU, and
harvests completed frames (detections on the host) as they finish.

Admission is bounded by HBM.  With a plan of ``RC_MEMORY_BUDGET`` (the
server's ``hbm_budget_bytes``), the library holds one device arena of that size
and admits each frame by the bytes its own sizes need (``rc_frame_bytes``:
table, pixel tables, partial images, detection buffers and the beat cube,
which the library copies from the sensor's pinned host memory itself), so
small frames do not pay for the largest one; a batch that does not fit what is
free is not enqueued (``RC_ENOTREADY``) and waits.  Without a budget, the
plan's fixed slots (each sized for the largest frame) bound the frames in
flight and the server copies each cube into a per-slot device buffer.  A frame
that cannot be admitted waits in a FIFO queue; its latency counts from its
arrival.

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
    raw_dev: object = None  # the beat cube already in HBM (Server(resident=True))


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

    def __init__(self, plan_cfg: "_rc.PlanConfig", n_streams: int = 2, keep_images: bool = False,
                 resident: bool = False):
        import torch

        self.torch = torch
        self.cfg = plan_cfg
        self.plan = _rc.Plan(plan_cfg)
        self.n_slots = plan_cfg.max_frames_in_flight
        self.resident = resident
        # a budget plan takes each cube from pinned host memory itself
        self.by_bytes = plan_cfg.frame_memory == _rc.RC_MEMORY_BUDGET
        dev = torch.device("cuda")
        n_in = plan_cfg.n_chirps_max * plan_cfg.n_channels_max * plan_cfg.n_samples_max
        # device input buffer per slot (the raw cube is copied in from pinned
        # memory), unless every sensor's cube is already resident in HBM or the
        # plan copies it into its own budget
        self.inputs = [] if resident or self.by_bytes else [
            torch.empty(n_in, dtype=torch.complex64, device=dev) for _ in range(self.n_slots)]
        self.images = [torch.empty((plan_cfg.n_pix_max, 2), dtype=torch.float32, device=dev)
                       for _ in range(self.n_slots)] if keep_images else None
        self.free = list(range(self.n_slots))
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        # the cubes' host-to-device copies run on a stream of their own: a
        # batch's kernels wait for its copies by an event, and the copies of
        # the next batch proceed while the current one computes
        self.copy_stream = torch.cuda.Stream()
        self.next_stream = 0
        self.inflight: Dict[int, tuple] = {}   # frame_id -> (slot, sensor_id, arrival, admitted)
        # per stream, the frame ids of its batches in submission order: a
        # stream's batches complete in that order, and a batch's frames together
        self.pending = [collections.deque() for _ in range(n_streams)]
        self.results: List[Completed] = []
        self.image_of: Dict[int, np.ndarray] = {}

    def close(self):
        self.torch.cuda.synchronize()
        self.plan.close()

    def submit(self, items) -> bool:
        """items: list of (frame_id, SensorStream, arrival_time), at most as many
        as free slots.  Admits all of them at once and returns True, or (a
        budget plan without room for them) none and returns False."""
        torch = self.torch
        if not items:
            return True
        stream = self.streams[self.next_stream]
        descs, taken = [], []
        now = time.perf_counter()
        copied = False
        with torch.cuda.stream(stream):
            for fid, sens, arrival in items:
                slot = self.free.pop()
                taken.append(slot)
                fr = sens.frame
                host = None
                if self.resident:
                    dst = sens.raw_dev
                elif self.by_bytes:
                    dst, host = None, sens.raw_pinned
                else:
                    # a free slot's buffer is no longer read by its last frame
                    dst = self.inputs[slot][:fr.raw.size]
                    with torch.cuda.stream(self.copy_stream):
                        dst.copy_(sens.raw_pinned.reshape(-1), non_blocking=True)
                    copied = True
                img = self.images[slot] if self.images is not None else None
                descs.append(_rc.Plan.make_frame(
                    fid, data=dst, q_tx=fr.q_tx, q_rx=fr.q_rx, vel=fr.vel, pixels=sens.pix_dev,
                    n_rows=fr.n_rows, n_cols=fr.n_cols, n_bins=fr.n_bins, n_fft=fr.n_fft, fs=fr.fs,
                    n_samples=fr.cfg.n_samples, image_out=img, sensor_id=sens.sensor_id,
                    height=fr.cfg.height, data_host=host))
        if copied:
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
            stream.wait_event(ev)
        if self.plan.try_process(descs, stream) != _rc.RC_OK:
            self.free.extend(reversed(taken))
            return False
        self.pending[self.next_stream].append([fid for fid, _, _ in items])
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        for (fid, sens, arrival), slot in zip(items, taken):
            self.inflight[fid] = (slot, sens.sensor_id, arrival, now)
        return True

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
        """Collects every completed frame (all in flight if block); returns how
        many.  Polls only the oldest batch of each stream: the later ones of a
        stream cannot have completed before it."""
        n = 0
        for q in self.pending:
            while q:
                batch = [f for f in q[0] if f in self.inflight]
                if batch and not block and not self.plan.poll(batch[-1]):
                    break
                q.popleft()
                for fid in batch:
                    self._complete(fid)
                n += len(batch)
        return n

    def harvest_until(self, max_inflight: int) -> int:
        """Waits for the oldest frames in flight until at most max_inflight remain."""
        n = 0
        while len(self.inflight) > max_inflight:
            self._complete(next(iter(self.inflight)))
            n += 1
        return n


def run_poisson(server: Server, sensors: List[SensorStream], rate_hz: float, duration_s: float,
                seed: int = 4000, max_batch: Optional[int] = None, max_wait_s: float = 2e-3,
                poll_s: float = 1e-4) -> dict:
    """Open-loop Poisson arrivals at rate_hz (sensors chosen uniformly) for
    duration_s; returns throughput and latency statistics.  Waiting frames are
    admitted as a batch when a full batch (max_batch) is waiting, when no batch
    is in flight, or when fewer batches than streams are in flight and the
    oldest has waited max_wait_s: under load the batches grow with the frames
    that arrive while others run (a batch's fixed costs are paid per batch),
    when idle a frame goes at once."""
    rng = np.random.default_rng(seed)
    n_expected = int(rate_hz * duration_s * 1.2) + 16
    gaps = rng.exponential(1.0 / rate_hz, n_expected)
    arrivals = np.cumsum(gaps)
    arrivals = arrivals[arrivals < duration_s]
    who = rng.integers(0, len(sensors), len(arrivals))
    queue = collections.deque()
    sizes = []   # frames per admitted batch
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
        in_flight = sum(len(q) for q in server.pending)
        ready = queue and (len(queue) >= max_batch or not server.inflight or
                           (in_flight < len(server.streams) and now - (queue[0][2] - t0) >= max_wait_s))
        if ready and server.free:
            # the largest leading part of the queue that fits (a budget plan
            # admits by bytes: halve the batch until it fits, or wait)
            k = min(len(queue), len(server.free), max_batch)
            while k and not server.submit([queue[j] for j in range(k)]):
                k //= 2
            for _ in range(k):
                queue.popleft()
            if k:
                sizes.append(k)
            else:
                server.harvest_until(max(0, len(server.inflight) - 1))
        elif not queue and i < len(arrivals) and not server.inflight:
            time.sleep(max(0.0, min(arrivals[i] - (time.perf_counter() - t0), 1e-3)))
        elif server.inflight:
            time.sleep(poll_s)  # between polls of the GPU, rather than spinning on the runtime
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
        "batches": len(sizes),
        "mean_batch": float(np.mean(sizes)) if sizes else None,
    }


# ---------------------------------------------------------------------------
# Continuous SAR: sensors streaming sub-apertures (rc_sliding)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class SubAperture:
    """One sub-aperture of a drive: beat cube in pinned host memory, geometry."""

    raw_pinned: object     # torch pinned CPU tensor, complex64 [S, CH, N_s]
    q_tx: np.ndarray       # float32 [S, CH, 2]
    q_rx: np.ndarray
    vel: np.ndarray        # float32 [S, 2]


@dataclasses.dataclass
class ContinuousSensor:
    """A sensor that emits the sub-apertures of `drive` one hop apart, starting
    at index `offset`; index 0 of the drive starts a new stream."""

    sensor_id: int
    drive: List[SubAperture]
    frame: object          # synth.Frame giving the sizes, lattice and radar constants
    pix_dev: object
    offset: int = 0


class ContinuousServer:
    """Admits sub-apertures of many sensors into the plan's slots (at most the
    plan's sliding_depth of one sensor at a time, in each sensor's order),
    copies each beat cube from pinned memory into its slot and keeps batches in
    flight on several streams; the plan forms every aperture."""

    def __init__(self, plan_cfg: "_rc.PlanConfig", n_streams: int = 2, keep_images: bool = False):
        import torch

        self.torch = torch
        self.plan = _rc.Plan(plan_cfg)
        self.n_slots = plan_cfg.max_frames_in_flight
        self.depth = plan_cfg.sliding_depth
        dev = torch.device("cuda")
        n_in = plan_cfg.n_chirps_max * plan_cfg.n_channels_max * plan_cfg.n_samples_max
        self.inputs = [torch.empty(n_in, dtype=torch.complex64, device=dev) for _ in range(self.n_slots)]
        self.images = [torch.empty((plan_cfg.n_pix_max, 2), dtype=torch.float32, device=dev)
                       for _ in range(self.n_slots)] if keep_images else None
        self.image_of: Dict[int, np.ndarray] = {}
        self.sub_of: Dict[int, tuple] = {}     # frame_id -> (drive index, rc_sliding mode)
        self.free = list(range(self.n_slots))
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.next_stream = 0
        self.inflight: Dict[int, tuple] = {}   # frame_id -> (slot, sensor_id, arrival)
        self.per_sensor = collections.Counter()
        self.started = set()                     # sensors whose stream has begun
        self.results: List[Completed] = []

    def close(self):
        self.torch.cuda.synchronize()
        self.plan.close()

    def admissible(self, sensor_id: int) -> bool:
        return bool(self.free) and self.per_sensor[sensor_id] < self.depth

    def submit(self, items):
        """items: (frame_id, ContinuousSensor, drive index, arrival time)."""
        if not items:
            return
        torch = self.torch
        stream = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        descs = []
        with torch.cuda.stream(stream):
            for fid, sens, k, arrival in items:
                slot = self.free.pop()
                sub = sens.drive[k]
                fr = sens.frame
                dst = self.inputs[slot][:sub.raw_pinned.numel()]
                dst.copy_(sub.raw_pinned.reshape(-1), non_blocking=True)
                mode = _rc.RC_SLIDE_START if k == 0 or sens.sensor_id not in self.started else _rc.RC_SLIDE_NEXT
                img = self.images[slot] if self.images is not None else None
                descs.append(_rc.Plan.make_frame(
                    fid, data=dst, q_tx=sub.q_tx, q_rx=sub.q_rx, vel=sub.vel, pixels=sens.pix_dev,
                    n_rows=fr.n_rows, n_cols=fr.n_cols, n_bins=fr.n_bins, n_fft=fr.n_fft, fs=fr.fs,
                    n_samples=fr.cfg.n_samples, sensor_id=sens.sensor_id, height=fr.cfg.height,
                    image_out=img, sliding=mode))
                self.started.add(sens.sensor_id)
                self.sub_of[fid] = (k, mode)
                self.inflight[fid] = (slot, sens.sensor_id, arrival)
                self.per_sensor[sens.sensor_id] += 1
        self.plan.process(descs, stream)

    def harvest(self) -> int:
        n = 0
        for fid in list(self.inflight):
            if not self.plan.poll(fid):
                continue
            slot, sid, arrival = self.inflight.pop(fid)
            dets = self.plan.detections(fid)
            done = time.perf_counter()
            if self.images is not None:
                self.torch.cuda.synchronize()
                self.image_of[fid] = self.images[slot].cpu().numpy().copy()
            self.plan.release(fid)
            self.free.append(slot)
            self.per_sensor[sid] -= 1
            self.results.append(Completed(fid, sid, arrival, arrival, done, dets))
            n += 1
        return n


def run_continuous(server: ContinuousServer, sensors: List[ContinuousSensor], hop_s: float, duration_s: float,
                   seed: int = 4100, max_batch: Optional[int] = None) -> dict:
    """Each sensor emits its next sub-aperture every hop_s (the radar time a
    sub-aperture takes), from a random phase; sub-apertures wait in arrival
    order and are admitted as slots and each sensor's depth allow.  Returns
    throughput and latency (arrival to detections on the host) statistics."""
    rng = np.random.default_rng(seed)
    events = []
    for s in sensors:
        phase = rng.uniform(0.0, hop_s)
        n = int((duration_s - phase) / hop_s) + 1
        for j in range(n):
            t = phase + j * hop_s
            if t < duration_s:
                events.append((t, s, (s.offset + j) % len(s.drive)))
    events.sort(key=lambda e: e[0])
    queue = collections.deque()
    max_batch = max_batch or server.n_slots
    t0 = time.perf_counter()
    i, fid = 0, 1
    while i < len(events) or queue or server.inflight:
        now = time.perf_counter() - t0
        while i < len(events) and events[i][0] <= now:
            t, s, k = events[i]
            queue.append((fid, s, k, t0 + t))
            fid += 1
            i += 1
        server.harvest()
        batch, held = [], set()
        # in arrival order; a sensor whose earlier sub-aperture must wait holds
        # back its later ones
        for item in list(queue):
            if len(batch) == max_batch or not server.free or len(batch) == len(server.free):
                break
            sid = item[1].sensor_id
            if sid in held:
                continue
            if server.per_sensor[sid] + sum(1 for b in batch if b[1].sensor_id == sid) < server.depth:
                batch.append(item)
            else:
                held.add(sid)
        for item in batch:
            queue.remove(item)
        if batch:
            server.submit(batch)
        elif not queue and i < len(events) and not server.inflight:
            time.sleep(max(0.0, min(events[i][0] - (time.perf_counter() - t0), 1e-3)))
    wall = time.perf_counter() - t0
    lat = np.array([r.done - r.arrival for r in server.results])
    per_sensor = collections.defaultdict(list)
    for r in server.results:
        per_sensor[r.sensor_id].append(r.done - r.arrival)
    return {
        "sensors": len(sensors),
        "subapertures": len(server.results),
        "wall_s": wall,
        "apertures_per_s": len(server.results) / wall,
        "offered_per_s": len(sensors) / hop_s,
        "hop_ms": 1e3 * hop_s,
        "p50_ms": 1e3 * float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": 1e3 * float(np.percentile(lat, 99)) if len(lat) else None,
        "max_ms": 1e3 * float(lat.max()) if len(lat) else None,
        "worst_sensor_p99_ms": 1e3 * max(float(np.percentile(v, 99)) for v in per_sensor.values())
        if per_sensor else None,
    }
