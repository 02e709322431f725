"""The serving loop's admission logic on the host, against a stand-in server
that completes each batch a fixed time after it starts on its stream (no
GPU): every arriving frame is admitted once and completes; no batch exceeds
max_batch or the free slots; under load batches grow; a server that refuses a batch (an HBM budget
without room) gets a smaller one, or the loop waits for a completion; the loop
ends with nothing in flight."""
import collections
import dataclasses
import time

import numpy as np

from paper_2306_09784_amd import serve


@dataclasses.dataclass
class _Sensor:
    sensor_id: int


class _StandIn:
    """The part of serve.Server that run_poisson uses.  A batch occupies its
    stream for `service_s` after the stream's previous batch; `cap_frames`
    (when set) refuses a batch that would hold more frames in flight."""

    def __init__(self, n_slots=16, n_streams=2, service_s=2e-3, cap_frames=None):
        self.n_slots = n_slots
        self.free = list(range(n_slots))
        self.streams = [object() for _ in range(n_streams)]
        self.pending = [collections.deque() for _ in range(n_streams)]
        self.inflight = {}
        self.results = []
        self.next_stream = 0
        self.service_s = service_s
        self.cap_frames = cap_frames
        self.stream_free_at = [0.0] * n_streams
        self.done_at = {}
        self.sizes = []
        self.refused = 0

    def submit(self, items):
        assert 0 < len(items) <= len(self.free)
        if self.cap_frames is not None and len(self.inflight) + len(items) > self.cap_frames:
            self.refused += 1
            return False
        now = time.perf_counter()
        s = self.next_stream
        end = max(now, self.stream_free_at[s]) + self.service_s
        self.stream_free_at[s] = end
        for fid, sens, arrival in items:
            slot = self.free.pop()
            self.inflight[fid] = (slot, sens.sensor_id, arrival, now)
            self.done_at[fid] = end
        self.pending[s].append([fid for fid, _, _ in items])
        self.next_stream = (s + 1) % len(self.streams)
        self.sizes.append(len(items))
        return True

    def _complete(self, fid):
        slot, sid, arrival, admitted = self.inflight.pop(fid)
        while time.perf_counter() < self.done_at[fid]:
            pass
        self.free.append(slot)
        self.results.append(serve.Completed(fid, sid, arrival, admitted, time.perf_counter(), None))

    def harvest(self, block=False):
        n = 0
        now = time.perf_counter()
        for q in self.pending:
            while q:
                batch = [f for f in q[0] if f in self.inflight]
                if batch and not block and self.done_at[batch[-1]] > now:
                    break
                q.popleft()
                for f in batch:
                    self._complete(f)
                n += len(batch)
        return n

    def harvest_until(self, max_inflight):
        n = 0
        while len(self.inflight) > max_inflight:
            self._complete(next(iter(self.inflight)))
            n += 1
        return n


def _check_all_served(srv, res):
    ids = sorted(r.frame_id for r in srv.results)
    assert res["frames"] == len(ids) > 0
    assert ids == list(range(1, len(ids) + 1))          # each arrival admitted and completed once
    assert not srv.inflight and sorted(srv.free) == list(range(srv.n_slots))
    assert all(r.done >= r.admitted >= r.arrival - 1e-3 for r in srv.results)


def test_poisson_admission_serves_every_frame_in_bounded_batches():
    srv = _StandIn(n_slots=16, service_s=2e-3)
    sensors = [_Sensor(i) for i in range(5)]
    res = serve.run_poisson(srv, sensors, rate_hz=3000.0, duration_s=0.3, seed=1, max_batch=8)
    _check_all_served(srv, res)
    assert max(srv.sizes) <= 8
    assert res["batches"] == len(srv.sizes) and abs(res["mean_batch"] - np.mean(srv.sizes)) < 1e-12
    # two streams of 2 ms batches of up to 8 frames serve 8000 frames/s: 3000/s keeps up
    assert res["p99_ms"] < 100.0


def test_batches_grow_under_load_and_stay_small_when_idle():
    busy = _StandIn(n_slots=32, service_s=4e-3)
    res_busy = serve.run_poisson(busy, [_Sensor(0)], rate_hz=4000.0, duration_s=0.3, seed=2, max_batch=16)
    idle = _StandIn(n_slots=32, service_s=2e-4)
    res_idle = serve.run_poisson(idle, [_Sensor(0)], rate_hz=200.0, duration_s=0.3, seed=3, max_batch=16)
    _check_all_served(busy, res_busy)
    _check_all_served(idle, res_idle)
    assert res_busy["mean_batch"] > 4 * res_idle["mean_batch"]
    assert res_idle["mean_batch"] < 1.5          # an idle server takes a frame at once
    assert res_idle["p50_ms"] < 3.0              # no 2 ms batching wait when nothing is in flight


def test_refused_batches_shrink_or_wait():
    srv = _StandIn(n_slots=16, service_s=1e-3, cap_frames=3)
    res = serve.run_poisson(srv, [_Sensor(i) for i in range(3)], rate_hz=3000.0, duration_s=0.2, seed=4,
                            max_batch=8)
    _check_all_served(srv, res)
    assert srv.refused > 0
    assert max(srv.sizes) <= 3
