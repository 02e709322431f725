"""Continuous batching on the GPU: frames of many sensors arriving at random
times are admitted into the plan's slots while others are in flight, on two
streams; every frame's result is the same as the frame processed alone."""
import dataclasses

import numpy as np
import pytest

from paper_2306_09784_amd import synth
from tests import sar_cases as SC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def rc():
    from paper_2306_09784_amd import rc as mod

    return mod


def _sensors(torch, n, samples=(32, 64)):
    from paper_2306_09784_amd import serve

    rng = np.random.default_rng(41)
    out = []
    for i in range(n):
        cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name=f"s{i}",
                                  n_samples=int(rng.choice(samples)), n_chirps=int(rng.choice([8, 16])),
                                  n_rx=int(rng.choice([2, 4, 8])), nx=int(rng.choice([24, 40])),
                                  ny=int(rng.choice([1, 24, 33])), box=(-4.0, 4.0, 1.5, 7.0), seed=500 + i)
        fr = synth.make_frame(cfg, frame_index=i)
        out.append(serve.SensorStream(i, fr, torch.from_numpy(fr.raw).pin_memory(),
                                      torch.from_numpy(fr.pix).to("cuda")))
    return out


@pytest.mark.parametrize("precision", ["RC_PREC_FP32", "RC_PREC_FP16"])
def test_poisson_serving_results_equal_alone(rc, torch, precision):
    """Either form: plain single precision, and the spectrum formed on the
    matrix cores in FP16 (DFT lengths 256 and 512 here, the shortest it takes)."""
    from paper_2306_09784_amd import serve

    fp16 = precision == "RC_PREC_FP16"
    sensors = _sensors(torch, 6, samples=(128, 256) if fp16 else (32, 64))
    cfg = SC.plan_config(rc, [s.frame for s in sensors], max_frames_in_flight=4,
                         precision=getattr(rc, precision))
    srv = serve.Server(cfg, n_streams=2, keep_images=True)
    peak = [0]
    orig_submit = srv.submit

    def submit(items):
        ok = orig_submit(items)
        peak[0] = max(peak[0], len(srv.inflight))
        return ok

    srv.submit = submit
    try:
        res = serve.run_poisson(srv, sensors, rate_hz=400.0, duration_s=0.5, seed=7)
        assert res["frames"] == len(srv.results) > 50
        assert peak[0] <= 4                                   # admission never exceeds the slots
        assert res["p50_ms"] > 0 and res["p99_ms"] >= res["p50_ms"]
        by_sensor = {}
        for r in srv.results:
            by_sensor.setdefault(r.sensor_id, []).append(r)
        alone = {}
        for s in sensors:
            out = SC.run_gpu(rc, srv.plan, s.frame, torch, frame_id=10**7 + s.sensor_id)
            alone[s.sensor_id] = out
        for sid, rs in by_sensor.items():
            fr = sensors[sid].frame
            ref = alone[sid]["image"].view(np.float32).reshape(-1, 2)
            for r in rs[:5]:
                img = srv.image_of[r.frame_id][: fr.n_rows * fr.n_cols]
                assert np.array_equal(img, ref), (sid, r.frame_id)
                assert np.array_equal(r.detections, alone[sid]["detections"]), (sid, r.frame_id)
    finally:
        srv.close()


def test_burst_waits_for_slots(rc, torch):
    """A burst larger than the slot count queues; every frame completes."""
    from paper_2306_09784_amd import serve

    sensors = _sensors(torch, 3)
    cfg = SC.plan_config(rc, [s.frame for s in sensors], max_frames_in_flight=2)
    srv = serve.Server(cfg, n_streams=2)
    try:
        res = serve.run_poisson(srv, sensors, rate_hz=20000.0, duration_s=0.002, seed=3)
        assert res["frames"] >= 10
        assert len(srv.free) == 2 and not srv.inflight
    finally:
        srv.close()


def test_continuous_sar_serving_equals_streams_alone(rc, torch):
    """Sensors streaming sub-apertures at their own hops, admitted into shared
    batches on two streams (at most two of a sensor in flight): each aperture
    equals the one its sensor's stream gives processed alone, bitwise."""
    from paper_2306_09784_amd import serve

    K, S, n_sub = 3, 8, 6
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="drive", n_samples=64, n_chirps=n_sub * S,
                              n_rx=4, nx=40, ny=33, box=(-4.0, 4.0, 1.5, 7.0), seed=700)
    fr = synth.make_frame(cfg)
    drive = [serve.SubAperture(torch.from_numpy(np.ascontiguousarray(fr.raw[j * S:(j + 1) * S])).pin_memory(),
                               np.ascontiguousarray(fr.q_tx[j * S:(j + 1) * S]),
                               np.ascontiguousarray(fr.q_rx[j * S:(j + 1) * S]),
                               np.ascontiguousarray(fr.vel[j * S:(j + 1) * S])) for j in range(n_sub)]
    pix = torch.from_numpy(fr.pix).to("cuda")
    sensors = [serve.ContinuousSensor(i, drive, fr, pix, offset=(2 * i) % n_sub) for i in range(4)]
    pc = SC.plan_config(rc, [fr], n_chirps_max=S, max_frames_in_flight=6, sliding_sensors=4,
                        sliding_subapertures=K, sliding_depth=2)
    srv = serve.ContinuousServer(pc, n_streams=2, keep_images=True)
    try:
        res = serve.run_continuous(srv, sensors, hop_s=0.004, duration_s=0.1, seed=11, max_batch=4)
        assert res["subapertures"] == len(srv.results) >= 80
        by_sensor = {}
        for r in sorted(srv.results, key=lambda r: r.frame_id):
            by_sensor.setdefault(r.sensor_id, []).append(r)
        n_pix = fr.n_rows * fr.n_cols
        # each sensor's sequence again, alone, on a plan of one sensor
        ref_cfg = dataclasses.replace(pc, sliding_sensors=1, max_frames_in_flight=2)
        with rc.Plan(ref_cfg) as plan:
            dev = torch.device("cuda")
            for sid, rs in by_sensor.items():
                for r in rs:
                    k, mode = srv.sub_of[r.frame_id]
                    sub = drive[k]
                    img = torch.empty((n_pix, 2), dtype=torch.float32, device=dev)
                    raw = sub.raw_pinned.to(dev)
                    f = rc.Plan.make_frame(1, data=raw, q_tx=sub.q_tx, q_rx=sub.q_rx, vel=sub.vel, pixels=pix,
                                           n_rows=fr.n_rows, n_cols=fr.n_cols, n_bins=fr.n_bins, n_fft=fr.n_fft,
                                           fs=fr.fs, n_samples=cfg.n_samples, image_out=img, sliding=mode)
                    plan.process([f])
                    dets = plan.detections(1)
                    torch.cuda.synchronize()
                    plan.release(1)
                    assert np.array_equal(srv.image_of[r.frame_id][:n_pix], img.cpu().numpy()), (sid, r.frame_id)
                    assert np.array_equal(r.detections, dets), (sid, r.frame_id)
    finally:
        srv.close()
