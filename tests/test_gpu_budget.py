"""HBM-budget admission on the GPU (RC_MEMORY_BUDGET): a frame takes from the
plan's arena the bytes its own sizes need and gives them back at release.
Checked here: the same frames give bitwise the same image and detections as a
plan of fixed slots, with the input handed over on the device or in pinned
host memory (a lone frame's copied in chirp-block pieces, in every precision
form); a batch that does not fit what is free is refused without
enqueuing anything and is admitted once a frame is released; small frames
share a budget that holds only one frame of the plan's limits; the serving
loop admits by bytes; a continuous-SAR stream gives the slot plan's
apertures."""
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


def _frames():
    big = dataclasses.replace(synth.CONFIGS["plain-small"], name="big", n_samples=128, n_chirps=32, n_rx=8,
                              nx=64, ny=48, box=(-4.0, 4.0, 1.5, 7.0), seed=901)
    small = dataclasses.replace(big, name="small", n_samples=64, n_chirps=8, n_rx=2, nx=24, ny=20, seed=902)
    return synth.make_frame(big), synth.make_frame(small)


class _Inputs:
    """Device copies (and pinned host copies) of a frame's cube and pixels,
    kept alive while its work is in flight."""

    def __init__(self, fr, torch):
        self.fr = fr
        self.raw = torch.from_numpy(np.ascontiguousarray(fr.raw)).to("cuda")
        self.pinned = torch.from_numpy(np.ascontiguousarray(fr.raw)).pin_memory()
        self.pix = torch.from_numpy(np.ascontiguousarray(fr.pix)).to("cuda")

    def desc(self, rc, fid, host=False, image_out=None):
        fr = self.fr
        return rc.Plan.make_frame(fid, data=None if host else self.raw, data_host=self.pinned if host else None,
                                  q_tx=fr.q_tx, q_rx=fr.q_rx, vel=fr.vel, pixels=self.pix, n_rows=fr.n_rows,
                                  n_cols=fr.n_cols, n_bins=fr.n_bins, n_fft=fr.n_fft, fs=fr.fs,
                                  n_samples=fr.cfg.n_samples, image_out=image_out)


def _result(rc, plan, torch, fid, n_pix):
    dets = plan.detections(fid)
    img = torch.empty((n_pix, 2), dtype=torch.float32, device="cuda")
    plan.image(fid, img)
    torch.cuda.synchronize()
    return img.cpu().numpy(), dets


def test_budget_plan_equals_slot_plan(rc, torch):
    """Device and pinned-host inputs, image in the arena or the caller's buffer:
    bitwise the slot plan's image and detections."""
    big, small = _frames()
    ins = [_Inputs(f, torch) for f in (big, small)]
    base = SC.plan_config(rc, [big, small], max_frames_in_flight=4)
    ref = {}
    with rc.Plan(base) as plan:
        for k, x in enumerate(ins):
            plan.process([x.desc(rc, 1 + k)])
        for k, x in enumerate(ins):
            ref[k] = _result(rc, plan, torch, 1 + k, x.fr.n_rows * x.fr.n_cols)
            plan.release(1 + k)
    budget = dataclasses.replace(base, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=rc.slot_bytes(base) * 3)
    with rc.Plan(budget) as plan:
        for host in (False, True):
            fids = []
            for k, x in enumerate(ins):
                fid = 100 * (1 + host) + k
                plan.process([x.desc(rc, fid, host=host)])
                fids.append(fid)
            for k, (x, fid) in enumerate(zip(ins, fids)):
                img, dets = _result(rc, plan, torch, fid, x.fr.n_rows * x.fr.n_cols)
                plan.release(fid)
                assert np.array_equal(img, ref[k][0]), (host, k)
                assert np.array_equal(dets, ref[k][1]), (host, k)


@pytest.mark.parametrize("precision", ["RC_PREC_FP32_SPLIT", "RC_PREC_FP16", "RC_PREC_BF16"])
def test_host_input_in_chirp_block_pieces_equals_slot_plan(rc, torch, precision):
    """A lone frame handed over in pinned memory is copied in its chirp
    blocks' pieces, each block's range compression (on the FP32 FFT or the
    matrix cores) and back-projection waiting only for its piece: bitwise the
    image and detections of the whole launches in a slot plan."""
    big, _ = _frames()
    fr = synth.make_frame(dataclasses.replace(big.cfg, name="pieces", n_samples=256, seed=903))
    x = _Inputs(fr, torch)
    base = SC.plan_config(rc, [fr], max_frames_in_flight=2, precision=getattr(rc, precision))
    with rc.Plan(base) as plan:
        plan.process([x.desc(rc, 1)])
        ref = _result(rc, plan, torch, 1, fr.n_rows * fr.n_cols)
    budget = dataclasses.replace(base, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=rc.slot_bytes(base) * 3)
    with rc.Plan(budget) as plan:
        for fid in (2, 3):
            plan.process([x.desc(rc, fid, host=True)])
            got = _result(rc, plan, torch, fid, fr.n_rows * fr.n_cols)
            plan.release(fid)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), fid


def test_budget_admission_waits_for_release(rc, torch):
    """A budget of one large frame: a second batch is refused (nothing
    enqueued, the first frame's results untouched) until the first is
    released; several small frames fit where one slot of the limits would."""
    big, small = _frames()
    xb, xs = _Inputs(big, torch), _Inputs(small, torch)
    base = SC.plan_config(rc, [big, small], max_frames_in_flight=8)
    one_big = rc.frame_bytes(dataclasses.replace(base, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=1 << 40),
                             xb.desc(rc, 0, host=True))
    small_b = rc.frame_bytes(dataclasses.replace(base, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=1 << 40),
                             xs.desc(rc, 0, host=True))
    assert small_b * 4 < one_big
    cfg = dataclasses.replace(base, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=one_big + (one_big >> 2))
    with rc.Plan(cfg) as plan:
        plan.process([xb.desc(rc, 1, host=True)])
        ref = _result(rc, plan, torch, 1, big.n_rows * big.n_cols)
        assert plan.try_process([xb.desc(rc, 2, host=True)]) == rc.RC_ENOTREADY
        assert "HBM budget" in rc.last_error()
        assert plan.try_process([xs.desc(rc, 3, host=True), xb.desc(rc, 4, host=True)]) == rc.RC_ENOTREADY
        with pytest.raises(rc.RcError) as ei:      # never enqueued
            plan.poll(3)
        assert ei.value.status == rc.RC_ENOTFOUND
        again = _result(rc, plan, torch, 1, big.n_rows * big.n_cols)
        assert np.array_equal(again[0], ref[0]) and np.array_equal(again[1], ref[1])
        plan.release(1)
        assert plan.try_process([xb.desc(rc, 2, host=True)]) == rc.RC_OK
        img, dets = _result(rc, plan, torch, 2, big.n_rows * big.n_cols)
        plan.release(2)
        assert np.array_equal(img, ref[0]) and np.array_equal(dets, ref[1])
        # four small frames at once in the budget of one large one
        descs = [xs.desc(rc, 10 + k, host=True) for k in range(4)]
        assert plan.try_process(descs) == rc.RC_OK
        outs = [_result(rc, plan, torch, 10 + k, small.n_rows * small.n_cols) for k in range(4)]
        for k in range(4):
            plan.release(10 + k)
        for o in outs[1:]:
            assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def test_frame_larger_than_arena_is_refused(rc, torch):
    big, small = _frames()
    xb = _Inputs(big, torch)
    base = SC.plan_config(rc, [big, small], max_frames_in_flight=2)
    need = rc.frame_bytes(dataclasses.replace(base, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=1 << 40),
                          xb.desc(rc, 0, host=True))
    cfg = dataclasses.replace(base, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=need // 2)
    with rc.Plan(cfg) as plan:
        with pytest.raises(rc.RcError) as ei:
            plan.try_process([xb.desc(rc, 1, host=True)])
        assert ei.value.status == rc.RC_ENOMEM and "whole arena" in rc.last_error()


def test_serving_admits_by_bytes(rc, torch):
    """Poisson arrivals of a large and a small sensor through a budget that
    holds one and a half large frames: every frame completes and results
    equal the frames processed alone."""
    from paper_2306_09784_amd import serve

    big, small = _frames()
    sensors = [serve.SensorStream(i, fr, torch.from_numpy(fr.raw).pin_memory(), torch.from_numpy(fr.pix).to("cuda"))
               for i, fr in enumerate((big, small))]
    base = SC.plan_config(rc, [big, small], max_frames_in_flight=6)
    probe = dataclasses.replace(base, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=1 << 40)
    xb = _Inputs(big, torch)
    one_big = rc.frame_bytes(probe, xb.desc(rc, 0, host=True))
    cfg = dataclasses.replace(probe, hbm_budget_bytes=one_big + (one_big >> 1))
    srv = serve.Server(cfg, n_streams=2, keep_images=True)
    try:
        assert srv.by_bytes and not srv.inputs
        res = serve.run_poisson(srv, sensors, rate_hz=3000.0, duration_s=0.05, seed=5)
        assert res["frames"] == len(srv.results) > 20
        assert len(srv.free) == 6 and not srv.inflight
        ref_cfg = dataclasses.replace(base, max_frames_in_flight=2)
        with rc.Plan(ref_cfg) as plan:
            alone = {s.sensor_id: SC.run_gpu(rc, plan, s.frame, torch) for s in sensors}
        for r in srv.results[:12]:
            fr = sensors[r.sensor_id].frame
            ref = alone[r.sensor_id]["image"].view(np.float32).reshape(-1, 2)
            assert np.array_equal(srv.image_of[r.frame_id][: fr.n_rows * fr.n_cols], ref), r.frame_id
            assert np.array_equal(r.detections, alone[r.sensor_id]["detections"]), r.frame_id
    finally:
        srv.close()


def test_budget_plan_continuous_sar_equals_slot_plan(rc, torch):
    """A continuous-SAR stream (sub-apertures of 8 chirps, apertures of the
    last 3) through a budget plan, every sub-aperture handed over in pinned
    host memory: each aperture's image and detections bitwise the slot
    plan's."""
    from tests.test_gpu_sliding import _Runner, _plan_cfg, _stream

    K, S, nb = 3, 8, 5
    fr, blocks = _stream(nb, S, seed=41)
    base = _plan_cfg(rc, fr, S, K, slots=4)
    with rc.Plan(base) as plan:
        ref = _Runner(rc, torch, plan, fr).run(blocks)
    cfg = dataclasses.replace(base, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=1 << 30)
    pix = torch.from_numpy(np.ascontiguousarray(fr.pix)).to("cuda")
    n_pix = fr.n_rows * fr.n_cols
    with rc.Plan(cfg) as plan:
        for j, blk in enumerate(blocks):
            pinned = torch.from_numpy(blk["raw"]).pin_memory()
            img = torch.empty((n_pix, 2), dtype=torch.float32, device="cuda")
            f = rc.Plan.make_frame(50 + j, data=None, data_host=pinned, q_tx=blk["q_tx"], q_rx=blk["q_rx"],
                                   vel=blk["vel"], pixels=pix, n_rows=fr.n_rows, n_cols=fr.n_cols,
                                   n_bins=fr.n_bins, n_fft=fr.n_fft, fs=fr.fs, n_samples=fr.cfg.n_samples,
                                   image_out=img, sensor_id=0, height=fr.cfg.height,
                                   sliding=rc.RC_SLIDE_START if j == 0 else rc.RC_SLIDE_NEXT)
            plan.process([f])
            dets = plan.detections(50 + j)
            torch.cuda.synchronize()
            plan.release(50 + j)
            got = img.cpu().numpy().view(np.complex64).reshape(-1)
            np.testing.assert_array_equal(got, ref[j][0])
            assert np.array_equal(dets, ref[j][1]), j
