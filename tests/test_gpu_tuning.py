"""Plan-time tuning of back-projection's chirp split, per size class
(rc_plan_tune, rc_plan_set_tuning).  Checked here: the tuner returns one
valid entry per class and installs it, also under an HBM budget that holds
fewer copies; a class given another split changes its image by rounding
only, and plans given the same table agree bitwise; in a tuned plan a batch
of mixed frames gives each frame's result alone, bitwise; an invalid table is
refused and leaves the plan's table as it was."""
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


@pytest.fixture(scope="module")
def frames():
    """Two size classes: 64 chirps x 8 channels on 96 x 80, 32 x 4 on 48 x 40."""
    base = dataclasses.replace(synth.CONFIGS["plain-small"], n_samples=64, box=(-4.0, 4.0, 1.5, 7.0))
    a = synth.make_frame(dataclasses.replace(base, name="a", n_chirps=64, n_rx=8, nx=80, ny=96, seed=811))
    b = synth.make_frame(dataclasses.replace(base, name="b", n_chirps=32, n_rx=4, nx=40, ny=48, seed=812))
    return a, b


class _Dev:
    """Device inputs and an image buffer of one frame, kept alive."""

    def __init__(self, fr, torch):
        self.fr = fr
        self.raw = torch.from_numpy(np.ascontiguousarray(fr.raw)).to("cuda")
        self.pix = torch.from_numpy(np.ascontiguousarray(fr.pix)).to("cuda")
        self.img = torch.empty((fr.n_rows * fr.n_cols, 2), dtype=torch.float32, device="cuda")

    def desc(self, rc, fid):
        fr = self.fr
        return rc.Plan.make_frame(fid, data=self.raw, q_tx=fr.q_tx, q_rx=fr.q_rx, vel=fr.vel, pixels=self.pix,
                                  n_rows=fr.n_rows, n_cols=fr.n_cols, n_bins=fr.n_bins, n_fft=fr.n_fft, fs=fr.fs,
                                  n_samples=fr.cfg.n_samples, image_out=self.img)


def _cfg(rc, frames, **kw):
    return SC.plan_config(rc, frames, precision=rc.RC_PREC_FP32_SPLIT, max_frames_in_flight=4, **kw)


def _image(rc, plan, dev, torch, fid):
    plan.process([dev.desc(rc, fid)])
    dets = plan.detections(fid)
    torch.cuda.synchronize()
    plan.release(fid)
    return dev.img.cpu().numpy().copy(), dets


def _entry(fr, blocks):
    return dict(n_rows=fr.n_rows, n_cols=fr.n_cols, n_chirps=fr.cfg.n_chirps, n_channels=fr.cfg.n_channels,
                chirp_blocks=blocks)


def test_tune_gives_one_valid_entry_per_class(rc, torch, frames):
    a, b = frames
    da, db = _Dev(a, torch), _Dev(b, torch)
    with rc.Plan(_cfg(rc, frames)) as plan:
        out = plan.tune([da.desc(rc, 1), db.desc(rc, 2), da.desc(rc, 3)])
        assert len(out) == 2
        for e, fr in zip(out, (a, b)):
            assert (e["n_rows"], e["n_cols"], e["n_chirps"], e["n_channels"]) == (
                fr.n_rows, fr.n_cols, fr.cfg.n_chirps, fr.cfg.n_channels)
            assert 1 <= e["chirp_blocks"] <= min(16, fr.cfg.n_chirps)
            assert 1 <= e["default_blocks"] <= min(16, fr.cfg.n_chirps)
            assert e["ms_default"] > 0 and 0 < e["ms_chosen"] <= e["ms_default"]
            if e["chirp_blocks"] != e["default_blocks"]:
                assert e["ms_chosen"] < 0.98 * e["ms_default"]
        # the plan keeps working with the installed table, and the frames'
        # results equal those of a plan given the same table
        got = _image(rc, plan, da, torch, 10)
        with rc.Plan(_cfg(rc, frames)) as other:
            other.set_tuning(out)
            ref = _image(rc, other, da, torch, 10)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("blocks", [1, 2, 16])
def test_another_split_changes_the_image_by_rounding_only(rc, torch, frames, blocks):
    """64 chirps x 8 channels: the rule's split against 1, 2 and 16 blocks:
    within 1e-5 of the peak (the same terms summed in another order);
    bitwise the same in two plans of the same table."""
    a, _ = frames
    da = _Dev(a, torch)
    with rc.Plan(_cfg(rc, frames)) as plan:
        ref, ref_dets = _image(rc, plan, da, torch, 1)
        plan.set_tuning([_entry(a, blocks)])
        got, dets = _image(rc, plan, da, torch, 2)
    with rc.Plan(_cfg(rc, frames)) as other:
        other.set_tuning([_entry(a, blocks)])
        again, _ = _image(rc, other, da, torch, 3)
    peak = np.abs(ref.view(np.complex64)).max()
    assert np.abs(got.view(np.complex64) - ref.view(np.complex64)).max() <= 1e-5 * peak
    assert np.array_equal(got, again)
    # detections may differ only at cells the plan flags near the threshold
    differ = set(dets["pixel"].tolist()) ^ set(ref_dets["pixel"].tolist())
    near = set(dets["pixel"][(dets["flags"] & rc.RC_DET_NEAR_THRESHOLD) != 0].tolist()) | set(
        ref_dets["pixel"][(ref_dets["flags"] & rc.RC_DET_NEAR_THRESHOLD) != 0].tolist())
    assert differ <= near, sorted(differ - near)[:5]


def test_tuned_plan_batch_equals_each_frame_alone(rc, torch, frames):
    a, b = frames
    da, db = _Dev(a, torch), _Dev(b, torch)
    db2 = _Dev(b, torch)
    with rc.Plan(_cfg(rc, frames)) as plan:
        plan.set_tuning([_entry(a, 3), _entry(b, 1)])
        alone_a = _image(rc, plan, da, torch, 1)
        alone_b = _image(rc, plan, db, torch, 2)
        plan.process([da.desc(rc, 11), db.desc(rc, 12), db2.desc(rc, 13)])
        outs = {fid: plan.detections(fid) for fid in (11, 12, 13)}
        torch.cuda.synchronize()
        for fid in (11, 12, 13):
            plan.release(fid)
        for dev, fid, ref in ((da, 11, alone_a), (db, 12, alone_b), (db2, 13, alone_b)):
            assert np.array_equal(dev.img.cpu().numpy(), ref[0]), fid
            assert np.array_equal(outs[fid], ref[1]), fid


def test_tuning_under_an_hbm_budget(rc, torch, frames):
    """An arena of 2.5 frames: the tuner measures smaller batches and still
    installs a valid table; the plan's results equal those of a slot plan
    given the same table, bitwise."""
    a, b = frames
    da, db = _Dev(a, torch), _Dev(b, torch)
    slots = _cfg(rc, frames)
    probe = dataclasses.replace(slots, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=1 << 40)
    need = rc.frame_bytes(probe, da.desc(rc, 0))
    with rc.Plan(dataclasses.replace(probe, hbm_budget_bytes=int(2.5 * need))) as plan:
        table = plan.tune([da.desc(rc, 1), db.desc(rc, 2)])
        assert len(table) == 2 and all(1 <= e["chirp_blocks"] <= 16 for e in table)
        got = [_image(rc, plan, d, torch, 10 + k) for k, d in enumerate((da, db))]
    with rc.Plan(slots) as ref_plan:
        ref_plan.set_tuning(table)
        ref = [_image(rc, ref_plan, d, torch, 10 + k) for k, d in enumerate((da, db))]
    for g, r in zip(got, ref):
        assert np.array_equal(g[0], r[0]) and np.array_equal(g[1], r[1])


def test_invalid_table_is_refused_and_keeps_the_table(rc, torch, frames):
    a, b = frames
    da = _Dev(a, torch)
    with rc.Plan(_cfg(rc, frames)) as plan:
        plan.set_tuning([_entry(a, 2)])
        before = _image(rc, plan, da, torch, 1)
        bad = [[_entry(a, 0)], [_entry(a, 17)], [_entry(b, 33)],
               [dict(_entry(a, 2), n_chirps=10 ** 6)], [dict(_entry(a, 2), n_rows=0)]]
        for table in bad:
            with pytest.raises(rc.RcError) as ei:
                plan.set_tuning([_entry(b, 1)] + table)
            assert ei.value.status == rc.RC_EINVAL, table
        after = _image(rc, plan, da, torch, 2)
        assert np.array_equal(before[0], after[0])
        # a sub-aperture is refused by the tuner; too small an output table too
        fr = da.desc(rc, 5)
        fr.sliding = rc.RC_SLIDE_START
        with pytest.raises(rc.RcError) as ei:
            plan.tune([fr])
        assert ei.value.status == rc.RC_EINVAL
        # an output table shorter than the classes: RC_ETRUNC with the class
        # count, nothing measured or installed; no frames: no classes
        import ctypes as C
        two = (rc.rc_frame * 2)(da.desc(rc, 6), _Dev(b, torch).desc(rc, 7))
        one = (rc.rc_tuning_entry * 1)()
        n = C.c_int32()
        assert rc.lib.rc_plan_tune(plan.handle, two, 2, None, one, 1, C.byref(n)) == rc.RC_ETRUNC
        assert n.value == 2
        assert rc.lib.rc_plan_tune(plan.handle, two, 0, None, one, 0, C.byref(n)) == rc.RC_OK
        assert n.value == 0
        plan.set_tuning([])
        cleared = _image(rc, plan, da, torch, 3)
    with rc.Plan(_cfg(rc, frames)) as fresh:
        untuned = _image(rc, fresh, da, torch, 1)
    assert np.array_equal(cleared[0], untuned[0])
