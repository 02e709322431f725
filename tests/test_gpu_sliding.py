"""GPU parity of continuous SAR (rc_sliding): a sensor's chirp stream cut into
sub-apertures of S chirps, each frame's image the aperture of the stream's
last K sub-apertures, against the oracle's bp_sliding, which sums the
sub-apertures' Alg. 2 (or Alg. 1) images with the window over the whole
aperture directly (no decomposition of the window).

Tolerance per pixel.  The library forms three sums per sub-aperture (plain,
and weighted by the cosine and the sine of each chirp's window phase, weights
of magnitude <= 1) and combines them with coefficients whose magnitudes add
up to at most 1/2 + sqrt(2)/2 < 1.25.  Each sum obeys the single-precision
bound of the parity tests, (2 pi e_phase + gamma) times the sum of the
unweighted term magnitudes, so the aperture's error is at most 1.25 times
that bound summed over its sub-apertures, plus the rounding of the weights
and of the combination (a few float ulps of the same magnitudes)."""
import dataclasses
import math

import numpy as np
import pytest

import oracle as O
from paper_2306_09784_amd import synth
from tests import sar_cases as SC
from tests.test_gpu_parity import BP_FLOOR, PLAIN, PLAIN_TOL, SPLIT, SPLIT_TOL, _report

pytestmark = pytest.mark.gpu

R = synth.RADAR


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


def _stream(n_blocks, S, nx=40, ny=32, n_rx=4, seed=31, speed=4.0, yaw=0.0, n_samples=128, n_tx=1,
            height=0.0):
    """One continuous drive cut into n_blocks sub-apertures of S chirps."""
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="stream", n_samples=n_samples,
                              n_chirps=n_blocks * S, nx=nx, ny=ny, n_rx=n_rx, n_tx=n_tx, seed=seed,
                              speed=speed, yaw_rate=yaw, height=height)
    fr = synth.make_frame(cfg)
    blocks = []
    for j in range(n_blocks):
        sl = slice(j * S, (j + 1) * S)
        blocks.append(dict(raw=np.ascontiguousarray(fr.raw[sl]), q_tx=np.ascontiguousarray(fr.q_tx[sl]),
                           q_rx=np.ascontiguousarray(fr.q_rx[sl]), vel=np.ascontiguousarray(fr.vel[sl])))
    return fr, blocks


def _plan_cfg(rc, fr, S, K, depth=2, sensors=2, slots=4, **kw):
    return SC.plan_config(rc, [fr], n_chirps_max=S, max_frames_in_flight=slots, sliding_sensors=sensors,
                          sliding_subapertures=K, sliding_depth=depth, **kw)


class _Runner:
    """Submits sub-apertures of a stream and collects each aperture's image."""

    def __init__(self, rc, torch, plan, fr):
        self.rc, self.torch, self.plan, self.fr = rc, torch, plan, fr
        self.dev = torch.device("cuda")
        self.pix = torch.from_numpy(np.ascontiguousarray(fr.pix)).to(self.dev)
        self.n_pix = fr.n_rows * fr.n_cols
        self.keep = {}

    def frame(self, fid, blk, mode, sensor=0, pixels=None, n_chirps=None):
        raw = self.torch.from_numpy(blk["raw"]).to(self.dev)
        img = self.torch.empty((self.n_pix, 2), dtype=self.torch.float32, device=self.dev)
        self.keep[fid] = (raw, img, blk)
        f = self.rc.Plan.make_frame(fid, data=raw, q_tx=blk["q_tx"], q_rx=blk["q_rx"], vel=blk["vel"],
                                    pixels=self.pix if pixels is None else pixels, n_rows=self.fr.n_rows,
                                    n_cols=self.fr.n_cols, n_bins=self.fr.n_bins, n_fft=self.fr.n_fft,
                                    fs=self.fr.fs, n_samples=self.fr.cfg.n_samples, image_out=img,
                                    sensor_id=sensor, sliding=mode, height=self.fr.cfg.height)
        return f

    def finish(self, fid):
        dets = self.plan.detections(fid)
        self.torch.cuda.synchronize()
        img = self.keep[fid][1].cpu().numpy().view(np.complex64).reshape(-1)
        self.plan.release(fid)
        del self.keep[fid]
        return img, dets

    def run(self, blocks, sensor=0, start_id=1, per_batch=1, stream=None):
        """All sub-apertures in order, per_batch per rc_process_batch."""
        rc = self.rc
        out = []
        for j0 in range(0, len(blocks), per_batch):
            fs = [self.frame(start_id + j, blocks[j], rc.RC_SLIDE_START if j == 0 else rc.RC_SLIDE_NEXT, sensor)
                  for j in range(j0, min(j0 + per_batch, len(blocks)))]
            self.plan.process(fs, stream=stream)
            for f in fs:
                out.append(self.finish(f.frame_id))
        return out


def _oracle_blocks(fr, blocks):
    k = SC.oracle_constants(fr)
    out = []
    for blk in blocks:
        s = O.range_compress(blk["raw"], O.window("hann", fr.cfg.n_samples), fr.n_fft, fr.n_bins)
        out.append(dict(q_tx=blk["q_tx"], q_rx=blk["q_rx"], vel=blk["vel"], s=s))
    return k, out


def _bound(fr, k, oblocks, b, K, precision, scale):
    """Per-pixel bound on |P_gpu - P_oracle| of the aperture ending at b."""
    pix = fr.pix.astype(np.float64)
    lam = R["c"] / R["f0"]
    h = fr.cfg.height
    S_abs = np.zeros(pix.shape[0])
    e_phase = 0.0
    for j in range(max(0, b - K + 1), b + 1):
        blk = oblocks[j]
        fd = O.doppler_table(pix, blk["q_tx"], blk["q_rx"], blk["vel"], k["kd"], height=h)
        S_abs += O.bp_alg2_abs(pix, blk["q_tx"], blk["q_rx"], fd, blk["s"], np.ones(len(blk["s"])), k["a1"],
                               height=h)
        q = np.concatenate([blk["q_tx"].reshape(-1, 2), blk["q_rx"].reshape(-1, 2)]).astype(np.float64)
        if precision == SPLIT:
            Q = np.sqrt(((q - q.mean(0)) ** 2).sum(-1)).max()
            e = 2.0 ** -19 * Q / lam + 2e-6
        else:
            lo, hi = pix.min(0), pix.max(0)
            corners = np.array([[lo[0], lo[1]], [hi[0], hi[1]], [lo[0], hi[1]], [hi[0], lo[1]]])
            d_max = 2 * np.sqrt(((corners[:, None, :] - q[None]) ** 2).sum(-1) + h * h).max()
            e = 2.0 ** -22 * d_max / lam + 1e-5
        e_phase = max(e_phase, e)
    S = len(oblocks[b]["s"])
    gamma = (S * oblocks[b]["s"].shape[1] + 3 * K + 4) * 2.0 ** -24
    return 1.25 * (2 * math.pi * e_phase + gamma) * S_abs + BP_FLOOR * scale


FORMS = [pytest.param(PLAIN, 0, id="fp32"), pytest.param(SPLIT, 0, id="split"), pytest.param(PLAIN, 1, id="exact")]


@pytest.mark.parametrize("precision,exact", FORMS)
def test_sliding_stream_parity(rc, torch, precision, exact):
    """Six sub-apertures of 16 chirps, apertures of K = 3 (48 chirps, Hann over
    48): every frame's image against the oracle, the first two before the
    stream holds K sub-apertures; two sub-apertures per batch (depth 2)."""
    K, S, nb = 3, 16, 6
    fr, blocks = _stream(nb, S, yaw=0.3 if exact else 0.0)
    kw = dict(precision=rc.RC_PREC_FP32_SPLIT if precision == SPLIT else rc.RC_PREC_FP32,
              doppler=rc.RC_DOPPLER_EXACT if exact else rc.RC_DOPPLER_AVERAGE)
    with rc.Plan(_plan_cfg(rc, fr, S, K, **kw)) as plan:
        got = _Runner(rc, torch, plan, fr).run(blocks, per_batch=2)
    k, ob = _oracle_blocks(fr, blocks)
    name = ["fp32", "split", "exact"][2 if exact else precision]
    worst_rel = 0.0
    for b in range(nb):
        P = O.bp_sliding(fr.pix.astype(np.float64), ob, b, K, k["a1"], k["a2"], k["kd"],
                         doppler="exact" if exact else "average", f0=R["f0"], mu=k["mu"], df=k["df"])
        G = got[b][0].astype(np.complex128)
        err = np.abs(G - P)
        pmax = np.abs(P).max()
        bound = _bound(fr, k, ob, b, K, precision, pmax)
        ratio = float((err / bound).max())
        rel = float(err.max() / pmax)
        worst_rel = max(worst_rel, rel)
        assert ratio <= 1.0, f"aperture {b}: per-pixel bound exceeded by {ratio:.3f}"
    _report(f"sliding_{name}", max_rel=worst_rel, apertures=nb)
    assert worst_rel <= (SPLIT_TOL if precision == SPLIT else PLAIN_TOL)


@pytest.mark.slow
def test_sliding_full_size_sampled_pixels(rc, torch):
    """The benchmark's continuous-SAR workload at full size: the plain-large
    sensor (1024 samples, 4 TX x 4 RX, 1201 x 1201 grid) driving on for five
    sub-apertures of 128 TDM cycles, apertures of the last K = 4 (512 cycles,
    Hann over the aperture), each sub-aperture one chirp block; the two full
    apertures and a partial one against the oracle on sampled pixels and the
    image's strongest ones."""
    K, S, nb = 4, 128, 5
    cfg = dataclasses.replace(synth.CONFIGS["plain-large"], name="plain-large-stream", n_chirps=nb * S)
    fr = synth.make_frame(cfg, device="cuda")
    blocks = []
    for j in range(nb):
        sl = slice(j * S, (j + 1) * S)
        blocks.append(dict(raw=np.ascontiguousarray(fr.raw[sl]), q_tx=np.ascontiguousarray(fr.q_tx[sl]),
                           q_rx=np.ascontiguousarray(fr.q_rx[sl]), vel=np.ascontiguousarray(fr.vel[sl])))
    with rc.Plan(_plan_cfg(rc, fr, S, K, sensors=1)) as plan:
        got = _Runner(rc, torch, plan, fr).run(blocks, per_batch=1)
    k, ob = _oracle_blocks(fr, blocks)
    rng = np.random.default_rng(79)
    worst_rel = 0.0
    for b in (1, 3, 4):
        G_all = got[b][0]
        idx = np.unique(np.concatenate([rng.integers(0, fr.n_rows * fr.n_cols, 400),
                                        np.argsort(-np.abs(G_all))[:50]]))
        frs = dataclasses.replace(fr, pix=np.ascontiguousarray(fr.pix[idx]))
        P = O.bp_sliding(frs.pix.astype(np.float64), ob, b, K, k["a1"], k["a2"], k["kd"])
        err = np.abs(G_all[idx].astype(np.complex128) - P)
        pmax = np.abs(P).max()
        bound = _bound(frs, k, ob, b, K, PLAIN, pmax)
        ratio = float((err / bound).max())
        worst_rel = max(worst_rel, float(err.max() / pmax))
        assert ratio <= 1.0, f"aperture {b}: per-pixel bound exceeded by {ratio:.3f}"
    _report("sliding_full_size_sampled", max_rel=worst_rel, apertures=3)
    assert worst_rel <= PLAIN_TOL


@pytest.mark.parametrize("n_tx,n_rx,height", [(2, 2, 0.0), (1, 3, 0.8), (1, 1, 0.0), (4, 2, 0.5)],
                         ids=["tdm2x2", "rx3-height", "rx1", "tdm4x2-height"])
def test_sliding_channel_layouts(rc, torch, n_tx, n_rx, height):
    """The chirp's channel sum joins the three sums at the end of every chirp:
    TX groups narrower than a chirp (several pipeline stages per chirp), odd
    and single channel counts (one-row stages), antennas above the pixels."""
    K, S, nb = 2, 12, 4
    fr, blocks = _stream(nb, S, n_tx=n_tx, n_rx=n_rx, height=height, seed=41 + n_rx, nx=24, ny=20)
    with rc.Plan(_plan_cfg(rc, fr, S, K)) as plan:
        got = _Runner(rc, torch, plan, fr).run(blocks, per_batch=2)
    k, ob = _oracle_blocks(fr, blocks)
    for b in range(nb):
        P = O.bp_sliding(fr.pix.astype(np.float64), ob, b, K, k["a1"], k["a2"], k["kd"], height=height)
        err = np.abs(got[b][0].astype(np.complex128) - P)
        ratio = float((err / _bound(fr, k, ob, b, K, PLAIN, np.abs(P).max())).max())
        assert ratio <= 1.0, f"aperture {b}: per-pixel bound exceeded by {ratio:.3f}"


def test_sliding_detections_match_oracle(rc, torch):
    """CA-CFAR on the last aperture of a stream: the detection list equals the
    oracle's except cells whose decision is not robust to the image bound."""
    K, S, nb = 4, 16, 5
    fr, blocks = _stream(nb, S, nx=96, ny=80, seed=33)
    with rc.Plan(_plan_cfg(rc, fr, S, K, max_rechecks=64)) as plan:
        got = _Runner(rc, torch, plan, fr).run(blocks)
    k, ob = _oracle_blocks(fr, blocks)
    b = nb - 1
    P = O.bp_sliding(fr.pix.astype(np.float64), ob, b, K, k["a1"], k["a2"], k["kd"])
    pw = (np.abs(P) ** 2).reshape(fr.n_rows, fr.n_cols)
    cf = O.ca_cfar(pw, 2, 8, 1e-4)
    bound = _bound(fr, k, ob, b, K, PLAIN, np.abs(P).max()).reshape(fr.n_rows, fr.n_cols)
    bad, n_diff, n_fragile = SC.detection_mismatch(got[b][1], cf, pw, bound, fr.n_cols, 2, 8, 1e-4)
    _report("sliding_detections", n_gpu=len(got[b][1]), n_oracle=len(cf[0]), n_diff=n_diff, fragile=n_fragile)
    assert not bad
    assert len(cf[0]) > 0
    # no recheck for continuous-SAR apertures (even with the plan's recheck on):
    # band cells keep the near-threshold flag
    assert not np.any(got[b][1]["flags"] & rc.RC_DET_RECHECKED)


def test_sliding_rect_window_sums_subaperture_images(rc, torch):
    """With the rectangular window the aperture is the plain sum of its
    sub-apertures' images (one partial image per sub-aperture)."""
    K, S, nb = 3, 8, 5
    fr, blocks = _stream(nb, S, seed=35)
    with rc.Plan(_plan_cfg(rc, fr, S, K, sar_window="rect")) as plan:
        got = _Runner(rc, torch, plan, fr).run(blocks, per_batch=2)
    k, ob = _oracle_blocks(fr, blocks)
    for b in range(nb):
        P = O.bp_sliding(fr.pix.astype(np.float64), ob, b, K, k["a1"], k["a2"], k["kd"], window_kind="rect")
        err = np.abs(got[b][0].astype(np.complex128) - P)
        assert float((err / _bound(fr, k, ob, b, K, PLAIN, np.abs(P).max())).max()) <= 1.0, b


def test_sliding_batching_streams_and_restart_are_bitwise_stable(rc, torch):
    """The same stream gives the same bits whether its sub-apertures come one
    per batch, two per batch interleaved with another sensor's, or alternate
    between two HIP streams; RC_SLIDE_START begins a new aperture history."""
    K, S, nb = 3, 8, 5
    fr, blocks = _stream(nb, S, seed=37)
    _, other = _stream(nb, S, seed=38)
    with rc.Plan(_plan_cfg(rc, fr, S, K, slots=6)) as plan:
        run = _Runner(rc, torch, plan, fr)
        ref = [g[0] for g in run.run(blocks)]
        # interleaved with sensor 1, two sub-apertures of each per batch
        imgs = {}
        for j0 in range(0, nb, 2):
            fs = []
            for j in range(j0, min(j0 + 2, nb)):
                mode = rc.RC_SLIDE_START if j == 0 else rc.RC_SLIDE_NEXT
                fs.append(run.frame(100 + j, blocks[j], mode, sensor=0))
                fs.append(run.frame(200 + j, other[j], mode, sensor=1))
            plan.process(fs)
            for f in fs:
                imgs[f.frame_id] = run.finish(f.frame_id)[0]
        for j in range(nb):
            np.testing.assert_array_equal(imgs[100 + j], ref[j])
        # alternating HIP streams, all sub-apertures submitted before any completes
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        ids = []
        for j in range(nb):
            if len(ids) == 2:
                done = ids.pop(0)
                imgs[done] = run.finish(done)[0]
            f = run.frame(300 + j, blocks[j], rc.RC_SLIDE_START if j == 0 else rc.RC_SLIDE_NEXT)
            plan.process([f], stream=s1 if j % 2 == 0 else s2)
            ids.append(300 + j)
        for fid in ids:
            imgs[fid] = run.finish(fid)[0]
        for j in range(nb):
            np.testing.assert_array_equal(imgs[300 + j], ref[j])
        # a restart mid-stream: its first apertures are the fresh stream's
        restart = run.run(blocks[:2], start_id=400)
        for j in range(2):
            np.testing.assert_array_equal(restart[j][0], ref[j])


def test_sliding_state_errors(rc, torch):
    K, S = 2, 8
    fr, blocks = _stream(3, S, seed=39)
    with rc.Plan(_plan_cfg(rc, fr, S, K, depth=1, slots=3)) as plan:
        run = _Runner(rc, torch, plan, fr)

        def status(f):
            arr = (rc.rc_frame * 1)(f)
            return rc.lib.rc_process_batch(plan.handle, arr, 1, torch.cuda.current_stream().cuda_stream)

        # a continuation without a stream
        assert status(run.frame(1, blocks[0], rc.RC_SLIDE_NEXT)) == rc.RC_EINVAL
        assert "RC_SLIDE_START" in rc.last_error()
        # a sensor outside the plan, an unknown mode
        assert status(run.frame(2, blocks[0], rc.RC_SLIDE_START, sensor=2)) == rc.RC_EINVAL
        assert status(run.frame(3, blocks[0], 7)) == rc.RC_EINVAL
        assert plan.try_process([run.frame(4, blocks[0], rc.RC_SLIDE_START)]) == rc.RC_OK
        # depth 1: a second sub-aperture of sensor 0 waits until the first is released
        assert status(run.frame(5, blocks[1], rc.RC_SLIDE_NEXT)) == rc.RC_ENOTREADY
        # other sensors are not held back
        assert plan.try_process([run.frame(6, blocks[0], rc.RC_SLIDE_START, sensor=1)]) == rc.RC_OK
        run.finish(4)
        run.finish(6)
        # a different lattice pointer or chirp count is not the same stream
        other_pix = torch.from_numpy(np.ascontiguousarray(fr.pix)).to(run.dev)
        assert status(run.frame(7, blocks[1], rc.RC_SLIDE_NEXT, pixels=other_pix)) == rc.RC_EINVAL
        short = {k: np.ascontiguousarray(v[: S // 2]) for k, v in blocks[1].items()}
        assert status(run.frame(8, short, rc.RC_SLIDE_NEXT)) == rc.RC_EINVAL
        # the failed calls left the stream where it was: this is its second sub-aperture
        assert plan.try_process([run.frame(9, blocks[1], rc.RC_SLIDE_NEXT)]) == rc.RC_OK
        run.finish(9)
    # a plan without continuous-SAR sensors refuses sub-apertures
    with rc.Plan(SC.plan_config(rc, [fr], n_chirps_max=S)) as plan:
        run = _Runner(rc, torch, plan, fr)
        with pytest.raises(rc.RcError) as ei:
            plan.process([run.frame(1, blocks[0], rc.RC_SLIDE_START)])
        assert ei.value.status == rc.RC_EINVAL
