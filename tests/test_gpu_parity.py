"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, stage
by stage and end to end, on seeded synthetic frames.

Tolerances (derivation in the design notes):
  * range spectrum, FP32 FFT: relative L2 error <= 1e-5 per frame;
  * Doppler table (double evaluation, rounded once): <= 1e-6 bins;
  * back-projection image, per pixel: |dP| <= (2 pi e_phase + gamma) S(p) +
    floor, where S(p) is the oracle's sum of term magnitudes, e_phase the
    bound on a term's phase error in turns and gamma the bound on the
    accumulation rounding (terms per accumulator x 2^-24); e_phase is
    2^-22 d_max / lambda for plain single precision (two ulps of the longest
    two-way path in wavelengths: the square root's biased rounding and the
    path's sums each stay within an ulp) and 2^-19 Q / lambda + 2e-6 for the
    split-phase form (Q: largest antenna offset from the aperture centre);
  * image-level max |dP| / max |P|: PLAIN_TOL (single precision, the paper's
    form: a pixel's mean phase error reaches ~4e-4 turns) and SPLIT_TOL;
  * detections: identical lists except cells whose oracle decision is not
    robust to the per-pixel image error bound (see sar_cases); for the
    split-phase form, every disagreement within the plan's band of the
    oracle's threshold.
"""
import dataclasses
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2306_09784_amd import synth
from tests import sar_cases as SC

pytestmark = pytest.mark.gpu

SPEC_TOL = 1e-5
DOP_TOL = 1e-6
PLAIN_TOL = 5e-3
SPLIT_TOL = 2e-4
BP_FLOOR = 1e-5
PLAIN, SPLIT = 0, 1
MARGIN = 3e-2    # the plan's CFAR band (relative to the threshold) in the end-to-end cases
R = synth.RADAR
PRECISIONS = [pytest.param(PLAIN, id="fp32"), pytest.param(SPLIT, id="split")]


def _report(name, **vals):
    vals = {k: (float(v) if isinstance(v, (np.floating, float)) else int(v)) for k, v in vals.items()}
    path = os.environ.get("RC_REPORT")
    print(name, vals, flush=True)
    if path:
        with open(path, "a") as f:
            f.write(json.dumps({"case": name, **vals}) + "\n")


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


def _phase_bound(frame, precision):
    lam = synth.RADAR["c"] / synth.RADAR["f0"]
    q = np.concatenate([frame.q_tx.reshape(-1, 2), frame.q_rx.reshape(-1, 2)]).astype(np.float64)
    if precision == SPLIT:
        Q = np.sqrt(((q - q.mean(0)) ** 2).sum(-1)).max()
        return 2.0 ** -19 * Q / lam + 2e-6
    corners = np.array([[frame.pix[:, 0].min(), frame.pix[:, 1].min()], [frame.pix[:, 0].max(), frame.pix[:, 1].max()],
                        [frame.pix[:, 0].min(), frame.pix[:, 1].max()], [frame.pix[:, 0].max(), frame.pix[:, 1].min()]])
    d_max = 2 * np.sqrt(((corners[:, None, :] - q[None]) ** 2).sum(-1) + frame.cfg.height ** 2).max()
    return 2.0 ** -22 * d_max / lam + 1e-5


def _amp_bound(frame, ora, precision, pix_index=None):
    """Per-pixel bound on |P_gpu - P_oracle| (see module docstring)."""
    k = ora["k"]
    pix = frame.pix.astype(np.float64) if pix_index is None else frame.pix.astype(np.float64)[pix_index]
    S = O.bp_alg2_abs(pix, frame.q_tx, frame.q_rx, ora["doppler"], ora["spectrum"], ora["w_sar"], k["a1"],
                      height=frame.cfg.height)
    gamma = (frame.cfg.n_chirps * frame.cfg.n_channels / 2 + 2) * 2.0 ** -24
    pmax = np.abs(ora["image"]).max()
    return (2 * math.pi * _phase_bound(frame, precision) + gamma) * S + BP_FLOOR * pmax


def _check_image(name, frame, gpu_img, ora, precision, pix_index=None, tol=None):
    P = ora["image"]
    G = gpu_img if pix_index is None else gpu_img[pix_index]
    err = np.abs(G.astype(np.complex128) - P)
    pmax = np.abs(P).max()
    rel = float(err.max() / pmax)
    bound = _amp_bound(frame, ora, precision, pix_index)
    worst = float((err / bound).max())
    tol = tol if tol is not None else SPLIT_TOL if precision == SPLIT else PLAIN_TOL
    _report(f"{name}_{'split' if precision == SPLIT else 'fp32'}", max_rel=rel,
            rms_rel=float(np.sqrt(np.mean(err ** 2)) / pmax), bound_ratio=worst)
    assert rel <= tol, f"{name}: max|dP|/max|P| = {rel:.3e}"
    assert worst <= 1.0, f"{name}: per-pixel bound exceeded by {worst:.3f}"
    return bound


# ---------------------------------------------------------------------------
# stage parity
# ---------------------------------------------------------------------------
def test_range_and_doppler_parity_plain_small(rc, torch):
    fr = SC.small_frame(nx=64, ny=48)
    with rc.Plan(SC.plan_config(rc, [fr])) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, want_spectrum=True, want_doppler=True)
    ora = SC.run_oracle(fr, cfar=None)
    s, so = out["spectrum"].astype(np.complex128), ora["spectrum"]
    rel_l2 = float(np.linalg.norm(s - so) / np.linalg.norm(so))
    row_rel = float((np.abs(s - so).max(-1) / np.abs(so).max(-1)).max())
    dd = float(np.abs(out["doppler"] - ora["doppler"]).max())
    _report("range_doppler_small", rel_l2=rel_l2, row_max_rel=row_rel, doppler_abs=dd)
    assert rel_l2 <= SPEC_TOL
    assert row_rel <= 10 * SPEC_TOL
    assert dd <= DOP_TOL
    _check_image("image_small_64x48", fr, out["image"], ora, PLAIN)


@pytest.mark.parametrize("log2n,n_s,n_bins", [(2, 3, 4), (3, 8, 5), (4, 9, 16), (5, 32, 7), (6, 40, 33),
                                                (7, 64, 27), (8, 200, 256), (9, 256, 101), (10, 1000, 433),
                                                (11, 1024, 432), (12, 2048, 900), (12, 4096, 2)])
def test_range_parity_every_fft_size(rc, torch, log2n, n_s, n_bins):
    """Range compression alone over every supported DFT length (4 .. 4096),
    ragged sample counts and kept-bin counts, on 9 rows (not a multiple of
    the rows a workgroup holds for short rows): the spectrum output against the
    oracle's FP64 DFT of the same windowed, zero-padded rows."""
    n_fft = 1 << log2n
    M, CH = 3, 3
    rng = np.random.default_rng(1000 + log2n)
    raw = (rng.standard_normal((M, CH, n_s)) + 1j * rng.standard_normal((M, CH, n_s))).astype(np.complex64)
    q = np.zeros((M, CH, 2), np.float32)
    q[..., 0] = np.arange(M * CH, dtype=np.float32).reshape(M, CH) * 1e-3
    vel = np.zeros((M, 2), np.float32)
    pix = np.array([[0.0, 5.0], [0.1, 5.0]], np.float32)
    dev = torch.device("cuda")
    d_raw = torch.from_numpy(raw).to(dev)
    d_pix = torch.from_numpy(pix).to(dev)
    spec = torch.empty((M, CH, n_bins, 2), dtype=torch.float32, device=dev)
    img = torch.empty((2, 2), dtype=torch.float32, device=dev)
    # (the split-phase form: at fs = 10 MHz the kept bins of the short DFTs
    # reach paths far beyond what the plain form's phase takes)
    cfg = rc.PlanConfig(radar=synth.RADAR, n_samples_max=n_s, n_fft_max=max(n_fft, 4), n_bins_max=max(n_bins, 2),
                        n_chirps_max=M, n_channels_max=CH, n_pix_max=2, max_frames_in_flight=1,
                        precision=rc.RC_PREC_FP32_SPLIT)
    with rc.Plan(cfg) as plan:
        fr = rc.Plan.make_frame(1, data=d_raw, q_tx=q, q_rx=q, vel=vel, pixels=d_pix, n_rows=1, n_cols=2,
                                n_bins=n_bins, n_fft=n_fft, fs=1e7, n_samples=n_s, image_out=img, spectrum_out=spec)
        plan.process([fr])
        plan.detections(1)
        torch.cuda.synchronize()
        got = spec.cpu().numpy().view(np.complex64)[..., 0].astype(np.complex128)
        plan.release(1)
    ref = O.range_compress(raw, O.window("hann", n_s), n_fft, n_bins)
    rel_l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    row_rel = float((np.abs(got - ref).max(-1) / np.abs(ref).max(-1)).max())
    _report(f"range_n{n_fft}_s{n_s}_b{n_bins}", rel_l2=rel_l2, row_max_rel=row_rel)
    assert rel_l2 <= SPEC_TOL
    assert row_rel <= 10 * SPEC_TOL


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("n_tx,n_rx,n_chirps", [(1, 4, 16), (4, 4, 8), (2, 1, 12), (1, 16, 6), (1, 8, 9),
                                                (1, 2, 10), (1, 1, 1), (3, 1, 5)])
def test_bp_parity_spectrum_input(rc, torch, n_tx, n_rx, n_chirps, precision):
    """Alg. 2 alone on a seeded random spectrum over a ragged 37 x 45 lattice
    (several 16 x 16 tiles plus partial ones); covers every TX-group width."""
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="bp", n_samples=64, n_chirps=n_chirps,
                              n_tx=n_tx, n_rx=n_rx, nx=45, ny=37, box=(-4.0, 4.0, 1.5, 7.0),
                              n_targets=1, noise=False, seed=7 + n_tx * 10 + n_rx)
    fr = synth.make_frame(cfg)
    rng = np.random.default_rng(100 + n_tx * 16 + n_rx)
    spec = synth.random_spectrum(rng, (cfg.n_chirps, cfg.n_channels, fr.n_bins))
    with rc.Plan(SC.plan_config(rc, [fr], precision=precision)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, spectrum=spec)
    ora = SC.run_oracle(fr, spectrum=spec, cfar=None)
    _check_image(f"bp_spectrum_tx{n_tx}_rx{n_rx}_m{n_chirps}", fr, out["image"], ora, precision)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("n_rx,n_chirps,nx,ny,sampled", [(4, 100, 45, 37, False), (8, 333, 512, 256, True)],
                         ids=["16_blocks_of_6_or_7", "5_blocks_of_66_or_67"])
def test_bp_parity_uneven_chirp_blocks(rc, torch, n_rx, n_chirps, nx, ny, sampled, precision):
    """Chirp counts that the frame's chirp blocks do not divide evenly.  A
    37 x 45 lattice (36 waves) with 100 chirps x 4 channels is split into 16
    blocks (one generation of resident waves needs more than 16) of 6 or 7
    chirps; a 256 x 512 lattice (2048 waves) with 333 chirps x 8 channels into
    5 blocks (at least 512 of its 2664 rows each; one generation needs only 4)
    of 66 or 67 chirps, its oracle on sampled pixels."""
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="uneven", n_samples=64, n_chirps=n_chirps,
                              n_tx=1, n_rx=n_rx, nx=nx, ny=ny, box=(-6.0, 6.0, 1.5, 9.0), n_targets=1,
                              noise=False, seed=31 + n_chirps)
    fr = synth.make_frame(cfg)
    rng = np.random.default_rng(300 + n_chirps)
    spec = synth.random_spectrum(rng, (cfg.n_chirps, cfg.n_channels, fr.n_bins))
    with rc.Plan(SC.plan_config(rc, [fr], precision=precision)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, spectrum=spec)
    idx = None
    if sampled:
        idx = np.unique(np.concatenate([rng.integers(0, fr.n_rows * fr.n_cols, 400),
                                        np.argsort(-np.abs(out["image"]))[:50]]))
    ora = SC.run_oracle(fr, spectrum=spec, pix_index=idx, cfar=None)
    _check_image(f"uneven_blocks_m{n_chirps}", fr, out["image"], ora, precision, pix_index=idx)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_bp_parity_indices_out_of_range(rc, torch, precision):
    """Too few kept bins: many terms fall outside [0, n_bins - 1] and must
    contribute zero (range-tested path), others stay in range."""
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="oor", n_samples=64, n_chirps=8, n_rx=4,
                              nx=40, ny=40, box=(-6.0, 6.0, 1.0, 13.0), n_targets=1, noise=False, seed=5)
    fr = synth.make_frame(cfg)
    fr = dataclasses.replace(fr, n_bins=fr.n_bins // 2)
    rng = np.random.default_rng(55)
    spec = synth.random_spectrum(rng, (cfg.n_chirps, cfg.n_channels, fr.n_bins))
    with rc.Plan(SC.plan_config(rc, [fr], precision=precision)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, spectrum=spec)
    ora = SC.run_oracle(fr, spectrum=spec, cfar=None)
    zero = np.abs(ora["image"]) == 0
    assert zero.sum() > 100                         # whole pixels beyond the band
    assert np.all(out["image"][zero] == 0)
    _check_image("bp_out_of_range", fr, out["image"], ora, precision)


@pytest.mark.parametrize("n_tx,n_rx,yaw", [(1, 4, 0.0), (4, 4, 25.0), (1, 8, -40.0)])
def test_alg1_exact_doppler_parity(rc, torch, n_tx, n_rx, yaw):
    """Alg. 1 (per-chirp radial velocities) on straight and curved drives; on a
    curved drive it must differ from Alg. 2 by more than its tolerance."""
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="alg1", n_samples=64, n_chirps=24,
                              n_tx=n_tx, n_rx=n_rx, nx=45, ny=37, box=(-4.0, 4.0, 1.5, 7.0), speed=8.0,
                              yaw_rate=yaw, n_targets=1, noise=False, seed=17 + n_rx)
    fr = synth.make_frame(cfg)
    rng = np.random.default_rng(200 + n_rx)
    spec = synth.random_spectrum(rng, (cfg.n_chirps, cfg.n_channels, fr.n_bins))
    with rc.Plan(SC.plan_config(rc, [fr], doppler=rc.RC_DOPPLER_EXACT)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, spectrum=spec)
    ora = SC.run_oracle(fr, spectrum=spec, cfar=None, doppler="exact")
    _check_image(f"alg1_tx{n_tx}_rx{n_rx}_yaw{yaw}", fr, out["image"], ora, PLAIN)
    if yaw != 0.0:
        # the per-chirp Doppler of a turning vehicle is visible: Alg. 2 (averaged)
        # departs from Alg. 1 by far more than the GPU's error against Alg. 1
        alg2 = SC.run_oracle(fr, spectrum=spec, cfar=None)["image"]
        gpu_err = np.abs(out["image"].astype(np.complex128) - ora["image"]).max()
        assert np.abs(alg2 - ora["image"]).max() > 5 * gpu_err


@pytest.mark.parametrize("n_tx,n_rx,yaw", [(1, 4, 0.0), (4, 4, 25.0)])
def test_alg1_direct_form_parity(rc, torch, n_tx, n_rx, yaw):
    """Alg. 1 as the paper states it (metres and seconds, tau, f_hyp in Hz,
    the index f_hyp / df and the phase f0 tau per term, the reference of
    Tab. II's "Opt." row) against the oracle's Alg. 1.  Its phase rounds tau
    and f0 tau once each on top of the distances: within the same per-term
    bound as the plain form (2^-21 of the path in wavelengths), and 1e-2 of
    the peak (twice the plain form's tolerance)."""
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="alg1d", n_samples=64, n_chirps=24,
                              n_tx=n_tx, n_rx=n_rx, nx=45, ny=37, box=(-4.0, 4.0, 1.5, 7.0), speed=8.0,
                              yaw_rate=yaw, n_targets=1, noise=False, seed=27 + n_rx)
    fr = synth.make_frame(cfg)
    rng = np.random.default_rng(300 + n_rx)
    spec = synth.random_spectrum(rng, (cfg.n_chirps, cfg.n_channels, fr.n_bins))
    with rc.Plan(SC.plan_config(rc, [fr], doppler=rc.RC_DOPPLER_EXACT_DIRECT)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, spectrum=spec)
    ora = SC.run_oracle(fr, spectrum=spec, cfar=None, doppler="exact")
    _check_image(f"alg1_direct_tx{n_tx}_rx{n_rx}_yaw{yaw}", fr, out["image"], ora, PLAIN, tol=1e-2)


def test_end_to_end_direct_form(rc, torch):
    fr = SC.small_frame(nx=96, ny=80, n_chirps=64)
    with rc.Plan(SC.plan_config(rc, [fr], doppler=rc.RC_DOPPLER_EXACT_DIRECT)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch)
    ora = SC.run_oracle(fr, cfar=None, doppler="exact")
    _check_image("end_to_end_direct", fr, out["image"], ora, PLAIN, tol=1e-2)


def test_end_to_end_exact_doppler(rc, torch):
    fr = SC.small_frame(nx=96, ny=80, n_chirps=64)
    with rc.Plan(SC.plan_config(rc, [fr], doppler=rc.RC_DOPPLER_EXACT)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch)
    ora = SC.run_oracle(fr, cfar=None, doppler="exact")
    _check_image("end_to_end_exact", fr, out["image"], ora, PLAIN)


@pytest.mark.parametrize("precision,doppler", [(PLAIN, 0), (SPLIT, 0), (PLAIN, 1)], ids=["fp32", "split", "exact"])
def test_antenna_height(rc, torch, precision, doppler):
    """Antennas 0.8 m above the pixel plane (3-D distances): every form against
    the oracle with the same height, on a scene simulated with that height."""
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="height", n_samples=128, n_chirps=48, n_rx=4,
                              nx=48, ny=40, box=(-3.0, 3.0, 1.0, 6.0), n_targets=4, height=0.8, seed=31,
                              yaw_rate=0.4 if doppler else 0.0)
    fr = synth.make_frame(cfg)
    kw = dict(precision=precision, doppler=rc.RC_DOPPLER_EXACT if doppler else rc.RC_DOPPLER_AVERAGE)
    with rc.Plan(SC.plan_config(rc, [fr], **kw)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, want_doppler=not doppler)
    ora = SC.run_oracle(fr, cfar=None, doppler="exact" if doppler else "average")
    if not doppler:
        assert np.abs(out["doppler"] - ora["doppler"]).max() <= DOP_TOL
    _check_image(f"height_{['avg', 'exact'][doppler]}", fr, out["image"], ora, precision)


@pytest.mark.parametrize("n_rows,n_cols", [(1, 300), (5, 70), (8, 8), (9, 17)])
def test_bp_parity_small_lattices(rc, torch, n_rows, n_cols):
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="lat", n_samples=32, n_chirps=6, n_rx=4,
                              nx=n_cols, ny=n_rows, box=(-3.0, 3.0, 2.0, 5.0), n_targets=2, noise=True,
                              seed=9)
    fr = synth.make_frame(cfg)
    with rc.Plan(SC.plan_config(rc, [fr])) as plan:
        out = SC.run_gpu(rc, plan, fr, torch)
    ora = SC.run_oracle(fr, cfar=None)
    _check_image(f"lattice_{n_rows}x{n_cols}", fr, out["image"], ora, PLAIN)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("n_samples,n_chirps,n_rx,n_rows,n_cols", [
    (32, 1, 1, 1, 1),       # one chirp of one channel, one pixel (the chirp window is one sample)
    (64, 1, 4, 1, 64),      # one chirp, one row of pixels
    (2048, 3, 2, 9, 17),    # the longest DFT (4096 points), a ragged lattice
])
def test_degenerate_and_longest_shapes(rc, torch, precision, n_samples, n_chirps, n_rx, n_rows, n_cols):
    """Degenerate frames and the longest range DFT, raw input end to end
    against the oracle's image."""
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="deg", n_samples=n_samples, n_chirps=n_chirps,
                              n_rx=n_rx, nx=n_cols, ny=n_rows, box=(-3.0, 3.0, 2.0, 5.0), n_targets=2,
                              noise=True, seed=19)
    fr = synth.make_frame(cfg)
    with rc.Plan(SC.plan_config(rc, [fr], precision=precision)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch)
    ora = SC.run_oracle(fr, cfar=None)
    _check_image(f"shape_{n_samples}x{n_chirps}x{n_rx}_{n_rows}x{n_cols}", fr, out["image"], ora, precision)


# ---------------------------------------------------------------------------
# end to end
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", PRECISIONS)
def test_end_to_end_plain_small(rc, torch, precision):
    """256 samples x 128 chirps x 4 RX on a 256 x 256 grid: image and detections."""
    fr = SC.small_frame()
    with rc.Plan(SC.plan_config(rc, [fr], precision=precision, cfar_margin_rel=MARGIN)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch)
    ora = SC.run_oracle(fr)
    bound = _check_image("end_to_end_small", fr, out["image"], ora, precision)
    dets = out["detections"]
    assert np.all(np.diff(dets["pixel"]) > 0)       # ascending pixel order
    amp_err = bound.reshape(fr.n_rows, fr.n_cols)
    bad, n_diff, n_fragile = SC.detection_mismatch(dets, ora["cfar"], ora["power"], amp_err, fr.n_cols, 2, 8, 1e-4)
    _report(f"detections_small_{'split' if precision == SPLIT else 'fp32'}", n_gpu=len(dets),
            n_oracle=len(ora["cfar"][0]), n_diff=n_diff, n_fragile=n_fragile, n_robust_mismatch=len(bad))
    assert not bad, bad[:5]
    assert len(dets) > 0
    if precision == SPLIT:
        # the detection contract: the lists differ only within the plan's band
        # of the oracle's threshold, where the GPU flags its own detections
        out_band, n_d = SC.band_mismatch(dets, ora["power"], fr.n_cols, 2, 8, 1e-4, MARGIN)
        assert not out_band, out_band[:5]
        g_rel = np.abs(dets["power"].astype(np.float64) - dets["threshold"]) / dets["threshold"]
        assert np.array_equal((dets["flags"] & rc.RC_DET_NEAR_THRESHOLD) != 0, g_rel <= MARGIN)
    # reported power / threshold match the oracle's at common cells
    common, gi, oi = np.intersect1d(dets["pixel"], ora["cfar"][0], return_indices=True)
    pw_err = 2 * np.sqrt(ora["cfar"][1][oi]) * amp_err.reshape(-1)[common] + amp_err.reshape(-1)[common] ** 2
    assert np.all(np.abs(dets["power"][gi] - ora["cfar"][1][oi]) <= pw_err + 1e-6 * ora["cfar"][1][oi])
    # every point target of SNR >= 20 dB is detected within one pixel
    for tp, a in zip(fr.targets, fr.target_amp):
        if 20 * np.log10(abs(a)) < 20:
            continue
        d = np.hypot(fr.pix[dets["pixel"], 0] - tp[0], fr.pix[dets["pixel"], 1] - tp[1])
        assert d.min() < 0.15


@pytest.mark.slow
@pytest.mark.parametrize("precision", PRECISIONS)
def test_plain_large_sampled_pixels(rc, torch, precision):
    """Full-size frame (1024 samples x 512 cycles x 16 channels, 1201^2 grid) in
    the benchmark's launch configuration; oracle on sampled pixels."""
    fr = synth.make_frame(synth.CONFIGS["plain-large"], device="cuda")
    with rc.Plan(SC.plan_config(rc, [fr], precision=precision)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, want_spectrum=True)
    s = O.range_compress(fr.raw, O.window("hann", fr.cfg.n_samples), fr.n_fft, fr.n_bins)
    rel_l2 = float(np.linalg.norm(out["spectrum"] - s) / np.linalg.norm(s))
    _report("range_large", rel_l2=rel_l2)
    assert rel_l2 <= SPEC_TOL
    rng = np.random.default_rng(77)
    idx = np.unique(np.concatenate([rng.integers(0, fr.n_rows * fr.n_cols, 400),
                                    np.argsort(-np.abs(out["image"]))[:50]]))
    ora = SC.run_oracle(fr, spectrum=s, pix_index=idx, cfar=None)
    _check_image("image_large_sampled", fr, out["image"], ora, precision, pix_index=idx)


@pytest.mark.slow
@pytest.mark.parametrize("precision", PRECISIONS)
def test_paper_configuration_sampled_pixels(rc, torch, precision):
    """The paper's combined setting (Sec. IV, Tab. II rows 7-8) at full size in
    the benchmark's launch configuration: 1024 samples x 1024 chirps x 8 RX on
    the 557 x 520 polar lattice of Sec. III-E (sixteen chirp blocks); oracle on
    sampled pixels and the image's strongest ones."""
    cfg = synth.CONFIGS["paper-polar"]
    fr = synth.make_frame(cfg, device="cuda")
    q = np.concatenate([fr.q_tx.reshape(-1, 2), fr.q_rx.reshape(-1, 2)])
    g = rc.grid_polar_params(R, cfg.box, (float(q[:, 0].mean()), float(q[:, 1].mean())), float(np.ptp(q[:, 0])))
    pol = rc.grid_polar(g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"])
    fr = dataclasses.replace(fr, pix=pol, n_rows=g["nth"], n_cols=g["nr"])
    assert (fr.n_rows, fr.n_cols) == (557, 520)
    with rc.Plan(SC.plan_config(rc, [fr], precision=precision)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, want_spectrum=True)
    s = O.range_compress(fr.raw, O.window("hann", cfg.n_samples), fr.n_fft, fr.n_bins)
    rel_l2 = float(np.linalg.norm(out["spectrum"] - s) / np.linalg.norm(s))
    _report("range_paper", rel_l2=rel_l2)
    assert rel_l2 <= SPEC_TOL
    rng = np.random.default_rng(78)
    idx = np.unique(np.concatenate([rng.integers(0, fr.n_rows * fr.n_cols, 400),
                                    np.argsort(-np.abs(out["image"]))[:50]]))
    ora = SC.run_oracle(fr, spectrum=s, pix_index=idx, cfar=None)
    _check_image("image_paper_sampled", fr, out["image"], ora, precision, pix_index=idx)


@pytest.mark.slow
def test_alg1_reference_frame_sampled_pixels(rc, torch):
    """The reference of the paper's Tab. II ablation at full size: Alg. 1 (per
    chirp Doppler) on 1024 samples x 1024 chirps x 16 RX and the 1201 x 1201
    Cartesian grid, as the benchmark runs it; oracle on sampled pixels and the
    image's strongest ones."""
    fr = synth.make_frame(synth.CONFIGS["paper-ref"], device="cuda")
    with rc.Plan(SC.plan_config(rc, [fr], doppler=rc.RC_DOPPLER_EXACT)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch)
    s = O.range_compress(fr.raw, O.window("hann", fr.cfg.n_samples), fr.n_fft, fr.n_bins)
    rng = np.random.default_rng(80)
    idx = np.unique(np.concatenate([rng.integers(0, fr.n_rows * fr.n_cols, 400),
                                    np.argsort(-np.abs(out["image"]))[:50]]))
    ora = SC.run_oracle(fr, spectrum=s, pix_index=idx, cfar=None, doppler="exact")
    _check_image("alg1_reference_sampled", fr, out["image"], ora, PLAIN, pix_index=idx)


# ---------------------------------------------------------------------------
# ABI behaviour on the device
# ---------------------------------------------------------------------------
def _caller_inputs(fr, seed):
    """A chirp window and a Doppler table of the caller's own: positive
    weights in [0.2, 1.2] and the computed table moved by up to +-2 bins."""
    rng = np.random.default_rng(seed)
    k = SC.oracle_constants(fr)
    w = (0.2 + rng.random(fr.cfg.n_chirps)).astype(np.float32)
    fd = O.doppler_table(fr.pix.astype(np.float64), fr.q_tx, fr.q_rx, fr.vel, k["kd"])
    fd = (fd + rng.uniform(-2.0, 2.0, fd.shape)).astype(np.float32)
    return w, fd


@pytest.mark.parametrize("precision", PRECISIONS)
def test_caller_window_and_doppler_table(rc, torch, precision):
    """Alg. 2 with the caller's w_sar and f_doppler (its inputs in the
    paper's statement of the problem) against the oracle given the same."""
    fr = SC.small_frame(nx=64, ny=48, n_chirps=48)
    w, fd = _caller_inputs(fr, 61)
    kw = dict(precision=rc.RC_PREC_FP32_SPLIT if precision == SPLIT else rc.RC_PREC_FP32)
    with rc.Plan(SC.plan_config(rc, [fr], **kw)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, want_doppler=True, w_sar=w, f_doppler=fd)
    assert np.array_equal(out["doppler"], fd)          # the table is taken as given
    ora = SC.run_oracle(fr, cfar=None, w_sar=w, f_doppler=fd)
    _check_image("caller_inputs", fr, out["image"], ora, precision)
    # not the plan's own window and table: the images differ far beyond the bound
    own = SC.run_oracle(fr, cfar=None)
    assert np.abs(own["image"] - ora["image"]).max() > 0.1 * np.abs(ora["image"]).max()


def test_abi_errors_on_device(rc, torch):
    fr = SC.small_frame(nx=96, ny=96)
    cfg = SC.plan_config(rc, [fr], max_frames_in_flight=1, max_detections=1)
    with rc.Plan(cfg) as plan:
        t = SC.to_device(fr, torch)
        img = torch.empty((96 * 96, 2), dtype=torch.float32, device="cuda")
        mk = lambda fid, **kw: rc.Plan.make_frame(fid, data=t["raw"], q_tx=fr.q_tx, q_rx=fr.q_rx, vel=fr.vel,
                                                  pixels=t["pix"], n_rows=96, n_cols=96, n_bins=fr.n_bins,
                                                  n_fft=fr.n_fft, fs=fr.fs, n_samples=fr.cfg.n_samples,
                                                  image_out=img, **kw)
        over = mk(1)
        over.n_fft = fr.n_fft * 2                           # over n_fft_max
        with pytest.raises(rc.RcError) as ei:
            plan.process([over])
        assert ei.value.status == rc.RC_EINVAL
        bad = mk(2)
        bad.n_bins = fr.n_bins + 1
        with pytest.raises(rc.RcError) as ei:
            plan.process([bad])
        assert ei.value.status == rc.RC_EINVAL
        plan.process([mk(3)])
        assert plan.try_process([mk(4)]) == rc.RC_ENOTREADY  # single slot busy
        with pytest.raises(rc.RcError) as ei:
            plan.detections(99)
        assert ei.value.status == rc.RC_ENOTFOUND
        import ctypes as C
        buf = np.zeros(1, dtype=rc.DETECTION_DTYPE)
        n = C.c_int64()
        st = rc.lib.rc_detections(plan.handle, 3, buf.ctypes.data_as(C.POINTER(rc.rc_detection)), 0, C.byref(n))
        assert n.value >= 1, "the frame's targets must be detected"
        assert st == rc.RC_ETRUNC
        # more detections than the plan's capacity of one: truncated, true count reported
        st = rc.lib.rc_detections(plan.handle, 3, buf.ctypes.data_as(C.POINTER(rc.rc_detection)), 1, C.byref(n))
        assert st == (rc.RC_ETRUNC if n.value > 1 else rc.RC_OK)
        while not plan.poll(3):
            pass
        plan.release(3)
        plan.process([mk(4)])
        plan.release(4)
        # a caller's window with a non-finite weight, a window of a sub-aperture
        w = np.ones(fr.cfg.n_chirps, np.float32)
        w[3] = np.nan
        with pytest.raises(rc.RcError) as ei:
            plan.process([mk(6, w_sar=w)])
        assert ei.value.status == rc.RC_EINVAL
    with rc.Plan(SC.plan_config(rc, [fr], doppler=rc.RC_DOPPLER_EXACT)) as plan:
        fd = torch.zeros(96 * 96, dtype=torch.float32, device="cuda")
        with pytest.raises(rc.RcError) as ei:                # Alg. 1 has no Doppler table
            plan.process([mk(7, f_doppler=fd)])
        assert ei.value.status == rc.RC_EINVAL and "f_doppler" in rc.last_error()
    # a destroyed plan: the binding passes a null handle, which every entry
    # point rejects
    with pytest.raises(rc.RcError) as ei:
        plan.process([mk(5)])
    assert ei.value.status == rc.RC_EINVAL
    with pytest.raises(rc.RcError) as ei:
        plan.release(4)
    assert ei.value.status == rc.RC_EINVAL


# ---------------------------------------------------------------------------
# batches of frames of mixed sizes
# ---------------------------------------------------------------------------
def _mixed_frames(n):
    rng = np.random.default_rng(3000)
    frames = []
    for i in range(n):
        n_tx, n_rx = [(1, 4), (1, 8), (2, 4), (1, 2)][i % 4]
        shape = [(40, 37), (64, 64), (1, 300), (20, 90), (33, 16)][i % 5]
        cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name=f"mix{i}",
                                  n_samples=int(rng.choice([32, 64, 128])),
                                  n_chirps=int(rng.choice([6, 12, 24])), n_tx=n_tx, n_rx=n_rx,
                                  nx=shape[1], ny=shape[0], box=(-4.0, 4.0, 1.5, 7.0), n_targets=2,
                                  seed=3000 + i)
        frames.append(synth.make_frame(cfg, frame_index=i))
    return frames


@pytest.mark.parametrize("n_frames", [5, 19])
def test_batch_of_mixed_frames_matches_each_frame_alone(rc, torch, n_frames):
    """One rc_process_batch call over frames of different sizes, TX groupings
    and lattices: every image is bitwise identical to the same frame processed
    alone, and matches the oracle.  19 frames exceed one launch's 16."""
    frames = _mixed_frames(n_frames)
    cfg = SC.plan_config(rc, frames, max_frames_in_flight=n_frames)
    dev = torch.device("cuda")
    with rc.Plan(cfg) as plan:
        keep, descs, imgs = [], [], []
        for i, fr in enumerate(frames):
            t = SC.to_device(fr, torch)
            img = torch.empty((fr.n_rows * fr.n_cols, 2), dtype=torch.float32, device=dev)
            keep.append(t)
            imgs.append(img)
            descs.append(rc.Plan.make_frame(100 + i, data=t["raw"], q_tx=fr.q_tx, q_rx=fr.q_rx, vel=fr.vel,
                                            pixels=t["pix"], n_rows=fr.n_rows, n_cols=fr.n_cols,
                                            n_bins=fr.n_bins, n_fft=fr.n_fft, fs=fr.fs,
                                            n_samples=fr.cfg.n_samples, image_out=img))
        plan.process(descs)
        dets_mix = [plan.detections(100 + i) for i in range(n_frames)]
        torch.cuda.synchronize()
        mixed = [im.cpu().numpy().copy() for im in imgs]
        for i in range(n_frames):
            plan.release(100 + i)
        for i, fr in enumerate(frames):
            alone = SC.run_gpu(rc, plan, fr, torch, frame_id=500 + i)
            assert np.array_equal(alone["image"].view(np.float32).reshape(-1, 2), mixed[i]), f"frame {i}"
            assert np.array_equal(alone["detections"], dets_mix[i]), f"frame {i}"
    for i in (0, n_frames - 1):
        ora = SC.run_oracle(frames[i], cfar=None)
        _check_image(f"batch_frame{i}", frames[i], mixed[i].view(np.complex64).reshape(-1), ora, PLAIN)
