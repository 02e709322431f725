"""The reduced-precision spectrum forms (RC_PREC_FP16, RC_PREC_BF16): range
compression on the matrix cores against the FP64 oracle's DFT, and the
pipeline built on them (split-phase back-projection) against the oracle's
image.

Tolerances: the spectrum within 3e-3 relative L2 of the FP64 DFT for every
DFT length the form takes (256 .. 4096, n_samples <= n_fft / 2); derived from
the arithmetic, FP16 rounds the data operand twice (entry, between the
stages) at 2^-12 relative (~2.4e-4 rms each), BF16 splits it into hi + lo
(~2^-16); the twiddles are split hi + lo in both.  Expected: ~3e-4 (FP16) and
~1e-5 (BF16).  The image: the spectrum's relative error carries over to each
term, so max|dP| / max|P| stays at the spectrum's level: 3e-3.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2306_09784_amd import synth
from tests import sar_cases as SC

pytestmark = pytest.mark.gpu

SPEC_TOL = 3e-3
IMG_TOL = 3e-3
FORMS = [pytest.param(2, id="fp16"), pytest.param(3, id="bf16")]


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


def _report(name, **vals):
    vals = {k: (float(v) if isinstance(v, (np.floating, float)) else int(v)) for k, v in vals.items()}
    print(name, vals, flush=True)
    path = os.environ.get("RC_REPORT")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps({"case": name, **vals}) + "\n")


def _spectrum(rc, torch, raw, n_fft, n_bins, form):
    M, CH, n_s = raw.shape
    q = np.zeros((M, CH, 2), np.float32)
    vel = np.zeros((M, 2), np.float32)
    pix = np.array([[0.0, 5.0], [0.1, 5.0]], np.float32)
    dev = torch.device("cuda")
    d_raw = torch.from_numpy(raw).to(dev)
    d_pix = torch.from_numpy(pix).to(dev)
    spec = torch.empty((M, CH, n_bins, 2), dtype=torch.float32, device=dev)
    img = torch.empty((2, 2), dtype=torch.float32, device=dev)
    cfg = rc.PlanConfig(radar=synth.RADAR, n_samples_max=n_s, n_fft_max=n_fft, n_bins_max=n_bins,
                        n_chirps_max=M, n_channels_max=CH, n_pix_max=2, max_frames_in_flight=1, precision=form)
    with rc.Plan(cfg) as plan:
        fr = rc.Plan.make_frame(1, data=d_raw, q_tx=q, q_rx=q, vel=vel, pixels=d_pix, n_rows=1, n_cols=2,
                                n_bins=n_bins, n_fft=n_fft, fs=n_s / synth.RADAR["t_chirp"], n_samples=n_s,
                                image_out=img, spectrum_out=spec)
        plan.process([fr])
        plan.detections(1)
        torch.cuda.synchronize()
        got = spec.cpu().numpy().view(np.complex64)[..., 0].astype(np.complex128)
        plan.release(1)
    return got


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("log2n,n_s,n_bins", [(8, 128, 77), (8, 97, 256), (9, 256, 222), (9, 200, 512),
                                                (10, 512, 433), (10, 333, 101), (11, 1024, 432),
                                                (11, 1000, 2048), (12, 2048, 900), (12, 1500, 4096)])
def test_mfma_spectrum_every_dft_length(rc, torch, form, log2n, n_s, n_bins):
    """Every DFT length and ragged sample/bin counts, on 21 rows whose
    amplitudes span 1e-3 .. 1e4 (each row's FP16 scale is its own), with a
    strong tone inside the kept bins (a target in the scene)."""
    n_fft = 1 << log2n
    M, CH = 7, 3
    rng = np.random.default_rng(500 + log2n + n_s)
    raw = rng.standard_normal((M, CH, n_s)) + 1j * rng.standard_normal((M, CH, n_s))
    t = np.arange(n_s)
    raw = raw + 20.0 * np.exp(2j * np.pi * (0.37 * n_bins / n_fft) * t)   # a strong tone in the kept band
    raw *= np.logspace(-3, 4, M * CH).reshape(M, CH, 1)
    raw = raw.astype(np.complex64)
    got = _spectrum(rc, torch, raw, n_fft, n_bins, form)
    ref = O.range_compress(raw, O.window("hann", n_s), n_fft, n_bins)
    rel_rows = np.linalg.norm(got - ref, axis=-1) / np.linalg.norm(ref, axis=-1)
    _report(f"mfma_spectrum_{'fp16' if form == 2 else 'bf16'}_{n_fft}_{n_s}_{n_bins}",
            rel_l2_max_row=float(rel_rows.max()), rel_l2_median_row=float(np.median(rel_rows)))
    assert rel_rows.max() <= SPEC_TOL


@pytest.mark.parametrize("form", FORMS)
def test_mfma_spectrum_error_is_relative_to_the_whole_band(rc, torch, form):
    """The 16-bit data operand rounds relative to the row's largest sample, so
    the error is a fraction of the whole spectrum's energy (Parseval), not of
    the kept bins': a strong tone outside the kept band leaves an error that
    is 3e-3 of the full-band norm but can exceed that of the weak kept part."""
    n_fft, n_s, n_bins = 1024, 333, 101
    M, CH = 4, 2
    rng = np.random.default_rng(77)
    t = np.arange(n_s)
    raw = rng.standard_normal((M, CH, n_s)) + 1j * rng.standard_normal((M, CH, n_s))
    raw = (raw + 20.0 * np.exp(2j * np.pi * 0.173 * t)).astype(np.complex64)  # bin 177: not kept
    got = _spectrum(rc, torch, raw, n_fft, n_bins, form)
    w = O.window("hann", n_s)
    ref = O.range_compress(raw, w, n_fft, n_bins)
    full = O.range_compress(raw, w, n_fft, n_fft)
    rel_full = np.linalg.norm(got - ref, axis=-1) / np.linalg.norm(full, axis=-1)
    _report(f"mfma_spectrum_{'fp16' if form == 2 else 'bf16'}_out_of_band_tone",
            rel_full_band_max=float(rel_full.max()),
            rel_kept_max=float((np.linalg.norm(got - ref, axis=-1) / np.linalg.norm(ref, axis=-1)).max()))
    assert rel_full.max() <= SPEC_TOL


@pytest.mark.parametrize("form", FORMS)
def test_mfma_spectrum_refuses_other_lengths(rc, torch, form):
    raw = np.ones((2, 2, 100), np.complex64)
    with pytest.raises(rc.RcError) as ei:       # n_samples > n_fft / 2
        _spectrum(rc, torch, raw, 128, 50, form)
    assert ei.value.status == rc.RC_EINVAL and "matrix-core" in rc.last_error()


@pytest.mark.parametrize("form", FORMS)
def test_mfma_form_image_matches_oracle(rc, torch, form):
    """plain-small frame (256 samples x 128 chirps x 4 RX, DFT 512) through the
    reduced-precision spectrum and split-phase back-projection."""
    fr = SC.small_frame(nx=96, ny=80)
    with rc.Plan(SC.plan_config(rc, [fr], precision=form)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, want_spectrum=True)
    ora = SC.run_oracle(fr, cfar=None)
    s, so = out["spectrum"].astype(np.complex128), ora["spectrum"]
    spec_rel = float(np.linalg.norm(s - so) / np.linalg.norm(so))
    P = ora["image"]
    img_rel = float(np.abs(out["image"].astype(np.complex128) - P).max() / np.abs(P).max())
    _report(f"mfma_image_small_{'fp16' if form == 2 else 'bf16'}", spectrum_rel_l2=spec_rel, image_max_rel=img_rel)
    assert spec_rel <= SPEC_TOL
    assert img_rel <= IMG_TOL
