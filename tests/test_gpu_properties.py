"""Properties of back-projection checked on the GPU path (seeded Hypothesis):
linearity in the spectrum, pixel-list permutation (bitwise), coincident
points of a polar and a Cartesian list (bitwise), channel-subset additivity
(Sec. III-F), and the scaling of back-projection time with the pixel and
channel counts (Sec. III-E/F: time proportional to both)."""
import dataclasses
import math

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle as O
from paper_2306_09784_amd import synth
from tests import sar_cases as SC

pytestmark = pytest.mark.gpu

R = synth.RADAR
SETTINGS = settings(max_examples=4, deadline=None, derandomize=True)


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
def frame():
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="prop", n_samples=64, n_chirps=16, n_rx=8,
                              nx=40, ny=24, box=(-4.0, 4.0, 1.5, 7.0), seed=900)
    return synth.make_frame(cfg)


def _image(rc, torch, fr, spec, pix=None, n_rows=None, n_cols=None, chans=None, plan_kw=None):
    """Back-projects a spectrum [M, CH, NB] (optionally a channel subset) on a
    pixel list; returns the complex64 image."""
    pix = fr.pix if pix is None else pix
    n_rows = fr.n_rows if n_rows is None else n_rows
    n_cols = fr.n_cols if n_cols is None else n_cols
    q_tx, q_rx = fr.q_tx, fr.q_rx
    if chans is not None:
        spec = spec[:, chans]
        q_tx = np.ascontiguousarray(q_tx[:, chans])
        q_rx = np.ascontiguousarray(q_rx[:, chans])
    dev = torch.device("cuda")
    d_spec = torch.from_numpy(np.ascontiguousarray(spec.astype(np.complex64))).to(dev)
    d_pix = torch.from_numpy(np.ascontiguousarray(pix.astype(np.float32))).to(dev)
    img = torch.empty((n_rows * n_cols, 2), dtype=torch.float32, device=dev)
    cfg = rc.PlanConfig(radar=R, n_samples_max=4, n_fft_max=fr.n_fft, n_bins_max=fr.n_bins,
                        n_chirps_max=fr.cfg.n_chirps, n_channels_max=fr.cfg.n_channels,
                        n_pix_max=n_rows * n_cols, **(plan_kw or {}))
    with rc.Plan(cfg) as plan:
        f = rc.Plan.make_frame(1, data=d_spec, q_tx=q_tx, q_rx=q_rx, vel=fr.vel, pixels=d_pix, n_rows=n_rows,
                               n_cols=n_cols, n_bins=fr.n_bins, n_fft=fr.n_fft, fs=fr.fs,
                               input_kind=rc.RC_INPUT_SPECTRUM, image_out=img)
        plan.process([f])
        plan.detections(1)
        torch.cuda.synchronize()
    return img.cpu().numpy().view(np.complex64).reshape(-1)


def _bound(fr, spec, pix=None):
    """Single-precision error bound of an image (as in the parity tests, with
    the plain form's phase bound): (2 pi e + gamma) sum |terms| + floor."""
    pix = fr.pix.astype(np.float64) if pix is None else pix.astype(np.float64)
    k = SC.oracle_constants(fr)
    fd = O.doppler_table(pix, fr.q_tx, fr.q_rx, fr.vel, k["kd"])
    w = O.window("hann", fr.cfg.n_chirps)
    S = O.bp_alg2_abs(pix, fr.q_tx, fr.q_rx, fd, spec, w, k["a1"])
    q = np.concatenate([fr.q_tx.reshape(-1, 2), fr.q_rx.reshape(-1, 2)]).astype(np.float64)
    lo, hi = pix.min(0), pix.max(0)
    corners = np.array([[lo[0], lo[1]], [hi[0], hi[1]], [lo[0], hi[1]], [hi[0], lo[1]]])
    d_max = 2 * np.sqrt(((corners[:, None, :] - q[None]) ** 2).sum(-1)).max()
    e = 2.0 ** -22 * d_max / (R["c"] / R["f0"]) + 1e-5
    gamma = (fr.cfg.n_chirps * fr.cfg.n_channels / 2 + 2) * 2.0 ** -24
    return (2 * math.pi * e + gamma) * S


@SETTINGS
@given(a_re=st.floats(-2, 2), a_im=st.floats(-2, 2), b_re=st.floats(-2, 2), b_im=st.floats(-2, 2),
       seed=st.integers(0, 2 ** 16))
def test_linearity_in_the_spectrum(rc, torch, frame, a_re, a_im, b_re, b_im, seed):
    """P(a s1 + b s2) = a P(s1) + b P(s2) to the single-precision bound."""
    rng = np.random.default_rng(seed)
    shape = (frame.cfg.n_chirps, frame.cfg.n_channels, frame.n_bins)
    s1 = synth.random_spectrum(rng, shape).astype(np.complex128)
    s2 = synth.random_spectrum(rng, shape).astype(np.complex128)
    a, b = complex(a_re, a_im), complex(b_re, b_im)
    mix = (a * s1 + b * s2).astype(np.complex64)
    lhs = _image(rc, torch, frame, mix).astype(np.complex128)
    rhs = a * _image(rc, torch, frame, s1).astype(np.complex128) + b * _image(rc, torch, frame, s2)
    # each side within its own bound of the exact value
    bound = _bound(frame, mix) + abs(a) * _bound(frame, s1) + abs(b) * _bound(frame, s2)
    floor = 1e-5 * (np.abs(lhs).max() + 1e-30)
    assert np.all(np.abs(lhs - rhs) <= bound + floor)


@SETTINGS
@given(seed=st.integers(0, 2 ** 16))
def test_pixel_permutation_is_bitwise(rc, torch, frame, seed):
    """Back-projection is pointwise: the image of a permuted pixel list is the
    permuted image, bit for bit (same lattice shape, so the same chirp split)."""
    rng = np.random.default_rng(seed)
    spec = synth.random_spectrum(rng, (frame.cfg.n_chirps, frame.cfg.n_channels, frame.n_bins))
    perm = rng.permutation(frame.pix.shape[0])
    img = _image(rc, torch, frame, spec)
    img_p = _image(rc, torch, frame, spec, pix=frame.pix[perm])
    assert np.array_equal(img_p.view(np.uint32), img[perm].view(np.uint32))


def test_polar_and_cartesian_coincident_points_are_bitwise(rc, torch, frame):
    """Points shared by a polar lattice and a Cartesian list get the same value,
    bit for bit: the grid only chooses where P is evaluated (Sec. III-E)."""
    rng = np.random.default_rng(5)
    spec = synth.random_spectrum(rng, (frame.cfg.n_chirps, frame.cfg.n_channels, frame.n_bins))
    # a polar lattice of the Cartesian list's shape (same chirp split and
    # summation order), theta slow
    pol = rc.grid_polar(0.0, 0.0, 2.0, 0.05, frame.n_cols, -0.5, 0.04, frame.n_rows)
    cart = frame.pix.copy()
    take = rng.choice(pol.shape[0], 200, replace=False)
    where = rng.choice(cart.shape[0], 200, replace=False)
    cart[where] = pol[take]
    img_p = _image(rc, torch, frame, spec, pix=pol)
    img_c = _image(rc, torch, frame, spec, pix=cart)
    assert np.array_equal(img_c[where].view(np.uint32), img_p[take].view(np.uint32))


@SETTINGS
@given(seed=st.integers(0, 2 ** 16))
def test_channel_subsets_add_up(rc, torch, frame, seed):
    """P(channels 0..3) + P(channels 4..7) = P(all 8) (Sec. III-F), to the bound."""
    rng = np.random.default_rng(seed)
    spec = synth.random_spectrum(rng, (frame.cfg.n_chirps, frame.cfg.n_channels, frame.n_bins))
    full = _image(rc, torch, frame, spec).astype(np.complex128)
    half_a = _image(rc, torch, frame, spec, chans=slice(0, 4)).astype(np.complex128)
    half_b = _image(rc, torch, frame, spec, chans=slice(4, 8)).astype(np.complex128)
    bound = 2 * _bound(frame, spec.astype(np.complex128))
    assert np.all(np.abs(half_a + half_b - full) <= bound + 1e-5 * np.abs(full).max())


def test_bp_time_scales_with_pixels_and_channels(rc, torch):
    """Back-projection time is proportional to the pixel count and to the
    channel count (Sec. III-E/F): the median device time of frames with 4x the
    pixels and 2x the channels is 4x and 2x, within 15 % (1024 x 1024 pixels,
    256 chirps x 8 channels as the base, about 1 ms, so that fixed costs and
    the launch's ragged end are a few per cent).  Both ratios come out a
    little low: the larger frames split their chirps into fewer blocks (two
    instead of four at 2048 x 2048), so they write and sum fewer partial images
    per term (measured 3.55x and 1.90x), and twice the channels share each TX
    distance among more of them."""
    def bp_ms(nx, n_rx):
        cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="scale", n_samples=256, n_chirps=256,
                                  n_rx=n_rx, nx=nx, ny=nx, seed=950)
        fr = synth.make_frame(cfg, device="cuda")
        dev = torch.device("cuda")
        raw = torch.from_numpy(fr.raw).to(dev)
        pix = torch.from_numpy(fr.pix).to(dev)
        img = torch.empty((fr.n_rows * fr.n_cols, 2), dtype=torch.float32, device=dev)
        pc = SC.plan_config(rc, [fr], stage_timing=True)
        times = []
        with rc.Plan(pc) as plan:
            for i in range(7):
                f = rc.Plan.make_frame(i, data=raw, q_tx=fr.q_tx, q_rx=fr.q_rx, vel=fr.vel, pixels=pix,
                                       n_rows=fr.n_rows, n_cols=fr.n_cols, n_bins=fr.n_bins, n_fft=fr.n_fft,
                                       fs=fr.fs, n_samples=cfg.n_samples, image_out=img)
                plan.process([f])
                times.append(plan.stage_times(i)[2])
                plan.release(i)
        return float(np.median(times[2:]))

    base = bp_ms(1024, 8)
    px = bp_ms(2048, 8) / base
    ch = bp_ms(1024, 16) / base
    print(f"bp time ratios: 4x pixels {px:.3f}, 2x channels {ch:.3f}", flush=True)
    assert 0.85 * 4 <= px <= 1.15 * 4
    assert 0.85 * 2 <= ch <= 1.15 * 2
