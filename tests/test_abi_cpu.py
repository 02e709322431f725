"""Host-side checks of the C ABI (no GPU work): the library loads, exports every
entry point rc.h declares, the ctypes mirror has the C layout, descriptor
validation and the host grid generators."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2306_09784_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rc.h")
LIB = os.path.join(ROOT, "paper_2306_09784_amd", "librc.so")


@pytest.fixture(scope="module")
def rc():
    if not os.path.exists(LIB):
        from paper_2306_09784_amd import build

        build.build()
    from paper_2306_09784_amd import rc as mod

    return mod


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rc_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_entry_point(rc):
    declared = _declared_functions()
    assert "rc_plan_create" in declared and "rc_process_batch" in declared
    lib = C.CDLL(LIB)
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(rc.ENTRY_POINTS) == declared


_LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "rc.h"
#define P(T, F) printf(#T "." #F " %zu\n", offsetof(T, F));
int main(void) {
  printf("rc_radar %zu\nrc_plan_desc %zu\nrc_frame %zu\nrc_detection %zu\nrc_tuning_entry %zu\n",
         sizeof(rc_radar), sizeof(rc_plan_desc), sizeof(rc_frame), sizeof(rc_detection), sizeof(rc_tuning_entry));
  P(rc_plan_desc, radar) P(rc_plan_desc, n_pix_max) P(rc_plan_desc, range_window)
  P(rc_plan_desc, range_kaiser_beta) P(rc_plan_desc, sar_kaiser_beta) P(rc_plan_desc, precision) P(rc_plan_desc, doppler)
  P(rc_plan_desc, cfar_pfa) P(rc_plan_desc, max_rechecks) P(rc_plan_desc, hbm_budget_bytes) P(rc_plan_desc, stage_timing)
  P(rc_plan_desc, sliding_sensors) P(rc_plan_desc, sliding_subapertures) P(rc_plan_desc, sliding_depth)
  P(rc_frame, fs) P(rc_frame, input_kind) P(rc_frame, data) P(rc_frame, pixels)
  P(rc_frame, n_rows) P(rc_frame, image_out) P(rc_frame, spectrum_out) P(rc_frame, height) P(rc_frame, sliding) P(rc_frame, w_sar) P(rc_frame, f_doppler)
  P(rc_detection, threshold) P(rc_detection, flags)
  P(rc_tuning_entry, n_channels) P(rc_tuning_entry, chirp_blocks) P(rc_tuning_entry, ms_chosen)
  return 0;
}
"""


def test_ctypes_layout_matches_header(rc, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(_LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    assert int(got["rc_radar"]) == C.sizeof(rc.rc_radar)
    assert int(got["rc_plan_desc"]) == C.sizeof(rc.rc_plan_desc)
    assert int(got["rc_frame"]) == C.sizeof(rc.rc_frame)
    assert int(got["rc_detection"]) == C.sizeof(rc.rc_detection) == rc.DETECTION_DTYPE.itemsize
    assert int(got["rc_tuning_entry"]) == C.sizeof(rc.rc_tuning_entry) == 32
    for key, val in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(getattr(rc, t), f).offset == int(val), key


def _cfg(rc, **kw):
    base = dict(radar=synth.RADAR, n_samples_max=256, n_fft_max=512, n_bins_max=256, n_chirps_max=128,
                n_channels_max=4, n_pix_max=65536)
    base.update(kw)
    return rc.PlanConfig(**base)


def test_descriptor_validation(rc):
    good = rc.slot_bytes(_cfg(rc))
    # pairs (16 B/bin) + image + tables per pixel dominate the slot
    assert good >= 128 * 4 * 256 * 16 + 65536 * (8 + 4 + 8 + 16)
    bad = [dict(n_fft_max=500), dict(n_fft_max=8192, n_samples_max=256), dict(n_bins_max=1024),
           dict(n_samples_max=1024), dict(cfar_guard=10, cfar_train=10), dict(cfar_pfa=1.5),
           dict(max_frames_in_flight=0), dict(precision=7), dict(range_window="bogus"), dict(doppler=5),
           dict(doppler=1, precision=1), dict(max_rechecks=-1), dict(max_rechecks=(1 << 20) + 1)]
    for kw in bad:
        with pytest.raises((rc.RcError, KeyError)) as ei:
            rc.slot_bytes(_cfg(rc, **kw))
        if isinstance(ei.value, rc.RcError):
            assert ei.value.status == rc.RC_EINVAL, kw
    # the recheck adds the double spectrum (16 B/bin), the cell list and the
    # window powers (441 doubles per listed cell)
    extra = rc.slot_bytes(_cfg(rc, max_rechecks=1000)) - good
    assert extra >= 128 * 4 * 256 * 16 + 1000 * (4 + 441 * 8)
    d = _cfg(rc).desc()
    d.abi_version = 99
    h = C.c_void_p()
    assert rc.lib.rc_plan_create(C.byref(d), C.byref(h)) == rc.RC_EINVAL
    assert "abi_version" in rc.last_error()


def test_sliding_descriptor_validation(rc):
    """Continuous SAR: K in [1, 64], depth in [1, max_frames_in_flight], and a
    chirp window that is a sum of cosines (Hann or rectangular); the ring of
    (K + depth - 1) partial images per sensor counts against the HBM budget."""
    ok = dict(sliding_sensors=2, sliding_subapertures=4, sliding_depth=2, max_frames_in_flight=4)
    rc.slot_bytes(_cfg(rc, **ok))
    rc.slot_bytes(_cfg(rc, **ok, sar_window="rect"))
    for kw in (dict(sliding_subapertures=0), dict(sliding_subapertures=65), dict(sliding_depth=0),
               dict(sliding_depth=5), dict(sar_window="kaiser"), dict(sliding_sensors=-1)):
        with pytest.raises(rc.RcError) as ei:
            rc.slot_bytes(_cfg(rc, **{**ok, **kw}))
        assert ei.value.status == rc.RC_EINVAL, kw
    # the Kaiser window is fine without continuous SAR
    rc.slot_bytes(_cfg(rc, sar_window="kaiser"))
    # 2 sensors x 5 ring slots x 3 planes x 65536 pixels x 8 B = 15.7 MB over a 15 MB budget
    slots = rc.slot_bytes(_cfg(rc, **ok)) * 4
    with pytest.raises(rc.RcError) as ei:
        rc.Plan(_cfg(rc, **ok, hbm_budget_bytes=slots + (1 << 20)))
    assert ei.value.status == rc.RC_ENOMEM and "budget" in rc.last_error()


def test_budget_rejection_before_any_device_call(rc):
    cfg = _cfg(rc, hbm_budget_bytes=1 << 20)
    with pytest.raises(rc.RcError) as ei:
        rc.Plan(cfg)
    assert ei.value.status == rc.RC_ENOMEM


def test_null_arguments(rc):
    assert rc.lib.rc_process_batch(None, None, 0, None) == rc.RC_EINVAL
    assert rc.lib.rc_poll(None, 1) == rc.RC_EINVAL
    assert rc.lib.rc_plan_destroy(None) == rc.RC_EINVAL


def test_cartesian_grid_matches_oracle(rc):
    g = rc.grid_cartesian(-15.0, 0.025, 1201, 1.0, 0.025, 1201)
    o = O.cartesian_grid(-15.0, 0.025, 1201, 1.0, 0.025, 1201).astype(np.float32)
    np.testing.assert_array_equal(g, o)


def test_polar_grid_matches_oracle(rc):
    lam = synth.RADAR["c"] / synth.RADAR["f0"]
    for box, L in [((-15, 15, 1, 31), 0.13), ((-7.5, 7.5, 1, 16), 0.5), ((2, 9, 3, 20), 1.7)]:
        p = rc.grid_polar_params(synth.RADAR, box, (0.0, 0.0), L)
        q = O.polar_grid_params(box, (0.0, 0.0), synth.RADAR["bandwidth"], lam, L)
        for k in ("r0", "dr", "th0", "dth"):
            assert p[k] == pytest.approx(q[k], rel=1e-15, abs=1e-15), k
        assert (p["nr"], p["nth"]) == (q["nr"], q["nth"])
        if p["nr"] * p["nth"] > 4_000_000:
            continue
        g = rc.grid_polar(p["ox"], p["oy"], p["r0"], p["dr"], p["nr"], p["th0"], p["dth"], p["nth"])
        o = O.polar_grid(q["ox"], q["oy"], q["r0"], q["dr"], q["nr"], q["th0"], q["dth"], q["nth"])
        # both round the same double expression once; libm and numpy may differ by
        # one double ulp in sin/cos, which can move a float by at most one ulp
        diff = np.abs(g.astype(np.float64) - o.astype(np.float32).astype(np.float64))
        ulp = np.spacing(np.abs(o).astype(np.float32)).astype(np.float64)
        assert np.all(diff <= ulp)


def test_polar_pixel_count_reported():
    """The paper's 165 061 polar pixels are not reproducible from the text
    (aperture length unstated); record what the grid rule gives at the paper's
    combined setting (1024 chirps at 1.2 m/s -> L = 0.131 m)."""
    lam = synth.RADAR["c"] / synth.RADAR["f0"]
    L = 1024 * synth.RADAR["t_pri"] * 1.2
    q = O.polar_grid_params((-15, 15, 1, 31), (0.0, 0.0), synth.RADAR["bandwidth"], lam, L)
    n = q["nr"] * q["nth"]
    assert 100_000 < n < 400_000


def _long_frame(rc, n_bins, n_samples=2048, f_doppler=None):
    """A frame of 2048 samples (fs = N / T_P, DFT 4096) keeping n_bins bins,
    4 chirps x 2 RX at 2 m/s; data and pixels are placeholders the check does
    not read."""
    M, CH = 4, 2
    q = np.zeros((M, CH, 2), np.float32)
    q[..., 0] = np.arange(CH) * 0.002
    vel = np.tile(np.array([[2.0, 0.0]], np.float32), (M, 1))
    fs = n_samples / synth.RADAR["t_chirp"]
    dummy = np.zeros(16, np.float32)
    return rc.Plan.make_frame(1, data=dummy, q_tx=q, q_rx=q.copy(), vel=vel, pixels=dummy, n_rows=4, n_cols=4,
                              n_bins=n_bins, n_fft=2 * n_samples, fs=fs, n_samples=n_samples,
                              f_doppler=f_doppler), (q, vel)


def test_single_precision_phase_range_guard(rc):
    """Alg. 2's exp(a2 d_hyp): the single-precision forms hand the whole path in
    wavelengths to the hardware sine/cosine, verified to 2^16 turns.  A frame
    whose bins reach paths beyond that is refused for RC_PREC_FP32 and the
    exact form, and accepted by the split-phase form."""
    R = synth.RADAR
    lam = R["c"] / R["f0"]
    df = 2048 / R["t_chirp"] / 4096
    a1 = R["bandwidth"] / R["t_chirp"] / (R["c"] * df)        # bins per metre of path
    limit_bins = int(65536 * lam * a1)                           # ~1630 bins here
    base = dict(n_samples_max=2048, n_fft_max=4096, n_bins_max=4096, n_chirps_max=4, n_channels_max=2,
                n_pix_max=16)
    ok_bins, bad_bins = limit_bins - 8, limit_bins + 8
    for prec, dop in ((rc.RC_PREC_FP32, rc.RC_DOPPLER_AVERAGE), (rc.RC_PREC_FP32, rc.RC_DOPPLER_EXACT)):
        cfg = _cfg(rc, **base, precision=prec, doppler=dop)
        fr, keep = _long_frame(rc, ok_bins)
        assert rc.validate_frame(cfg, fr) == rc.RC_OK, rc.last_error()
        fr, keep = _long_frame(rc, bad_bins)
        assert rc.validate_frame(cfg, fr) == rc.RC_EINVAL
        assert "RC_PREC_FP32_SPLIT" in rc.last_error()
    split = _cfg(rc, **base, precision=rc.RC_PREC_FP32_SPLIT)
    fr, keep = _long_frame(rc, 4096)
    assert rc.validate_frame(split, fr) == rc.RC_OK, rc.last_error()
    # a caller's Doppler table may hold up to n_bins - 1 bins: the bound doubles
    plain = _cfg(rc, **base)
    table = np.zeros(16, np.float32)
    half = limit_bins // 2 - 8
    fr, keep = _long_frame(rc, half)
    assert rc.validate_frame(plain, fr) == rc.RC_OK
    fr, keep = _long_frame(rc, ok_bins, f_doppler=table)
    assert rc.validate_frame(plain, fr) == rc.RC_EINVAL
    fr, keep = _long_frame(rc, half, f_doppler=table)
    assert rc.validate_frame(plain, fr) == rc.RC_OK, rc.last_error()


def test_benchmark_frames_pass_the_phase_range_guard(rc):
    """The benchmark's and the paper's frames stay far inside 2^16 turns."""
    for name in ("plain-large", "paper-polar", "plain-small"):
        cfg = synth.CONFIGS[name]
        M, CH = cfg.n_chirps, cfg.n_channels
        q = np.zeros((M, CH, 2), np.float32)
        vel = np.tile(np.array([[9.0, 0.0]], np.float32), (M, 1))
        fs = synth.sample_rate(cfg)
        n_bins = int(synth.required_bins(cfg, q, q, vel))
        dummy = np.zeros(16, np.float32)
        fr = rc.Plan.make_frame(1, data=dummy, q_tx=q, q_rx=q.copy(), vel=vel, pixels=dummy, n_rows=4, n_cols=4,
                                n_bins=n_bins, n_fft=cfg.n_fft, fs=fs, n_samples=cfg.n_samples)
        pc = _cfg(rc, n_samples_max=cfg.n_samples, n_fft_max=cfg.n_fft, n_bins_max=n_bins, n_chirps_max=M,
                  n_channels_max=CH, n_pix_max=16)
        assert rc.validate_frame(pc, fr) == rc.RC_OK, (name, rc.last_error())


def test_static_entry_point_refuses_before_any_device_call(rc):
    """rc_process_frame_static works in RC_STATIC_SCRATCH_BYTES of device
    memory it never allocates: a frame whose table alone exceeds it (1024
    chirps x 8 channels x 512 bins x 16 B = 64 MiB), a plan with the recheck,
    and missing outputs are refused on the host, before any HIP call."""
    M, CH, NB = 1024, 8, 512
    q = np.zeros((M, CH, 2), np.float32)
    vel = np.zeros((M, 2), np.float32)
    dummy = np.zeros(16, np.float32)
    img = np.zeros(32, np.float32)
    cfg = _cfg(rc, n_samples_max=1024, n_fft_max=2048, n_bins_max=NB, n_chirps_max=M, n_channels_max=CH,
               n_pix_max=16)
    fr = rc.Plan.make_frame(1, data=dummy, q_tx=q, q_rx=q.copy(), vel=vel, pixels=dummy, n_rows=4, n_cols=4,
                            n_bins=NB, n_fft=2048, fs=1024 / synth.RADAR["t_chirp"], n_samples=1024,
                            image_out=img)
    det = np.zeros(64, np.float32)
    cnt = np.zeros(1, np.int64)
    with pytest.raises(rc.RcError) as ei:
        rc.process_frame_static(cfg, fr, None, None, 0)
    assert ei.value.status == rc.RC_EINVAL
    import ctypes as C
    d = cfg.desc()
    st = rc.lib.rc_process_frame_static(C.byref(d), C.byref(fr), det.ctypes.data, 4, cnt.ctypes.data, None)
    assert st == rc.RC_EINVAL and "scratch" in rc.last_error()
    assert rc.STATIC_SCRATCH_BYTES == 32 << 20
    small = _cfg(rc, max_rechecks=8)
    d = small.desc()
    st = rc.lib.rc_process_frame_static(C.byref(d), C.byref(fr), det.ctypes.data, 4, cnt.ctypes.data, None)
    assert st == rc.RC_EINVAL and "recheck" in rc.last_error()


def _small_frame_desc(rc, n_chirps=16, n_ch=4, n_s=128, n_bins=100, rows=40, cols=50, image=True, host=False):
    q = np.zeros((n_chirps, n_ch, 2), np.float32)
    q[..., 0] = np.arange(n_ch) * 0.002
    vel = np.tile(np.array([[2.0, 0.0]], np.float32), (n_chirps, 1))
    dummy = np.zeros(16, np.float32)
    fr = rc.Plan.make_frame(1, data=None if host else dummy, q_tx=q, q_rx=q.copy(), vel=vel, pixels=dummy,
                            n_rows=rows, n_cols=cols, n_bins=n_bins, n_fft=2 * n_s,
                            fs=n_s / synth.RADAR["t_chirp"], n_samples=n_s, image_out=dummy if image else None,
                            data_host=dummy if host else None)
    return fr, (q, vel, dummy)


def test_frame_bytes_follow_the_frames_own_sizes(rc):
    """RC_MEMORY_BUDGET admits a frame by the device bytes its own sizes need:
    the interpolation table (16 B per chirp, channel and bin) and per-pixel
    buffers grow with the frame, a plan's image buffer is counted only without
    image_out, the input only when it comes from pinned host memory."""
    cfg = _cfg(rc, hbm_budget_bytes=1 << 30, frame_memory=rc.RC_MEMORY_BUDGET)
    base, k1 = _small_frame_desc(rc)
    b0 = rc.frame_bytes(cfg, base)
    twice, k2 = _small_frame_desc(rc, n_chirps=32)
    assert rc.frame_bytes(cfg, twice) - b0 >= 16 * 4 * 100 * 16     # 16 more chirps of table
    no_img, k3 = _small_frame_desc(rc, image=False)
    assert rc.frame_bytes(cfg, no_img) - b0 >= 40 * 50 * 8            # the image in the arena
    host, k4 = _small_frame_desc(rc, host=True)
    assert rc.frame_bytes(cfg, host) - b0 >= 16 * 4 * 128 * 8         # the input cube
    # far below a slot sized for the plan's limits (128 chirps x 4 x 256 bins, 65536 px)
    assert b0 < rc.slot_bytes(_cfg(rc)) / 4


def test_budget_mode_refusals(rc):
    """The arena is the budget: a budget plan without a budget, host input
    outside budget mode, host input next to a device pointer, and a budget
    smaller than the plan's fixed needs are refused before any device call."""
    with pytest.raises(rc.RcError) as ei:
        rc.slot_bytes(_cfg(rc, frame_memory=rc.RC_MEMORY_BUDGET))
    assert ei.value.status == rc.RC_EINVAL and "hbm_budget_bytes" in rc.last_error()
    host, keep = _small_frame_desc(rc, host=True)
    assert rc.validate_frame(_cfg(rc), host) == rc.RC_EINVAL and "data_host" in rc.last_error()
    both, keep2 = _small_frame_desc(rc, host=True)
    both.data = keep2[2].ctypes.data
    assert rc.validate_frame(_cfg(rc, hbm_budget_bytes=1 << 30, frame_memory=rc.RC_MEMORY_BUDGET),
                             both) == rc.RC_EINVAL
    with pytest.raises(rc.RcError) as ei:   # the recheck's twiddles alone exceed 4 kB
        rc.Plan(_cfg(rc, hbm_budget_bytes=4096, frame_memory=rc.RC_MEMORY_BUDGET, max_rechecks=8))
    assert ei.value.status == rc.RC_ENOMEM
