"""GPU parity of the double-precision recheck of near-threshold CFAR decisions.

With ``max_rechecks`` > 0 every cell whose single-precision statistic lies in
the band |p - thr| <= cfar_margin_rel * thr is decided again from its own
pixel and every training pixel formed by back-projection in double, from a
beat spectrum formed again in double.  The test knows the band exactly: the
single-precision image is an output of the same call, and p and thr of every
cell follow from it in double as the CFAR kernel forms them.  So:

  * outside the band the decision is the single-precision one, p > thr of the
    returned image, and a detection carries no flag;
  * inside the band a detection carries RC_DET_RECHECKED, and the decision
    is the oracle's, except where the oracle's own margin |p - thr| is within
    the double-precision rounding of the two evaluations.

That rounding is bounded through the spectrum: a radix-2 FFT in double has a
relative L2 error of a few log2(N) * 2^-53, so no bin is off by more than
1e-12 max_bins |s| on either side (the oracle's FFT included) and, with

  B = sum over (chirp, channel) of w_sar[m] * 2e-12 * max_bins |s|,

|P_recheck - P_oracle| <= B at every pixel up to the far smaller rounding of
the sum itself (linear interpolation never exceeds the larger error of its two
bins).  A cell's power is then uncertain by 2|P|B + B^2 and its threshold by
alpha/N times the training sum of that.  Rechecked detections report the
oracle's power and threshold within the same bound plus the rounding of the
single-precision record.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2306_09784_amd import synth
from tests import sar_cases as SC
from tests.test_gpu_parity import PLAIN, SPLIT, _report

pytestmark = pytest.mark.gpu

GUARD, TRAIN, PFA = 2, 8, 1e-4
H = GUARD + TRAIN
N_TRAIN = (2 * H + 1) ** 2 - (2 * GUARD + 1) ** 2
ALPHA = O.cfar_alpha(N_TRAIN, PFA)
MARGIN = 0.5
EDGE = 1e-9   # summation-order slack between the CFAR kernel and numpy


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


def _train_sum(x):
    R, C = x.shape
    view = np.lib.stride_tricks.sliding_window_view
    outer = view(x, (2 * H + 1, 2 * H + 1)).sum(axis=(-1, -2))
    inner = view(x, (2 * GUARD + 1, 2 * GUARD + 1)).sum(axis=(-1, -2))
    off = H - GUARD
    return outer - inner[off:off + R - 2 * H, off:off + C - 2 * H]


def _stat(power):
    """(cell power, threshold) over the tested cells of a power lattice."""
    R, C = power.shape
    return power[H:R - H, H:C - H], ALPHA * _train_sum(power) / N_TRAIN


def _table_bound(spec_oracle, w_sar):
    m = np.abs(spec_oracle.astype(np.complex128)).max(-1)
    return float((w_sar[:, None] * 2e-12 * m).sum())


def _run(rc, torch, frame, spectrum=None, **plan_kw):
    with rc.Plan(SC.plan_config(rc, [frame], cfar_margin_rel=MARGIN, **plan_kw)) as plan:
        return SC.run_gpu(rc, plan, frame, torch, spectrum=spectrum)


def _classify(frame, ora, out, table_err):
    """Per tested cell: GPU single-precision p, thr, band membership; oracle
    decision and whether the recheck bound covers the oracle's margin."""
    R, C = frame.n_rows, frame.n_cols
    z = out["image"].reshape(R, C)
    pw_g = z.real.astype(np.float64) ** 2 + z.imag.astype(np.float64) ** 2
    p_g, thr_g = _stat(pw_g)
    gap_g = np.abs(p_g - thr_g)
    in_band = gap_g <= MARGIN * thr_g
    ambiguous = (np.abs(gap_g - MARGIN * thr_g) <= EDGE * thr_g) | (gap_g <= EDGE * thr_g)
    p_o, thr_o = _stat(ora["power"])
    dpow = 2.0 * np.sqrt(ora["power"]) * table_err + table_err ** 2
    d_cell, d_thr = _stat(dpow)
    unc = d_cell + d_thr
    fragile64 = np.abs(p_o - thr_o) <= unc
    det_o = np.zeros((R, C), bool)
    det_o.flat[ora["cfar"][0]] = True
    return dict(p_g=p_g, thr_g=thr_g, in_band=in_band, ambiguous=ambiguous, det32=p_g > thr_g,
                det_o=det_o[H:R - H, H:C - H], fragile64=fragile64, p_o=p_o, thr_o=thr_o, unc=unc)


def _check(name, frame, ora, out, table_err, cap=None):
    R, C = frame.n_rows, frame.n_cols
    k = _classify(frame, ora, out, table_err)
    assert not k["ambiguous"].any()
    dets = out["detections"]
    assert np.all(np.diff(dets["pixel"]) > 0)
    det_g = np.zeros((R, C), bool)
    det_g.flat[dets["pixel"]] = True
    det_g = det_g[H:R - H, H:C - H]
    flags = np.zeros((R, C), np.int64)
    flags.flat[dets["pixel"]] = dets["flags"]
    flags = flags[H:R - H, H:C - H]
    band, det32, det_o = k["in_band"], k["det32"], k["det_o"]
    n_band = int(band.sum())

    # outside the band: the single-precision decision, no flag
    assert np.array_equal(det_g[~band], det32[~band])
    assert not flags[~band].any()
    # inside the band: rechecked cells take the oracle's decision
    rechecked = det_g & ((flags & 2) != 0)
    assert not (rechecked & ~band).any()
    if cap is None or n_band <= cap:
        assert not ((flags & 1) != 0).any()
        bad = band & (det_g != det_o) & ~k["fragile64"]
    else:
        # the listed subset is unknown; a band cell shows either decision, a
        # rechecked detection the oracle's, an unrechecked one the FP32 one
        near = det_g & ((flags & 1) != 0)
        assert int(rechecked.sum()) <= cap
        assert np.array_equal(det_g[near], det32[near])
        bad = rechecked & ~det_o & ~k["fragile64"]
    idx = np.argwhere(bad)
    assert idx.size == 0, [(int(r + H) * C + int(c + H), float(k["p_o"][r, c]), float(k["thr_o"][r, c]))
                           for r, c in idx[:5]]
    # rechecked detections report the oracle's power and threshold
    worst_p = worst_t = 0.0
    for d in dets[(dets["flags"] & 2) != 0]:
        r, c = divmod(int(d["pixel"]), C)
        r, c = r - H, c - H
        p_o, t_o, u = k["p_o"][r, c], k["thr_o"][r, c], k["unc"][r, c]
        dp, dt = abs(float(d["power"]) - p_o), abs(float(d["threshold"]) - t_o)
        worst_p, worst_t = max(worst_p, dp / p_o), max(worst_t, dt / t_o)
        assert dp <= u + 2.0 ** -23 * p_o and dt <= u + 2.0 ** -23 * t_o, (int(d["pixel"]), dp, dt, u)
    n_fix = int((band & (det32 != det_o) & (det_g == det_o)).sum())
    _report(f"recheck_{name}", n_dets=len(dets), n_oracle=int(det_o.sum()), band_cells=n_band,
            rechecked_dets=int(rechecked.sum()), fp32_band_mismatch=int((band & (det32 != det_o)).sum()),
            fixed_by_recheck=n_fix, fragile_after=int((band & k["fragile64"]).sum()),
            table_bound=table_err, power_rel=worst_p, thr_rel=worst_t)
    assert n_band > 0
    return k


def test_recheck_caller_window_and_doppler_table(rc, torch):
    """The recheck forms its pixels in double with the caller's window and
    Doppler table too."""
    from tests.test_gpu_parity import _caller_inputs

    fr = SC.small_frame(nx=160, ny=160)
    w, fd = _caller_inputs(fr, 62)
    with rc.Plan(SC.plan_config(rc, [fr], cfar_margin_rel=MARGIN, max_rechecks=1 << 16)) as plan:
        out = SC.run_gpu(rc, plan, fr, torch, w_sar=w, f_doppler=fd)
    ora = SC.run_oracle(fr, cfar=(GUARD, TRAIN, PFA), w_sar=w, f_doppler=fd)
    _check("caller_inputs", fr, ora, out, _table_bound(ora["spectrum"], ora["w_sar"]))


@pytest.mark.parametrize("precision", [pytest.param(PLAIN, id="fp32"), pytest.param(SPLIT, id="split")])
def test_recheck_end_to_end(rc, torch, precision):
    fr = SC.small_frame(nx=192, ny=192)
    ora = SC.run_oracle(fr)
    out = _run(rc, torch, fr, precision=precision, max_rechecks=8192)
    tb = _table_bound(ora["spectrum"], ora["w_sar"])
    _check("raw_" + ("split" if precision == SPLIT else "fp32"), fr, ora, out, tb)


def test_recheck_spectrum_input(rc, torch):
    """Spectrum input: the oracle and the recheck start from the same complex64 samples."""
    fr = SC.small_frame(nx=128, ny=112)
    spec = SC.run_oracle(fr, cfar=None)["spectrum"].astype(np.complex64)
    ora = SC.run_oracle(fr, spectrum=spec)
    out = _run(rc, torch, fr, spectrum=spec, max_rechecks=8192)
    _check("spectrum", fr, ora, out, _table_bound(spec, ora["w_sar"]))


def test_recheck_exact_doppler(rc, torch):
    """Exact-Doppler plans recheck with Alg. 1 (per-chirp radial velocities) on a turning drive."""
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="yaw-recheck", nx=96, ny=80, n_chirps=64,
                              yaw_rate=25.0, seed=23)
    fr = synth.make_frame(cfg)
    ora = SC.run_oracle(fr, doppler="exact")
    out = _run(rc, torch, fr, doppler=rc.RC_DOPPLER_EXACT, max_rechecks=8192)
    _check("exact", fr, ora, out, _table_bound(ora["spectrum"], ora["w_sar"]))


def test_recheck_capacity(rc, torch):
    """A capacity below the band size: at most that many cells are rechecked,
    the rest keep the single-precision decision, flagged near-threshold."""
    fr = SC.small_frame(nx=128, ny=128)
    ora = SC.run_oracle(fr)
    out = _run(rc, torch, fr, max_rechecks=3)
    k = _check("capacity", fr, ora, out, _table_bound(ora["spectrum"], ora["w_sar"]), cap=3)
    assert int(k["in_band"].sum()) > 3
