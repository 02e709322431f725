"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the pin it checks: figures the paper prints, closed forms,
library routines the oracle does not call, brute force on tiny inputs and
invariants of back-projection.  CPU only.
"""
import dataclasses
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2306_09784_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
R = synth.RADAR


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# Figures printed in the paper
# ---------------------------------------------------------------------------
def test_paper_printed_numbers():
    g = _golden("paper_numbers.json")
    tab1 = g["radar_tab1"]
    # Tab. I parameters are the ones the simulator uses
    assert tab1["f0_hz"] == R["f0"] and tab1["bandwidth_hz"] == R["bandwidth"]
    assert tab1["t_chirp_s"] == R["t_chirp"] and tab1["t_pri_s"] == R["t_pri"]
    # real-time bound N_m T_P0 (Sec. III)
    assert round(tab1["n_chirps"] * tab1["t_pri_s"] * 1e3, 1) == g["realtime_bound_ms"]["value"]
    # 30 m at 2.5 cm -> 1201 x 1201 (Sec. II)
    cg = g["cartesian_grid"]
    n = int(round(cg["extent_m"] / cg["step_m"])) + 1
    assert n == cg["n_side"] and n * n == cg["n_pix"]
    pix = O.cartesian_grid(-15.0, 0.025, n, 1.0, 0.025, n)
    assert pix.shape == (cg["n_pix"], 2)
    # window sizes in float32 (Sec. III-B)
    assert round(tab1["n_chirps"] * 4 / 1e3, 2) == g["window_vector_kb"]["value"]
    assert round(cg["n_pix"] * tab1["n_chirps"] * 4 / 1e9, 2) == g["window_full_gb"]["value"]
    # polar share of the Cartesian grid (Sec. III-E); the paper rounds 11.44 % to 11.5 %
    share = 100.0 * g["polar_pixels"]["n_pix"] / cg["n_pix"]
    assert abs(share - g["polar_pixels"]["percent"]) < 0.1
    # chirps combined (abstract) = chirps x reduced RX count (Sec. III-F)
    assert tab1["n_chirps"] * g["rx_reduction"]["to"] == g["chirps_combined"]["value"]
    # RX halving costs at most 20 log10(2) = 6.02 dB of coherent gain (Sec. III-F)
    assert 20 * math.log10(g["rx_reduction"]["from"] / g["rx_reduction"]["to"]) == pytest.approx(6.0206, abs=1e-4)


def test_radar_constants_closed_form():
    fs, nfft = 10e6, 2048
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], fs, nfft)
    # df = 1 / (Z T_P) when fs = N_s / T_P and n_fft = Z N_s
    assert k["df"] == pytest.approx(1.0 / (2 * R["t_chirp"]), rel=1e-15)
    # a1: one metre of two-way path is mu / c Hz of beat frequency
    assert k["a1"] * k["df"] == pytest.approx(R["bandwidth"] / R["t_chirp"] / R["c"], rel=1e-15)
    # a2 d over one wavelength of path is one full turn
    assert abs(k["a2"] * k["lam"]) == pytest.approx(2 * math.pi, rel=1e-15)
    # range resolution c / 2B = 16.1 cm and the paper's polar step = 1 / 2.5 of it
    assert R["c"] / (2 * R["bandwidth"]) == pytest.approx(0.16100, abs=1e-5)


# ---------------------------------------------------------------------------
# Windows: against scipy's independent implementations
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 7, 64, 1024])
def test_window_hann_matches_scipy(n):
    from scipy.signal import windows

    np.testing.assert_allclose(O.window("hann", n), windows.hann(n, sym=True), atol=1e-15)


@pytest.mark.parametrize("beta", [0.0, 2.5, 4.0, 8.6])
def test_window_kaiser_matches_scipy(beta):
    from scipy.signal import windows

    np.testing.assert_allclose(O.window("kaiser", 129, beta), windows.kaiser(129, beta, sym=True),
                               rtol=1e-12, atol=1e-15)


def test_window_hann_closed_form_sum():
    # sum of a symmetric Hann of length N is (N - 1) / 2
    for n in (5, 128, 1023):
        assert O.window("hann", n).sum() == pytest.approx((n - 1) / 2.0, rel=1e-13)


# ---------------------------------------------------------------------------
# Range compression (the DFT producing s): closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("method", ["direct", "fft"])
def test_range_tone_on_bin(method):
    n_s, k0, A = 64, 11, 0.7 - 0.2j
    t = np.arange(n_s)
    x = A * np.exp(2j * np.pi * k0 * t / n_s)
    # Z = 1, rect window: all energy in bin k0, N_s A
    X = O.range_compress(x, np.ones(n_s), n_s, n_s, method=method)
    expect = np.zeros(n_s, complex)
    expect[k0] = n_s * A
    np.testing.assert_allclose(X, expect, atol=1e-10)
    # Z = 2: the tone sits on bin 2 k0 of the zero-padded axis
    X2 = O.range_compress(x, np.ones(n_s), 2 * n_s, 2 * n_s, method=method)
    assert X2[2 * k0] == pytest.approx(n_s * A, abs=1e-10)


def test_range_parseval_uncropped():
    rng = np.random.default_rng(5)
    n_s, nfft = 100, 256
    x = rng.standard_normal(n_s) + 1j * rng.standard_normal(n_s)
    w = O.window("hann", n_s)
    X = O.range_compress(x, w, nfft, nfft, method="fft")
    assert np.sum(np.abs(X) ** 2) == pytest.approx(nfft * np.sum(np.abs(w * x) ** 2), rel=1e-12)


def test_range_direct_equals_fft():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((3, 2, 48)) + 1j * rng.standard_normal((3, 2, 48))
    w = O.window("hann", 48)
    a = O.range_compress(x, w, 96, 40, method="direct")
    b = O.range_compress(x, w, 96, 40, method="fft")
    np.testing.assert_allclose(a, b, atol=1e-12 * np.abs(a).max())


def _dirichlet(nu, n):
    """sum_{t<n} exp(j 2 pi nu t) in closed form."""
    nu = np.asarray(nu, dtype=np.float64)
    out = np.empty(nu.shape, dtype=np.complex128)
    s = np.sin(np.pi * nu)
    small = np.abs(s) < 1e-14
    out[~small] = np.exp(1j * np.pi * nu[~small] * (n - 1)) * np.sin(np.pi * nu[~small] * n) / s[~small]
    out[small] = n * np.exp(1j * np.pi * np.round(nu[small]) * (n - 1))
    return out


def test_range_hann_off_bin_tone_matches_dirichlet():
    """Hann = 0.5 - 0.25 e^{+j2pi t/(N-1)} - 0.25 e^{-j2pi t/(N-1)}: three Dirichlet kernels."""
    n_s, nfft, nb = 256, 512, 200
    f_norm = 0.1234567     # tone frequency in cycles per sample (off-bin)
    A = 1.3 * np.exp(0.4j)
    t = np.arange(n_s)
    x = A * np.exp(2j * np.pi * f_norm * t)
    X = O.range_compress(x, O.window("hann", n_s), nfft, nb)
    nu = f_norm - np.arange(nb) / nfft
    e = 1.0 / (n_s - 1)
    closed = A * (0.5 * _dirichlet(nu, n_s) - 0.25 * _dirichlet(nu + e, n_s) - 0.25 * _dirichlet(nu - e, n_s))
    np.testing.assert_allclose(X, closed, atol=1e-9 * np.abs(closed).max())


# ---------------------------------------------------------------------------
# Index interpolation rules
# ---------------------------------------------------------------------------
def test_interp_index_rules():
    row = np.array([[1.0 + 1j, 3.0, -1.0j, 5.0]])
    f = np.array([[0.0, 0.5, 1.25, 2.999, 3.0, 3.0000001, -1e-9, -0.5, 7.0]])
    v = O.interp_index(row, f)[0]
    assert v[0] == row[0, 0]
    assert v[1] == pytest.approx(0.5 * (1 + 1j) + 0.5 * 3.0)
    assert v[2] == pytest.approx(0.75 * 3.0 + 0.25 * (-1j))
    assert v[3] == pytest.approx(0.001 * (-1j) + 0.999 * 5.0)
    assert v[4] == row[0, 3]                  # last sample exactly at f = n - 1
    assert v[5] == 0 and v[6] == 0 and v[7] == 0 and v[8] == 0


def test_interp_linear_ramp_exact():
    k = np.arange(50.0)
    row = (2.0 - 0.5j) + (0.25 + 0.1j) * k
    f = np.random.default_rng(1).uniform(0, 49, size=1000)
    v = O.interp_index(row[None], f[None])[0]
    np.testing.assert_allclose(v, (2.0 - 0.5j) + (0.25 + 0.1j) * f, rtol=1e-14, atol=1e-13)


# ---------------------------------------------------------------------------
# Back-projection (Alg. 2 / Alg. 1)
# ---------------------------------------------------------------------------
def _geometry(M=24, CH=4, speed=3.0, seed=0):
    cfg = synth.SceneConfig("t", n_samples=64, n_chirps=M, n_tx=1, n_rx=CH, speed=speed, seed=seed)
    q_tx, q_rx, vel = synth._trajectory(cfg, speed)
    return q_tx, q_rx, vel


def _dist(p, q):
    return np.sqrt(np.sum((p - q) ** 2, axis=-1))


def test_bp_closed_form_coherent_gain():
    """P1: a spectrum linear in k and matched at p0 focuses to exactly N_ch sum(w)."""
    q_tx, q_rx, vel = _geometry(M=20, CH=3)
    M, CH, _ = q_tx.shape
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], 2.5e6, 512)
    rng = np.random.default_rng(3)
    pix = np.stack([rng.uniform(-3, 3, 40), rng.uniform(4, 9, 40)], -1)
    fd = rng.uniform(-0.5, 0.5, 40)
    p0 = 7
    beta = 0.013 - 0.02j
    dh0 = _dist(pix[p0], q_tx) + _dist(pix[p0], q_rx)        # [M, CH]
    f0 = k["a1"] * dh0 + fd[p0]
    kk = np.arange(160.0)
    # s[m, ch, k] = e^{+j 2 pi d0 / lam} (1 + beta (k - f0))
    s = np.exp(2j * np.pi * dh0 / k["lam"])[:, :, None] * (1 + beta * (kk[None, None, :] - f0[:, :, None]))
    w = O.window("hann", M) + 0.1
    P = O.bp_alg2(pix, q_tx, q_rx, fd, s, w, k["a1"], k["a2"])
    # exact up to the FP64 rounding of phases of ~1e4 rad
    assert P[p0] == pytest.approx(CH * w.sum(), rel=1e-9)
    # every other in-range pixel: no interpolation error either
    dh = _dist(pix[:, None, None, :], q_tx[None]) + _dist(pix[:, None, None, :], q_rx[None])
    f = k["a1"] * dh + fd[:, None, None]
    assert f.min() > 0 and f.max() < kk[-1]
    expect = np.sum(w[None, :, None] * np.exp(-2j * np.pi * (dh - dh0[None]) / k["lam"])
                    * (1 + beta * (f - f0[None])), axis=(1, 2))
    np.testing.assert_allclose(P, expect, rtol=1e-10, atol=1e-10 * np.abs(expect).max())


def test_bp_linearity():
    """P2: P is linear in s."""
    q_tx, q_rx, _ = _geometry(M=10, CH=2)
    rng = np.random.default_rng(4)
    pix = np.stack([rng.uniform(-2, 2, 30), rng.uniform(2, 6, 30)], -1)
    fd = rng.uniform(-1, 1, 30)
    s1 = synth.random_spectrum(rng, (10, 2, 120)).astype(np.complex128)
    s2 = synth.random_spectrum(rng, (10, 2, 120)).astype(np.complex128)
    w = O.window("hann", 10)
    a, b = 0.3 - 1.1j, -2.0 + 0.5j
    args = (6.2, -1605.4j)
    P = O.bp_alg2(pix, q_tx, q_rx, fd, a * s1 + b * s2, w, *args)
    Q = a * O.bp_alg2(pix, q_tx, q_rx, fd, s1, w, *args) + b * O.bp_alg2(pix, q_tx, q_rx, fd, s2, w, *args)
    np.testing.assert_allclose(P, Q, atol=1e-11 * np.abs(P).max())


def test_alg1_equals_alg2_when_doppler_is_exact():
    """P3: with a static aperture the averaged Doppler is exact, so Alg. 2 == Alg. 1.

    Alg. 1 is written with mu, f0, c, df and tau; Alg. 2 with a1, a2 and kd; the
    two agree only if the constants are derived correctly.
    """
    rng = np.random.default_rng(8)
    M, CH = 12, 3
    base_tx = np.array([0.1, -0.05])
    # every chirp and channel sees the same TX and RX position, so the mean
    # position (aperture centre) is every position and the average is exact
    rx_off = np.array([0.0, 0.03])
    q_tx = np.broadcast_to(base_tx, (M, CH, 2)).copy()
    q_rx = np.broadcast_to(base_tx + rx_off, (M, CH, 2)).copy()
    vel = np.broadcast_to(np.array([4.0, 1.5]), (M, 2)).copy()
    pix = np.stack([rng.uniform(-4, 4, 50), rng.uniform(1, 9, 50)], -1)
    fs, nfft = 2.5e6, 512
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], fs, nfft)
    s = synth.random_spectrum(rng, (M, CH, 150)).astype(np.complex128)
    w = O.window("kaiser", M, 3.0)
    fd = O.doppler_table(pix, q_tx, q_rx, vel, k["kd"])
    P2 = O.bp_alg2(pix, q_tx, q_rx, fd, s, w, k["a1"], k["a2"])
    P1 = O.bp_alg1(pix, q_tx, q_rx, vel, s, w, R["f0"], k["mu"], k["df"])
    np.testing.assert_allclose(P1, P2, atol=1e-10 * np.abs(P1).max())
    # a moving aperture at zero velocity has no Doppler in either form
    q_tx, q_rx, _ = _geometry(M=M, CH=CH)
    vel0 = np.zeros((M, 2))
    fd0 = O.doppler_table(pix, q_tx, q_rx, vel0, k["kd"])
    assert np.all(fd0 == 0)
    P2 = O.bp_alg2(pix, q_tx, q_rx, fd0, s, w, k["a1"], k["a2"])
    P1 = O.bp_alg1(pix, q_tx, q_rx, vel0, s, w, R["f0"], k["mu"], k["df"])
    np.testing.assert_allclose(P1, P2, atol=1e-10 * np.abs(P1).max())


def test_bp_bruteforce_mpmath_tiny():
    """P6: 50-digit evaluation of the definition on a tiny input."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    rng = np.random.default_rng(9)
    M, CH, NB = 4, 2, 40
    q_tx, q_rx, _ = _geometry(M=M, CH=CH)
    pix = np.stack([rng.uniform(-1, 1, 5), rng.uniform(1.0, 2.5, 5)], -1)
    fd = rng.uniform(-0.3, 0.3, 5)
    s = synth.random_spectrum(rng, (M, CH, NB)).astype(np.complex128)
    w = O.window("hann", M) + 0.25
    a1, a2 = 6.210963452589591, -1605.417286814988j
    P = O.bp_alg2(pix, q_tx, q_rx, fd, s, w, a1, a2)
    mp = mpmath.mpf
    for p in range(5):
        acc = mpmath.mpc(0)
        for m in range(M):
            for c in range(CH):
                dt = mpmath.sqrt((mp(pix[p, 0]) - mp(q_tx[m, c, 0])) ** 2 + (mp(pix[p, 1]) - mp(q_tx[m, c, 1])) ** 2)
                dr = mpmath.sqrt((mp(pix[p, 0]) - mp(q_rx[m, c, 0])) ** 2 + (mp(pix[p, 1]) - mp(q_rx[m, c, 1])) ** 2)
                d = dt + dr
                f = mp(a1) * d + mp(fd[p])
                if f < 0 or f > NB - 1:
                    continue
                i = int(mpmath.floor(f))
                phi = f - i
                lo = mpmath.mpc(s[m, c, i].real, s[m, c, i].imag)
                hi = mpmath.mpc(s[m, c, min(i + 1, NB - 1)].real, s[m, c, min(i + 1, NB - 1)].imag)
                acc += mpmath.exp(mpmath.mpc(0, mp(a2.imag)) * d) * ((1 - phi) * lo + phi * hi) * mp(w[m])
        ref = complex(acc)
        assert abs(P[p] - ref) <= 1e-10 * max(1.0, abs(ref))


def test_bp_pointwise_and_permutation():
    """P7: back-projection is pointwise; permuting pixels permutes the image."""
    q_tx, q_rx, _ = _geometry(M=8, CH=2)
    rng = np.random.default_rng(10)
    pix = np.stack([rng.uniform(-2, 2, 64), rng.uniform(2, 6, 64)], -1)
    fd = rng.uniform(-1, 1, 64)
    s = synth.random_spectrum(rng, (8, 2, 100))
    w = O.window("hann", 8)
    P = O.bp_alg2(pix, q_tx, q_rx, fd, s, w, 6.2, -1605.4j)
    perm = rng.permutation(64)
    Pp = O.bp_alg2(pix[perm], q_tx, q_rx, fd[perm], s, w, 6.2, -1605.4j)
    np.testing.assert_array_equal(Pp, P[perm])
    sub = O.bp_alg2(pix[10:13], q_tx, q_rx, fd[10:13], s, w, 6.2, -1605.4j)
    np.testing.assert_array_equal(sub, P[10:13])


def _indices_by_loops(pix, q_tx, q_rx, fd, a1, height=0.0):
    """f_ind(p, m, ch) = a1 (|p - q_tx| + |p - q_rx|) + f_doppler(p) written out
    term by term with math.sqrt, independent of the oracle's array code."""
    P, (M, CH) = len(pix), q_tx.shape[:2]
    f = np.zeros((P, M, CH))
    for p in range(P):
        for m in range(M):
            for c in range(CH):
                dt = math.sqrt((pix[p][0] - q_tx[m, c, 0]) ** 2 + (pix[p][1] - q_tx[m, c, 1]) ** 2 + height ** 2)
                dr = math.sqrt((pix[p][0] - q_rx[m, c, 0]) ** 2 + (pix[p][1] - q_rx[m, c, 1]) ** 2 + height ** 2)
                f[p, m, c] = a1 * (dt + dr) + fd[p]
    return f


def test_bp_abs_row_constant_spectrum():
    """S(p) = sum_m sum_ch |w_sar[m] s(f_ind)|, the scale of every per-pixel
    error bound.  A spectrum constant along each (m, ch) row, s = a e^{i theta},
    interpolates to that row's value at any in-range index, so S(p) is the sum
    of |w_sar[m]| a(m, ch) over the terms whose index lies in [0, n_bins - 1]
    (Alg. 2's rule: other terms add nothing).  Negative window weights check
    the magnitude of w_sar; a pixel whose every index is out of range gets 0."""
    q_tx, q_rx, _ = _geometry(M=6, CH=3, seed=2)
    M, CH, _ = q_tx.shape
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], 2.5e6, 512)
    rng = np.random.default_rng(21)
    pix = np.stack([rng.uniform(-3, 3, 14), rng.uniform(1.5, 9, 14)], -1)
    pix[-1] = [0.0, 40.0]                                # far beyond the kept bins
    fd = rng.uniform(-2, 2, 14)
    amp = rng.uniform(0.5, 2.0, (M, CH))
    theta = rng.uniform(-np.pi, np.pi, (M, CH))
    w = rng.uniform(-1.0, 1.0, M)
    f = _indices_by_loops(pix, q_tx, q_rx, fd, k["a1"])
    for nb in (int(f[:-1].max()) + 3, int(np.median(f[:-1])) + 1):   # all in range / about half out
        s = np.broadcast_to((amp * np.exp(1j * theta))[:, :, None], (M, CH, nb)).copy()
        S = O.bp_alg2_abs(pix, q_tx, q_rx, fd, s, w, k["a1"])
        inside = (f >= 0) & (f <= nb - 1)
        expect = np.sum(np.abs(w)[None, :, None] * amp[None] * inside, axis=(1, 2))
        np.testing.assert_allclose(S, expect, rtol=1e-13, atol=0)
        assert S[-1] == 0.0
    assert 0 < inside[:-1].mean() < 1                    # the second case drops part of the terms
    # every term in range: N_ch sum |w| for unit rows
    s1 = np.broadcast_to(np.exp(1j * theta)[:, :, None], (M, CH, int(f[:-1].max()) + 3)).copy()
    S1 = O.bp_alg2_abs(pix[:-1], q_tx, q_rx, fd[:-1], s1, w, k["a1"])
    np.testing.assert_allclose(S1, CH * np.abs(w).sum(), rtol=1e-13)


@pytest.mark.parametrize("height", [0.0, 0.7])
def test_bp_abs_linear_ramp_closed_form(height):
    """A row e^{i theta} (1 + beta k) with real beta > 0 interpolates to
    e^{i theta} (1 + beta f) exactly, so S(p) = sum |w_sar[m]| (1 + beta
    f_ind(p, m, ch)) with the indices from the distances written out term by
    term: pins the index (a1, the Doppler table, the 3-D distances) inside S."""
    q_tx, q_rx, _ = _geometry(M=7, CH=2, seed=3)
    M, CH, _ = q_tx.shape
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], 2.5e6, 512)
    rng = np.random.default_rng(22)
    pix = np.stack([rng.uniform(-3, 3, 12), rng.uniform(2, 8, 12)], -1)
    fd = rng.uniform(-1.5, 1.5, 12)
    beta = 0.037
    f = _indices_by_loops(pix, q_tx, q_rx, fd, k["a1"], height)
    nb = int(f.max()) + 4
    theta = rng.uniform(-np.pi, np.pi, (M, CH))
    s = np.exp(1j * theta)[:, :, None] * (1 + beta * np.arange(nb))[None, None, :]
    w = rng.uniform(-1.0, 1.0, M)
    S = O.bp_alg2_abs(pix, q_tx, q_rx, fd, s, w, k["a1"], height=height)
    expect = np.sum(np.abs(w)[None, :, None] * (1 + beta * f), axis=(1, 2))
    np.testing.assert_allclose(S, expect, rtol=1e-12)


def test_bp_abs_bounds_the_image_and_is_reached_when_coherent():
    """|P(p)| <= S(p) (triangle inequality) on random spectra and windows, and
    equality where every term has the same phase: the matched spectrum of the
    coherent-gain pin focuses p0 to S(p0) = N_ch sum(w)."""
    q_tx, q_rx, _ = _geometry(M=16, CH=3)
    M, CH, _ = q_tx.shape
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], 2.5e6, 512)
    rng = np.random.default_rng(23)
    pix = np.stack([rng.uniform(-3, 3, 60), rng.uniform(1, 9, 60)], -1)
    fd = rng.uniform(-1, 1, 60)
    for _ in range(3):
        s = synth.random_spectrum(rng, (M, CH, 130)).astype(np.complex128)
        w = rng.uniform(-1, 1, M)
        P = O.bp_alg2(pix, q_tx, q_rx, fd, s, w, k["a1"], k["a2"])
        S = O.bp_alg2_abs(pix, q_tx, q_rx, fd, s, w, k["a1"])
        assert np.all(np.abs(P) <= S * (1 + 1e-12))
        assert np.all(S > 0)
    p0 = 11
    dh0 = _dist(pix[p0], q_tx) + _dist(pix[p0], q_rx)
    f0 = k["a1"] * dh0 + fd[p0]
    kk = np.arange(160.0)
    s = np.exp(2j * np.pi * dh0 / k["lam"])[:, :, None] * (1 + 0.01 * (kk[None, None, :] - f0[:, :, None]))
    w = O.window("hann", M) + 0.1
    P = O.bp_alg2(pix, q_tx, q_rx, fd, s, w, k["a1"], k["a2"])
    S = O.bp_alg2_abs(pix, q_tx, q_rx, fd, s, w, k["a1"])
    assert S[p0] == pytest.approx(CH * w.sum(), rel=1e-12)
    assert abs(P[p0]) == pytest.approx(S[p0], rel=1e-9)
    others = np.arange(60) != p0
    assert np.all(np.abs(P[others]) < S[others])


def _point_target_frame(n_rx=8, speed=2.0, seed=11):
    cfg = synth.SceneConfig("pt", n_samples=128, n_chirps=64, n_tx=1, n_rx=n_rx,
                            box=(-2.0, 2.0, 3.0, 7.0), nx=41, ny=41, speed=speed,
                            n_targets=1, snr_db=(20.0, 20.0), noise=False, seed=seed)
    return cfg, synth.make_frame(cfg)


def test_point_target_focuses_and_rx_halving_costs_6db():
    """P5/P8: a noise-free point target focuses at its position; half the RX
    channels give 20 log10(2) = 6.02 dB less coherent gain; channel subsets add."""
    cfg, fr = _point_target_frame()
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], fr.fs, fr.n_fft)
    s = O.range_compress(fr.raw, O.window("hann", cfg.n_samples), fr.n_fft, fr.n_bins)
    w = O.window("hann", cfg.n_chirps)
    tp = fr.targets[0][None, :]
    pix = np.concatenate([tp, fr.pix.astype(np.float64)])
    fd = O.doppler_table(pix, fr.q_tx, fr.q_rx, fr.vel, k["kd"])
    P = O.bp_alg2(pix, fr.q_tx, fr.q_rx, fd, s, w, k["a1"], k["a2"])
    img = np.abs(P[1:])
    ipk = int(np.argmax(img))
    step = np.array([(cfg.box[1] - cfg.box[0]) / (cfg.nx - 1), (cfg.box[3] - cfg.box[2]) / (cfg.ny - 1)])
    assert np.all(np.abs(fr.pix[ipk] - tp[0]) <= 1.5 * step)
    # at the scatterer the image is within the worst-case scalloping of linear
    # interpolation between bins that are 90 degrees apart (|(1-phi) - j phi| >= 1/sqrt 2)
    assert abs(P[0]) >= 0.7 * img.max()
    # coherent gain bound: |P| <= |A| N_ch sum(w_sar) sum(w_range)
    bound = abs(fr.target_amp[0]) * cfg.n_channels * w.sum() * O.window("hann", cfg.n_samples).sum()
    assert abs(P[0]) <= bound
    assert abs(P[0]) > 0.5 * bound          # linear interpolation loses < 6 dB
    # RX halving
    h = cfg.n_channels // 2
    Ph = O.bp_alg2(pix[:1], fr.q_tx[:, :h], fr.q_rx[:, :h], fd[:1], s[:, :h], w, k["a1"], k["a2"])
    loss = 20 * np.log10(abs(P[0]) / abs(Ph[0]))
    assert loss == pytest.approx(20 * np.log10(2), abs=0.05)
    Pb = O.bp_alg2(pix[:1], fr.q_tx[:, h:], fr.q_rx[:, h:], fd[:1], s[:, h:], w, k["a1"], k["a2"])
    assert Ph[0] + Pb[0] == pytest.approx(P[0], rel=1e-12)


def test_bp_closed_form_coherent_gain_with_height():
    """P1 with the antennas h above the pixel plane: s matched to the 3-D paths
    of p0 focuses to exactly N_ch sum(w); Alg. 1 agrees on a static aperture."""
    q_tx, q_rx, vel = _geometry(M=16, CH=2)
    M, CH, _ = q_tx.shape
    h = 0.9
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], 2.5e6, 512)
    rng = np.random.default_rng(13)
    pix = np.stack([rng.uniform(-3, 3, 20), rng.uniform(3, 8, 20)], -1)
    p0 = 5
    d3 = lambda p, q: np.sqrt(np.sum((p - q) ** 2, axis=-1) + h * h)  # noqa: E731
    dh0 = d3(pix[p0], q_tx) + d3(pix[p0], q_rx)
    f0 = k["a1"] * dh0
    kk = np.arange(160.0)
    s = np.exp(2j * np.pi * dh0 / k["lam"])[:, :, None] * (1 + 0.01 * (kk[None, None, :] - f0[:, :, None]))
    w = O.window("hann", M) + 0.1
    P = O.bp_alg2(pix, q_tx, q_rx, np.zeros(20), s, w, k["a1"], k["a2"], height=h)
    assert P[p0] == pytest.approx(CH * w.sum(), rel=1e-9)
    # Alg. 1 at zero velocity with the same height gives Alg. 2's image
    P1 = O.bp_alg1(pix, q_tx, q_rx, np.zeros_like(vel), s, w, R["f0"], k["mu"], k["df"], height=h)
    np.testing.assert_allclose(P1, P, rtol=1e-9, atol=1e-9 * abs(P[p0]))


def test_doppler_table_with_height_closed_form():
    """A pixel on the line of motion at distance x from the (co-located) aperture
    centre, antennas h above the plane: f_d = kd 2 v x / sqrt(x^2 + h^2)."""
    h, v, x, kd = 1.2, 3.0, 4.0, 37.5
    q = np.zeros((2, 1, 2))
    vel = np.array([[v, 0.0], [v, 0.0]])
    fd = O.doppler_table(np.array([[x, 0.0], [-x, 0.0], [0.0, 5.0]]), q, q, vel, kd, height=h)
    assert fd[0] == pytest.approx(kd * 2 * v * x / math.hypot(x, h), rel=1e-14)
    assert fd[1] == pytest.approx(-fd[0], rel=1e-14)
    assert fd[2] == 0.0


def test_point_target_with_height_focuses_only_with_it():
    """A point target simulated with the radar 1 m above the ground focuses at its
    position when back-projected with that height, and loses gain without it."""
    cfg = dataclasses.replace(synth.CONFIGS["plain-small"], name="h", n_samples=128, n_chirps=64, n_rx=4,
                              nx=9, ny=9, box=(-0.4, 0.4, 2.6, 3.4), n_targets=1, noise=False, height=1.0,
                              speed=4.0, seed=77)
    fr = synth.make_frame(cfg)
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], fr.fs, fr.n_fft)
    s = O.range_compress(fr.raw, O.window("hann", cfg.n_samples), fr.n_fft, fr.n_bins)
    w = O.window("hann", cfg.n_chirps)
    tp = fr.targets[0][None, :]
    amp = {}
    for h in (1.0, 0.0):
        fd = O.doppler_table(tp, fr.q_tx, fr.q_rx, fr.vel, k["kd"], height=h)
        amp[h] = abs(O.bp_alg2(tp, fr.q_tx, fr.q_rx, fd, s, w, k["a1"], k["a2"], height=h)[0])
    bound = abs(fr.target_amp[0]) * cfg.n_channels * w.sum() * O.window("hann", cfg.n_samples).sum()
    assert 0.5 * bound < amp[1.0] <= bound
    assert amp[0.0] < 0.7 * amp[1.0]            # the planar reading loses more than 3 dB


# ---------------------------------------------------------------------------
# Continuous SAR: overlapping apertures of one chirp stream (Sec. V)
# ---------------------------------------------------------------------------
def _stream(n_blocks, S, CH=2, speed=3.0, seed=5, nb=150, yaw=0.0):
    cfg = synth.SceneConfig("st", n_samples=64, n_chirps=n_blocks * S, n_tx=1, n_rx=CH, speed=speed,
                            seed=seed, yaw_rate=yaw)
    q_tx, q_rx, vel = synth._trajectory(cfg, speed)
    rng = np.random.default_rng(seed + 1)
    s = synth.random_spectrum(rng, (n_blocks * S, CH, nb)).astype(np.complex128)
    blocks = [dict(q_tx=q_tx[j * S:(j + 1) * S], q_rx=q_rx[j * S:(j + 1) * S], vel=vel[j * S:(j + 1) * S],
                   s=s[j * S:(j + 1) * S]) for j in range(n_blocks)]
    return blocks, (q_tx, q_rx, vel, s)


def test_sliding_exact_doppler_equals_whole_aperture():
    """With per-term Doppler (Alg. 1) the aperture of sub-aperture b is Alg. 1
    over its N = K S chirps with the window over N; before the stream has K
    sub-apertures, the available chirps take the last positions of the window
    (numpy's own Hann, not the oracle's)."""
    K, S, nb = 3, 5, 6
    blocks, (q_tx, q_rx, vel, s) = _stream(nb, S, yaw=0.05)
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], 2.5e6, 512)
    rng = np.random.default_rng(17)
    pix = np.stack([rng.uniform(-3, 3, 30), rng.uniform(3, 8, 30)], -1)
    N = K * S
    for b in range(nb):
        P = O.bp_sliding(pix, blocks, b, K, k["a1"], k["a2"], k["kd"], doppler="exact", f0=R["f0"],
                         mu=k["mu"], df=k["df"])
        lo = max(0, (b - K + 1) * S)
        hi = (b + 1) * S
        w = np.hanning(N)[N - (hi - lo):]
        ref = O.bp_alg1(pix, q_tx[lo:hi], q_rx[lo:hi], vel[lo:hi], s[lo:hi], w, R["f0"], k["mu"], k["df"])
        np.testing.assert_allclose(P, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_sliding_average_doppler_at_rest_equals_whole_aperture():
    """At zero velocity every Doppler table is zero, so the aperture of the
    averaged-Doppler form is Alg. 2 over its chirps; a rectangular window
    makes it the plain sum of the sub-aperture images."""
    K, S = 4, 3
    blocks, (q_tx, q_rx, _, s) = _stream(6, S)
    for blk in blocks:
        blk["vel"] = np.zeros_like(blk["vel"])
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], 2.5e6, 512)
    rng = np.random.default_rng(18)
    pix = np.stack([rng.uniform(-3, 3, 25), rng.uniform(3, 8, 25)], -1)
    b = 5
    P = O.bp_sliding(pix, blocks, b, K, k["a1"], k["a2"], k["kd"])
    lo, hi = (b - K + 1) * S, (b + 1) * S
    ref = O.bp_alg2(pix, q_tx[lo:hi], q_rx[lo:hi], np.zeros(25), s[lo:hi], np.hanning(K * S), k["a1"], k["a2"])
    np.testing.assert_allclose(P, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    Pr = O.bp_sliding(pix, blocks, b, K, k["a1"], k["a2"], k["kd"], window_kind="rect")
    parts = [O.bp_alg2(pix, blocks[j]["q_tx"], blocks[j]["q_rx"], np.zeros(25), blocks[j]["s"], np.ones(S),
                       k["a1"], k["a2"]) for j in range(b - K + 1, b + 1)]
    np.testing.assert_allclose(Pr, np.sum(parts, axis=0), rtol=0, atol=1e-12 * np.abs(Pr).max())


def test_sliding_closed_form_gain_with_subaperture_doppler():
    """P1 on a moving stream: a spectrum whose every sub-aperture j is matched
    at p0 to the index a1 d_hyp + f_doppler_j(p0) of that sub-aperture's own
    Doppler table focuses to N_ch times the sum of the window positions the
    available chirps take (numpy's Hann)."""
    K, S, CH, nbk = 4, 6, 2, 7
    blocks, (q_tx, q_rx, vel, _) = _stream(nbk, S, CH=CH, speed=5.0, yaw=0.2)
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], 2.5e6, 512)
    p0 = np.array([[0.7, 5.5]])
    kk = np.arange(200.0)
    beta = 0.8 + 0.3j   # steep ramps: a Doppler table off by 0.01 bins shows
    for j, blk in enumerate(blocks):
        # velocities that differ from one sub-aperture to the next, so that
        # every sub-aperture's Doppler table is its own
        vx = (1.0, 7.0, 2.0, 8.0, 1.5, 6.0, 3.0)[j]
        blk["vel"] = np.broadcast_to([vx, 0.1 * (-1) ** j], blk["vel"].shape).copy()
        fdj = O.doppler_table(p0, blk["q_tx"], blk["q_rx"], blk["vel"], k["kd"])[0]
        d0 = _dist(p0[0], blk["q_tx"]) + _dist(p0[0], blk["q_rx"])
        f = k["a1"] * d0 + fdj
        blk["s"] = np.exp(2j * np.pi * d0 / k["lam"])[:, :, None] * (1 + beta * (kk - f[:, :, None]))
    N = K * S
    for b in (1, 3, 6):
        P = O.bp_sliding(p0, blocks, b, K, k["a1"], k["a2"], k["kd"])
        n_avail = min(b + 1, K) * S
        assert P[0] == pytest.approx(CH * np.hanning(N)[N - n_avail:].sum(), rel=1e-9)
    # the whole-aperture table (Alg. 2 over the N chirps) does not match the ramps
    lo, hi = 3 * S, 7 * S
    vel_all = np.concatenate([blk["vel"] for blk in blocks[3:7]])
    fd_ap = O.doppler_table(p0, q_tx[lo:hi], q_rx[lo:hi], vel_all, k["kd"])
    s_all = np.concatenate([blk["s"] for blk in blocks[3:7]])
    P_ap = O.bp_alg2(p0, q_tx[lo:hi], q_rx[lo:hi], fd_ap, s_all, np.hanning(N), k["a1"], k["a2"])
    assert abs(P_ap[0] - CH * np.hanning(N).sum()) > 1e-3 * CH * np.hanning(N).sum()


def test_doppler_average_error_below_100hz():
    """P9 (Sec. III-D): on a straight drive at parking speed the averaged table
    stays within 100 Hz of Alg. 1's per-chirp Doppler, the deviation obeys the
    geometric bound 2 (f0 / c) |v| (L / 2) / d_min (direction change across the
    aperture), and the table has Alg. 1's sign."""
    cfg = synth.CONFIGS["plain-small"]
    speed = 2.0
    q_tx, q_rx, vel = synth._trajectory(cfg, speed)
    fs = synth.sample_rate(cfg)
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], fs, cfg.n_fft)
    pix = synth.cartesian_pixels(cfg.box, 33, 33).astype(np.float64)
    fd = O.doppler_table(pix, q_tx, q_rx, vel, k["kd"])          # bins
    worst = 0.0
    for m in range(cfg.n_chirps):
        for c in range(cfg.n_channels):
            rt = pix - q_tx[m, c]
            rr = pix - q_rx[m, c]
            vr = (rt @ vel[m]) / _dist(pix, q_tx[m, c]) + (rr @ vel[m]) / _dist(pix, q_rx[m, c])
            exact = R["f0"] * vr / R["c"]                           # Hz, Alg. 1
            worst = max(worst, float(np.max(np.abs(exact - fd * k["df"]))))
    assert worst < 100.0
    L = np.ptp(q_rx[:, :, 0]) + np.ptp(q_tx[:, :, 0])
    d_min = float(pix[:, 1].min())
    assert worst <= 2 * R["f0"] / R["c"] * speed * (L / 2) / d_min * 1.05
    # approaching pixels (ahead of the car, +x) have a positive shift
    ahead = pix[:, 0] > 1.0
    assert np.all(fd[ahead] > 0) and np.all(fd[pix[:, 0] < -1.0] < 0)


# ---------------------------------------------------------------------------
# Grids
# ---------------------------------------------------------------------------
def test_polar_grid_steps_and_coverage():
    lam = R["c"] / R["f0"]
    L = 1.0
    g = O.polar_grid_params((-15, 15, 1, 31), (0.0, 0.0), R["bandwidth"], lam, L)
    assert g["dr"] == pytest.approx(R["c"] / (2 * R["bandwidth"]) / 2.5, rel=1e-15)
    assert g["dth"] == pytest.approx(lam / (2 * L) / 2.5, rel=1e-15)
    pts = O.polar_grid(g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"])
    assert pts.shape == (g["nr"] * g["nth"], 2)
    r = np.hypot(pts[:, 0], pts[:, 1])
    th = np.arctan2(pts[:, 0], pts[:, 1])
    np.testing.assert_allclose(r.reshape(g["nth"], g["nr"])[0], g["r0"] + g["dr"] * np.arange(g["nr"]), rtol=1e-12)
    np.testing.assert_allclose(th.reshape(g["nth"], g["nr"])[:, 0], g["th0"] + g["dth"] * np.arange(g["nth"]), atol=1e-12)
    # every box point is within half a step of a lattice point (coverage)
    assert g["r0"] == pytest.approx(1.0) and g["r0"] + (g["nr"] - 1) * g["dr"] >= math.hypot(15, 31) - g["dr"]
    assert g["th0"] <= math.atan2(-15, 1) + 1e-12 and g["th0"] + g["nth"] * g["dth"] >= math.atan2(15, 1)


def _polar_fixture():
    g = dict(ox=0.3, oy=-0.2, r0=2.0, dr=0.05, nr=40, th0=-0.6, dth=0.02, nth=50)
    r = g["r0"] + g["dr"] * np.arange(g["nr"])
    th = g["th0"] + g["dth"] * np.arange(g["nth"])
    return g, r, th


def test_resample_polar_reproduces_bilinear_functions():
    """Bilinear interpolation in (theta, r) is exact for a + b r + c theta + d r theta."""
    g, r, th = _polar_fixture()
    a, b, c, d = 5.0, 0.7, 1.3, 0.4
    f = lambda rr, tt: a + b * rr + c * tt + d * rr * tt  # noqa: E731  (positive on the lattice)
    img = (f(r[None, :], th[:, None]) * np.exp(1j * 2.1)).astype(np.complex128)  # phase must not matter
    rng = np.random.default_rng(5)
    rr = rng.uniform(r[0], r[-1], 500)
    tt = rng.uniform(th[0], th[-1], 500)
    pts = np.stack([g["ox"] + rr * np.sin(tt), g["oy"] + rr * np.cos(tt)], axis=1)
    out = O.resample_polar(img, g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"], pts)
    np.testing.assert_allclose(out, f(rr, tt), rtol=1e-12)


def test_resample_polar_nodes_edges_and_outside():
    g, r, th = _polar_fixture()
    rng = np.random.default_rng(6)
    img = rng.standard_normal((g["nth"], g["nr"])) + 1j * rng.standard_normal((g["nth"], g["nr"]))
    # lattice nodes, including the last row and column, return the node magnitude
    iv = np.array([0, 7, g["nth"] - 1, g["nth"] - 1, 0])
    iu = np.array([0, 13, g["nr"] - 1, 0, g["nr"] - 1])
    pts = np.stack([g["ox"] + r[iu] * np.sin(th[iv]), g["oy"] + r[iu] * np.cos(th[iv])], axis=1)
    out = O.resample_polar(img, g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"], pts)
    np.testing.assert_allclose(out, np.abs(img[iv, iu]), rtol=1e-9)
    # halfway between two range samples: their mean magnitude
    pm = np.array([[g["ox"] + (r[3] + r[4]) / 2 * np.sin(th[9]), g["oy"] + (r[3] + r[4]) / 2 * np.cos(th[9])]])
    mid = O.resample_polar(img, g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"], pm)
    assert mid[0] == pytest.approx((abs(img[9, 3]) + abs(img[9, 4])) / 2, rel=1e-9)
    # beyond the last range, before the first angle, at the origin: zero
    far = np.array([[g["ox"], g["oy"] + r[-1] + 0.01], [g["ox"] + 3.0 * np.sin(th[0] - 0.01), g["oy"] + 3.0 * np.cos(th[0] - 0.01)],
                    [g["ox"], g["oy"]]])
    out = O.resample_polar(img, g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"], far)
    assert np.all(out == 0.0)


def test_cartesian_grid_layout():
    p = O.cartesian_grid(-1.0, 0.5, 5, 2.0, 0.25, 3)
    assert p.shape == (15, 2)
    assert tuple(p[0]) == (-1.0, 2.0) and tuple(p[4]) == (1.0, 2.0) and tuple(p[5]) == (-1.0, 2.25)


# ---------------------------------------------------------------------------
# Detection stage (CA-CFAR, not part of the paper)
# ---------------------------------------------------------------------------
def test_cfar_alpha_closed_form():
    # N = 21^2 - 5^2 = 416 training cells for guard 2, train 8
    n = (2 * 10 + 1) ** 2 - (2 * 2 + 1) ** 2
    assert n == 416
    a = O.cfar_alpha(n, 1e-4)
    assert a == pytest.approx(9.31306, abs=5e-5)
    # the scale reproduces the false-alarm rate (1 + alpha / N)^-N exactly
    assert (1 + a / n) ** (-n) == pytest.approx(1e-4, rel=1e-12)


def test_cfar_bruteforce_tiny():
    rng = np.random.default_rng(12)
    pw = rng.exponential(1.0, (30, 27))
    pw[15, 13] = 40.0
    pw[11, 11] = 25.0
    g, t, pfa = 1, 3, 1e-2
    idx, pv, th = O.ca_cfar(pw, g, t, pfa)
    h = g + t
    n = (2 * h + 1) ** 2 - (2 * g + 1) ** 2
    a = O.cfar_alpha(n, pfa)
    exp_idx, exp_th = [], []
    for r in range(h, 30 - h):
        for c in range(h, 27 - h):
            tot = 0.0
            for dr in range(-h, h + 1):
                for dc in range(-h, h + 1):
                    if max(abs(dr), abs(dc)) > g:
                        tot += pw[r + dr, c + dc]
            thr = a * tot / n
            if pw[r, c] > thr:
                exp_idx.append(r * 27 + c)
                exp_th.append(thr)
    assert list(idx) == exp_idx
    np.testing.assert_allclose(th, exp_th, rtol=1e-12)
    np.testing.assert_array_equal(pv, pw.ravel()[exp_idx])
    assert 15 * 27 + 13 in exp_idx


@pytest.mark.slow
def test_cfar_false_alarm_rate_on_exponential_noise():
    """P10: on i.i.d. exponential cells the detection count matches Pfa."""
    rng = np.random.default_rng(13)
    pw = rng.exponential(1.0, (1100, 1100))
    idx, _, _ = O.ca_cfar(pw, 2, 8, 1e-4)
    n_cells = (1100 - 20) ** 2
    expect = 1e-4 * n_cells                      # 116.6
    # overlapping windows correlate neighbours only weakly; a 4-sigma Poisson band
    assert abs(len(idx) - expect) < 4 * math.sqrt(expect) + 2


def test_to_db_normalisation():
    P = np.array([1.0, -2.0j, 0.5 + 0.5j, 0.0])
    d = O.to_db(P)
    assert d[1] == 0.0 and d[0] == pytest.approx(-6.0206, abs=1e-4) and d[3] == -np.inf
