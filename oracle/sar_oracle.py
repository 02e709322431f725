"""Plain FP64 CPU oracle for real-time automotive FMCW SAR back-projection.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct reference
that the HIP path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the HIP library or its Python binding, and it imports nothing from them.

Everything is NumPy in float64 / complex128.  Each function names the part of
Hoffmann et al., "Implementation of Real-Time Automotive SAR Imaging"
(arXiv 2306.09784) it follows:

* Alg. 1 (Sec. II): standard back-projection with per-chirp Doppler.
* Alg. 2 (Sec. IV): the optimised back-projection the paper times, i.e. Alg. 1
  with the chirp-only window (Sec. III-B), hoisted constants a1/a2 and
  index-domain interpolation (Sec. III-C), the averaged-velocity Doppler table
  (Sec. III-D), any pixel list such as the polar grid (Sec. III-E) and any
  channel subset (Sec. III-F).

Readings taken where the paper is silent or garbled (each is listed in the
design notes of the repository):

* s_hyp uses the carrier: exp(-j 2 pi f0 tau), so a2 = -j 2 pi f0 / c.  The
  printed Alg. 1 omits f0, which is dimensionally impossible.
* The beat spectrum s is the unnormalised DFT of the Hann-windowed IQ beat
  signal, zero-padded to n_fft and cropped to the first n_bins bins; the
  fast-time origin is the chirp start.
* Linear interpolation on the index axis: i = floor(f), phi = f - i, value
  (1 - phi) s[i] + phi s[i+1]; a term contributes only when 0 <= f <= n_bins - 1
  (f = n_bins - 1 gives s[n_bins - 1]); otherwise it contributes zero.
* f_doppler is in bins, taken at the aperture centre (mean TX and mean RX
  position over all chirps and channels) with the mean velocity; a velocity
  pointing towards the pixel gives a positive shift, as in Alg. 1.
* Geometry is planar (2-D distances) unless a radar height above the pixels'
  plane is given (3-D distances, the pixels' plane below the antennas).
* Continuous SAR (Sec. V): an aperture is the last n_sub sub-apertures of a
  sensor's chirp stream, windowed over all of its chirps; with the averaged
  Doppler each sub-aperture uses its own Doppler table.
* The CA-CFAR detector is not part of the paper; it is the detection stage
  layered on the image: square-law cell-averaging over the 2-D pixel lattice.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299_792_458.0

__all__ = [
    "C_LIGHT",
    "radar_constants",
    "window",
    "range_compress",
    "interp_index",
    "doppler_table",
    "bp_alg2",
    "bp_alg1",
    "bp_alg2_abs",
    "bp_sliding",
    "cartesian_grid",
    "polar_grid_params",
    "polar_grid",
    "resample_polar",
    "cfar_alpha",
    "ca_cfar",
    "to_db",
]


# ---------------------------------------------------------------------------
# Constants (Sec. II after Alg. 1; Sec. III-C; Alg. 2 constants a1, a2)
# ---------------------------------------------------------------------------
def radar_constants(f0: float, bandwidth: float, t_chirp: float, fs: float,
                    n_fft: int, c: float = C_LIGHT) -> dict:
    """Derived constants of the FMCW chirp and the beat-frequency axis.

    mu = B / T_P is the chirp rate (Sec. II).  The beat spectrum is sampled on an
    equidistant axis with spacing df = fs / n_fft (Sec. III-C), so a beat
    frequency f maps to the fractional bin f / df.  Alg. 1's beat-frequency
    hypothesis is
    f_hyp = mu * tau + f0 * v / c with tau = d_hyp / c, hence in bins
        f_ind = a1 * d_hyp + kd * v,   a1 = mu / (c df),   kd = f0 / (c df),
    and s_hyp = exp(a2 d_hyp) with a2 = -j 2 pi f0 / c (carrier-phase reading).
    """
    mu = bandwidth / t_chirp
    df = fs / n_fft
    return {
        "mu": mu,
        "df": df,
        "a1": mu / (c * df),
        "kd": f0 / (c * df),
        "a2": -2j * np.pi * f0 / c,
        "lam": c / f0,
        "c": c,
        "f0": f0,
    }


# ---------------------------------------------------------------------------
# Windows (Sec. III-B: chirp-only w_sar, Hann by default, Kaiser as option)
# ---------------------------------------------------------------------------
def window(kind: str, n: int, beta: float = 4.0) -> np.ndarray:
    """Symmetric window of length n in float64.

    hann:   0.5 - 0.5 cos(2 pi t / (n - 1))
    kaiser: I0(beta sqrt(1 - (2 t / (n - 1) - 1)^2)) / I0(beta)
    rect:   ones
    """
    if n <= 0:
        raise ValueError("window length must be positive")
    if kind == "rect" or n == 1:
        return np.ones(n)
    t = np.arange(n, dtype=np.float64)
    if kind == "hann":
        return 0.5 - 0.5 * np.cos(2.0 * np.pi * t / (n - 1))
    if kind == "kaiser":
        u = 2.0 * t / (n - 1) - 1.0
        return np.i0(beta * np.sqrt(np.maximum(0.0, 1.0 - u * u))) / np.i0(beta)
    raise ValueError(f"unknown window kind {kind!r}")


# ---------------------------------------------------------------------------
# Range compression: beat signal -> beat spectrum s (input of Alg. 1 / Alg. 2)
# ---------------------------------------------------------------------------
def range_compress(raw: np.ndarray, w_range: np.ndarray, n_fft: int, n_bins: int,
                   method: str = "auto") -> np.ndarray:
    """s[..., k] = sum_t w_range[t] raw[..., t] exp(-j 2 pi k t / n_fft), k < n_bins.

    The spectrum that Alg. 1 and Alg. 2 interpolate lives on an
    equidistant beat-frequency axis (Sec. III-C).  ``method='direct'`` evaluates
    the definition with exact integer phase indices (t k mod n_fft);
    ``method='fft'`` uses numpy's FFT of the zero-padded row.
    """
    raw = np.asarray(raw)
    n_s = raw.shape[-1]
    if n_fft < n_s or n_bins > n_fft or n_bins < 1:
        raise ValueError("need n_s <= n_fft and 1 <= n_bins <= n_fft")
    x = raw.astype(np.complex128) * np.asarray(w_range, dtype=np.float64)
    if method == "auto":
        method = "direct" if n_s * n_bins <= 1 << 16 else "fft"
    if method == "direct":
        t = np.arange(n_s, dtype=np.int64)
        k = np.arange(n_bins, dtype=np.int64)
        idx = np.outer(t, k) % n_fft
        kernel = np.exp(-2j * np.pi * idx / n_fft)
        return x @ kernel
    if method == "fft":
        return np.fft.fft(x, n=n_fft, axis=-1)[..., :n_bins]
    raise ValueError(f"unknown method {method!r}")


def interp_index(row: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Linear interpolation of ``row`` (last axis) at fractional indices ``f``.

    Sec. III-C: the interpolation runs on the index of s.  Out-of-range
    indices contribute zero; f = n - 1 exactly yields row[n - 1].
    ``row`` has shape [..., n] and ``f`` shape [..., q] with matching leading
    axes (broadcast); the result has the shape of ``f``.
    """
    n = row.shape[-1]
    f = np.asarray(f, dtype=np.float64)
    valid = (f >= 0.0) & (f <= n - 1)
    fs = np.where(valid, f, 0.0)
    i0 = np.floor(fs).astype(np.int64)
    i1 = np.minimum(i0 + 1, n - 1)
    phi = fs - i0
    lo = np.take_along_axis(row, i0, axis=-1)
    hi = np.take_along_axis(row, i1, axis=-1)
    val = (1.0 - phi) * lo + phi * hi
    return np.where(valid, val, 0.0)


# ---------------------------------------------------------------------------
# Doppler table (Sec. III-D; the f_doppler term of Alg. 2's index)
# ---------------------------------------------------------------------------
def doppler_table(pix: np.ndarray, q_tx: np.ndarray, q_rx: np.ndarray,
                  vel: np.ndarray, kd: float, height: float = 0.0) -> np.ndarray:
    """Per-pixel Doppler shift in bins from the average velocity.

    Sec. III-D: the velocity is taken as constant over the chirp sequence, so
    the radial velocity components of Alg. 1 are evaluated once per
    pixel with the mean velocity, at the aperture centre (mean TX and mean RX
    position over every chirp and channel).  A pixel that coincides with a
    reference position gets a zero radial term.  With the radar ``height``
    above the pixels' plane the distance is 3-D and the (horizontal) velocity
    projects on the 3-D line of sight.
    """
    pix = np.asarray(pix, dtype=np.float64).reshape(-1, 2)
    qt = np.asarray(q_tx, dtype=np.float64).reshape(-1, 2).mean(axis=0)
    qr = np.asarray(q_rx, dtype=np.float64).reshape(-1, 2).mean(axis=0)
    v = np.asarray(vel, dtype=np.float64).reshape(-1, 2).mean(axis=0)

    def radial(q):
        r = pix - q
        d = np.sqrt(np.sum(r * r, axis=1) + height * height)
        num = r @ v
        out = np.zeros_like(d)
        nz = d > 0
        out[nz] = num[nz] / d[nz]
        return out

    return kd * (radial(qt) + radial(qr))


# ---------------------------------------------------------------------------
# Alg. 2: optimised back-projection
# ---------------------------------------------------------------------------
def _norm2(a: np.ndarray, height: float = 0.0) -> np.ndarray:
    """Distance for in-plane differences a [..., 2] with the radar `height`
    above the plane (the paper's planar geometry is height 0)."""
    return np.sqrt(np.sum(a * a, axis=-1) + height * height)


def bp_alg2(pix, q_tx, q_rx, f_doppler, s, w_sar, a1, a2, chunk: int = 4096, height: float = 0.0):
    """P(p) = sum_m sum_ch w_sar[m] exp(a2 d_hyp) s(a1 d_hyp + f_doppler(p), m, ch).

    Alg. 2: d_tx = ||p - q_tx(m, ch)||, d_rx = ||p - q_rx(m, ch)||,
    d_hyp = d_tx + d_rx, f_ind = a1 d_hyp + f_doppler(p), s_hyp = exp(a2 d_hyp),
    contribution s_hyp * s(f_ind, m, ch) * w_sar[m], summed over chirps m and
    channels ch.  TX positions are given per (m, ch) so that time-multiplexed
    MIMO channels are covered; with one TX every channel of a chirp repeats it.

    pix [P, 2]; q_tx, q_rx [M, CH, 2]; f_doppler [P]; s [M, CH, NB] complex;
    w_sar [M].  Returns complex128 [P].  Pixels are processed in chunks only to
    bound memory; every pixel's sum runs over m in order.  ``height`` puts the
    antennas that far above the pixels' plane (3-D distances).
    """
    pix = np.asarray(pix, dtype=np.float64).reshape(-1, 2)
    q_tx = np.asarray(q_tx, dtype=np.float64)
    q_rx = np.asarray(q_rx, dtype=np.float64)
    fd = np.asarray(f_doppler, dtype=np.float64).reshape(-1)
    s = np.asarray(s).astype(np.complex128)
    w = np.asarray(w_sar, dtype=np.float64)
    M, CH, _ = s.shape
    out = np.zeros(pix.shape[0], dtype=np.complex128)
    for p0 in range(0, pix.shape[0], chunk):
        p = pix[p0:p0 + chunk]
        acc = np.zeros(p.shape[0], dtype=np.complex128)
        for m in range(M):
            d_tx = _norm2(p[:, None, :] - q_tx[m][None, :, :], height)      # [P, CH]
            d_rx = _norm2(p[:, None, :] - q_rx[m][None, :, :], height)
            d_hyp = d_tx + d_rx
            f_ind = a1 * d_hyp + fd[p0:p0 + chunk, None]
            s_hyp = np.exp(a2 * d_hyp)
            val = interp_index(s[m][None, :, :], f_ind[:, :, None])[:, :, 0]
            acc += np.sum(s_hyp * val, axis=1) * w[m]
        out[p0:p0 + chunk] = acc
    return out


def bp_alg2_abs(pix, q_tx, q_rx, f_doppler, s, w_sar, a1, chunk: int = 4096, height: float = 0.0):
    """Sum of magnitudes of the Alg. 2 terms, sum_m sum_ch |w_sar[m] s(f_ind)|.

    Not an image: it is the scale against which the rounding error of a
    reduced-precision evaluation of Alg. 2 is bounded term by term.
    """
    pix = np.asarray(pix, dtype=np.float64).reshape(-1, 2)
    q_tx = np.asarray(q_tx, dtype=np.float64)
    q_rx = np.asarray(q_rx, dtype=np.float64)
    fd = np.asarray(f_doppler, dtype=np.float64).reshape(-1)
    s = np.asarray(s).astype(np.complex128)
    w = np.asarray(w_sar, dtype=np.float64)
    M, CH, _ = s.shape
    out = np.zeros(pix.shape[0], dtype=np.float64)
    for p0 in range(0, pix.shape[0], chunk):
        p = pix[p0:p0 + chunk]
        acc = np.zeros(p.shape[0], dtype=np.float64)
        for m in range(M):
            d_hyp = (_norm2(p[:, None, :] - q_tx[m][None, :, :], height)
                     + _norm2(p[:, None, :] - q_rx[m][None, :, :], height))
            f_ind = a1 * d_hyp + fd[p0:p0 + chunk, None]
            val = interp_index(s[m][None, :, :], f_ind[:, :, None])[:, :, 0]
            acc += np.sum(np.abs(val), axis=1) * abs(w[m])
        out[p0:p0 + chunk] = acc
    return out


# ---------------------------------------------------------------------------
# Alg. 1: standard back-projection (per-chirp, per-channel Doppler)
# ---------------------------------------------------------------------------
def bp_alg1(pix, q_tx, q_rx, vel, s, w_sar, f0, mu, df, c: float = C_LIGHT,
            chunk: int = 4096, height: float = 0.0):
    """Alg. 1 with the chirp-only window vector (Sec. III-B).

    For every pixel, chirp m and channel ch: the distances d_tx and d_rx;
    radial velocities v_tx, v_rx from the per-chirp velocity vel[m], summed;
    tau = (d_tx + d_rx) / c; f_hyp = mu tau + f0 v / c;
    s_hyp = exp(-j 2 pi f0 tau) (carrier reading); the spectrum is
    interpolated at the fractional bin f_hyp / df and weighted by
    w_sar[m].  The per-pixel-per-chirp window of the original reference
    implementation is never defined by the paper and is not reproduced.
    """
    pix = np.asarray(pix, dtype=np.float64).reshape(-1, 2)
    q_tx = np.asarray(q_tx, dtype=np.float64)
    q_rx = np.asarray(q_rx, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64).reshape(-1, 2)
    s = np.asarray(s).astype(np.complex128)
    w = np.asarray(w_sar, dtype=np.float64)
    M, CH, _ = s.shape
    out = np.zeros(pix.shape[0], dtype=np.complex128)
    for p0 in range(0, pix.shape[0], chunk):
        p = pix[p0:p0 + chunk]
        acc = np.zeros(p.shape[0], dtype=np.complex128)
        for m in range(M):
            r_tx = p[:, None, :] - q_tx[m][None, :, :]
            r_rx = p[:, None, :] - q_rx[m][None, :, :]
            d_tx = _norm2(r_tx, height)
            d_rx = _norm2(r_rx, height)
            v_tx = np.sum(r_tx * vel[m], axis=-1) / d_tx
            v_rx = np.sum(r_rx * vel[m], axis=-1) / d_rx
            tau = (d_tx + d_rx) / c
            f_hyp = mu * tau + f0 * (v_tx + v_rx) / c
            s_hyp = np.exp(-2j * np.pi * f0 * tau)
            val = interp_index(s[m][None, :, :], (f_hyp / df)[:, :, None])[:, :, 0]
            acc += np.sum(s_hyp * val, axis=1) * w[m]
        out[p0:p0 + chunk] = acc
    return out


# ---------------------------------------------------------------------------
# Continuous SAR: overlapping apertures of one sensor's chirp stream (Sec. V)
# ---------------------------------------------------------------------------
def bp_sliding(pix, blocks, b, n_sub, a1, a2, kd, window_kind="hann", doppler="average",
               f0=None, mu=None, df=None, c: float = C_LIGHT, height: float = 0.0):
    """Image of the aperture that ends with sub-aperture ``b`` of a stream.

    The conclusion (Sec. V) argues that a continuous measurement can be imaged
    as it arrives.  Reading taken here: a sensor's chirp stream is cut into
    sub-apertures of S chirps each; the aperture of sub-aperture b is the last
    ``n_sub`` of them (N = n_sub S chirps, sub-apertures b - n_sub + 1 .. b),
    weighted by the chirp window over N positions (Sec. III-B) with chirp i of
    sub-aperture j at position (j - (b - n_sub + 1)) S + i.  Sub-apertures
    before the start of the stream (j < 0) hold no chirps and add nothing.
    With the averaged Doppler (Alg. 2) each sub-aperture's terms use the
    Doppler table of that sub-aperture (its mean positions and velocity,
    Sec. III-D); with doppler="exact" each term has its own (Alg. 1).

    blocks[j]: dict with q_tx, q_rx [S, CH, 2], vel [S, 2] and s [S, CH, NB]
    (the beat spectrum of those chirps).  Alg. 1 needs f0, mu and df.
    Returns complex128 [P].
    """
    pix = np.asarray(pix, dtype=np.float64).reshape(-1, 2)
    S = int(np.asarray(blocks[b]["s"]).shape[0])
    N = n_sub * S
    w = window(window_kind, N)
    first = b - n_sub + 1
    out = np.zeros(pix.shape[0], dtype=np.complex128)
    for j in range(max(first, 0), b + 1):
        blk = blocks[j]
        if np.asarray(blk["s"]).shape[0] != S:
            raise ValueError("every sub-aperture of a stream has the same chirp count")
        w_j = w[(j - first) * S:(j - first + 1) * S]
        if doppler == "exact":
            out += bp_alg1(pix, blk["q_tx"], blk["q_rx"], blk["vel"], blk["s"], w_j, f0, mu, df, c=c,
                           height=height)
        else:
            fd = doppler_table(pix, blk["q_tx"], blk["q_rx"], blk["vel"], kd, height=height)
            out += bp_alg2(pix, blk["q_tx"], blk["q_rx"], fd, blk["s"], w_j, a1, a2, height=height)
    return out


# ---------------------------------------------------------------------------
# Reconstruction grids (Sec. II: Cartesian reference grid; Sec. III-E: polar)
# ---------------------------------------------------------------------------
def cartesian_grid(x0: float, dx: float, nx: int, y0: float, dy: float, ny: int) -> np.ndarray:
    """Row-major lattice, y slow: pixel (iy, ix) -> (x0 + ix dx, y0 + iy dy)."""
    ix = np.arange(nx, dtype=np.float64)
    iy = np.arange(ny, dtype=np.float64)
    x = x0 + ix * dx
    y = y0 + iy * dy
    out = np.empty((ny, nx, 2))
    out[:, :, 0] = x[None, :]
    out[:, :, 1] = y[:, None]
    return out.reshape(-1, 2)


def polar_grid_params(box, origin, bandwidth, lam, aperture_len, factor=2.5,
                      c: float = C_LIGHT) -> dict:
    """Polar lattice covering an axis-aligned box (Sec. III-E).

    The grid originates at the synthetic-aperture centre ``origin``; its steps
    are the range resolution c / (2 B) and the azimuth resolution
    lam / (2 L) (L = aperture length) each divided by ``factor`` (2.5 in the
    paper).  Azimuth theta is measured from +y towards +x, so a point is
    origin + r (sin theta, cos theta).  The lattice spans the range and angle
    extent of the box corners; it is the full n_th x n_r lattice (pixels
    outside the box are kept so the lattice stays rectangular).
    """
    x0, x1, y0, y1 = (float(v) for v in box)
    ox, oy = float(origin[0]), float(origin[1])
    if not (y0 > oy):
        raise ValueError("box must lie in front of the aperture (y0 > origin y)")
    dr = c / (2.0 * bandwidth) / factor
    dth = lam / (2.0 * aperture_len) / factor
    xs = np.array([x0, x1]) - ox
    ys = np.array([y0, y1]) - oy
    # nearest range: the box point closest to the origin (the box is in front of it)
    cx = min(max(0.0, xs[0]), xs[1])
    r_min = float(np.hypot(cx, ys[0]))
    r_max = float(max(np.hypot(x, y) for x in xs for y in ys))
    th = [np.arctan2(x, y) for x in xs for y in ys]
    th_min, th_max = float(min(th)), float(max(th))
    nr = int(np.floor((r_max - r_min) / dr)) + 1
    nth = int(np.floor((th_max - th_min) / dth)) + 1
    return {"r0": r_min, "dr": dr, "nr": nr, "th0": th_min, "dth": dth, "nth": nth,
            "ox": ox, "oy": oy}


def polar_grid(ox: float, oy: float, r0: float, dr: float, nr: int,
               th0: float, dth: float, nth: int) -> np.ndarray:
    """Row-major polar lattice, theta slow: (ith, ir) -> origin + r (sin th, cos th)."""
    r = r0 + np.arange(nr, dtype=np.float64) * dr
    th = th0 + np.arange(nth, dtype=np.float64) * dth
    out = np.empty((nth, nr, 2))
    out[:, :, 0] = ox + r[None, :] * np.sin(th)[:, None]
    out[:, :, 1] = oy + r[None, :] * np.cos(th)[:, None]
    return out.reshape(-1, 2)


def resample_polar(img_polar: np.ndarray, ox: float, oy: float, r0: float, dr: float, nr: int,
                   th0: float, dth: float, nth: int, points: np.ndarray) -> np.ndarray:
    """Magnitude of a polar-grid image at arbitrary points (metres).

    Sec. III-E forms the image on a polar lattice; showing it on the
    Cartesian reference grid (the comparison of Fig. 3) needs the magnitude
    at Cartesian points.  A point's range r and azimuth theta (from +y
    towards +x, as in ``polar_grid``) give fractional lattice indices
    u = (r - r0) / dr, v = (theta - th0) / dth; |P| is interpolated
    bilinearly in (v, u) with the rule of ``interp_index`` on each axis (an
    index equal to the last one takes that sample; outside [0, n - 1] the
    result is 0).  The magnitude, not the complex value, is interpolated: the
    image's phase turns over once per half wavelength of range, far faster
    than the lattice samples it.
    """
    A = np.abs(np.asarray(img_polar)).astype(np.float64).reshape(nth, nr)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    dx, dy = pts[:, 0] - ox, pts[:, 1] - oy
    u = (np.hypot(dx, dy) - r0) / dr
    v = (np.arctan2(dx, dy) - th0) / dth
    valid = (u >= 0) & (u <= nr - 1) & (v >= 0) & (v <= nth - 1)
    us, vs = np.where(valid, u, 0.0), np.where(valid, v, 0.0)
    iu = np.minimum(np.floor(us).astype(np.int64), nr - 1)
    iv = np.minimum(np.floor(vs).astype(np.int64), nth - 1)
    fu, fv = us - iu, vs - iv
    iu1, iv1 = np.minimum(iu + 1, nr - 1), np.minimum(iv + 1, nth - 1)
    out = ((1 - fv) * ((1 - fu) * A[iv, iu] + fu * A[iv, iu1]) +
           fv * ((1 - fu) * A[iv1, iu] + fu * A[iv1, iu1]))
    return np.where(valid, out, 0.0)


# ---------------------------------------------------------------------------
# Detection stage on the image (not part of the paper): 2-D CA-CFAR
# ---------------------------------------------------------------------------
def cfar_alpha(n_train: int, pfa: float) -> float:
    """Scale of the cell-averaging threshold for exponential (square-law) cells.

    With N i.i.d. exponential training cells, P(x > alpha mean) = (1 + alpha/N)^-N,
    so alpha = N (Pfa^(-1/N) - 1) yields the requested false-alarm rate.
    """
    return float(n_train * (pfa ** (-1.0 / n_train) - 1.0))


def ca_cfar(power: np.ndarray, guard: int, train: int, pfa: float):
    """Square-law cell-averaging CFAR on a 2-D lattice.

    The training set of a cell is the (2(g+t)+1)^2 square centred on it minus
    the (2g+1)^2 guard square.  A cell is tested only when its whole window
    lies inside the lattice.  It is a detection iff power > alpha * mean(train)
    (strict).  Returns (flat indices ascending, power, threshold) as arrays.
    """
    power = np.asarray(power, dtype=np.float64)
    R, C = power.shape
    h = guard + train
    n_train = (2 * h + 1) ** 2 - (2 * guard + 1) ** 2
    alpha = cfar_alpha(n_train, pfa)
    if R < 2 * h + 1 or C < 2 * h + 1:
        return np.zeros(0, np.int64), np.zeros(0), np.zeros(0)
    view = np.lib.stride_tricks.sliding_window_view
    outer = view(power, (2 * h + 1, 2 * h + 1)).sum(axis=(-1, -2))
    inner = view(power, (2 * guard + 1, 2 * guard + 1)).sum(axis=(-1, -2))
    off = h - guard
    inner = inner[off:off + R - 2 * h, off:off + C - 2 * h]
    thresh = alpha * (outer - inner) / n_train
    cells = power[h:R - h, h:C - h]
    rr, cc = np.nonzero(cells > thresh)
    idx = (rr + h) * C + (cc + h)
    order = np.argsort(idx)
    return idx[order], cells[rr, cc][order], thresh[rr, cc][order]


def to_db(P: np.ndarray) -> np.ndarray:
    """Image amplitude in dB normalised to its maximum, 20 log10(|P| / max |P|)."""
    a = np.abs(np.asarray(P))
    m = a.max()
    with np.errstate(divide="ignore"):
        return 20.0 * np.log10(a / m)
