"""Seeded synthetic radar frames: the inputs of the SAR pipeline.

This module only *generates inputs*: vehicle trajectory, antenna positions,
scatterers and the FMCW beat signal they would produce, plus the pixel list of
a Cartesian reconstruction grid.  It contains none of the back-projection
arithmetic; both the HIP path and the CPU oracle consume what it returns.

Radar parameters are those of the paper's Tab. I (77 GHz FMCW, f0 = 76.6 GHz,
B = 931 MHz, T_P = 102.4 us, T_P0 = 106.7 us).  The real measured data of the
paper is not available, so scenes are drawn from a seeded generator:

* The vehicle drives along +x (optionally with a constant yaw rate) and the
  radar looks towards +y.  The aperture centre (mid-time of the frame) is at
  the origin.  Each chirp is transmitted at t = (j - (J - 1) / 2) T_P0 where j
  is the chirp's slot; time-multiplexed MIMO frames use n_tx slots per cycle.
* RX elements are spaced lambda/2 along the vehicle axis, TX elements
  n_rx lambda/2 (a filled virtual array).
* A point scatterer at x with complex amplitude A adds, per chirp m, channel
  ch and fast-time sample k (t_k = k / fs from the chirp start),
      A exp(j 2 pi [f0 tau + (mu tau + f_D) t_k]),
  tau = (|x - q_tx| + |x - q_rx|) / c and f_D the two-way Doppler shift
  f0 / c (<x - q_tx, v> / |x - q_tx| + <x - q_rx, v> / |x - q_rx|), evaluated at
  the chirp start (stop-and-go).  Complex white noise CN(0, 1) is added, so a
  target's per-sample SNR is |A|^2.
* All random draws use numpy's PCG64 seeded generator on the host; the tone
  synthesis itself is deterministic and may run on any torch device in float64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

C_LIGHT = 299_792_458.0

#: Tab. I of the paper.
RADAR = {
    "f0": 76.6e9,
    "bandwidth": 931e6,
    "t_chirp": 102.4e-6,
    "t_pri": 106.7e-6,
    "c": C_LIGHT,
}


@dataclasses.dataclass(frozen=True)
class SceneConfig:
    """Sizes and scene statistics of one synthetic frame."""

    name: str
    n_samples: int                 # fast-time IQ samples per chirp
    n_chirps: int                  # chirp cycles (one per TX slot group)
    n_tx: int = 1
    n_rx: int = 4
    zero_pad: int = 2              # n_fft = zero_pad * n_samples
    box: tuple = (-7.5, 7.5, 1.0, 16.0)   # x0, x1, y0, y1 in metres
    nx: int = 256
    ny: int = 256
    speed: Optional[float] = None  # m/s; None draws U[1, 9]
    yaw_rate: float = 0.0          # rad/s, 0 = straight path
    height: float = 0.0            # radar above the ground plane of targets and pixels, m
    n_targets: int = 8
    snr_db: tuple = (10.0, 30.0)
    n_clutter: int = 0             # extended clutter patches
    clutter_db: float = -10.0      # mean scatterer power of a patch (per sample)
    clutter_size: float = 0.2      # patch edge, metres
    clutter_step: float = 0.02     # scatterer lattice inside a patch, metres
    noise: bool = True
    seed: int = 1000

    @property
    def n_channels(self) -> int:
        return self.n_tx * self.n_rx

    @property
    def n_fft(self) -> int:
        return self.zero_pad * self.n_samples

    @property
    def n_pix(self) -> int:
        return self.nx * self.ny


#: Named workloads.  "plain-small" is a 256-sample x 128-chirp x 4-RX frame on a
#: 256 x 256 Cartesian grid; "plain-large" is a 1024-sample x 512-cycle frame of
#: a 4 TX x 4 RX time-multiplexed array (16 virtual channels) on the paper's
#: 1201 x 1201, 2.5 cm Cartesian grid over 30 m x 30 m; "paper-polar" is the
#: paper's combined setting, 1024 chirps x 8 RX.
CONFIGS = {
    "plain-small": SceneConfig("plain-small", n_samples=256, n_chirps=128, n_tx=1, n_rx=4,
                               box=(-7.5, 7.5, 1.0, 16.0), nx=256, ny=256, n_targets=8,
                               snr_db=(10.0, 30.0), seed=1000),
    "plain-large": SceneConfig("plain-large", n_samples=1024, n_chirps=512, n_tx=4, n_rx=4,
                               box=(-15.0, 15.0, 1.0, 31.0), nx=1201, ny=1201, speed=2.0,
                               n_targets=64, snr_db=(0.0, 30.0), n_clutter=3, seed=1001),
    "paper-polar": SceneConfig("paper-polar", n_samples=1024, n_chirps=1024, n_tx=1, n_rx=8,
                               box=(-15.0, 15.0, 1.0, 31.0), nx=1201, ny=1201, speed=1.2,
                               n_targets=64, snr_db=(0.0, 30.0), n_clutter=3, seed=1002),
    # the paper's reference setting (Sec. II, Tab. I): one TX, 16 RX, 1024 chirps
    "paper-ref": SceneConfig("paper-ref", n_samples=1024, n_chirps=1024, n_tx=1, n_rx=16,
                             box=(-15.0, 15.0, 1.0, 31.0), nx=1201, ny=1201, speed=1.2,
                             n_targets=64, snr_db=(0.0, 30.0), n_clutter=3, seed=1002),
}


def wavelength(radar=RADAR) -> float:
    return radar["c"] / radar["f0"]


def sample_rate(cfg: SceneConfig, radar=RADAR) -> float:
    """IQ sampling spans the chirp: fs = n_samples / T_P."""
    return cfg.n_samples / radar["t_chirp"]


def cartesian_pixels(box, nx: int, ny: int) -> np.ndarray:
    """float32 [ny * nx, 2] pixel list, row-major with y slow, edges included."""
    x0, x1, y0, y1 = box
    xs = x0 + (x1 - x0) * np.arange(nx, dtype=np.float64) / max(nx - 1, 1)
    ys = y0 + (y1 - y0) * np.arange(ny, dtype=np.float64) / max(ny - 1, 1)
    out = np.empty((ny, nx, 2), dtype=np.float64)
    out[:, :, 0] = xs[None, :]
    out[:, :, 1] = ys[:, None]
    return out.reshape(-1, 2).astype(np.float32)


def _trajectory(cfg: SceneConfig, speed: float, radar=RADAR):
    """Antenna positions q_tx, q_rx [M, CH, 2] and per-cycle velocity [M, 2] (float64)."""
    lam = wavelength(radar)
    M, ntx, nrx = cfg.n_chirps, cfg.n_tx, cfg.n_rx
    slots = M * ntx
    j = np.arange(slots, dtype=np.float64).reshape(M, ntx)
    t = (j - (slots - 1) / 2.0) * radar["t_pri"]
    if cfg.yaw_rate == 0.0:
        head = np.zeros_like(t)
        px = speed * t
        py = np.zeros_like(t)
    else:
        w = cfg.yaw_rate
        head = w * t
        px = speed * np.sin(head) / w
        py = speed * (1.0 - np.cos(head)) / w
    rx_off = (np.arange(nrx) - (nrx - 1) / 2.0) * lam / 2.0
    tx_off = (np.arange(ntx) - (ntx - 1) / 2.0) * nrx * lam / 2.0
    ch, sh = np.cos(head), np.sin(head)
    q_tx = np.empty((M, ntx, nrx, 2))
    q_rx = np.empty((M, ntx, nrx, 2))
    q_tx[..., 0] = (px + ch * tx_off[None, :])[:, :, None]
    q_tx[..., 1] = (py + sh * tx_off[None, :])[:, :, None]
    q_rx[..., 0] = px[:, :, None] + ch[:, :, None] * rx_off[None, None, :]
    q_rx[..., 1] = py[:, :, None] + sh[:, :, None] * rx_off[None, None, :]
    vel = np.stack([speed * ch[:, 0], speed * sh[:, 0]], axis=-1)
    return q_tx.reshape(M, ntx * nrx, 2), q_rx.reshape(M, ntx * nrx, 2), vel


def _scatterers(cfg: SceneConfig, rng: np.random.Generator):
    """Point targets uniform in the box plus optional Rayleigh clutter patches."""
    x0, x1, y0, y1 = cfg.box
    n = cfg.n_targets
    pos = np.stack([rng.uniform(x0, x1, n), rng.uniform(y0, y1, n)], axis=-1)
    snr = rng.uniform(cfg.snr_db[0], cfg.snr_db[1], n)
    amp = 10.0 ** (snr / 20.0) * np.exp(2j * np.pi * rng.uniform(0.0, 1.0, n))
    pos_l, amp_l = [pos], [amp]
    if cfg.n_clutter:
        k = max(1, int(round(cfg.clutter_size / cfg.clutter_step)))
        g = (np.arange(k) - (k - 1) / 2.0) * cfg.clutter_step
        gx, gy = np.meshgrid(g, g)
        p_mean = 10.0 ** (cfg.clutter_db / 10.0)
        for _ in range(cfg.n_clutter):
            cx = rng.uniform(x0 + cfg.clutter_size, x1 - cfg.clutter_size)
            cy = rng.uniform(y0 + cfg.clutter_size, y1 - cfg.clutter_size)
            pos_l.append(np.stack([cx + gx.ravel(), cy + gy.ravel()], axis=-1))
            z = rng.standard_normal((2, k * k))
            amp_l.append(np.sqrt(p_mean / 2.0) * (z[0] + 1j * z[1]))
    return np.concatenate(pos_l), np.concatenate(amp_l), pos, amp


def required_bins(cfg: SceneConfig, q_tx, q_rx, vel, radar=RADAR, margin: int = 2) -> int:
    """Spectrum bins to keep so every pixel of the box maps inside the kept band.

    The largest two-way path from any box corner to any antenna position, plus
    the largest possible Doppler shift, expressed on the beat-frequency axis.
    """
    fs = sample_rate(cfg, radar)
    df = fs / cfg.n_fft
    mu = radar["bandwidth"] / radar["t_chirp"]
    x0, x1, y0, y1 = cfg.box
    corners = np.array([[x0, y0], [x0, y1], [x1, y0], [x1, y1]])
    qt = q_tx.reshape(-1, 2)
    qr = q_rx.reshape(-1, 2)
    h2 = cfg.height ** 2
    dmax = (np.sqrt(((corners[:, None, :] - qt[None]) ** 2).sum(-1) + h2).max()
            + np.sqrt(((corners[:, None, :] - qr[None]) ** 2).sum(-1) + h2).max())
    vmax = float(np.sqrt((vel ** 2).sum(-1)).max())
    fmax = mu * dmax / radar["c"] + 2.0 * radar["f0"] * vmax / radar["c"]
    nb = int(math.ceil(fmax / df)) + margin
    return min(nb, cfg.n_fft)


def beat_signal(scat_pos, scat_amp, q_tx, q_rx, vel, n_samples: int, fs: float,
                radar=RADAR, device: str = "cpu", chunk: Optional[int] = None, height: float = 0.0):
    """Noise-free beat signal complex128 [M, CH, n_samples] as a torch tensor.

    Evaluated in float64 on ``device``; the carrier phase f0 tau is reduced to
    its fractional cycle before it is scaled by 2 pi.  Scatterers lie on the
    ground plane, the antennas ``height`` above it (3-D distances; the
    horizontal velocity projects on the 3-D line of sight).
    """
    import torch

    dev = torch.device(device)
    f64 = torch.float64
    qt = torch.as_tensor(q_tx, dtype=f64, device=dev)          # [M, CH, 2]
    qr = torch.as_tensor(q_rx, dtype=f64, device=dev)
    v = torch.as_tensor(vel, dtype=f64, device=dev)[:, None, :]  # [M, 1, 2]
    M, CH, _ = qt.shape
    k = torch.arange(n_samples, dtype=f64, device=dev) / fs     # fast time, s
    out = torch.zeros((M, CH, n_samples), dtype=torch.complex128, device=dev)
    c, f0 = radar["c"], radar["f0"]
    mu = radar["bandwidth"] / radar["t_chirp"]
    pos = np.asarray(scat_pos, dtype=np.float64)
    amp = np.asarray(scat_amp, dtype=np.complex128)
    if chunk is None:
        per = M * CH * n_samples * 16 * 3
        chunk = max(1, int((1 << 30) // per))
    for s0 in range(0, pos.shape[0], chunk):
        x = torch.as_tensor(pos[s0:s0 + chunk], dtype=f64, device=dev)[:, None, None, :]
        a = torch.as_tensor(amp[s0:s0 + chunk], dtype=torch.complex128, device=dev)
        rt = x - qt[None]
        rr = x - qr[None]
        dt = torch.sqrt((rt * rt).sum(-1) + height * height)
        dr = torch.sqrt((rr * rr).sum(-1) + height * height)
        tau = (dt + dr) / c
        fdop = f0 / c * ((rt * v[None]).sum(-1) / dt + (rr * v[None]).sum(-1) / dr)
        ph0 = torch.remainder(f0 * tau, 1.0)                     # [S, M, CH]
        fb = mu * tau + fdop                                     # Hz
        cyc = ph0[..., None] + fb[..., None] * k                 # [S, M, CH, K]
        cyc = torch.remainder(cyc, 1.0)
        tone = torch.polar(torch.ones_like(cyc), 2.0 * math.pi * cyc)
        out += (a[:, None, None, None] * tone).sum(0)
    return out


@dataclasses.dataclass
class Frame:
    """One synthetic frame; arrays are numpy on the host unless noted."""

    cfg: SceneConfig
    raw: np.ndarray            # complex64 [M, CH, n_samples]
    q_tx: np.ndarray           # float32 [M, CH, 2]
    q_rx: np.ndarray           # float32 [M, CH, 2]
    vel: np.ndarray            # float32 [M, 2]
    pix: np.ndarray            # float32 [n_rows * n_cols, 2]
    n_rows: int
    n_cols: int
    fs: float
    n_fft: int
    n_bins: int
    targets: np.ndarray        # float64 [n_targets, 2] point-target positions
    target_amp: np.ndarray     # complex128 [n_targets]
    speed: float


def make_frame(cfg: SceneConfig, frame_index: int = 0, device: str = "cpu",
               radar=RADAR) -> Frame:
    """Draw and synthesise one frame.

    The scene (targets, clutter, speed) depends on ``cfg.seed``; the noise on
    ``2000 + frame_index``, so frames of one scene differ only in noise.
    """
    rng = np.random.default_rng(cfg.seed)
    speed = float(cfg.speed) if cfg.speed is not None else float(rng.uniform(1.0, 9.0))
    q_tx, q_rx, vel = _trajectory(cfg, speed, radar)
    # antenna positions and pixels are handed over in float32; the signal is
    # synthesised from exactly those float32 positions
    q_tx32 = q_tx.astype(np.float32)
    q_rx32 = q_rx.astype(np.float32)
    vel32 = vel.astype(np.float32)
    pos, amp, tpos, tamp = _scatterers(cfg, rng)
    fs = sample_rate(cfg, radar)
    sig = beat_signal(pos, amp, q_tx32, q_rx32, vel32, cfg.n_samples, fs, radar, device, height=cfg.height)
    raw = sig.to("cpu").numpy()
    if cfg.noise:
        nrng = np.random.default_rng(2000 + frame_index)
        z = nrng.standard_normal((2,) + raw.shape)
        raw = raw + (z[0] + 1j * z[1]) * math.sqrt(0.5)
    pix = cartesian_pixels(cfg.box, cfg.nx, cfg.ny)
    return Frame(cfg=cfg, raw=raw.astype(np.complex64), q_tx=q_tx32, q_rx=q_rx32, vel=vel32,
                 pix=pix, n_rows=cfg.ny, n_cols=cfg.nx, fs=fs, n_fft=cfg.n_fft,
                 n_bins=required_bins(cfg, q_tx, q_rx, vel, radar), targets=tpos,
                 target_amp=tamp, speed=speed)


def random_spectrum(rng: np.random.Generator, shape: Sequence[int]) -> np.ndarray:
    """complex64 CN(0, 1) array, e.g. a beat spectrum [M, CH, NB] for stage tests."""
    z = rng.standard_normal((2,) + tuple(shape))
    return ((z[0] + 1j * z[1]) * math.sqrt(0.5)).astype(np.complex64)


def mixed_configs(n: int, seed: int = 3000):
    """Scene configurations of a mixed-size sensor population: n_samples in
    {128, 256, 512, 1024}, n_chirps in {64, 128, 256, 512}, channels in
    {4, 8, 16} (one TX), a G x G Cartesian grid with G in {128, 256, 512}, all
    drawn uniformly; 8 point targets at 10-30 dB in a 15 m box, which keeps the
    farthest path inside the unambiguous range of the smallest sample count."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        g = int(rng.choice([128, 256, 512]))
        out.append(SceneConfig(
            f"mixed-{i}", n_samples=int(rng.choice([128, 256, 512, 1024])),
            n_chirps=int(rng.choice([64, 128, 256, 512])), n_tx=1, n_rx=int(rng.choice([4, 8, 16])),
            box=(-7.5, 7.5, 1.0, 16.0), nx=g, ny=g, n_targets=8, snr_db=(10.0, 30.0),
            seed=int(seed + 1 + i)))
    return out
