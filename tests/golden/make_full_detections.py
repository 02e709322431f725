#!/usr/bin/env python3
"""Writes the oracle's CA-CFAR detection lists of the two full-size frames.

    python tests/golden/make_full_detections.py [--procs N] [--only NAME] [--fingerprint-only]

For the benchmark's frame (plain-large: 1024 IQ samples x 512 TDM cycles x 16
channels on the 1201 x 1201 Cartesian grid) and the paper's configuration
(paper-polar: 1024 samples x 1024 chirps x 8 RX on the polar lattice of
Sec. III-E), this script forms the whole image with the FP64 oracle (range
DFT, Doppler table of Sec. III-D, Alg. 2 over every pixel), runs its CA-CFAR
(guard 2, train 8, Pfa 1e-4) over the whole lattice, and stores

  * every detection (flat cell index, |P|^2, threshold),
  * every tested cell whose power lies within 5 % of its threshold (the cells
    whose decision a reduced-precision image may legitimately flip), and
  * SHA-256 digests of the synthetic beat cube and pixel list the values were
    formed from, and a seeded sample of their values, so a test can confirm it
    feeds the GPU the same frame (to the last-bit rounding another host's or
    the GPU's synthesis may differ by).

Only the oracle and the seeded input generator are used; nothing here touches
the HIP library.  Alg. 2 runs on disjoint pixel slices in a pool of
single-threaded processes (back-projection is pointwise, so the slices are
independent and the result is the same as one pass).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GUARD, TRAIN, PFA = 2, 8, 1e-4
NEAR = 0.05
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_detections_{}.json")

_ARGS = None


def _init(args):
    global _ARGS
    _ARGS = args


def _bp_slice(bounds):
    import oracle as O

    pix, fd, q_tx, q_rx, s, w, a1, a2 = _ARGS
    lo, hi = bounds
    return lo, O.bp_alg2(pix[lo:hi], q_tx, q_rx, fd[lo:hi], s, w, a1, a2, chunk=1024)


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


SAMPLE_SEED, SAMPLE_N = 4242, 2048


def sample_index(n: int) -> np.ndarray:
    """Seeded positions of the elements a fingerprint records."""
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, size=min(n, SAMPLE_N), replace=False))


def fingerprint(fr) -> dict:
    """A seeded sample of the beat cube and of the pixel list.  Another host's
    libm (or the GPU) may round the synthesis differently in the last bit, so
    a test recognises the frame by these values to a tolerance, not by its
    digest alone."""
    raw = np.ascontiguousarray(fr.raw).reshape(-1)
    pix = np.ascontiguousarray(fr.pix).reshape(-1)
    ri, pi = sample_index(raw.size), sample_index(pix.size)
    return {"sample_seed": SAMPLE_SEED,
            "raw_sample": [[float(v.real), float(v.imag)] for v in raw[ri]],
            "pix_sample": [float(v) for v in pix[pi]]}


def frame_of(name: str):
    """The frame the GPU tests build for this workload (CPU synthesis)."""
    import oracle as O
    from paper_2306_09784_amd import synth

    fr = synth.make_frame(synth.CONFIGS[name], device="cpu")
    if name == "paper-polar":
        fr = polar_frame(fr)
    return fr


def polar_frame(fr):
    """The polar lattice of Sec. III-E around the aperture centre, spanning the
    scene box, with the aperture length the antennas' extent along x."""
    import dataclasses

    import oracle as O
    from paper_2306_09784_amd import synth

    q = np.concatenate([fr.q_tx.reshape(-1, 2), fr.q_rx.reshape(-1, 2)]).astype(np.float64)
    g = O.polar_grid_params(fr.cfg.box, (float(q[:, 0].mean()), float(q[:, 1].mean())),
                            synth.RADAR["bandwidth"], synth.RADAR["c"] / synth.RADAR["f0"],
                            float(np.ptp(q[:, 0])))
    pix = O.polar_grid(g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"]).astype(np.float32)
    return dataclasses.replace(fr, pix=pix, n_rows=g["nth"], n_cols=g["nr"])


def oracle_power(fr, procs: int):
    import oracle as O
    from paper_2306_09784_amd import synth

    R = synth.RADAR
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], fr.fs, fr.n_fft)
    s = O.range_compress(fr.raw, O.window("hann", fr.cfg.n_samples), fr.n_fft, fr.n_bins)
    pix = fr.pix.astype(np.float64)
    fd = O.doppler_table(pix, fr.q_tx, fr.q_rx, fr.vel, k["kd"])
    w = O.window("hann", fr.cfg.n_chirps)
    n = pix.shape[0]
    step = 4096
    P = np.zeros(n, np.complex128)
    args = (pix, fd, fr.q_tx, fr.q_rx, s, w, k["a1"], k["a2"])
    # single-threaded workers, one per core
    saved = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        with mp.get_context("spawn").Pool(procs, initializer=_init, initargs=(args,)) as pool:
            for lo, part in pool.imap_unordered(_bp_slice, [(i, min(n, i + step)) for i in range(0, n, step)]):
                P[lo:lo + part.shape[0]] = part
    finally:
        if saved is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = saved
    return (np.abs(P) ** 2).reshape(fr.n_rows, fr.n_cols)


def cfar_stat(power):
    """(cell power, threshold) of every tested cell, as the oracle's CA-CFAR forms them."""
    import oracle as O

    R, C = power.shape
    h = GUARD + TRAIN
    n_train = (2 * h + 1) ** 2 - (2 * GUARD + 1) ** 2
    alpha = O.cfar_alpha(n_train, PFA)
    view = np.lib.stride_tricks.sliding_window_view
    outer = view(power, (2 * h + 1, 2 * h + 1)).sum(axis=(-1, -2))
    inner = view(power, (2 * GUARD + 1, 2 * GUARD + 1)).sum(axis=(-1, -2))
    off = h - GUARD
    thr = alpha * (outer - inner[off:off + R - 2 * h, off:off + C - 2 * h]) / n_train
    return power[h:R - h, h:C - h], thr


def make(name: str, procs: int) -> dict:
    import oracle as O

    t0 = time.perf_counter()
    fr = frame_of(name)
    t1 = time.perf_counter()
    power = oracle_power(fr, procs)
    t2 = time.perf_counter()
    idx, pw, thr = O.ca_cfar(power, GUARD, TRAIN, PFA)
    p, t = cfar_stat(power)
    h = GUARD + TRAIN
    near = np.argwhere(np.abs(p - t) <= NEAR * t)
    near_idx = (near[:, 0] + h) * fr.n_cols + (near[:, 1] + h)
    order = np.argsort(near_idx)
    rec = {
        "_cite": "Alg. 2 (Sec. IV) with the Doppler table of Sec. III-D on the paper's scene geometry; "
                 "square-law CA-CFAR on |P|^2 (the detection stage layered on the image)",
        "_command": "python tests/golden/make_full_detections.py",
        "workload": name,
        "n_rows": fr.n_rows, "n_cols": fr.n_cols, "n_bins": fr.n_bins,
        "guard": GUARD, "train": TRAIN, "pfa": PFA, "near_rel": NEAR,
        "raw_sha256": digest(fr.raw), "pix_sha256": digest(fr.pix),
        **fingerprint(fr),
        "max_power": float(power.max()),
        "detections": [[int(i), float(a), float(b)] for i, a, b in zip(idx, pw, thr)],
        "near": [[int(near_idx[j]), float(p[tuple(near[j])]), float(t[tuple(near[j])])] for j in order],
    }
    print(f"{name}: synthesis {t1 - t0:.0f} s, oracle image {t2 - t1:.0f} s, {len(idx)} detections, "
          f"{len(near_idx)} cells within {NEAR:.0%} of the threshold", flush=True)
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", default=None)
    ap.add_argument("--fingerprint-only", action="store_true",
                    help="re-synthesise the frames and refresh only their digests and samples, after checking "
                         "that the frames are the ones the stored lists were formed from")
    a = ap.parse_args()
    for name in ("plain-large", "paper-polar"):
        if a.only and name != a.only:
            continue
        if a.fingerprint_only:
            with open(OUT.format(name)) as f:
                rec = json.load(f)
            fr = frame_of(name)
            if digest(fr.raw) != rec["raw_sha256"] or digest(fr.pix) != rec["pix_sha256"]:
                raise SystemExit(f"{name}: this host synthesises another frame; recompute the lists instead")
            rec.update(fingerprint(fr))
        else:
            rec = make(name, a.procs)
        with open(OUT.format(name), "w") as f:
            json.dump(rec, f, separators=(",", ":"))
            f.write("\n")


if __name__ == "__main__":
    main()
