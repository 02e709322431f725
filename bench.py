#!/usr/bin/env python3
"""Benchmark: real-time FMCW SAR imaging (range compression -> Doppler table ->
Alg. 2 back-projection -> CA-CFAR detection) on one MI355X.

One step = one radar frame through the whole pipeline: rc_process_batch on a
frame whose beat cube is already resident in HBM (geometry travels from host
memory through pinned staging, as every frame's ego pose does), then the
detection list back on the host.  Prints one JSON line.

Workload (the single-GPU large configuration): 1024 IQ samples x 512 TDM cycles
x 16 virtual channels (4 TX x 4 RX), complex64; 64 point targets, SNR uniform
0-30 dB, plus 3 Rayleigh clutter patches at -10 dB; Hann range window, DFT
2048 cropped to the bins the 30 m x 30 m scene needs; Hann chirp window;
1201 x 1201 Cartesian grid at 2.5 cm; CA-CFAR guard 2, train 8, Pfa 1e-4.
"""
from __future__ import annotations

import argparse
import contextlib
import dataclasses
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "radar frames/s and p50/p99 frame latency at 1 MI355X; % HBM roofline"

# gfx950 issue rates, in lanes per clock per CU (x 256 CUs x 2.4 GHz), as
# measured with independent instruction streams on the GPU: FP32 add, multiply
# and FMA 128 (78.6e12 lane-instructions/s, the published 157.3 TFLOP/s FP32
# vector peak with an FMA counted as two flops); conversions, fractions and
# integer shifts 64; transcendentals (sqrt, sin, cos) 32.  Costs below are in
# issue slots of the fastest class.
VALU_LANE_OPS = 256 * 128 * 2.4e9
HALF_SLOTS = 2.0
TRANS_SLOTS = 4.0
# the same classes' rates as the microbenchmarks measured them (midpoints of
# the measured ranges: v_fma/v_fmac/v_add/v_mul 57-64, v_cvt/v_fract 36-37,
# v_sqrt/v_sin 18-19 T lane-instructions/s); nominal full rate is 78.6 T
MEASURED_LANE_RATES = {"full": 60.5e12, "half": 36.5e12, "trans": 18.5e12}
HBM_PEAK_GBS = 8000.0
PUBLISHED_FP32_TFLOPS = 157.3


def alg2_cost(chg: int):
    """(algorithmic FP32 flops, issue slots) per back-projection term.

    Flops, those of the algorithm as written (FMA = 2; sqrt, sin, cos,
    floor/fraction = 1): squared RX distance and its square root 6, path sum
    1, index 2, index fraction 1, sin + cos 2 (the hardware takes the phase in
    turns and reduces it), interpolation 4 (value and slope of the segment),
    complex multiply-accumulate 8 = 24 per term, plus the TX distance with the
    pixel's correction term (7) once per group of chg channels that share a
    TX position.
    Slots, those of the compiled loop: 11 add/mul/FMA (squared distance 3,
    path sum 1, index 1, interpolation 2, multiply-accumulate 4), 1 half-rate
    (the index conversion: the table holds each segment's intercept and
    slope in the fractional index itself, so no fraction is formed, and the
    table load takes the bin index, which the buffer descriptor's 16-byte
    stride scales) and 3 transcendentals (sqrt, sin, cos) per term, plus 4
    add/FMA and 1 sqrt per TX distance.
    """
    flops = 24.0 + 7.0 / chg
    slots = 11.0 + HALF_SLOTS + 3 * TRANS_SLOTS + (4.0 + TRANS_SLOTS) / chg
    return flops, slots


def alg2_classes(chg: int):
    """VALU instructions per back-projection term by rate class (full-rate
    add/mul/FMA, half-rate conversion, transcendental), as alg2_cost counts
    them: slots = full + HALF_SLOTS half + TRANS_SLOTS trans."""
    return {"full": 11.0 + 4.0 / chg, "half": 1.0, "trans": 3.0 + 1.0 / chg}


def measured_rate_ceiling(chg: int) -> float:
    """Terms/s if every instruction class of the loop issued at its measured
    rate (MEASURED_LANE_RATES), one class after another."""
    return 1.0 / sum(n / MEASURED_LANE_RATES[k] for k, n in alg2_classes(chg).items())


def _kernel_sources_digest() -> str:
    """sha256 over the back-projection kernel's sources (bp.hip, rc_kernels.hpp)."""
    import hashlib

    h = hashlib.sha256()
    for name in ("bp.hip", "rc_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2306_09784_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per bp_kernel launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a device copy of known size), or None when the summary is missing or
    was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"bp_kernel_{workload}.traffic.txt")
    try:
        with open(path) as f:
            kv = dict(line.split(None, 1) for line in f if line.strip() and not line.startswith("#"))
    except OSError:
        return None
    if kv.get("kernel_sources_sha256", "").strip() != _kernel_sources_digest():
        return None
    return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])


_POOL_ARGS = None


def _pool_init(args):
    global _POOL_ARGS
    _POOL_ARGS = args


def _pool_bp(bounds):
    """Worker of the process pool: Alg. 2 of the oracle on pixels [lo, hi)."""
    import oracle as O

    pix, fd, q_tx, q_rx, s, w, a1, a2 = _POOL_ARGS
    lo, hi = bounds
    t0 = time.perf_counter()
    O.bp_alg2(pix[lo:hi], q_tx, q_rx, fd[lo:hi], s, w, a1, a2)
    return time.perf_counter() - t0


def _pool_bp_image(bounds):
    """Worker of the process pool: Alg. 2 of the oracle on pixels [lo, hi), the values."""
    import oracle as O

    pix, fd, q_tx, q_rx, s, w, a1, a2 = _POOL_ARGS
    lo, hi = bounds
    return O.bp_alg2(pix[lo:hi], q_tx, q_rx, fd[lo:hi], s, w, a1, a2)


def cpu_baseline(frame, budget_s: float = 20.0, procs: int = 16):
    """The FP64 oracle on this host's cores: range compression, Doppler table
    and CFAR over the whole frame in this process, Alg. 2 on disjoint pixel
    slices in a pool of single-threaded processes (one per core, at most
    `procs`), extrapolated linearly in pixels (back-projection is pointwise)."""
    import multiprocessing as mp

    import oracle as O
    from paper_2306_09784_amd import synth

    R = synth.RADAR
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], frame.fs, frame.n_fft)
    t0 = time.perf_counter()
    s = O.range_compress(frame.raw, O.window("hann", frame.cfg.n_samples), frame.n_fft, frame.n_bins)
    t_range = time.perf_counter() - t0
    pix = frame.pix.astype(np.float64)
    t0 = time.perf_counter()
    fd = O.doppler_table(pix, frame.q_tx, frame.q_rx, frame.vel, k["kd"])
    t_dop = time.perf_counter() - t0
    w = O.window("hann", frame.cfg.n_chirps)
    n_pix = pix.shape[0]
    # calibrate a slice that takes about budget_s on one core
    n = 256
    t0 = time.perf_counter()
    O.bp_alg2(pix[:n], frame.q_tx, frame.q_rx, fd[:n], s, w, k["a1"], k["a2"])
    t_cal = time.perf_counter() - t0
    n2 = int(min(n_pix // max(1, procs), max(n, n * (budget_s - t_cal) / max(t_cal, 1e-3))))
    P = max(1, min(procs, os.cpu_count() or 1))
    env_keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {key: os.environ.get(key) for key in env_keys}
    for key in env_keys:
        os.environ[key] = "1"
    try:
        ctx = mp.get_context("spawn")
        args = (pix, fd, frame.q_tx, frame.q_rx, s, w, k["a1"], k["a2"])
        with ctx.Pool(P, initializer=_pool_init, initargs=(args,)) as pool:
            pool.map(_pool_bp, [(0, 8)] * P)  # start-up outside the timed region
            t0 = time.perf_counter()
            per_proc = pool.map(_pool_bp, [(n + i * n2, n + (i + 1) * n2) for i in range(P)])
            t_bp = time.perf_counter() - t0
    finally:
        for key, v in saved.items():
            if v is None:
                os.environ.pop(key, None)
            else:
                os.environ[key] = v
    pix_per_s = P * n2 / t_bp
    rng = np.random.default_rng(0)
    pw = rng.exponential(1.0, (frame.n_rows, frame.n_cols))
    t0 = time.perf_counter()
    O.ca_cfar(pw, 2, 8, 1e-4)
    t_cfar = time.perf_counter() - t0
    t_frame = t_range + t_dop + n_pix / pix_per_s + t_cfar
    t_one = t_range + t_dop + n_pix * float(np.mean(per_proc)) / n2 + t_cfar
    return {
        "value": 1.0 / t_frame,
        "unit": "frames/s",
        "cores": P,
        "kind": "oracle",
        "sample": (f"FP64 NumPy oracle: range DFT of all {frame.cfg.n_chirps * frame.cfg.n_channels} rows "
                   f"({t_range:.2f} s), Doppler table ({t_dop:.2f} s) and CA-CFAR on the {frame.n_rows}x"
                   f"{frame.n_cols} lattice ({t_cfar:.2f} s) in one process; Alg. 2 on {P} x {n2} of {n_pix} "
                   f"pixels by {P} single-threaded processes in {t_bp:.1f} s, extrapolated linearly: "
                   f"{t_frame:.4g} s per frame ({t_one:.4g} s on one core)"),
    }


def cpu_full_frame(frame, pix, n_rows, n_cols, procs: int = 16):
    """The FP64 oracle over one whole frame on this host's cores, nothing
    extrapolated: range DFT, Doppler table and CA-CFAR in this process, Alg. 2
    over every pixel in slices by a pool of single-threaded processes.
    Returns (seconds, processes)."""
    import multiprocessing as mp

    import oracle as O
    from paper_2306_09784_amd import synth

    R = synth.RADAR
    P = max(1, min(procs, os.cpu_count() or 1))
    env_keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {key: os.environ.get(key) for key in env_keys}
    for key in env_keys:
        os.environ[key] = "1"
    try:
        pixd = np.asarray(pix, dtype=np.float64)
        k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], frame.fs, frame.n_fft)
        ctx = mp.get_context("spawn")
        t0 = time.perf_counter()
        s = O.range_compress(frame.raw, O.window("hann", frame.cfg.n_samples), frame.n_fft, frame.n_bins)
        fd = O.doppler_table(pixd, frame.q_tx, frame.q_rx, frame.vel, k["kd"])
        w = O.window("hann", frame.cfg.n_chirps)
        t_pre = time.perf_counter() - t0
        n = pixd.shape[0]
        step = max(256, -(-n // (4 * P)))
        args = (pixd, fd, frame.q_tx, frame.q_rx, s, w, k["a1"], k["a2"])
        with ctx.Pool(P, initializer=_pool_init, initargs=(args,)) as pool:
            pool.map(abs, range(P))  # interpreter start-up outside the timed parts
            t0 = time.perf_counter()
            parts = pool.map(_pool_bp_image, [(i, min(n, i + step)) for i in range(0, n, step)])
            t_bp = time.perf_counter() - t0
        t0 = time.perf_counter()
        P_img = np.concatenate(parts)
        O.ca_cfar((np.abs(P_img) ** 2).reshape(n_rows, n_cols), 2, 8, 1e-4)
        return t_pre + t_bp + time.perf_counter() - t0, P
    finally:
        for key, v in saved.items():
            if v is None:
                os.environ.pop(key, None)
            else:
                os.environ[key] = v


def form_outputs(rc, synth, torch, frame, precision):
    """One frame in one precision form: its spectrum (before w_sar), image and
    detections, on the host."""
    dev = torch.device("cuda:0")
    cfg = frame.cfg
    n_pix = frame.n_rows * frame.n_cols
    raw = torch.from_numpy(frame.raw).to(dev)
    pix = torch.from_numpy(np.ascontiguousarray(frame.pix)).to(dev)
    img = torch.empty((n_pix, 2), dtype=torch.float32, device=dev)
    spec = torch.empty((cfg.n_chirps, cfg.n_channels, frame.n_bins, 2), dtype=torch.float32, device=dev)
    pc = rc.PlanConfig(radar=synth.RADAR, n_samples_max=cfg.n_samples, n_fft_max=frame.n_fft,
                       n_bins_max=frame.n_bins, n_chirps_max=cfg.n_chirps, n_channels_max=cfg.n_channels,
                       n_pix_max=n_pix, max_detections=1 << 16, precision=precision, cfar_margin_rel=1e-2)
    with rc.Plan(pc) as plan:
        f = rc.Plan.make_frame(1, data=raw, q_tx=frame.q_tx, q_rx=frame.q_rx, vel=frame.vel, pixels=pix,
                               n_rows=frame.n_rows, n_cols=frame.n_cols, n_bins=frame.n_bins, n_fft=frame.n_fft,
                               fs=frame.fs, n_samples=cfg.n_samples, image_out=img, spectrum_out=spec,
                               height=cfg.height)
        plan.process([f])
        dets = plan.detections(1)
        plan.release(1)
    torch.cuda.synchronize()
    return {"spectrum": spec.cpu().numpy().view(np.complex64)[..., 0], "image": img.cpu().numpy().view(np.complex64)
            .reshape(-1), "detections": dets}


def oracle_errors(frame, forms, workload, n_pixels=300):
    """Per-stage error of every precision form against the FP64 oracle (part of
    the oracle's leg of the benchmark): the spectrum's relative L2 error over
    all rows, the image's max |dP| / max |P| on n_pixels sampled pixels and the
    brightest ones, and the detection list against the oracle's list of the
    whole image (stored by tests/golden/make_full_detections.py for this
    frame), as cells that differ and how many of them lie outside 1 % of the
    oracle's threshold."""
    import oracle as O
    from paper_2306_09784_amd import synth

    R = synth.RADAR
    k = O.radar_constants(R["f0"], R["bandwidth"], R["t_chirp"], frame.fs, frame.n_fft)
    s = O.range_compress(frame.raw, O.window("hann", frame.cfg.n_samples), frame.n_fft, frame.n_bins)
    rng = np.random.default_rng(91)
    any_img = next(iter(forms.values()))["image"]
    idx = np.unique(np.concatenate([rng.integers(0, any_img.size, n_pixels), np.argsort(-np.abs(any_img))[:50]]))
    pix = frame.pix.astype(np.float64)[idx]
    fd = O.doppler_table(pix, frame.q_tx, frame.q_rx, frame.vel, k["kd"])
    P = O.bp_alg2(pix, frame.q_tx, frame.q_rx, fd, s, O.window("hann", frame.cfg.n_chirps), k["a1"], k["a2"])
    gold = None
    path = os.path.join(ROOT, "tests", "golden", f"full_detections_{workload}.json")
    if os.path.exists(path):
        with open(path) as f:
            gold = json.load(f)
    out = {}
    for name, o in forms.items():
        e = {"spectrum_rel_l2": float(np.linalg.norm(o["spectrum"] - s) / np.linalg.norm(s)),
             "image_max_rel": float(np.abs(o["image"][idx].astype(np.complex128) - P).max() / np.abs(P).max())}
        if gold is not None:
            g = set(int(c) for c in o["detections"]["pixel"])
            ol = set(int(d[0]) for d in gold["detections"])
            near = {int(c): (p, t) for c, p, t in gold["near"]}
            diff = g ^ ol
            e["detections"] = len(g)
            e["oracle_detections"] = len(ol)
            e["detections_differing"] = len(diff)
            e["differing_beyond_1pct_of_threshold"] = sum(
                1 for c in diff if c not in near or abs(near[c][0] - near[c][1]) > 1e-2 * near[c][1])
        out[name] = e
    return out


def time_pipeline(rc, synth, torch, frame, pix_host, n_rows, n_cols, precision, steps, warmup,
                  doppler=0, want_image=False, depth=2, n_streams=None, plan_kw=None, upload=False):
    """Times `steps` frames through rc_process_batch + rc_detections, `depth`
    frames in flight: frame i + 1 is prepared on the host and enqueued while
    the GPU still processes frame i (a sensor streams frames back to back).
    With two or more in flight, frames alternate between n_streams HIP streams
    (default two, each with its own image buffer), so one frame's short stages
    run beside the other's back-projection.  Latency is per frame, from its
    submission to its detections on the host.

    upload=True: each frame's beat cube starts in pinned host memory (the
    paper's Load with pinned memory, Tab. II row 8) and is copied to the
    frame's device buffer on a copy stream; the frame's stream waits for that
    copy's event, so the copy of one frame overlaps the other frame's
    back-projection; latency then runs from the cube being ready in pinned
    memory to the detections on the host.  upload="plan": the plan itself
    takes the cube from pinned memory (an HBM-budget plan, rc_frame.data_host)
    and copies it on its copy stream in chirp-block pieces, each block's
    kernels waiting only for its own piece."""
    dev = torch.device("cuda:0")
    cfg = frame.cfg
    raw = torch.from_numpy(frame.raw).to(dev)
    pix = torch.from_numpy(np.ascontiguousarray(pix_host)).to(dev)
    n_pix = n_rows * n_cols
    if n_streams is None:
        n_streams = 2 if depth >= 2 else 1
    imgs = [torch.empty((n_pix, 2), dtype=torch.float32, device=dev) for _ in range(n_streams)]
    if upload:
        host = torch.empty(frame.raw.shape, dtype=torch.complex64, pin_memory=True)
        host.copy_(torch.from_numpy(frame.raw))
        raws = [torch.empty_like(raw) for _ in range(n_streams)]
        copy_stream = torch.cuda.Stream()
    else:
        raws = [raw] * n_streams
    by_plan = upload == "plan"
    pc = rc.PlanConfig(radar=synth.RADAR, n_samples_max=cfg.n_samples, n_fft_max=frame.n_fft,
                       n_bins_max=frame.n_bins, n_chirps_max=cfg.n_chirps, n_channels_max=cfg.n_channels,
                       n_pix_max=n_pix, max_frames_in_flight=max(2, depth), max_detections=1 << 16,
                       precision=precision, doppler=doppler, stage_timing=True, **(plan_kw or {}))
    if by_plan:  # an arena for the frames in flight plus one
        probe = dataclasses.replace(pc, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=1 << 40)
        one = rc.frame_bytes(probe, rc.Plan.make_frame(
            0, data=None, data_host=host, q_tx=frame.q_tx, q_rx=frame.q_rx, vel=frame.vel, pixels=pix,
            n_rows=n_rows, n_cols=n_cols, n_bins=frame.n_bins, n_fft=frame.n_fft, fs=frame.fs,
            n_samples=cfg.n_samples, height=cfg.height))
        pc = dataclasses.replace(probe, hbm_budget_bytes=(max(2, depth) + 1) * one)
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(n_streams - 1)]
    lat, stages, n_det = [], [], 0
    last_dets = None
    with rc.Plan(pc) as plan:
        def submit(fid):
            k = fid % n_streams
            if upload and not by_plan:  # the copy on its own stream, then the frame's kernels after it
                # (buffer k was last read by frame fid - n_streams, which the
                # loop below has already waited for)
                with torch.cuda.stream(copy_stream):
                    raws[k].copy_(host, non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(copy_stream)
                streams[k].wait_event(ev)
            fr = rc.Plan.make_frame(fid, data=None if by_plan else raws[k], q_tx=frame.q_tx, q_rx=frame.q_rx,
                                    vel=frame.vel, pixels=pix, n_rows=n_rows, n_cols=n_cols, n_bins=frame.n_bins,
                                    n_fft=frame.n_fft, fs=frame.fs, n_samples=cfg.n_samples, image_out=imgs[k],
                                    height=cfg.height, data_host=host if by_plan else None)
            plan.process([fr], streams[k])

        # the collector runs before the warm-up, not between it and the timed
        # frames: a pause there lets the GPU's clock drop again
        with no_gc():
            for i in range(warmup):
                submit(i)
                plan.detections(i)
                plan.release(i)
            torch.cuda.synchronize()
            t_start = time.perf_counter()
            t_sub = {}
            queue = []
            for i in range(steps):
                fid = 1000 + i
                t_sub[fid] = time.perf_counter()
                submit(fid)
                queue.append(fid)
                while len(queue) >= depth or (i == steps - 1 and queue):
                    done = queue.pop(0)
                    dets = plan.detections(done)
                    last_dets = dets
                    lat.append(time.perf_counter() - t_sub[done])
                    stages.append(plan.stage_times(done))
                    plan.release(done)
                    n_det = len(dets)
            torch.cuda.synchronize()
            total = time.perf_counter() - t_start
    res = {"total_s": total, "fps": steps / total, "lat": lat, "stages": np.array(stages), "n_det": n_det,
           "detections": last_dets}
    if want_image:  # the last frame's
        res["image"] = imgs[(1000 + steps - 1) % n_streams].cpu().numpy().view(np.complex64).reshape(-1)
    return res


def paper_config(rc, synth, torch, steps, warmup):
    """The paper's combined setting (Sec. IV, Tab. II rows 7-8): 1024 chirps x
    8 RX, 30 m x 30 m scene on the polar grid of Sec. III-E, synthetic data."""
    cfg = synth.CONFIGS["paper-polar"]
    frame = synth.make_frame(cfg, device="cuda")
    q = np.concatenate([frame.q_tx.reshape(-1, 2), frame.q_rx.reshape(-1, 2)])
    L = float(np.ptp(q[:, 0]))
    g = rc.grid_polar_params(synth.RADAR, cfg.box, (float(q[:, 0].mean()), float(q[:, 1].mean())), L)
    pix = rc.grid_polar(g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"])
    x0, x1, y0, y1 = cfg.box
    in_box = int(np.sum((pix[:, 0] >= x0) & (pix[:, 0] <= x1) & (pix[:, 1] >= y0) & (pix[:, 1] <= y1)))
    # frames this short (1.2 ms of back-projection) take many frames for the
    # GPU's clock to settle: at least 20 untimed and 100 timed ones
    run = time_pipeline(rc, synth, torch, frame, pix, g["nth"], g["nr"], rc.RC_PREC_FP32, max(100, steps),
                        max(20, warmup), want_image=True)
    one = time_pipeline(rc, synth, torch, frame, pix, g["nth"], g["nr"], rc.RC_PREC_FP32, 20, max(20, warmup),
                        depth=1)
    n_pix = g["nth"] * g["nr"]
    terms = float(n_pix) * cfg.n_chirps * cfg.n_channels
    bp_ms = float(one["stages"][:, 2].mean())
    # Fig. 3's comparison: the polar image shown on the 2.5 cm Cartesian grid
    # (rc_resample_polar) against the image formed on that grid directly
    cart = time_pipeline(rc, synth, torch, frame, frame.pix, frame.n_rows, frame.n_cols, rc.RC_PREC_FP32, 1, 1,
                         want_image=True)
    dev = torch.device("cuda")
    d_img = torch.from_numpy(run["image"]).to(dev)
    d_pts = torch.from_numpy(np.ascontiguousarray(frame.pix)).to(dev)
    shown = torch.empty(frame.pix.shape[0], dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rc.resample_polar(d_img, g, d_pts, shown, stream)  # warm-up
    e0.record(stream)
    rc.resample_polar(d_img, g, d_pts, shown, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    shown_h = shown.cpu().numpy()
    return {
        "workload": (f"paper-polar: {cfg.n_samples} samples x {cfg.n_chirps} chirps x {cfg.n_channels} RX, polar "
                     f"lattice {g['nth']} x {g['nr']} (dr {g['dr'] * 100:.2f} cm, dth {g['dth'] * 1e3:.2f} mrad, "
                     f"aperture {L:.3f} m; {in_box} pixels inside the 30 m x 30 m box)"),
        "frames_per_s": run["fps"],
        "ms_per_frame": 1e3 / run["fps"],
        "stages_ms": {"range": float(one["stages"][:, 0].mean()), "tables": float(one["stages"][:, 1].mean()),
                      "backprojection": bp_ms, "detection": float(one["stages"][:, 3].mean())},
        "backprojection_ms": bp_ms,
        "bp_terms_per_s": terms / (bp_ms * 1e-3),
        "p99_ms": 1e3 * float(np.percentile(one["lat"], 99)),
        "polar_on_cartesian": {
            "resample_ms": e0.elapsed_time(e1),
            "target_gain_db_vs_cartesian_image": _target_gain_db(shown_h, frame.pix, frame.targets,
                                                                 cart["image"], frame.pix),
            "region_snr_db_polar_shown": _region_snr_db(shown_h, frame.pix, frame.targets),
            "region_snr_db_cartesian": _region_snr_db(cart["image"], frame.pix, frame.targets),
            "cartesian_bp_ms": float(cart["stages"][:, 2].mean()),
        },
        "paper_tab2_row8": {"gpu": "GTX 1080 Ti (FP32, pyCUDA)", "bp_ms": 15.5, "total_ms": 18.8,
                            "bp_terms": 165061 * 1024 * 8, "bp_terms_per_s": 165061 * 1024 * 8 / 15.5e-3},
    }


def make_drive(synth, torch, n_sub=24, sub_cycles=128):
    """The plain-large sensor driving on for n_sub sub-apertures of sub_cycles
    TDM cycles (one synthesis of the whole drive, cut into sub-apertures):
    device and pinned host copies of each beat cube, geometry per sub-aperture."""
    import dataclasses

    cfg = dataclasses.replace(synth.CONFIGS["plain-large"], name="plain-large-stream", n_chirps=n_sub * sub_cycles)
    t0 = time.perf_counter()
    fr = synth.make_frame(cfg, device="cuda")
    t_synth = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    subs = []
    for j in range(n_sub):
        sl = slice(j * sub_cycles, (j + 1) * sub_cycles)
        host = torch.from_numpy(np.ascontiguousarray(fr.raw[sl]))
        subs.append(dict(raw=host.to(dev), raw_pinned=host.pin_memory(), q_tx=np.ascontiguousarray(fr.q_tx[sl]),
                         q_rx=np.ascontiguousarray(fr.q_rx[sl]), vel=np.ascontiguousarray(fr.vel[sl])))
    pix = torch.from_numpy(np.ascontiguousarray(fr.pix)).to(dev)
    return cfg, fr, subs, pix, t_synth


def continuous_serving(rc, synth, torch, drive, capacity, sub_cycles=128, K=4, load=0.7, duration_s=20.0,
                       max_batch=8):
    """Sensors like the continuous-SAR one, each emitting a sub-aperture every
    hop (its radar time, 128 cycles x 4 TX x T_P0 = 54.6 ms) from a random
    phase, as many as make load x the measured aperture capacity; beat cubes
    uploaded from pinned memory; the sensors share the synthesised drive
    (each from its own offset; the drive's first sub-aperture starts a new
    stream)."""
    from paper_2306_09784_amd import serve

    cfg, fr, subs, pix, _ = drive
    hop = sub_cycles * cfg.n_tx * synth.RADAR["t_pri"]
    n_sensors = max(1, int(load * capacity * hop))
    pc = rc.PlanConfig(radar=synth.RADAR, n_samples_max=cfg.n_samples, n_fft_max=fr.n_fft, n_bins_max=fr.n_bins,
                       n_chirps_max=sub_cycles, n_channels_max=cfg.n_channels, n_pix_max=fr.n_rows * fr.n_cols,
                       max_frames_in_flight=16, max_detections=1 << 14, sliding_sensors=n_sensors,
                       sliding_subapertures=K, sliding_depth=2)
    drive_subs = [serve.SubAperture(s["raw_pinned"], s["q_tx"], s["q_rx"], s["vel"]) for s in subs]
    sensors = [serve.ContinuousSensor(i, drive_subs, fr, pix, offset=(5 * i) % len(subs)) for i in range(n_sensors)]
    srv = serve.ContinuousServer(pc, n_streams=2)
    try:
        with no_gc():
            res = serve.run_continuous(srv, sensors, hop, duration_s, max_batch=max_batch)
    finally:
        srv.close()
    res["load"] = load
    return res


def continuous_sar(rc, synth, torch, main_fps, drive, sub_cycles=128, K=4, depth=2):
    """Continuous SAR (the conclusion's continuous measurement): the large
    workload's sensor drives on; its stream is cut into sub-apertures of
    sub_cycles TDM cycles and every sub-aperture completes an aperture of the
    last K (K * sub_cycles = the large workload's 512 cycles, overlapping by
    (K - 1) / K).  Each chirp is back-projected once (three sums) and every
    aperture is formed from the sums of its K sub-apertures.  The stream is
    processed once untimed, then started again and timed over its full
    apertures (sub-apertures K - 1 .. n_sub - 1), two in flight."""
    import dataclasses

    cfg, fr, subs, pix, t_synth = drive
    n_sub = len(subs)
    dev = torch.device("cuda:0")
    S = sub_cycles
    n_pix = fr.n_rows * fr.n_cols
    imgs = [torch.empty((n_pix, 2), dtype=torch.float32, device=dev) for _ in range(depth)]
    pc = rc.PlanConfig(radar=synth.RADAR, n_samples_max=cfg.n_samples, n_fft_max=fr.n_fft, n_bins_max=fr.n_bins,
                       n_chirps_max=S, n_channels_max=cfg.n_channels, n_pix_max=n_pix,
                       max_frames_in_flight=depth, max_detections=1 << 16, stage_timing=True,
                       sliding_sensors=1, sliding_subapertures=K, sliding_depth=depth)
    # sub-apertures alternate between two streams; the plan orders each
    # aperture after the sensor's previous one
    streams = [torch.cuda.current_stream(), torch.cuda.Stream()]
    stages, lat = [], []
    with rc.Plan(pc) as plan:
        def submit(j):
            s = subs[j]
            f = rc.Plan.make_frame(j, data=s["raw"], q_tx=s["q_tx"], q_rx=s["q_rx"], vel=s["vel"], pixels=pix,
                                   n_rows=fr.n_rows, n_cols=fr.n_cols, n_bins=fr.n_bins, n_fft=fr.n_fft, fs=fr.fs,
                                   n_samples=cfg.n_samples, image_out=imgs[j % depth], sliding=(
                                       rc.RC_SLIDE_START if j == 0 else rc.RC_SLIDE_NEXT))
            plan.process([f], streams[j % 2])

        # the collector runs before the untimed pass, not between it and the
        # timed apertures (a pause there lets the GPU's clock drop again)
        with no_gc():
            for n, j in enumerate(list(range(n_sub)) + list(range(K - 1))):
                # an untimed pass over the stream, one sub-aperture at a time
                # (its full apertures give the stage times: kernels of
                # concurrent sub-apertures would overlap), then the restarted
                # stream's first, partial apertures
                submit(j)
                if K - 1 <= n < n_sub:
                    stages.append(plan.stage_times(j))
                plan.release(j)
            torch.cuda.synchronize()
            t_start = time.perf_counter()
            t_sub, queue = {}, []
            for j in range(K - 1, n_sub):
                t_sub[j] = time.perf_counter()
                submit(j)
                queue.append(j)
                while len(queue) >= depth or (j == n_sub - 1 and queue):
                    done = queue.pop(0)
                    plan.detections(done)
                    lat.append(time.perf_counter() - t_sub[done])
                    if done != n_sub - 1:
                        plan.release(done)
            torch.cuda.synchronize()
            total = time.perf_counter() - t_start
        last = imgs[(n_sub - 1) % depth].cpu().numpy().view(np.complex64).reshape(-1)
        plan.release(n_sub - 1)
    # the same aperture formed at once (Alg. 2 over its 512 cycles, one
    # Doppler table for all of them): how far the per-sub-aperture tables move it
    lo = (n_sub - K) * S
    whole = dataclasses.replace(fr, cfg=dataclasses.replace(cfg, n_chirps=K * S),
                                raw=np.ascontiguousarray(fr.raw[lo:]), q_tx=np.ascontiguousarray(fr.q_tx[lo:]),
                                q_rx=np.ascontiguousarray(fr.q_rx[lo:]), vel=np.ascontiguousarray(fr.vel[lo:]))
    ref = time_pipeline(rc, synth, torch, whole, fr.pix, fr.n_rows, fr.n_cols, rc.RC_PREC_FP32, 1, 1,
                        want_image=True)["image"]
    st = np.array(stages)
    n_ap = n_sub - (K - 1)
    fps = n_ap / total
    hop_s = S * cfg.n_tx * synth.RADAR["t_pri"]
    terms = float(n_pix) * S * cfg.n_channels
    bp_ms = float(st[:, 2].mean())
    return {
        "workload": (f"plain-large sensor driving on: sub-apertures of {S} TDM cycles x {cfg.n_channels} channels, "
                     f"apertures of the last {K} ({K * S} cycles, {100 * (K - 1) / K:.0f} % overlap), "
                     f"{fr.n_rows}x{fr.n_cols} grid, Hann window over the aperture"),
        "apertures": n_ap,
        "apertures_per_s": fps,
        "ms_per_aperture": 1e3 / fps,
        "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "stages_ms": {"range": float(st[:, 0].mean()), "tables": float(st[:, 1].mean()),
                      "backprojection_and_combine": bp_ms, "detection": float(st[:, 3].mean())},
        "bp_terms_per_s": terms / (bp_ms * 1e-3),
        "vs_independent_apertures": fps / main_fps if main_fps else None,
        "hop_ms_of_radar_time": 1e3 * hop_s,
        "sensors_in_real_time": fps * hop_s,
        "image_vs_whole_aperture_alg2": float(np.abs(last.astype(np.complex128) - ref).max() / np.abs(ref).max()),
        "synth_s": t_synth,
    }


def _region_snr_db(img, pix, targets, rad=0.06, r_in=1.0, r_out=2.0):
    """Synthetic region SNR (the paper measures SNR over regions of its real
    scenes): mean over point targets of 10 log10(peak |P|^2 within rad of the
    target / mean |P|^2 over the ring r_in..r_out around it), the ring without
    the pixels within r_out of any other target.  The ring lies beyond the
    point response's main lobe and near side lobes, so its mean is mostly the
    image of the receiver noise (and of the scene's clutter patches, which
    are not excluded)."""
    t = np.asarray(targets, dtype=np.float64)[:, :2]
    p2 = np.abs(np.asarray(img)).astype(np.float64) ** 2
    out = []
    for i, (tx, ty) in enumerate(t):
        d = np.hypot(pix[:, 0] - tx, pix[:, 1] - ty)
        peak = p2[d < rad]
        ring = np.flatnonzero((d >= r_in) & (d < r_out))
        others = np.delete(t, i, axis=0)
        if len(others) and ring.size:
            dd = np.hypot(pix[ring, 0][:, None] - others[None, :, 0], pix[ring, 1][:, None] - others[None, :, 1])
            ring = ring[(dd >= r_out).all(axis=1)]
        if peak.size and ring.size and p2[ring].mean() > 0:
            out.append(10 * np.log10(peak.max() / p2[ring].mean()))
    return float(np.mean(out)) if out else None


def _target_gain_db(img, pix, targets, ref_img, ref_pix, rad=0.06):
    """Mean over point targets of 20 log10(peak |P| near the target / the same
    in the reference image): the synthetic stand-in for the paper's region SNR."""
    out = []
    for t in targets:
        a = np.abs(img[np.hypot(pix[:, 0] - t[0], pix[:, 1] - t[1]) < rad])
        b = np.abs(ref_img[np.hypot(ref_pix[:, 0] - t[0], ref_pix[:, 1] - t[1]) < rad])
        if a.size and b.size and b.max() > 0:
            out.append(20 * np.log10(a.max() / b.max()))
    return float(np.mean(out)) if out else None


def ablation(rc, synth, torch, steps=5, warmup=5):
    """The measures of the paper's Tab. II on one synthetic frame of its
    reference setting (1024 chirps x 16 RX, 30 m x 30 m): Alg. 1 as stated on
    the 2.5 cm Cartesian grid (reference: metres and seconds, tau, f_hyp in Hz
    and its division by df per term), then its constants folded (row 3,
    "Opt.", Sec. III-C), the Doppler table (Alg. 2, Sec. III-D), the polar grid
    (Sec. III-E), 8 of the 16 RX (Sec. III-F) and all combined.  Row 2 (the
    chirp window as a vector instead of a per-pixel, per-chirp weight, Sec.
    III-B) has no measurement here: the per-pixel window is not defined, so
    every row already uses the vector.  Reports BP time and its share of the
    reference, next to the paper's shares, and the mean coherent gain change at
    the point targets."""
    cfg = synth.CONFIGS["paper-ref"]
    frame = synth.make_frame(cfg, device="cuda")
    q = np.concatenate([frame.q_tx.reshape(-1, 2), frame.q_rx.reshape(-1, 2)])
    g = rc.grid_polar_params(synth.RADAR, cfg.box, (float(q[:, 0].mean()), float(q[:, 1].mean())),
                             float(np.ptp(q[:, 0])))
    polar = rc.grid_polar(g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"])
    half = synth.Frame(**{**frame.__dict__, "raw": np.ascontiguousarray(frame.raw[:, :8]),
                          "q_tx": np.ascontiguousarray(frame.q_tx[:, :8]),
                          "q_rx": np.ascontiguousarray(frame.q_rx[:, :8]),
                          "cfg": synth.dataclasses.replace(cfg, n_rx=8)})
    runs = {
        "ref_alg1_cartesian_16rx": (frame, frame.pix, frame.n_rows, frame.n_cols, rc.RC_DOPPLER_EXACT_DIRECT),
        "opt_constants": (frame, frame.pix, frame.n_rows, frame.n_cols, rc.RC_DOPPLER_EXACT),
        "doppler_table": (frame, frame.pix, frame.n_rows, frame.n_cols, rc.RC_DOPPLER_AVERAGE),
        "polar_grid": (frame, polar, g["nth"], g["nr"], rc.RC_DOPPLER_AVERAGE),
        "rx_8": (half, frame.pix, frame.n_rows, frame.n_cols, rc.RC_DOPPLER_AVERAGE),
        "combined": (half, polar, g["nth"], g["nr"], rc.RC_DOPPLER_AVERAGE),
    }
    paper = {"opt_constants": (83.7, 70.5), "doppler_table": (63.7, 65.0), "polar_grid": (11.9, 10.4),
             "rx_8": (51.7, 52.6), "combined": (2.9, 2.4)}
    out, ref_ms, ref_img = {}, None, None
    for name, (fr, pix, nr, nc, dop) in runs.items():
        run = time_pipeline(rc, synth, torch, fr, pix, nr, nc, rc.RC_PREC_FP32, steps, warmup, doppler=dop,
                            want_image=True, depth=1)
        bp_ms = float(run["stages"][:, 2].mean())
        ref_ms = ref_ms or bp_ms
        if ref_img is None:
            ref_img = run["image"]
        out[name] = {"bp_ms": bp_ms, "bp_share_pct": 100.0 * bp_ms / ref_ms,
                     "paper_share_pct_gpu1_gpu2": paper.get(name),
                     "target_gain_db_vs_ref": _target_gain_db(run["image"], pix, frame.targets, ref_img,
                                                               frame.pix),
                     "region_snr_db": _region_snr_db(run["image"], pix, frame.targets),
                     "pixels": nr * nc}
    out["row2_w_sar_vector"] = ("not measured: the per-pixel, per-chirp window of the initial reference is not "
                                "defined in the paper; every row uses the chirp window as a vector")
    return out


def make_sensors(rc, synth, torch, n_sensors, seed=3000):
    """Mixed-size sensor population (see synth.mixed_configs): one frame per
    sensor, beat cube in pinned host memory, pixel grid resident on the GPU."""
    from paper_2306_09784_amd import serve

    sensors = []
    for i, cfg in enumerate(synth.mixed_configs(n_sensors, seed)):
        fr = synth.make_frame(cfg, frame_index=i, device="cuda")
        raw = torch.from_numpy(fr.raw).pin_memory()
        pix = torch.from_numpy(fr.pix).to("cuda")
        sensors.append(serve.SensorStream(i, fr, raw, pix, raw.to("cuda")))
    return sensors


def mixed_plan_config(rc, synth, sensors, slots, **kw):
    """Plan for the mixed-size sensors; serving runs the split-phase form, whose
    detection lists match the FP64 oracle's outside the CFAR band."""
    frs = [s.frame for s in sensors]
    kw.setdefault("precision", rc.RC_PREC_FP32_SPLIT)
    return rc.PlanConfig(radar=synth.RADAR, n_samples_max=max(f.cfg.n_samples for f in frs),
                         n_fft_max=max(f.n_fft for f in frs), n_bins_max=max(f.n_bins for f in frs),
                         n_chirps_max=max(f.cfg.n_chirps for f in frs),
                         n_channels_max=max(f.cfg.n_channels for f in frs),
                         n_pix_max=max(f.n_rows * f.n_cols for f in frs), max_frames_in_flight=slots,
                         max_detections=1 << 14, **kw)


def batched_mixed_median(rc, synth, torch, sensors, repeats=3, **kw):
    """batched_mixed repeated; the run with the median throughput, plus every
    run's; then the same with the beat cubes resident in HBM."""
    runs = [batched_mixed(rc, synth, torch, sensors, **kw) for _ in range(repeats)]
    runs.sort(key=lambda r: r["frames_per_s"])
    med = dict(runs[len(runs) // 2])
    med["frames_per_s_runs"] = [r["frames_per_s"] for r in runs]
    res = sorted((batched_mixed(rc, synth, torch, sensors, resident=True, **kw) for _ in range(repeats)),
                 key=lambda r: r["frames_per_s"])
    med["resident"] = {"frames_per_s": res[len(res) // 2]["frames_per_s"],
                       "frames_per_s_runs": [r["frames_per_s"] for r in res],
                       "bp_terms_per_s_incl_all_stages": res[len(res) // 2]["bp_terms_per_s_incl_all_stages"]}
    # the paper's plain single-precision form on the same resident batches
    res = sorted((batched_mixed(rc, synth, torch, sensors, resident=True, precision="fp32", **kw)
                  for _ in range(repeats)), key=lambda r: r["frames_per_s"])
    med["resident_fp32"] = {"frames_per_s": res[len(res) // 2]["frames_per_s"],
                            "frames_per_s_runs": [r["frames_per_s"] for r in res],
                            "bp_terms_per_s_incl_all_stages": res[len(res) // 2]["bp_terms_per_s_incl_all_stages"]}
    # the chirp split tuned per size class (rc_plan_tune) on the resident batches
    t0 = time.perf_counter()
    table = tune_sensors(rc, synth, sensors)
    t_tune = time.perf_counter() - t0
    res = sorted((batched_mixed(rc, synth, torch, sensors, resident=True, tuning=table, **kw)
                  for _ in range(repeats)), key=lambda r: r["frames_per_s"])
    med["resident_tuned"] = {"frames_per_s": res[len(res) // 2]["frames_per_s"],
                             "frames_per_s_runs": [r["frames_per_s"] for r in res],
                             "classes": len(table),
                             "classes_changed": sum(e["chirp_blocks"] != e["default_blocks"] for e in table),
                             "tuning_s": t_tune}
    return med


def tune_sensors(rc, synth, sensors, precision="fp32-split"):
    """rc_plan_tune over one frame of every sensor (their cubes resident): the
    table of chirp splits per size class."""
    cfg = mixed_plan_config(rc, synth, sensors, 2, precision=getattr(rc, FORMS[precision]))
    descs = []
    for i, sn in enumerate(sensors):
        fr = sn.frame
        descs.append(rc.Plan.make_frame(i + 1, data=sn.raw_dev, q_tx=fr.q_tx, q_rx=fr.q_rx, vel=fr.vel,
                                        pixels=sn.pix_dev, n_rows=fr.n_rows, n_cols=fr.n_cols, n_bins=fr.n_bins,
                                        n_fft=fr.n_fft, fs=fr.fs, n_samples=fr.cfg.n_samples))
    with rc.Plan(cfg) as plan:
        return plan.tune(descs)


def batched_mixed(rc, synth, torch, sensors, n_frames=1024, batch=32, resident=False, precision="fp32-split",
                  tuning=None):
    """Frames of mixed sizes in batches of `batch` frames per rc_process_batch
    (one back-projection launch per TX-group width and 16 frames), each batch
    including the pinned-memory upload of its beat cubes (resident=False) or
    with every cube already in HBM (resident=True).  Two batches are in
    flight on two streams: the host prepares and enqueues the next batch while
    the GPU processes the current one.  tuning: a table of chirp splits per
    size class (rc_plan_tune) installed in the plan first."""
    from paper_2306_09784_amd import serve

    srv = serve.Server(mixed_plan_config(rc, synth, sensors, 2 * batch, precision=getattr(rc, FORMS[precision])),
                       n_streams=2, resident=resident)
    try:
        if tuning:
            srv.plan.set_tuning(tuning)
        order = [sensors[i % len(sensors)] for i in range(n_frames)]
        with no_gc():
            # warm-up batch (after the collector ran: no pause before the timed batches)
            srv.submit([(10**6 + i, order[i], time.perf_counter()) for i in range(min(batch, n_frames))])
            srv.harvest(block=True)
            srv.results.clear()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fid = 1
            for b0 in range(0, n_frames, batch):
                items = [(fid + i, order[b0 + i], time.perf_counter()) for i in range(min(batch, n_frames - b0))]
                fid += len(items)
                srv.submit(items)
                srv.harvest_until(batch)
            srv.harvest(block=True)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
    finally:
        srv.close()
    terms = sum(s.frame.n_rows * s.frame.n_cols * s.frame.cfg.n_chirps * s.frame.cfg.n_channels for s in order)
    out = {"frames": n_frames, "batch": batch, "batches_in_flight": 2, "precision": precision,
           "frames_per_s": n_frames / wall,
           "bp_terms_per_s_incl_all_stages": terms / wall, "wall_s": wall, "inputs": (
               "beat cubes resident in HBM" if resident else "beat cubes uploaded from pinned host memory")}
    if not resident:
        up = float(sum(s.frame.raw.nbytes for s in order))
        out["upload_bytes"] = up
        out["upload_gb_per_s"] = up / wall / 1e9
    return out


def serving(rc, synth, torch, sensors, capacity_fps, duration_s, load=0.7, slots=64, max_batch=32,
            precision="fp32-split"):
    """Poisson arrivals from all sensors at `load` x the measured batch capacity,
    continuous batching over the plan's slots (at most max_batch frames per
    batch, so a second batch can be admitted while one runs), two streams."""
    from paper_2306_09784_amd import serve

    srv = serve.Server(mixed_plan_config(rc, synth, sensors, slots, precision=getattr(rc, FORMS[precision])),
                       n_streams=2)
    try:
        with no_gc():
            res = serve.run_poisson(srv, sensors, rate_hz=load * capacity_fps, duration_s=duration_s,
                                    max_batch=max_batch)
    finally:
        srv.close()
    res["load"] = load
    res["precision"] = precision
    res["realtime_bound_ms"] = 1024 * synth.RADAR["t_pri"] * 1e3
    return res


def serving_legs(rc, synth, torch, sensors, capacity_fps, seconds):
    """Poisson serving at 70 % of the uploaded batch capacity (0.3 of the
    time), at 50 % (0.15), at 70 % with admission by bytes (0.15), at 70 % in
    the paper's plain single-precision form (0.2), and at 70 % with the
    spectrum formed on the matrix cores in FP16 (0.2)."""
    res = serving(rc, synth, torch, sensors, capacity_fps, 0.3 * seconds)
    progress("serving done")
    res["at_half_load"] = serving(rc, synth, torch, sensors, capacity_fps, 0.15 * seconds, load=0.5)
    progress("serving at half load done")
    res["by_bytes"] = serving_budget(rc, synth, torch, sensors, capacity_fps, 0.15 * seconds)
    progress("serving by bytes done")
    res["plain_fp32"] = serving(rc, synth, torch, sensors, capacity_fps, 0.2 * seconds, precision="fp32")
    progress("serving in the plain form done")
    res["fp16_spectrum"] = serving(rc, synth, torch, sensors, capacity_fps, 0.2 * seconds,
                                   precision="fp16-spectrum")
    progress("serving with the FP16 matrix-core spectrum done")
    return res


def serving_budget(rc, synth, torch, sensors, capacity_fps, duration_s, load=0.7, slots=64, max_batch=32):
    """serving() with admission by bytes: one HBM arena sized for two batches
    of the sensors' mean frame (each frame's cube copied from pinned memory
    into it by the plan), against the slots of the plan's limits plus a device
    input buffer per slot that the slot plan needs for the same run."""
    from paper_2306_09784_amd import serve

    base = mixed_plan_config(rc, synth, sensors, slots)
    probe = dataclasses.replace(base, frame_memory=rc.RC_MEMORY_BUDGET, hbm_budget_bytes=1 << 40)
    sizes = []
    for sn in sensors:
        fr = sn.frame
        sizes.append(rc.frame_bytes(probe, rc.Plan.make_frame(
            0, data=None, data_host=sn.raw_pinned, q_tx=fr.q_tx, q_rx=fr.q_rx, vel=fr.vel, pixels=sn.pix_dev,
            n_rows=fr.n_rows, n_cols=fr.n_cols, n_bins=fr.n_bins, n_fft=fr.n_fft, fs=fr.fs,
            n_samples=fr.cfg.n_samples)))
    budget = int(max(2 * max(sizes), 2 * max_batch * float(np.mean(sizes))))
    n_in = base.n_chirps_max * base.n_channels_max * base.n_samples_max
    slot_mode = rc.slot_bytes(base) * slots + slots * n_in * 8
    srv = serve.Server(dataclasses.replace(probe, hbm_budget_bytes=budget), n_streams=2)
    try:
        with no_gc():
            res = serve.run_poisson(srv, sensors, rate_hz=load * capacity_fps, duration_s=duration_s,
                                    max_batch=max_batch)
    finally:
        srv.close()
    res.update(load=load, precision="fp32-split", hbm_budget_bytes=budget, slot_mode_hbm_bytes=slot_mode,
               frame_bytes_min=min(sizes), frame_bytes_max=max(sizes), frame_bytes_mean=float(np.mean(sizes)))
    return res


@contextlib.contextmanager
def no_gc():
    """Python's cyclic collector paused during a timed host loop (collected before)."""
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()


def progress(msg: str) -> None:
    """One line on stderr per finished section (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


#: precision forms by name (constants of the binding)
FORMS = {"fp32": "RC_PREC_FP32", "fp32-split": "RC_PREC_FP32_SPLIT", "fp16-spectrum": "RC_PREC_FP16",
         "bf16-spectrum": "RC_PREC_BF16"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="plain-large")
    ap.add_argument("--streams", type=int, default=2, choices=(1, 2),
                    help="HIP streams the main workload's frames alternate over (1 for profiling: kernels of "
                         "different frames then never overlap, so per-dispatch counters stay attributable)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="duration of the Poisson serving run (0 disables it)")
    ap.add_argument("--main-only", action="store_true",
                    help="skip the split-phase, paper-configuration, batched and serving runs")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the mixed-size batch run (printed as its own JSON line)")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the mixed-size batch capacity (uploaded inputs, one run) and the serving runs "
                         "(printed as their own JSON line)")
    ap.add_argument("--sliding-only", action="store_true",
                    help="only the continuous-SAR run (printed as its own JSON line)")
    ap.add_argument("--form-only", choices=tuple(FORMS), default=None,
                    help="only the main frame in one precision form, one frame in flight (printed as its own "
                         "JSON line; for profiling that form's kernels)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for HBM counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus}: the benchmark runs one frame pipeline on one GPU; "
              "frames and sensors shard across GPUs without communication, but only N=1 is measured",
              file=sys.stderr)
        return 2

    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    if args.copy_calibration:
        n = args.copy_calibration << 18
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "copies": 3}), flush=True)
        return 0
    from paper_2306_09784_amd import rc, synth

    if args.batched_only:
        sensors = make_sensors(rc, synth, torch, 32)
        print(json.dumps({"batched_mixed": batched_mixed_median(rc, synth, torch, sensors)}), flush=True)
        return 0
    if args.serving_only:
        sensors = make_sensors(rc, synth, torch, 32)
        cap = batched_mixed(rc, synth, torch, sensors)
        print(json.dumps({"batched_mixed": cap, "serving": serving_legs(
            rc, synth, torch, sensors, cap["frames_per_s"], args.serve_seconds)}), flush=True)
        return 0
    if args.form_only:
        prec = getattr(rc, FORMS[args.form_only])
        frame = synth.make_frame(synth.CONFIGS[args.workload], device="cuda")
        one = time_pipeline(rc, synth, torch, frame, frame.pix, frame.n_rows, frame.n_cols, prec, args.steps,
                            args.warmup, depth=1)
        st = one["stages"].mean(axis=0)
        print(json.dumps({"form": args.form_only, "workload": args.workload, "frames": args.steps,
                          "stages_ms": dict(zip(("range", "tables", "backprojection", "detection"),
                                                map(float, st)))}), flush=True)
        return 0
    if args.sliding_only:
        drive = make_drive(synth, torch)
        res = continuous_sar(rc, synth, torch, None, drive)
        if args.serve_seconds > 0:
            res["serving"] = continuous_serving(rc, synth, torch, drive, res["apertures_per_s"],
                                                duration_s=args.serve_seconds / 3)
        print(json.dumps({"continuous_sar": res}), flush=True)
        return 0
    cfg = synth.CONFIGS[args.workload]
    t0 = time.perf_counter()
    frame = synth.make_frame(cfg, device="cuda")
    t_synth = time.perf_counter() - t0
    main_run = time_pipeline(rc, synth, torch, frame, frame.pix, frame.n_rows, frame.n_cols,
                             rc.RC_PREC_FP32, args.steps, args.warmup, n_streams=args.streams)
    # frame latency alone (one frame in flight)
    lat_run = time_pipeline(rc, synth, torch, frame, frame.pix, frame.n_rows, frame.n_cols,
                            rc.RC_PREC_FP32, 20, args.warmup, depth=1)
    # the same with every cube copied from pinned host memory (Load + BP + detections)
    up_run = time_pipeline(rc, synth, torch, frame, frame.pix, frame.n_rows, frame.n_cols,
                           rc.RC_PREC_FP32, args.steps, args.warmup, n_streams=args.streams, upload="plan")
    up_lat = time_pipeline(rc, synth, torch, frame, frame.pix, frame.n_rows, frame.n_cols,
                           rc.RC_PREC_FP32, 20, args.warmup, depth=1, upload="plan")
    # per-stage device times (and the roofline) from the single-frame run: with
    # two frames on two streams, kernels of different frames overlap and a
    # launch's duration no longer measures the launch alone
    stages = lat_run["stages"]
    n_pix = frame.n_rows * frame.n_cols
    progress(f"main workload: {main_run['fps']:.1f} frames/s")

    M, CH = cfg.n_chirps, cfg.n_channels
    contrib = float(n_pix) * M * CH
    chg = cfg.n_rx if cfg.n_tx > 1 else CH
    flops, slots = alg2_cost(chg)
    bp_ms = float(stages[:, 2].mean())
    achieved = contrib / (bp_ms * 1e-3) * flops / 1e12
    peak = VALU_LANE_OPS / slots * flops / 1e12
    measured_peak = measured_rate_ceiling(chg) * flops / 1e12
    range_bytes = float(M * CH) * (8 * cfg.n_samples + 8 * frame.n_bins)
    range_ms = float(stages[:, 0].mean())
    total = main_run["total_s"]
    lat = lat_run["lat"]
    out = {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "p50_ms": 1e3 * float(np.percentile(up_lat["lat"], 50)),
        "p99_ms": 1e3 * float(np.percentile(up_lat["lat"], 99)),
        "latency_note": "p50/p99: one frame in flight (20 frames), from its beat cube ready in pinned host "
                        "memory (handed to the plan, which copies it in chirp-block pieces, each block's "
                        "kernels waiting for its own piece) to its detections on the host; value and "
                        "ms_per_step: frames streamed back to back, two in flight on "
                        f"{args.streams} stream(s), cubes resident in HBM; stages_ms: device stage times of "
                        "the resident one-frame run",
        "resident_p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "resident_p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "streamed_p50_ms": 1e3 * float(np.percentile(main_run["lat"], 50)),
        "with_upload": {
            "frames_per_s": up_run["fps"],
            "ms_per_frame": 1e3 * up_run["total_s"] / args.steps,
            "streamed_p50_ms": 1e3 * float(np.percentile(up_run["lat"], 50)),
            "streamed_p99_ms": 1e3 * float(np.percentile(up_run["lat"], 99)),
            "cube_bytes": int(frame.raw.nbytes),
            "note": "each frame's cube handed to the plan in pinned host memory; the plan copies it on its "
                    "copy stream in chirp-block pieces, each block's kernels waiting for its own piece; two "
                    "frames in flight, so the copies overlap both the other frame's and the frame's own "
                    "back-projection",
        },
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: {cfg.n_samples} IQ samples x {M} chirp cycles x {CH} channels "
                         f"({cfg.n_tx}TX x {cfg.n_rx}RX) complex64, DFT {frame.n_fft} -> {frame.n_bins} bins, "
                         f"{frame.n_rows}x{frame.n_cols} Cartesian grid over 30 m x 30 m, CA-CFAR g2/t8/Pfa 1e-4"),
            "n_samples": cfg.n_samples, "n_chirps": M, "n_channels": CH, "n_bins": frame.n_bins,
            "n_pix": n_pix, "terms_per_frame": contrib, "precision": "fp32",
        },
        "stages_ms": {"range": range_ms, "tables": float(stages[:, 1].mean()), "backprojection": bp_ms,
                      "detection": float(stages[:, 3].mean())},
        "bp_terms_per_s": contrib / (bp_ms * 1e-3),
        "range_hbm_gbs": range_bytes / (range_ms * 1e-3) / 1e9,
        "range_hbm_frac": range_bytes / (range_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "detections": main_run["n_det"],
        "roofline": {
            "bound": "alu",
            "kernel": "bp_kernel (Alg. 2 back-projection)",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "peak_note": "peak = the VALU issue ceiling of this loop's instruction mix: 256 CUs x 128 FP32 "
                         "lanes/clock x 2.4 GHz over the issue slots one term needs (full-rate add/FMA 1, "
                         "index conversion 2, sqrt/sin/cos 4), times its algorithmic flops per term",
            "published_fp32_peak": PUBLISHED_FP32_TFLOPS,
            "frac_of_published_fp32_peak": achieved / PUBLISHED_FP32_TFLOPS,
            "slots_per_term": slots,
            "measured_rates_peak": measured_peak,
            "frac_of_measured_rates": achieved / measured_peak,
            "measured_rates_note": "the same loop's ceiling with each instruction class at the rate "
                                   "microbenchmarks reach (full 60.5, half 36.5, transcendental 18.5 T "
                                   "lane-instructions/s, against the nominal 78.6 T full rate)",
            "flops_per_term": flops,
            "traffic": measured_traffic(args.workload),
            "measured": "HIP events around each back-projection launch of the one-frame-in-flight run (the "
                        "same launches as the streamed run, without other frames' kernels beside them)",
            # the same flops per frame over the streamed time per frame, all stages included
            "streamed_frac": contrib * flops / (total / args.steps) / 1e12 / peak,
        },
        "synth_s": t_synth,
    }
    forms_out = {}
    if not args.main_only:
        # the same frame in every precision form: split-phase back-projection
        # (oracle-matching detections) and the matrix-core spectrum forms
        out["precision_forms"] = {"fp32": {"frames_per_s": out["value"], "range_ms": range_ms, "backprojection_ms": bp_ms,
                                           "p99_ms": out["resident_p99_ms"]}}
        for name, prec in (("fp32-split", rc.RC_PREC_FP32_SPLIT), ("fp16-spectrum", rc.RC_PREC_FP16),
                           ("bf16-spectrum", rc.RC_PREC_BF16)):
            sp = time_pipeline(rc, synth, torch, frame, frame.pix, frame.n_rows, frame.n_cols, prec,
                               max(5, args.steps // 2), args.warmup)
            sp1 = time_pipeline(rc, synth, torch, frame, frame.pix, frame.n_rows, frame.n_cols, prec, 10,
                                args.warmup, depth=1)
            out["precision_forms"][name] = {
                "frames_per_s": sp["fps"], "range_ms": float(sp1["stages"][:, 0].mean()),
                "backprojection_ms": float(sp1["stages"][:, 2].mean()),
                "p99_ms": 1e3 * float(np.percentile(sp1["lat"], 99)),
                "vs_fp32_frames_per_s": sp["fps"] / out["value"]}
        for name, prec in (("fp32", rc.RC_PREC_FP32), ("fp32-split", rc.RC_PREC_FP32_SPLIT),
                           ("fp16-spectrum", rc.RC_PREC_FP16), ("bf16-spectrum", rc.RC_PREC_BF16)):
            forms_out[name] = form_outputs(rc, synth, torch, frame, prec)
        progress("precision forms done")
        # the same frame with the double-precision recheck of near-threshold cells
        rk = time_pipeline(rc, synth, torch, frame, frame.pix, frame.n_rows, frame.n_cols, rc.RC_PREC_FP32, 5,
                           args.warmup, depth=1, plan_kw=dict(max_rechecks=4096))
        flags = rk["detections"]["flags"]
        out["fp64_recheck"] = {
            "max_rechecks": 4096, "cfar_margin_rel": 0.03,
            # the double FFT of the frame runs with range compression, the
            # double back-projection of the listed cells with detection
            "range_ms": float(rk["stages"][:, 0].mean()), "range_ms_without": float(stages[:, 0].mean()),
            "detection_ms": float(rk["stages"][:, 3].mean()),
            "detection_ms_without": float(stages[:, 3].mean()),
            "detections": int(len(flags)), "decided_in_fp64": int(((flags & rc.RC_DET_RECHECKED) != 0).sum()),
            "still_near_threshold": int(((flags & rc.RC_DET_NEAR_THRESHOLD) != 0).sum())}
        progress("recheck done")
        out["paper_config"] = paper_config(rc, synth, torch, args.steps, args.warmup)
        progress("paper configuration done")
        out["tab2_ablation"] = ablation(rc, synth, torch)
        progress("Tab. II ablation done")
        drive = make_drive(synth, torch)
        out["continuous_sar"] = continuous_sar(rc, synth, torch, out["value"], drive)
        progress(f"continuous SAR: {out['continuous_sar']['apertures_per_s']:.0f} apertures/s")
        if args.serve_seconds > 0:
            out["continuous_sar"]["serving"] = continuous_serving(
                rc, synth, torch, drive, out["continuous_sar"]["apertures_per_s"], duration_s=args.serve_seconds / 3)
            progress("continuous-SAR serving done")
        del drive
        sensors = make_sensors(rc, synth, torch, 32)
        out["batched_mixed"] = batched_mixed_median(rc, synth, torch, sensors)
        progress(f"batched mixed: {out['batched_mixed']['frames_per_s']:.0f} frames/s")
        if args.serve_seconds > 0:
            out["serving"] = serving_legs(rc, synth, torch, sensors, out["batched_mixed"]["frames_per_s"],
                                          args.serve_seconds)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(frame, args.cpu_budget)
        if forms_out:
            out["errors_vs_oracle"] = oracle_errors(frame, forms_out, args.workload)
            progress("per-stage errors done")
        # the small frame and the paper's configuration, each timed whole
        full = {}
        small = synth.make_frame(synth.CONFIGS["plain-small"], device="cuda")
        t, P = cpu_full_frame(small, small.pix, small.n_rows, small.n_cols)
        full["plain-small"] = {"s_per_frame": t, "processes": P,
                               "terms": float(small.n_rows * small.n_cols) * small.cfg.n_chirps * small.cfg.n_channels}
        pcfg = synth.CONFIGS["paper-polar"]
        pf = synth.make_frame(pcfg, device="cuda")
        q = np.concatenate([pf.q_tx.reshape(-1, 2), pf.q_rx.reshape(-1, 2)])
        g = rc.grid_polar_params(synth.RADAR, pcfg.box, (float(q[:, 0].mean()), float(q[:, 1].mean())),
                                 float(np.ptp(q[:, 0])))
        ppix = rc.grid_polar(g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"])
        t, P = cpu_full_frame(pf, ppix, g["nth"], g["nr"])
        full["paper-polar"] = {"s_per_frame": t, "processes": P,
                               "terms": float(g["nth"] * g["nr"]) * pcfg.n_chirps * pcfg.n_channels}
        out["cpu_baseline"]["full_frames"] = full
        progress("CPU baseline done")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
