"""ctypes binding of librc.so (see include/rc.h).

Argument marshalling only: every step of the SAR pipeline runs in the HIP
kernels of the library.  PyTorch supplies device memory and the stream.  The
library must have been built (``python -m paper_2306_09784_amd.build``);
importing this module without it raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librc.so")

RC_ABI_VERSION = 5

# rc_status
RC_OK, RC_EINVAL, RC_ENOMEM, RC_ETRUNC, RC_EHIP, RC_ENOTREADY, RC_ENOTFOUND = range(7)
STATUS_NAMES = {0: "RC_OK", 1: "RC_EINVAL", 2: "RC_ENOMEM", 3: "RC_ETRUNC", 4: "RC_EHIP",
                5: "RC_ENOTREADY", 6: "RC_ENOTFOUND"}
# rc_window_kind
RC_WIN_RECT, RC_WIN_HANN, RC_WIN_KAISER = 0, 1, 2
WINDOWS = {"rect": RC_WIN_RECT, "hann": RC_WIN_HANN, "kaiser": RC_WIN_KAISER}
# rc_precision
RC_PREC_FP32, RC_PREC_FP32_SPLIT, RC_PREC_FP16, RC_PREC_BF16 = 0, 1, 2, 3
# rc_doppler_mode
RC_DOPPLER_AVERAGE, RC_DOPPLER_EXACT, RC_DOPPLER_EXACT_DIRECT = 0, 1, 2
RC_MEMORY_SLOTS, RC_MEMORY_BUDGET = 0, 1
# rc_input_kind
RC_INPUT_RAW, RC_INPUT_SPECTRUM = 0, 1
# rc_sliding (continuous SAR: sub-apertures of a sensor's chirp stream)
RC_SLIDE_OFF, RC_SLIDE_NEXT, RC_SLIDE_START = 0, 1, 2
RC_DET_NEAR_THRESHOLD = 1
RC_DET_RECHECKED = 2


class rc_radar(C.Structure):
    _fields_ = [("f0", C.c_double), ("bandwidth", C.c_double), ("t_chirp", C.c_double),
                ("c", C.c_double)]


class rc_plan_desc(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32),
        ("radar", rc_radar),
        ("n_samples_max", C.c_int32),
        ("n_fft_max", C.c_int32),
        ("n_bins_max", C.c_int32),
        ("n_chirps_max", C.c_int32),
        ("n_channels_max", C.c_int32),
        ("n_pix_max", C.c_int64),
        ("max_frames_in_flight", C.c_int32),
        ("max_detections", C.c_int32),
        ("range_window", C.c_int),
        ("range_kaiser_beta", C.c_double),
        ("sar_window", C.c_int),
        ("sar_kaiser_beta", C.c_double),
        ("precision", C.c_int),
        ("doppler", C.c_int),
        ("cfar_guard", C.c_int32),
        ("cfar_train", C.c_int32),
        ("cfar_pfa", C.c_double),
        ("cfar_margin_rel", C.c_double),
        ("max_rechecks", C.c_int32),
        ("hbm_budget_bytes", C.c_int64),
        ("stage_timing", C.c_int32),
        ("sliding_sensors", C.c_int32),
        ("sliding_subapertures", C.c_int32),
        ("sliding_depth", C.c_int32),
        ("frame_memory", C.c_int),
    ]


class rc_frame(C.Structure):
    _fields_ = [
        ("frame_id", C.c_int64),
        ("sensor_id", C.c_int32),
        ("n_samples", C.c_int32),
        ("n_fft", C.c_int32),
        ("n_bins", C.c_int32),
        ("n_chirps", C.c_int32),
        ("n_channels", C.c_int32),
        ("fs", C.c_double),
        ("input_kind", C.c_int),
        ("data", C.c_void_p),
        ("q_tx", C.c_void_p),
        ("q_rx", C.c_void_p),
        ("vel", C.c_void_p),
        ("pixels", C.c_void_p),
        ("n_rows", C.c_int32),
        ("n_cols", C.c_int32),
        ("image_out", C.c_void_p),
        ("doppler_out", C.c_void_p),
        ("spectrum_out", C.c_void_p),
        ("height", C.c_double),
        ("sliding", C.c_int),
        ("w_sar", C.c_void_p),
        ("f_doppler", C.c_void_p),
        ("data_host", C.c_void_p),
    ]


class rc_detection(C.Structure):
    _fields_ = [("pixel", C.c_int32), ("power", C.c_float), ("threshold", C.c_float),
                ("flags", C.c_uint32)]


DETECTION_DTYPE = np.dtype([("pixel", "<i4"), ("power", "<f4"), ("threshold", "<f4"),
                            ("flags", "<u4")])


class rc_tuning_entry(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_cols", C.c_int32), ("n_chirps", C.c_int32), ("n_channels", C.c_int32),
                ("chirp_blocks", C.c_int32), ("default_blocks", C.c_int32), ("ms_default", C.c_float),
                ("ms_chosen", C.c_float)]

#: every entry point declared in include/rc.h
ENTRY_POINTS = [
    "rc_plan_create", "rc_plan_slot_bytes", "rc_frame_bytes", "rc_frame_validate", "rc_process_batch", "rc_poll", "rc_detections",
    "rc_image", "rc_stage_times", "rc_frame_release", "rc_plan_destroy", "rc_last_error", "rc_grid_cartesian",
    "rc_grid_polar_params", "rc_grid_polar", "rc_resample_polar", "rc_process_frame_static", "rc_plan_tune",
    "rc_plan_set_tuning",
]


class RcError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    # librc.so needs libamdhip64.so.7.  Load torch first so that the library
    # binds to the HIP runtime torch already uses: one runtime per process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2306_09784_amd.build`")
    lib = C.CDLL(_LIB_PATH)
    i32, i64, vp, dp = C.c_int32, C.c_int64, C.c_void_p, C.POINTER(C.c_double)
    sig = {
        "rc_plan_create": (C.c_int, [C.POINTER(rc_plan_desc), C.POINTER(C.c_void_p)]),
        "rc_plan_slot_bytes": (C.c_int, [C.POINTER(rc_plan_desc), C.POINTER(C.c_int64)]),
        "rc_frame_validate": (C.c_int, [C.POINTER(rc_plan_desc), C.POINTER(rc_frame)]),
        "rc_frame_bytes": (C.c_int, [C.POINTER(rc_plan_desc), C.POINTER(rc_frame), C.POINTER(C.c_int64)]),
        "rc_process_batch": (C.c_int, [vp, C.POINTER(rc_frame), i32, vp]),
        "rc_poll": (C.c_int, [vp, i64]),
        "rc_detections": (C.c_int, [vp, i64, C.POINTER(rc_detection), i64, C.POINTER(C.c_int64)]),
        "rc_image": (C.c_int, [vp, i64, vp, i64, vp]),
        "rc_stage_times": (C.c_int, [vp, i64, C.POINTER(C.c_float)]),
        "rc_frame_release": (C.c_int, [vp, i64]),
        "rc_plan_destroy": (C.c_int, [vp]),
        "rc_last_error": (C.c_char_p, []),
        "rc_grid_cartesian": (C.c_int, [C.c_double, C.c_double, i32, C.c_double, C.c_double, i32, vp]),
        "rc_grid_polar_params": (C.c_int, [C.POINTER(rc_radar), C.c_double, C.c_double, C.c_double,
                                           C.c_double, C.c_double, C.c_double, C.c_double,
                                           C.c_double, dp]),
        "rc_grid_polar": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_double, i32, C.c_double,
                                    C.c_double, i32, vp]),
        "rc_resample_polar": (C.c_int, [vp, i32, i32, C.c_double, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_double, vp, i64, vp, vp]),
        "rc_process_frame_static": (C.c_int, [C.POINTER(rc_plan_desc), C.POINTER(rc_frame), vp, i64, vp, vp]),
        "rc_plan_tune": (C.c_int, [vp, C.POINTER(rc_frame), i32, vp, C.POINTER(rc_tuning_entry), i32,
                                   C.POINTER(C.c_int32)]),
        "rc_plan_set_tuning": (C.c_int, [vp, C.POINTER(rc_tuning_entry), i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    return lib.rc_last_error().decode()


def check(status: int, where: str):
    if status != RC_OK:
        raise RcError(status, where, last_error())


# ---------------------------------------------------------------------------
# Grids (host)
# ---------------------------------------------------------------------------
def grid_cartesian(x0: float, dx: float, nx: int, y0: float, dy: float, ny: int) -> np.ndarray:
    out = np.empty((ny * nx, 2), dtype=np.float32)
    check(lib.rc_grid_cartesian(x0, dx, nx, y0, dy, ny, out.ctypes.data), "rc_grid_cartesian")
    return out


def grid_polar_params(radar: dict, box, origin, aperture_len: float, factor: float = 2.5) -> dict:
    r = rc_radar(radar["f0"], radar["bandwidth"], radar["t_chirp"], radar.get("c", 0.0))
    out = (C.c_double * 6)()
    check(lib.rc_grid_polar_params(C.byref(r), box[0], box[1], box[2], box[3], origin[0], origin[1],
                                   aperture_len, factor, out), "rc_grid_polar_params")
    return {"r0": out[0], "dr": out[1], "th0": out[2], "dth": out[3], "nr": int(out[4]),
            "nth": int(out[5]), "ox": float(origin[0]), "oy": float(origin[1])}


def grid_polar(ox, oy, r0, dr, nr, th0, dth, nth) -> np.ndarray:
    out = np.empty((nth * nr, 2), dtype=np.float32)
    check(lib.rc_grid_polar(ox, oy, r0, dr, nr, th0, dth, nth, out.ctypes.data), "rc_grid_polar")
    return out


def resample_polar(polar_image, g: dict, points, out, stream=None) -> None:
    """rc_resample_polar: |image| on the polar lattice `g` (grid_polar_params
    keys) at device `points` (float32 [n, 2]) into device `out` (float32 [n])."""
    n = int(out.numel()) if hasattr(out, "numel") else int(np.asarray(out).size)
    check(lib.rc_resample_polar(_ptr(polar_image), int(g["nth"]), int(g["nr"]), float(g["ox"]), float(g["oy"]),
                                float(g["r0"]), float(g["dr"]), float(g["th0"]), float(g["dth"]), _ptr(points),
                                n, _ptr(out), _stream_handle(stream)), "rc_resample_polar")


# ---------------------------------------------------------------------------
# Plans
# ---------------------------------------------------------------------------
@dataclass
class PlanConfig:
    radar: dict
    n_samples_max: int
    n_fft_max: int
    n_bins_max: int
    n_chirps_max: int
    n_channels_max: int
    n_pix_max: int
    max_frames_in_flight: int = 2
    max_detections: int = 65536
    range_window: str = "hann"
    range_kaiser_beta: float = 4.0
    sar_window: str = "hann"
    sar_kaiser_beta: float = 4.0
    precision: int = RC_PREC_FP32
    doppler: int = RC_DOPPLER_AVERAGE
    cfar_guard: int = 2
    cfar_train: int = 8
    cfar_pfa: float = 1e-4
    cfar_margin_rel: float = 3e-2
    max_rechecks: int = 0
    hbm_budget_bytes: int = 0
    stage_timing: bool = False
    sliding_sensors: int = 0
    sliding_subapertures: int = 1
    sliding_depth: int = 1
    frame_memory: int = RC_MEMORY_SLOTS

    def desc(self) -> rc_plan_desc:
        r = self.radar
        return rc_plan_desc(
            RC_ABI_VERSION, rc_radar(r["f0"], r["bandwidth"], r["t_chirp"], r.get("c", 0.0)),
            self.n_samples_max, self.n_fft_max, self.n_bins_max, self.n_chirps_max,
            self.n_channels_max, self.n_pix_max, self.max_frames_in_flight, self.max_detections,
            WINDOWS[self.range_window], self.range_kaiser_beta, WINDOWS[self.sar_window],
            self.sar_kaiser_beta, self.precision, self.doppler, self.cfar_guard, self.cfar_train, self.cfar_pfa,
            self.cfar_margin_rel, self.max_rechecks, self.hbm_budget_bytes, int(self.stage_timing),
            self.sliding_sensors, self.sliding_subapertures, self.sliding_depth, self.frame_memory)


def slot_bytes(cfg: PlanConfig) -> int:
    out = C.c_int64()
    d = cfg.desc()
    check(lib.rc_plan_slot_bytes(C.byref(d), C.byref(out)), "rc_plan_slot_bytes")
    return out.value


def validate_frame(cfg: PlanConfig, frame) -> int:
    """rc_frame_validate: the status rc_process_batch would give the frame
    under a plan of this configuration (host only, no GPU)."""
    d = cfg.desc()
    return lib.rc_frame_validate(C.byref(d), C.byref(frame))


def frame_bytes(cfg: PlanConfig, frame) -> int:
    """rc_frame_bytes: the device bytes the frame takes from a RC_MEMORY_BUDGET
    plan of this configuration (host only)."""
    d = cfg.desc()
    out = C.c_int64()
    check(lib.rc_frame_bytes(C.byref(d), C.byref(frame), C.byref(out)), "rc_frame_bytes")
    return out.value


#: device scratch the no-allocation entry point works in (RC_STATIC_SCRATCH_BYTES)
STATIC_SCRATCH_BYTES = 32 << 20


def process_frame_static(cfg: PlanConfig, frame, detections, n_det, stream=None) -> None:
    """rc_process_frame_static: one frame through the pipeline with no
    allocation.  detections: device tensor of DETECTION_DTYPE records (any
    shape, its byte size / 16 is the capacity); n_det: device int64 tensor of
    one element."""
    d = cfg.desc()
    cap = detections.numel() * detections.element_size() // 16 if detections is not None else 0
    check(lib.rc_process_frame_static(C.byref(d), C.byref(frame), _ptr(detections), cap, _ptr(n_det),
                                      _stream_handle(stream)), "rc_process_frame_static")


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


class Plan:
    """Owns an rc plan.  Frames are described by plain dicts/arrays; device
    buffers are torch tensors on the current device."""

    def __init__(self, cfg: PlanConfig):
        self.cfg = cfg
        self._desc = cfg.desc()
        h = C.c_void_p()
        check(lib.rc_plan_create(C.byref(self._desc), C.byref(h)), "rc_plan_create")
        self.handle = h
        self._keep = {}

    def close(self):
        if self.handle:
            check(lib.rc_plan_destroy(self.handle), "rc_plan_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def make_frame(frame_id: int, *, data, q_tx: np.ndarray, q_rx: np.ndarray, vel: np.ndarray,
                   pixels, n_rows: int, n_cols: int, n_bins: int, n_fft: int, fs: float,
                   n_samples: int = 0, input_kind: int = RC_INPUT_RAW, image_out=None,
                   doppler_out=None, spectrum_out=None, sensor_id: int = 0, height: float = 0.0,
                   sliding: int = RC_SLIDE_OFF, w_sar: Optional[np.ndarray] = None,
                   f_doppler=None, data_host=None) -> rc_frame:
        """Builds an rc_frame.  q_tx, q_rx, vel (and w_sar, if given) must be
        C-contiguous float32 host arrays that stay alive until rc_process_batch
        returns; f_doppler is a device tensor of one float per pixel;
        data_host (a pinned host tensor) replaces data in a plan of
        RC_MEMORY_BUDGET (pass data=None)."""
        for a in (q_tx, q_rx, vel) + ((w_sar,) if w_sar is not None else ()):
            if not (isinstance(a, np.ndarray) and a.dtype == np.float32 and a.flags.c_contiguous):
                raise TypeError("q_tx, q_rx, vel and w_sar must be C-contiguous float32 numpy arrays")
        M, CH = q_tx.shape[0], q_tx.shape[1]
        if q_tx.shape != (M, CH, 2) or q_rx.shape != (M, CH, 2) or vel.shape != (M, 2):
            raise ValueError("geometry shapes must be q [M, CH, 2], vel [M, 2]")
        if w_sar is not None and w_sar.shape != (M,):
            raise ValueError("w_sar must have one weight per chirp")
        return rc_frame(frame_id, sensor_id, n_samples, n_fft, n_bins, M, CH, fs, input_kind,
                        _ptr(data), q_tx.ctypes.data, q_rx.ctypes.data, vel.ctypes.data,
                        _ptr(pixels), n_rows, n_cols, _ptr(image_out), _ptr(doppler_out),
                        _ptr(spectrum_out), float(height), int(sliding),
                        w_sar.ctypes.data if w_sar is not None else None, _ptr(f_doppler), _ptr(data_host))

    def process(self, frames, stream=None) -> int:
        arr = (rc_frame * len(frames))(*frames)
        st = lib.rc_process_batch(self.handle, arr, len(frames), _stream_handle(stream))
        if st != RC_OK:
            raise RcError(st, "rc_process_batch", last_error())
        return st

    def try_process(self, frames, stream=None) -> int:
        """Like process() but returns RC_ENOTREADY instead of raising it."""
        arr = (rc_frame * len(frames))(*frames)
        st = lib.rc_process_batch(self.handle, arr, len(frames), _stream_handle(stream))
        if st not in (RC_OK, RC_ENOTREADY):
            raise RcError(st, "rc_process_batch", last_error())
        return st

    def poll(self, frame_id: int) -> bool:
        st = lib.rc_poll(self.handle, frame_id)
        if st == RC_OK:
            return True
        if st == RC_ENOTREADY:
            return False
        raise RcError(st, "rc_poll", last_error())

    def detections(self, frame_id: int, cap: Optional[int] = None) -> np.ndarray:
        if cap is None:
            cap = self.cfg.max_detections
        buf = np.empty(cap, dtype=DETECTION_DTYPE)   # the first n records are written
        n = C.c_int64()
        st = lib.rc_detections(self.handle, frame_id,
                               buf.ctypes.data_as(C.POINTER(rc_detection)), cap, C.byref(n))
        if st not in (RC_OK, RC_ETRUNC):
            raise RcError(st, "rc_detections", last_error())
        if st == RC_ETRUNC:
            raise RcError(st, "rc_detections", last_error())
        return buf[: n.value].copy()

    def image(self, frame_id: int, dst, stream=None):
        check(lib.rc_image(self.handle, frame_id, _ptr(dst), dst.numel(), _stream_handle(stream)),
              "rc_image")

    def stage_times(self, frame_id: int) -> np.ndarray:
        """Device ms of (range compression, tables, back-projection, detection)."""
        out = (C.c_float * 4)()
        check(lib.rc_stage_times(self.handle, frame_id, out), "rc_stage_times")
        return np.array(out[:], dtype=np.float64)

    def release(self, frame_id: int):
        check(lib.rc_frame_release(self.handle, frame_id), "rc_frame_release")

    _TUNING_KEYS = ("n_rows", "n_cols", "n_chirps", "n_channels", "chirp_blocks", "default_blocks", "ms_default",
                    "ms_chosen")

    def tune(self, frames, stream=None) -> list:
        """rc_plan_tune: measures the chirp split of each size class among
        `frames` (rc_frame structs) and installs the fastest; returns one dict
        per class."""
        arr = (rc_frame * len(frames))(*frames)
        cap = max(1, len(frames))
        out = (rc_tuning_entry * cap)()
        n = C.c_int32()
        check(lib.rc_plan_tune(self.handle, arr, len(frames), _stream_handle(stream), out, cap, C.byref(n)),
              "rc_plan_tune")
        return [{k: getattr(out[i], k) for k in self._TUNING_KEYS} for i in range(n.value)]

    def set_tuning(self, entries) -> None:
        """rc_plan_set_tuning: installs a table of dicts with the class keys
        and chirp_blocks (the other keys are ignored); [] clears it."""
        arr = (rc_tuning_entry * max(1, len(entries)))()
        for i, e in enumerate(entries):
            for k in self._TUNING_KEYS[:5]:
                setattr(arr[i], k, int(e[k]))
        check(lib.rc_plan_set_tuning(self.handle, arr, len(entries)), "rc_plan_set_tuning")
