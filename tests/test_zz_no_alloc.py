"""The no-allocation entry point (rc_process_frame_static) against the plan
path (rc_process_batch) on the same frames, through the C ABI: two calls in a
row, the second with a smaller frame; images and detection lists must be
bitwise the same (the same kernels with the same chirp split run in both)."""
import numpy as np
import pytest

from tests import sar_cases as SC

pytestmark = pytest.mark.gpu


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


def _static(rc, torch, cfg, fr, cap=4096):
    dev = torch.device("cuda")
    t = SC.to_device(fr, torch)
    img = torch.full((fr.n_rows * fr.n_cols, 2), float("nan"), dtype=torch.float32, device=dev)
    dets = torch.zeros((cap, 4), dtype=torch.int32, device=dev)
    n_det = torch.full((1,), -1, dtype=torch.int64, device=dev)
    f = rc.Plan.make_frame(7, data=t["raw"], q_tx=fr.q_tx, q_rx=fr.q_rx, vel=fr.vel, pixels=t["pix"],
                           n_rows=fr.n_rows, n_cols=fr.n_cols, n_bins=fr.n_bins, n_fft=fr.n_fft, fs=fr.fs,
                           n_samples=fr.cfg.n_samples, image_out=img, height=fr.cfg.height)
    rc.process_frame_static(cfg, f, dets, n_det, torch.cuda.current_stream())
    torch.cuda.synchronize()
    n = int(n_det.item())
    out = dets.cpu().numpy().view(rc.DETECTION_DTYPE).reshape(-1)[:min(n, cap)]
    return img.cpu().numpy().view(np.complex64).reshape(-1), out, n


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "split"])
def test_static_entry_matches_plan_path(rc, torch, precision):
    big = SC.small_frame(nx=160, ny=144, n_chirps=96)
    small = SC.small_frame(nx=48, ny=40, n_chirps=32, n_samples=128, seed=1007)
    cfg = SC.plan_config(rc, [big, small], precision=precision)
    for fr in (big, small):
        img_s, det_s, n_s = _static(rc, torch, cfg, fr)
        with rc.Plan(cfg) as plan:
            ref = SC.run_gpu(rc, plan, fr, torch)
        assert np.array_equal(img_s.view(np.float32), ref["image"].view(np.float32)), "image differs"
        assert n_s == len(ref["detections"]) and n_s > 0
        assert np.array_equal(det_s, ref["detections"]), "detections differ"
    # the parity bar against the oracle, on the static path's own output
    ora = SC.run_oracle(small, cfar=None)
    rel = np.abs(img_s.astype(np.complex128) - ora["image"]).max() / np.abs(ora["image"]).max()
    assert rel <= (5e-3 if precision == 0 else 2e-4)


def test_static_entry_refuses_what_does_not_fit(rc, torch):
    fr = SC.small_frame(nx=64, ny=64, n_chirps=32)
    cfg = SC.plan_config(rc, [fr], max_rechecks=16)
    with pytest.raises(rc.RcError) as ei:
        _static(rc, torch, cfg, fr)
    assert ei.value.status == rc.RC_EINVAL and "recheck" in rc.last_error()
