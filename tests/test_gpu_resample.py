"""GPU parity of rc_resample_polar (a polar-grid image shown on Cartesian
points, Sec. III-E / Fig. 3) against the oracle's bilinear magnitude
resampling, on an analytic image and on a back-projected polar image.

The kernel evaluates coordinates, weights and magnitudes in double from the
same complex64 image and rounds the result once to float, so the tolerance is
a few float ulps of the image's largest magnitude."""
import numpy as np
import pytest

import oracle as O
from paper_2306_09784_amd import synth
from tests import sar_cases as SC

pytestmark = pytest.mark.gpu

TOL = 1e-6  # of max |P|


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


def _run(rc, torch, img, g, pts):
    dev = torch.device("cuda")
    d_img = torch.from_numpy(np.ascontiguousarray(img.astype(np.complex64))).to(dev)
    d_pts = torch.from_numpy(np.ascontiguousarray(pts.astype(np.float32))).to(dev)
    out = torch.full((pts.shape[0],), -1.0, dtype=torch.float32, device=dev)
    rc.resample_polar(d_img, g, d_pts, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_resample_analytic_image(rc, torch):
    """|image| = a + b r + c theta + d r theta with a random phase: bilinear
    interpolation reproduces it; points beyond the lattice get 0."""
    g = dict(ox=0.3, oy=-0.2, r0=2.0, dr=0.05, nr=40, th0=-0.6, dth=0.02, nth=50)
    r = g["r0"] + g["dr"] * np.arange(g["nr"])
    th = g["th0"] + g["dth"] * np.arange(g["nth"])
    f = lambda rr, tt: 5.0 + 0.7 * rr + 1.3 * tt + 0.4 * rr * tt  # noqa: E731
    rng = np.random.default_rng(21)
    img = f(r[None, :], th[:, None]) * np.exp(2j * np.pi * rng.random((g["nth"], g["nr"])))
    img = img.astype(np.complex64)
    # a ragged Cartesian lattice covering the polar sector and beyond it
    pts = O.cartesian_grid(-3.0, 0.037, 173, -0.5, 0.041, 131).astype(np.float32)
    out = _run(rc, torch, img, g, pts)
    ref = O.resample_polar(img, g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"],
                           pts.astype(np.float64))
    amax = np.abs(img).max()
    assert np.abs(out - ref).max() <= TOL * amax
    inside = ref > 0
    assert inside.sum() > 1000 and (~inside).sum() > 1000
    assert np.all(out[~inside] == 0.0)
    # against the closed form where the oracle says the point is inside
    p64 = pts.astype(np.float64)
    rr = np.hypot(p64[:, 0] - g["ox"], p64[:, 1] - g["oy"])
    tt = np.arctan2(p64[:, 0] - g["ox"], p64[:, 1] - g["oy"])
    assert np.abs(out[inside] - f(rr[inside], tt[inside])).max() <= 1e-5 * amax


def test_resample_backprojected_polar_image(rc, torch):
    """A frame back-projected on its polar lattice, resampled onto a Cartesian
    grid: equal to the oracle's resampling of the same image."""
    fr = SC.small_frame(nx=16, ny=16, n_chirps=32)
    q = np.concatenate([fr.q_tx.reshape(-1, 2), fr.q_rx.reshape(-1, 2)])
    g = rc.grid_polar_params(synth.RADAR, fr.cfg.box, (float(q[:, 0].mean()), float(q[:, 1].mean())),
                             float(np.ptp(q[:, 0])) + 0.05)
    polar = rc.grid_polar(g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"])
    pf = synth.Frame(**{**fr.__dict__, "pix": polar, "n_rows": g["nth"], "n_cols": g["nr"]})
    with rc.Plan(SC.plan_config(rc, [pf])) as plan:
        img = SC.run_gpu(rc, plan, pf, torch)["image"].reshape(g["nth"], g["nr"])
    pts = O.cartesian_grid(fr.cfg.box[0], 0.05, 301, fr.cfg.box[2], 0.05, 301).astype(np.float32)
    out = _run(rc, torch, img, g, pts)
    ref = O.resample_polar(img, g["ox"], g["oy"], g["r0"], g["dr"], g["nr"], g["th0"], g["dth"], g["nth"],
                           pts.astype(np.float64))
    assert np.abs(out - ref).max() <= TOL * np.abs(img).max()
    assert (ref > 0).mean() > 0.9  # the lattice covers the box


def test_resample_arguments(rc, torch):
    g = dict(ox=0.0, oy=0.0, r0=1.0, dr=0.1, nr=4, th0=-0.1, dth=0.05, nth=5)
    dev = torch.device("cuda")
    img = torch.zeros((5, 4, 2), dtype=torch.float32, device=dev)
    pts = torch.zeros((3, 2), dtype=torch.float32, device=dev)
    out = torch.zeros(3, dtype=torch.float32, device=dev)
    assert rc.lib.rc_resample_polar(img.data_ptr(), 5, 4, 0.0, 0.0, 1.0, 0.1, -0.1, 0.05, pts.data_ptr(), 0,
                                    out.data_ptr(), None) == rc.RC_OK
    for bad in ((img.data_ptr(), 5, 4, 0.0, 0.0, 1.0, 0.0, -0.1, 0.05),     # dr = 0
                (img.data_ptr(), 0, 4, 0.0, 0.0, 1.0, 0.1, -0.1, 0.05),     # nth = 0
                (None, 5, 4, 0.0, 0.0, 1.0, 0.1, -0.1, 0.05),               # no image
                (img.data_ptr(), 5, 4, 0.0, 0.0, 1.0, 0.1, -0.1, float("nan"))):
        assert rc.lib.rc_resample_polar(*bad, pts.data_ptr(), 3, out.data_ptr(), None) == rc.RC_EINVAL
    assert rc.lib.rc_resample_polar(img.data_ptr(), 5, 4, 0.0, 0.0, 1.0, 0.1, -0.1, 0.05, pts.data_ptr(), -1,
                                    out.data_ptr(), None) == rc.RC_EINVAL
    # a single-sample lattice: only its node is inside
    one = torch.tensor([[3.0, 4.0]], dtype=torch.float32, device=dev)
    pts1 = torch.tensor([[0.0, 1.0], [0.0, 1.01]], dtype=torch.float32, device=dev)
    out1 = torch.full((2,), -1.0, dtype=torch.float32, device=dev)
    rc.resample_polar(one, dict(ox=0.0, oy=0.0, r0=1.0, dr=0.1, nr=1, th0=0.0, dth=0.05, nth=1), pts1, out1)
    torch.cuda.synchronize()
    assert out1.cpu().numpy().tolist() == [5.0, 0.0]
