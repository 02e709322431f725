"""Host logic of bench.py (CPU only): the issue-slot model behind the ALU
roofline, the rule that measured HBM traffic is reported only for the kernel
sources it was measured on, and the refusal of more than one GPU before any
device work."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("chg", [1, 2, 4, 8, 16])
def test_alg2_cost_model(chg):
    """Flops: 24 per term plus the TX distance (7) shared by chg channels.
    Issue slots: 11 full-rate + 1 half-rate (x2, the index conversion) + 3
    transcendental (x4) per term, plus 4 full-rate + 1 sqrt per TX distance."""
    flops, slots = bench.alg2_cost(chg)
    assert flops == pytest.approx(24.0 + 7.0 / chg)
    assert slots == pytest.approx(11 + 1 * 2 + 3 * 4 + (4 + 4) / chg)
    # the ceiling in TFLOP/s is the lane-instruction rate spread over the slots
    peak = bench.VALU_LANE_OPS / slots * flops / 1e12
    assert peak < 157.3  # below the published FP32 vector peak (FMA = 2 flops)


def test_chg4_ceiling():
    """256 CUs x 128 lanes x 2.4 GHz / 27 slots = 2.91e12 terms/s at chg 4."""
    _, slots = bench.alg2_cost(4)
    assert slots == 27.0
    assert bench.VALU_LANE_OPS / slots == pytest.approx(2.9127e12, rel=1e-4)


@pytest.mark.parametrize("chg", [1, 2, 4, 8, 16])
def test_instruction_classes_match_the_slot_model(chg):
    """The classes count the same instructions as the slot model, and at the
    measured rates (each below its nominal one) the ceiling is lower."""
    c = bench.alg2_classes(chg)
    _, slots = bench.alg2_cost(chg)
    assert c["full"] + bench.HALF_SLOTS * c["half"] + bench.TRANS_SLOTS * c["trans"] == pytest.approx(slots)
    nominal = bench.VALU_LANE_OPS / slots
    assert bench.measured_rate_ceiling(chg) < nominal
    # chg 4: 12 full, 1 half, 3.25 transcendental instructions per term
    if chg == 4:
        t = 12 / 60.5e12 + 1 / 36.5e12 + 3.25 / 18.5e12
        assert bench.measured_rate_ceiling(4) == pytest.approx(1 / t)


def test_traffic_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    """A counter summary counts only for the kernel sources whose hash it
    records: the same sources give its bytes, changed sources give none."""
    fake = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "paper_2306_09784_amd", "csrc"), fake / "paper_2306_09784_amd" / "csrc")
    (fake / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(fake))
    digest = bench._kernel_sources_digest()
    (fake / "profiles" / "bp_kernel_plain-large.traffic.txt").write_text(
        "# counters\nkernel_sources_sha256 %s\nfetch_bytes_per_launch 5.0e+08\n"
        "write_bytes_per_launch 4.0e+07\n" % digest)
    assert bench.measured_traffic("plain-large") == pytest.approx(5.4e8)
    src = fake / "paper_2306_09784_amd" / "csrc" / "bp.hip"
    src.write_text(src.read_text() + "\n// changed\n")
    assert bench.measured_traffic("plain-large") is None
    assert bench.measured_traffic("no-such-workload") is None


def test_committed_traffic_summary_parses():
    """The committed summary names a source hash and both byte counts."""
    with open(os.path.join(ROOT, "profiles", "bp_kernel_plain-large.traffic.txt")) as f:
        kv = dict(line.split(None, 1) for line in f if line.strip() and not line.startswith("#"))
    assert len(kv["kernel_sources_sha256"].strip()) == 64
    assert 1e8 < float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"]) < 1e10


def test_more_than_one_gpu_is_refused():
    """--gpus 2 ends with exit status 2 and a message, before any GPU work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_region_snr_of_a_point_on_a_flat_floor():
    """One target of power 1e4 on a floor of unit power: 40 dB; a second target
    inside the first one's ring is left out of that ring's mean."""
    xs = np.arange(-1.0, 1.0, 0.025)
    X, Y = np.meshgrid(xs, xs)
    pix = np.stack([X.ravel(), Y.ravel()], 1)
    img = np.ones(len(pix), np.complex128)
    k = np.argmin(np.hypot(pix[:, 0], pix[:, 1]))
    img[k] = 100.0
    kw = dict(r_in=0.3, r_out=0.6)
    assert bench._region_snr_db(img, pix, np.array([[0.0, 0.0]]), **kw) == pytest.approx(40.0, abs=1e-9)
    j = np.argmin(np.hypot(pix[:, 0] - 0.45, pix[:, 1]))
    img2 = img.copy()
    img2[j] = 100.0
    snr = bench._region_snr_db(img2, pix, np.array([[0.0, 0.0], [pix[j, 0], pix[j, 1]]]), **kw)
    assert snr == pytest.approx(40.0, abs=1e-9)
