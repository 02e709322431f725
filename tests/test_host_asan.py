"""The host code of librc under AddressSanitizer (CPU only).

The runtime is compiled again with the sanitizer on its host part only (the
device code is unchanged; GPU sanitizers are not used), linked into a
separate library in a temporary directory, and a C driver calls every entry
point that needs no GPU: descriptor validation and slot sizing (with the
recheck and continuous-SAR state on), a frame's validation and its bytes
under an HBM-budget plan, the grid generators, the argument
checks of the batch and resampling calls, and plan creation refused by the
HBM budget before any device call.  Any out-of-bounds access or leak in those
paths fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2306_09784_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include "rc.h"
#define CHECK(cond) do { if (!(cond)) { printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond); return 1; } } while (0)
int main(void) {
  rc_plan_desc d = {0};
  d.abi_version = RC_ABI_VERSION;
  d.radar.f0 = 76.6e9; d.radar.bandwidth = 931e6; d.radar.t_chirp = 102.4e-6;
  d.n_samples_max = 256; d.n_fft_max = 512; d.n_bins_max = 300; d.n_chirps_max = 128; d.n_channels_max = 4;
  d.n_pix_max = 65536; d.max_frames_in_flight = 2; d.max_detections = 100;
  d.range_window = RC_WIN_HANN; d.sar_window = RC_WIN_HANN; d.cfar_guard = 2; d.cfar_train = 8;
  d.cfar_pfa = 1e-4; d.cfar_margin_rel = 0.03; d.max_rechecks = 16;
  d.sliding_sensors = 2; d.sliding_subapertures = 4; d.sliding_depth = 2;
  int64_t b = 0;
  CHECK(rc_plan_slot_bytes(&d, &b) == RC_OK && b > 0);
  d.sliding_subapertures = 0;
  CHECK(rc_plan_slot_bytes(&d, &b) == RC_EINVAL && rc_last_error()[0]);
  d.sliding_subapertures = 4;
  d.sar_window = RC_WIN_KAISER;
  CHECK(rc_plan_slot_bytes(&d, &b) == RC_EINVAL);
  d.sar_window = RC_WIN_HANN;
  float* xy = malloc(sizeof(float) * 2 * 37 * 41);
  CHECK(rc_grid_cartesian(-1, 0.1, 37, 2, 0.1, 41, xy) == RC_OK);
  CHECK(xy[2 * (37 * 41 - 1)] > 2.5f);
  double p6[6];
  CHECK(rc_grid_polar_params(&d.radar, -3, 3, 2, 8, 0, 0, 0.2, 2.5, p6) == RC_OK);
  float* pol = malloc(sizeof(float) * 2 * (size_t)p6[4] * (size_t)p6[5]);
  CHECK(rc_grid_polar(0, 0, p6[0], p6[1], (int)p6[4], p6[2], p6[3], (int)p6[5], pol) == RC_OK);
  CHECK(rc_grid_polar(0, 0, 1, 0.1, 0, 0, 0.1, 3, pol) == RC_EINVAL);
  CHECK(rc_process_batch(NULL, NULL, 0, NULL) == RC_EINVAL);
  CHECK(rc_resample_polar(NULL, 5, 4, 0, 0, 1, 0.1, 0, 0.1, NULL, -1, NULL, NULL) == RC_EINVAL);
  CHECK(rc_resample_polar(NULL, 5, 4, 0, 0, 1, 0.1, 0, 0.1, NULL, 0, NULL, NULL) == RC_OK);
  /* a frame checked and sized on the host: the limits, the bytes an HBM-budget
     plan gives it (more with its cube in pinned host memory), host input
     refused outside budget mode */
  float* q = calloc(8 * 4 * 2, sizeof(float));
  float* vel = calloc(8 * 2, sizeof(float));
  rc_frame f = {0};
  f.frame_id = 1; f.n_samples = 64; f.n_fft = 128; f.n_bins = 40; f.n_chirps = 8; f.n_channels = 4;
  f.fs = 64 / 102.4e-6; f.input_kind = RC_INPUT_RAW; f.data = q; f.q_tx = q; f.q_rx = q; f.vel = vel;
  f.pixels = q; f.n_rows = 10; f.n_cols = 12;
  CHECK(rc_frame_validate(&d, &f) == RC_OK);
  d.frame_memory = RC_MEMORY_BUDGET;
  d.hbm_budget_bytes = (int64_t)1 << 30;
  int64_t b_dev = 0, b_host = 0;
  CHECK(rc_frame_bytes(&d, &f, &b_dev) == RC_OK && b_dev > 0);
  f.data = NULL;
  f.data_host = q;
  CHECK(rc_frame_bytes(&d, &f, &b_host) == RC_OK && b_host > b_dev);
  d.frame_memory = RC_MEMORY_SLOTS;
  CHECK(rc_frame_validate(&d, &f) == RC_EINVAL && rc_last_error()[0]);
  f.n_bins = 0;
  CHECK(rc_frame_bytes(&d, &f, &b_dev) == RC_EINVAL);
  free(q);
  free(vel);
  void* plan = NULL;
  d.hbm_budget_bytes = 1;
  CHECK(rc_plan_create(&d, &plan) == RC_ENOMEM && plan == NULL);
  d.abi_version = 1;
  CHECK(rc_plan_create(&d, &plan) == RC_EINVAL);
  free(xy);
  free(pol);
  printf("ok\n");
  return 0;
}
"""


def _hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("hipcc not available")


def _clang():
    for cand in ("/opt/rocm/llvm/bin/clang", shutil.which("clang")):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("clang not available")


@pytest.mark.slow
def test_host_code_under_address_sanitizer(tmp_path):
    hipcc, clang = _hipcc(), _clang()
    from paper_2306_09784_amd import build

    objs = []
    for src in build.SOURCES:
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        extra = ["-g", "-Xarch_host", "-fsanitize=address"] if src == "runtime.hip" else []
        cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-c", "-I", INCLUDE, "-I", CSRC,
               *DEVICE_FLAGS, *extra, os.path.join(CSRC, src), "-o", obj]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        objs.append(obj)
    lib = str(tmp_path / "librc_asan.so")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                    "-o", lib, *objs], check=True, capture_output=True, text=True)
    drv_c = tmp_path / "drv.c"
    drv_c.write_text(DRIVER)
    drv = str(tmp_path / "drv")
    subprocess.run([clang, "-g", "-fsanitize=address", "-I", INCLUDE, str(drv_c), "-o", drv, lib,
                    f"-Wl,-rpath,{tmp_path}"], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23")
    r = subprocess.run([drv], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0 and "ok" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
