// C-ABI runtime of librc.so: plans, frame slots, host-side geometry
// preparation and the stream-ordered launch sequence of the pipeline
//   range compression -> Doppler table -> back-projection (Alg. 2) -> CA-CFAR
// described in rc.h, and the per-sensor state of continuous SAR (sub-aperture
// partial images in a ring, combined into each aperture).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rc.h"
#include "rc_kernels.hpp"

namespace {

thread_local std::string g_err;

rc_status fail(rc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define RC_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(RC_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),   \
                  __FILE__, __LINE__);                                               \
  } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr int kDetPrefix = 1024;  // detections the compaction writes straight into mapped pinned memory per frame
// longest two-way path, in wavelengths, whose phase the single-precision forms
// hand to the hardware sine and cosine (their argument reduction is verified
// to 2^16 turns)
constexpr double kMaxPathTurns = 65536.0;

// back-projection in the split-phase form: RC_PREC_FP32_SPLIT and the
// reduced-precision spectrum forms
bool split_phase(const rc_plan_desc& d) { return d.precision != RC_PREC_FP32; }
// range compression on the matrix cores (FP16 / BF16 operands)
bool mfma_spectrum(const rc_plan_desc& d) { return d.precision == RC_PREC_FP16 || d.precision == RC_PREC_BF16; }

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) {
  int r = 0;
  while ((int64_t(1) << r) < v) ++r;
  return r;
}

double bessel_i0(double x) {
  // power series sum_k ((x/2)^k / k!)^2, converged to double precision
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= q / ((double)k * k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

template <class T>
void make_window(rc_window_kind kind, double beta, int n, T* out) {
  for (int t = 0; t < n; ++t) {
    double w = 1.0;
    if (n > 1 && kind == RC_WIN_HANN) {
      w = 0.5 - 0.5 * std::cos(2.0 * kPi * t / (n - 1));
    } else if (n > 1 && kind == RC_WIN_KAISER) {
      const double u = 2.0 * t / (n - 1) - 1.0;
      w = bessel_i0(beta * std::sqrt(std::max(0.0, 1.0 - u * u))) / bessel_i0(beta);
    }
    out[t] = (T)w;
  }
}

struct Slot {
  // device
  float4* pairs = nullptr;
  float4* rowgeo = nullptr;   // rowq[rows], grpq[rows], w_sar[n_chirps_max], w_range[n_samples_max]
  float* fd = nullptr;
  float4* pixc = nullptr;
  float* fbase = nullptr;
  float2* partials = nullptr;
  int64_t partial_cap = 0;   // pixels x chirp blocks the partial buffer holds
  float2* image = nullptr;
  unsigned long long* mask = nullptr;
  rc_detection* det_cell = nullptr;
  rc_detection* det_out = nullptr;
  int64_t* det_count = nullptr;
  int* listed = nullptr;      // near-threshold cells for the double-precision recheck
  int* n_listed = nullptr;
  double* rpower = nullptr;   // recomputed powers of the pixels the listed windows need
  unsigned long long* need = nullptr;  // bitmap of those pixels (mask layout)
  int* plist = nullptr;       // those pixels, ascending
  int* pmap = nullptr;        // pixel -> place in plist
  int* n_need = nullptr;
  double2* spec64 = nullptr;  // beat spectrum in double for the recheck
  rc::RecheckArgs rk{};       // geometry part filled by prepare_frame
  // pinned host (staging: mapped and coherent, read by the upload kernel
  // through staging_dev)
  float* staging = nullptr;
  const float4* staging_dev = nullptr;
  int64_t* h_count = nullptr;        // mapped, coherent: the compaction kernel writes
  rc_detection* h_det = nullptr;      // the count and the first records here
  int64_t* h_count_dev = nullptr;     // (their device addresses)
  rc_detection* h_det_dev = nullptr;
  hipEvent_t done = nullptr;
  hipEvent_t stage_ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  // state
  bool busy = false;
  int64_t frame_id = -1;
  int32_t n_rows = 0, n_cols = 0;
  int32_t sensor = -1;        // continuous-SAR sensor of the frame in the slot, or -1
  float2* image_used = nullptr;
  // RC_MEMORY_BUDGET: the frame's share of the plan's arena and, for a frame
  // handed over in pinned host memory, its input copied there
  size_t arena_off = 0, arena_len = 0;
  void* input = nullptr;
};

// A sensor's continuous-SAR stream: sub-aperture b's partial images live in
// ring slot b % n_ring until n_ring newer sub-apertures have replaced them.
struct Sensor {
  bool started = false;
  int64_t next = 0;    // sub-apertures of the current stream so far
  int64_t stored = 0;  // sub-apertures ever stored (a new stream continues the ring)
  int32_t n_chirps = 0, n_channels = 0, n_rows = 0, n_cols = 0;
  const float* pixels = nullptr;
  double height = 0;
  hipEvent_t done = nullptr;  // recorded after the stream's last aperture was formed
  bool recorded = false;
};

// Where one sub-aperture's sums go and which aperture it completes.
struct Slide {
  int32_t sensor = -1;
  int64_t block = 0;   // index of the sub-aperture in its stream
  float2* dst = nullptr;
  int ring_slot = 0;
  int first_slot = 0;  // ring slot of the aperture's oldest sub-aperture
  int n_blk = 1;       // sub-apertures of the aperture present in the stream
};

struct Plan {
  rc_plan_desc d;
  int device = 0;
  // with the recheck on: double twiddles exp(-2 pi i k / n_fft_max) over the
  // half circle (single-precision range compression takes its twiddles from
  // the hardware sine and cosine)
  double2* twiddle64 = nullptr;
  int tw_log2 = 0;
  size_t geo_floats = 0;  // floats of the staging/rowgeo region
  std::vector<Slot> slots;
  // continuous SAR: ring[sensor][n_ring][planes][n_pix_max]
  std::vector<Sensor> sensors;
  float2* ring = nullptr;
  int n_ring = 0, planes = 0;
  int64_t ring_stride = 0;  // complex values per ring slot
  // RC_MEMORY_BUDGET: one device arena, handed out first fit in 256-byte
  // units; free_list maps the offset of each free range to its length
  char* arena = nullptr;
  size_t arena_bytes = 0;
  std::map<size_t, size_t> free_list;
  // inputs handed over in pinned host memory are copied on a stream of their
  // own (default priority), so that a batch's copies overlap the kernels of
  // the batches before it; the batch's stream waits for them by an event
  hipStream_t copy_stream = nullptr;
  hipEvent_t copied = nullptr;
  // a lone frame's input is copied in chirp-block pieces, one event each
  hipEvent_t pieces[16] = {};
  // back-projection's chirp blocks per size class (n_rows, n_cols, n_chirps,
  // n_channels), installed by rc_plan_tune / rc_plan_set_tuning; classes not
  // listed take the rule of rc::bp_chirp_blocks
  std::map<std::array<int32_t, 4>, int> tuned;
};

// First fit from the arena; returns the offset or SIZE_MAX when no free range holds len.
size_t arena_alloc(Plan* p, size_t len) {
  for (auto it = p->free_list.begin(); it != p->free_list.end(); ++it) {
    if (it->second < len) continue;
    const size_t off = it->first, rest = it->second - len;
    p->free_list.erase(it);
    if (rest) p->free_list.emplace(off + len, rest);
    return off;
  }
  return SIZE_MAX;
}

// Returns a range to the arena, merging it with free neighbours.
void arena_free(Plan* p, size_t off, size_t len) {
  if (!len) return;
  auto next = p->free_list.lower_bound(off);
  if (next != p->free_list.end() && off + len == next->first) {
    len += next->second;
    next = p->free_list.erase(next);
  }
  if (next != p->free_list.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += len;
      return;
    }
  }
  p->free_list.emplace(off, len);
}

int sliding_planes(const rc_plan_desc& d) { return d.sar_window == RC_WIN_HANN ? 3 : 1; }
int sliding_ring(const rc_plan_desc& d) { return d.sliding_subapertures + d.sliding_depth - 1; }
size_t ring_bytes(const rc_plan_desc& d) {
  if (d.sliding_sensors <= 0) return 0;
  return (size_t)d.sliding_sensors * sliding_ring(d) * sliding_planes(d) * (size_t)d.n_pix_max * sizeof(float2);
}

struct SlotSizes {
  size_t pairs, geo, fd, pixc, fbase, partials, image, mask, det_cell, det_out, listed, rpower, spec64, need,
      plist, pmap, input = 0;
  size_t total() const {
    return pairs + geo + fd + pixc + fbase + partials + image + mask + det_cell + det_out + listed + rpower +
           spec64 + need + plist + pmap + input + 64;
  }
};

int window_cells(const rc_plan_desc& d) {
  const int w = 2 * (d.cfar_guard + d.cfar_train) + 1;
  return w * w;
}

size_t round_up(size_t v) { return (v + 255) & ~size_t(255); }

// Detection records a frame can produce: at most one per pixel, and the
// plan's max_detections are kept.
int64_t det_capacity(const rc_plan_desc& d, const rc_frame& f) {
  return std::min<int64_t>(d.max_detections, (int64_t)f.n_rows * f.n_cols);
}

// Pixel-blocks of partial images a slot may need: a frame of W waves (64
// lanes each, covering at least its n_pix pixels) is split into
// n_kb = min(16, ceil(T 8192 / W)) chirp blocks (T generations of waves), so
// n_kb * n_pix <= min(16 n_pix, (T 8192 / W + 1) n_pix) <= min(16 n_pix, T 2^19 + n_pix);
// a continuous-SAR sub-aperture has three such images per block (Hann window).
int64_t partial_capacity(const rc_plan_desc& d) {
  const int64_t planes = d.sliding_sensors > 0 && d.sar_window == RC_WIN_HANN ? 3 : 1;
  return planes * std::min<int64_t>(16 * d.n_pix_max, (int64_t)rc::kBpTargetGenerations * (1 << 19) + d.n_pix_max);
}

// staging/device geometry region: rowq[rows] and grpq[rows] float4; with the
// recheck on, the antenna positions in metres (q_tx, q_rx) float4[rows], the
// velocities float2[n_chirps] and the windows in double, w_sar[n_chirps] and
// w_range[n_samples]; then the windows in single precision
size_t recheck_floats(int64_t rows, int64_t n_chirps, int64_t n_samples) {
  return 4 * rows + 2 * n_chirps + 2 * n_chirps + 2 * n_samples;
}
// (a sub-aperture frame has no recheck; its per-row window-phase weights,
// float2[rows], take the place of the recheck's region)
size_t geo_floats(const rc_plan_desc& d) {
  const size_t rows = (size_t)d.n_chirps_max * d.n_channels_max;
  const size_t metres = d.max_rechecks > 0 ? recheck_floats(rows, d.n_chirps_max, d.n_samples_max) : 0;
  const size_t weights = d.sliding_sensors > 0 ? 2 * rows : 0;
  // rounded up to whole 16-byte units for the upload kernel
  return (rows * 8 + std::max(metres, weights) + d.n_chirps_max + d.n_samples_max + 3) & ~size_t(3);
}

SlotSizes slot_sizes(const rc_plan_desc& d) {
  SlotSizes s;
  const size_t rows = (size_t)d.n_chirps_max * d.n_channels_max;
  s.pairs = round_up(rows * d.n_bins_max * sizeof(float4));
  s.geo = round_up(geo_floats(d) * sizeof(float));
  s.fd = round_up((size_t)d.n_pix_max * sizeof(float));
  s.pixc = round_up((size_t)d.n_pix_max * sizeof(float4));
  s.fbase = split_phase(d) ? round_up((size_t)d.n_pix_max * sizeof(float)) : 0;
  s.partials = round_up((size_t)partial_capacity(d) * sizeof(float2));
  s.image = round_up((size_t)d.n_pix_max * sizeof(float2));
  s.mask = round_up((size_t)d.n_pix_max * sizeof(unsigned long long));
  s.det_cell = round_up((size_t)d.n_pix_max * sizeof(rc_detection));
  s.det_out = round_up((size_t)d.max_detections * sizeof(rc_detection));
  s.listed = round_up((size_t)d.max_rechecks * sizeof(int));
  s.rpower = round_up((size_t)d.max_rechecks * window_cells(d) * sizeof(double));
  const bool rk = d.max_rechecks > 0;
  s.need = rk ? round_up((size_t)d.n_pix_max * sizeof(unsigned long long)) : 0;
  s.plist = rk ? round_up((size_t)d.max_rechecks * window_cells(d) * sizeof(int)) : 0;
  s.pmap = rk ? round_up((size_t)d.n_pix_max * sizeof(int)) : 0;
  s.spec64 = d.max_rechecks > 0 ? round_up(rows * d.n_bins_max * sizeof(double2)) : 0;
  return s;
}

// The device bytes of one frame under RC_MEMORY_BUDGET: the buffers of a slot
// sized for this frame (n_kb chirp blocks of `planes` partial images), plus its
// input when it comes from pinned host memory.
SlotSizes frame_sizes(const rc_plan_desc& d, const rc_frame& f, int n_kb, int planes) {
  SlotSizes s;
  const size_t rows = (size_t)f.n_chirps * f.n_channels;
  const size_t n_pix = (size_t)f.n_rows * f.n_cols;
  const size_t n_s = f.input_kind == RC_INPUT_RAW ? (size_t)f.n_samples : 0;
  const bool rk = d.max_rechecks > 0 && f.sliding == RC_SLIDE_OFF;
  const size_t metres = rk ? recheck_floats(rows, f.n_chirps, n_s) : f.sliding != RC_SLIDE_OFF ? 2 * rows : 0;
  s.pairs = round_up(rows * f.n_bins * sizeof(float4));
  s.geo = round_up(((rows * 8 + metres + f.n_chirps + n_s + 3) & ~size_t(3)) * sizeof(float));
  s.fd = round_up(n_pix * sizeof(float));
  s.pixc = round_up(n_pix * sizeof(float4));
  s.fbase = split_phase(d) ? round_up(n_pix * sizeof(float)) : 0;
  s.partials = n_kb > 1 ? round_up((size_t)n_kb * planes * n_pix * sizeof(float2)) : 0;
  s.image = f.image_out ? 0 : round_up(n_pix * sizeof(float2));
  s.mask = round_up(n_pix * sizeof(unsigned long long));
  s.det_cell = round_up(n_pix * sizeof(rc_detection));
  s.det_out = round_up((size_t)det_capacity(d, f) * sizeof(rc_detection));
  s.listed = rk ? round_up((size_t)d.max_rechecks * sizeof(int)) : 0;
  s.rpower = rk ? round_up((size_t)d.max_rechecks * window_cells(d) * sizeof(double)) : 0;
  s.need = rk ? round_up(n_pix * sizeof(unsigned long long)) : 0;
  s.plist = rk ? round_up((size_t)d.max_rechecks * window_cells(d) * sizeof(int)) : 0;
  s.pmap = rk ? round_up(n_pix * sizeof(int)) : 0;
  s.spec64 = rk ? round_up(rows * f.n_bins * sizeof(double2)) : 0;
  s.input = f.data_host ? round_up(rows * (f.input_kind == RC_INPUT_RAW ? (size_t)f.n_samples : (size_t)f.n_bins) *
                                   sizeof(float2))
                        : 0;
  return s;
}

// Points a slot's device buffers into [base, base + sz.total()).
void carve_slot(Slot& s, char* base, const SlotSizes& sz) {
  size_t off = 0;
  auto take = [&](size_t n) -> char* {
    char* q = n ? base + off : nullptr;
    off += n;
    return q;
  };
  s.pairs = reinterpret_cast<float4*>(take(sz.pairs));
  s.rowgeo = reinterpret_cast<float4*>(take(sz.geo));
  s.fd = reinterpret_cast<float*>(take(sz.fd));
  s.pixc = reinterpret_cast<float4*>(take(sz.pixc));
  s.fbase = reinterpret_cast<float*>(take(sz.fbase));
  s.partials = reinterpret_cast<float2*>(take(sz.partials));
  s.image = reinterpret_cast<float2*>(take(sz.image));
  s.mask = reinterpret_cast<unsigned long long*>(take(sz.mask));
  s.det_cell = reinterpret_cast<rc_detection*>(take(sz.det_cell));
  s.det_out = reinterpret_cast<rc_detection*>(take(sz.det_out));
  s.listed = reinterpret_cast<int*>(take(sz.listed));
  s.rpower = reinterpret_cast<double*>(take(sz.rpower));
  s.need = reinterpret_cast<unsigned long long*>(take(sz.need));
  s.plist = reinterpret_cast<int*>(take(sz.plist));
  s.pmap = reinterpret_cast<int*>(take(sz.pmap));
  s.spec64 = reinterpret_cast<double2*>(take(sz.spec64));
  s.input = take(sz.input);
  s.det_count = reinterpret_cast<int64_t*>(take(64));
  s.n_listed = reinterpret_cast<int*>(s.det_count + 1);
  s.n_need = s.n_listed + 1;
}

rc_status validate_desc(const rc_plan_desc* d) {
  if (!d) return fail(RC_EINVAL, "desc is NULL");
  if (d->abi_version != RC_ABI_VERSION)
    return fail(RC_EINVAL, "abi_version %d != %d", d->abi_version, RC_ABI_VERSION);
  if (!(d->radar.f0 > 0) || !(d->radar.bandwidth > 0) || !(d->radar.t_chirp > 0) ||
      d->radar.c < 0)
    return fail(RC_EINVAL, "radar constants must be positive");
  if (d->n_samples_max < 1 || !is_pow2(d->n_fft_max) || d->n_fft_max < 4 || d->n_fft_max > 4096 ||
      d->n_samples_max > d->n_fft_max)
    return fail(RC_EINVAL, "need 1 <= n_samples_max <= n_fft_max, n_fft_max a power of two in [4, 4096]");
  if (d->n_bins_max < 2 || d->n_bins_max > d->n_fft_max)
    return fail(RC_EINVAL, "need 2 <= n_bins_max <= n_fft_max");
  if (d->n_chirps_max < 1 || d->n_channels_max < 1 || d->n_pix_max < 1 ||
      d->n_pix_max > 0x7fffffffLL || (int64_t)d->n_chirps_max * d->n_channels_max >= (1LL << 31))
    return fail(RC_EINVAL, "chirp/channel/pixel limits out of range");
  if (d->max_frames_in_flight < 1 || d->max_frames_in_flight > 1024)
    return fail(RC_EINVAL, "max_frames_in_flight must be in [1, 1024]");
  if (d->max_detections < 1) return fail(RC_EINVAL, "max_detections must be >= 1");
  if (d->cfar_guard < 0 || d->cfar_train < 1 || d->cfar_guard + d->cfar_train > 16)
    return fail(RC_EINVAL, "need guard >= 0, train >= 1, guard + train <= 16");
  if (!(d->cfar_pfa > 0 && d->cfar_pfa < 1)) return fail(RC_EINVAL, "cfar_pfa must be in (0, 1)");
  if (d->cfar_margin_rel < 0) return fail(RC_EINVAL, "cfar_margin_rel must be >= 0");
  if (d->max_rechecks < 0 || d->max_rechecks > (1 << 20))
    return fail(RC_EINVAL, "max_rechecks must be in [0, 2^20]");
  if (d->precision != RC_PREC_FP32 && d->precision != RC_PREC_FP32_SPLIT && d->precision != RC_PREC_FP16 &&
      d->precision != RC_PREC_BF16)
    return fail(RC_EINVAL, "unknown precision %d", (int)d->precision);
  if (d->doppler != RC_DOPPLER_AVERAGE && d->doppler != RC_DOPPLER_EXACT && d->doppler != RC_DOPPLER_EXACT_DIRECT)
    return fail(RC_EINVAL, "unknown Doppler mode %d", (int)d->doppler);
  if (d->doppler != RC_DOPPLER_AVERAGE && d->precision != RC_PREC_FP32)
    return fail(RC_EINVAL, "the exact-Doppler forms are single precision only");
  if (d->frame_memory != RC_MEMORY_SLOTS && d->frame_memory != RC_MEMORY_BUDGET)
    return fail(RC_EINVAL, "unknown frame_memory %d", (int)d->frame_memory);
  if (d->frame_memory == RC_MEMORY_BUDGET && d->hbm_budget_bytes <= 0)
    return fail(RC_EINVAL, "RC_MEMORY_BUDGET needs hbm_budget_bytes > 0");
  if (d->doppler == RC_DOPPLER_EXACT_DIRECT && d->sliding_sensors > 0)
    return fail(RC_EINVAL, "the direct form of Alg. 1 does not form continuous-SAR apertures");
  for (rc_window_kind k : {d->range_window, d->sar_window})
    if (k != RC_WIN_RECT && k != RC_WIN_HANN && k != RC_WIN_KAISER)
      return fail(RC_EINVAL, "unknown window kind %d", (int)k);
  if (d->sliding_sensors < 0 || d->sliding_sensors > 4096)
    return fail(RC_EINVAL, "sliding_sensors must be in [0, 4096]");
  if (d->sliding_sensors > 0) {
    if (d->sliding_subapertures < 1 || d->sliding_subapertures > 64)
      return fail(RC_EINVAL, "sliding_subapertures must be in [1, 64]");
    if (d->sliding_depth < 1 || d->sliding_depth > d->max_frames_in_flight)
      return fail(RC_EINVAL, "sliding_depth must be in [1, max_frames_in_flight]");
    if (d->sar_window == RC_WIN_KAISER)
      return fail(RC_EINVAL, "continuous SAR needs the Hann or rectangular chirp window (a sum of cosines)");
  }
  return RC_OK;
}

void free_slot(Slot& s, bool owns_device) {
  if (owns_device && s.pairs) (void)hipFree(s.pairs);
  if (s.staging) (void)hipHostFree(s.staging);
  if (s.h_count) (void)hipHostFree(s.h_count);
  if (s.done) (void)hipEventDestroy(s.done);
  for (hipEvent_t& e : s.stage_ev)
    if (e) (void)hipEventDestroy(e);
  s = Slot();
}

void free_plan(Plan* p) {
  if (!p) return;
  for (Slot& s : p->slots) free_slot(s, !p->arena);
  if (p->copy_stream) (void)hipStreamSynchronize(p->copy_stream);
  if (p->arena) (void)hipFree(p->arena);
  if (p->copied) (void)hipEventDestroy(p->copied);
  for (hipEvent_t& e : p->pieces)
    if (e) (void)hipEventDestroy(e);
  if (p->copy_stream) (void)hipStreamDestroy(p->copy_stream);
  for (Sensor& s : p->sensors)
    if (s.done) (void)hipEventDestroy(s.done);
  if (p->ring) (void)hipFree(p->ring);
  if (p->twiddle64) (void)hipFree(p->twiddle64);
  delete p;
}

// Chirp blocks of a frame's back-projection; a sub-aperture's partial images
// have `planes` planes each and must fit the slot's partial buffer.
std::array<int32_t, 4> size_class(const rc_frame& f) { return {f.n_rows, f.n_cols, f.n_chirps, f.n_channels}; }

int frame_chirp_blocks(const Plan* p, const rc_frame& f) {
  if (f.sliding == RC_SLIDE_OFF && !p->tuned.empty()) {
    const auto it = p->tuned.find(size_class(f));
    if (it != p->tuned.end()) return it->second;
  }
  const int planes = f.sliding != RC_SLIDE_OFF ? p->planes : 1;
  int n_kb = rc::bp_chirp_blocks(f.n_rows, f.n_cols, f.n_chirps, f.n_channels, planes);
  if (f.sliding != RC_SLIDE_OFF && n_kb > 1) {
    const int64_t per = (int64_t)planes * f.n_rows * f.n_cols;
    const int64_t fit = partial_capacity(p->d) / per;
    if (fit < n_kb) n_kb = fit < 2 ? 1 : (int)fit;
  }
  return n_kb;
}

Slot* find_slot(Plan* p, int64_t id) {
  for (Slot& s : p->slots)
    if (s.busy && s.frame_id == id) return &s;
  return nullptr;
}

rc_status validate_frame(const Plan* p, const rc_frame& f) {
  const rc_plan_desc& d = p->d;
  if (f.n_chirps < 1 || f.n_chirps > d.n_chirps_max)
    return fail(RC_EINVAL, "frame %lld: n_chirps %d outside [1, %d]", (long long)f.frame_id, f.n_chirps, d.n_chirps_max);
  if (f.n_channels < 1 || f.n_channels > d.n_channels_max)
    return fail(RC_EINVAL, "frame %lld: n_channels %d outside [1, %d]", (long long)f.frame_id, f.n_channels, d.n_channels_max);
  if (f.n_bins < 2 || f.n_bins > d.n_bins_max)
    return fail(RC_EINVAL, "frame %lld: n_bins %d outside [2, %d]", (long long)f.frame_id, f.n_bins, d.n_bins_max);
  if (f.n_rows < 1 || f.n_cols < 1 || (int64_t)f.n_rows * f.n_cols > d.n_pix_max)
    return fail(RC_EINVAL, "frame %lld: lattice %d x %d outside n_pix_max %lld", (long long)f.frame_id, f.n_rows, f.n_cols, (long long)d.n_pix_max);
  if (f.n_rows > 65535 * 16)
    return fail(RC_EINVAL, "frame %lld: n_rows %d too large", (long long)f.frame_id, f.n_rows);
  if (!(f.fs > 0)) return fail(RC_EINVAL, "frame %lld: fs must be positive", (long long)f.frame_id);
  if (!std::isfinite(f.height)) return fail(RC_EINVAL, "frame %lld: height must be finite", (long long)f.frame_id);
  if (!(f.data || f.data_host) || !f.q_tx || !f.q_rx || !f.vel || !f.pixels)
    return fail(RC_EINVAL, "frame %lld: data, q_tx, q_rx, vel and pixels are required", (long long)f.frame_id);
  if (f.data_host && (f.data || d.frame_memory != RC_MEMORY_BUDGET))
    return fail(RC_EINVAL, "frame %lld: data_host (with data NULL) needs a RC_MEMORY_BUDGET plan",
                (long long)f.frame_id);
  const int64_t rows = (int64_t)f.n_chirps * f.n_channels;
  for (int64_t i = 0; i < 2 * rows; ++i)
    if (!std::isfinite(f.q_tx[i]) || !std::isfinite(f.q_rx[i]))
      return fail(RC_EINVAL, "frame %lld: non-finite antenna position", (long long)f.frame_id);
  for (int64_t i = 0; i < 2 * (int64_t)f.n_chirps; ++i)
    if (!std::isfinite(f.vel[i]))
      return fail(RC_EINVAL, "frame %lld: non-finite velocity", (long long)f.frame_id);
  if (f.w_sar) {
    if (f.sliding != RC_SLIDE_OFF)
      return fail(RC_EINVAL, "frame %lld: a sub-aperture takes the plan's window (it spans the aperture)",
                  (long long)f.frame_id);
    for (int m = 0; m < f.n_chirps; ++m)
      if (!std::isfinite(f.w_sar[m]))
        return fail(RC_EINVAL, "frame %lld: non-finite w_sar", (long long)f.frame_id);
  }
  if (f.f_doppler && d.doppler != RC_DOPPLER_AVERAGE)
    return fail(RC_EINVAL, "frame %lld: f_doppler with RC_DOPPLER_EXACT (Alg. 1 has no Doppler table)",
                (long long)f.frame_id);
  if (f.sliding != RC_SLIDE_OFF) {
    if (f.sliding != RC_SLIDE_NEXT && f.sliding != RC_SLIDE_START)
      return fail(RC_EINVAL, "frame %lld: unknown sliding mode %d", (long long)f.frame_id, (int)f.sliding);
    if (d.sliding_sensors <= 0)
      return fail(RC_EINVAL, "frame %lld: the plan has no continuous-SAR sensors", (long long)f.frame_id);
    if (f.sensor_id < 0 || f.sensor_id >= d.sliding_sensors)
      return fail(RC_EINVAL, "frame %lld: sensor %d outside [0, %d)", (long long)f.frame_id, f.sensor_id, d.sliding_sensors);
  }
  const int n_kb = frame_chirp_blocks(p, f);
  const int planes = f.sliding != RC_SLIDE_OFF ? p->planes : 1;
  if (n_kb > 1 && (int64_t)n_kb * planes * f.n_rows * f.n_cols > partial_capacity(d))
    return fail(RC_EINVAL, "frame %lld: %d chirp blocks exceed the partial-image buffer", (long long)f.frame_id, n_kb);
  if (f.input_kind == RC_INPUT_RAW) {
    if (f.n_samples < 1 || f.n_samples > d.n_samples_max)
      return fail(RC_EINVAL, "frame %lld: n_samples %d outside [1, %d]", (long long)f.frame_id, f.n_samples, d.n_samples_max);
    if (!is_pow2(f.n_fft) || f.n_fft < 4 || f.n_fft > d.n_fft_max || f.n_fft < f.n_samples)
      return fail(RC_EINVAL, "frame %lld: n_fft %d must be a power of two in [max(4, n_samples), %d]", (long long)f.frame_id, f.n_fft, d.n_fft_max);
    if (f.n_bins > f.n_fft)
      return fail(RC_EINVAL, "frame %lld: n_bins %d > n_fft %d", (long long)f.frame_id, f.n_bins, f.n_fft);
    if (mfma_spectrum(d) && !rc::range_mfma_supported(f.n_fft, f.n_samples))
      return fail(RC_EINVAL,
                  "frame %lld: the matrix-core spectrum takes DFT lengths %d..%d with n_samples <= n_fft / 2 "
                  "(n_fft %d, n_samples %d)", (long long)f.frame_id, rc::kRangeMfmaMinFft, rc::kRangeMfmaMaxFft,
                  f.n_fft, f.n_samples);
  } else if (f.input_kind == RC_INPUT_SPECTRUM) {
    if (f.n_fft < f.n_bins || f.n_fft < 1)
      return fail(RC_EINVAL, "frame %lld: n_fft %d must be >= n_bins (it defines the bin spacing)", (long long)f.frame_id, f.n_fft);
    if (f.spectrum_out)
      return fail(RC_EINVAL, "frame %lld: spectrum_out needs RAW input", (long long)f.frame_id);
  } else {
    return fail(RC_EINVAL, "frame %lld: unknown input_kind %d", (long long)f.frame_id, (int)f.input_kind);
  }
  // The single-precision forms feed a term's whole two-way path, in
  // wavelengths, to the hardware sine and cosine (Alg. 2's exp(a2 d_hyp)).
  // Their argument reduction is verified up to kMaxPathTurns turns, and the
  // path's float rounding stays below 1e-3 turns there.  A term contributes
  // only while its index a1 d_hyp + f_doppler lies in [0, n_bins - 1], so
  // every contributing path is at most (n_bins - 1 + F) / a1 long, F bounding
  // -f_doppler: twice kd |v| for the plan's own table and for Alg. 1, and
  // n_bins - 1 for a caller's table (the documented bound on its values).
  // Longer paths need the split-phase form, whose phase never holds the
  // whole path.
  if (!split_phase(d)) {
    const double c = d.radar.c > 0 ? d.radar.c : 299792458.0;
    const double df = f.fs / f.n_fft;
    const double a1 = d.radar.bandwidth / d.radar.t_chirp / (c * df);  // bins per metre of path
    double vmax = 0;
    for (int m = 0; m < f.n_chirps; ++m) vmax = std::max(vmax, std::hypot((double)f.vel[2 * m], (double)f.vel[2 * m + 1]));
    const double F = f.f_doppler ? (double)(f.n_bins - 1) : 2.0 * d.radar.f0 / (c * df) * vmax;
    const double turns = (f.n_bins - 1 + F) / a1 * d.radar.f0 / c;
    if (!(turns <= kMaxPathTurns))
      return fail(RC_EINVAL,
                  "frame %lld: paths up to %.0f wavelengths can contribute, beyond the %.0f the single-precision "
                  "phase supports; use RC_PREC_FP32_SPLIT",
                  (long long)f.frame_id, turns, kMaxPathTurns);
  }
  return RC_OK;
}

// Largest channel-group size (16, 8, 4, 2 or 1) dividing n_ch whose channels
// share the TX position in every chirp.
int tx_group(const rc_frame& f) {
  for (int g : {16, 8, 4, 2}) {
    if (f.n_channels % g) continue;
    bool ok = true;
    for (int64_t m = 0; m < f.n_chirps && ok; ++m)
      for (int c0 = 0; c0 < f.n_channels && ok; c0 += g)
        for (int j = 1; j < g && ok; ++j) {
          const float* a = f.q_tx + ((m * f.n_channels) + c0) * 2;
          const float* b = f.q_tx + ((m * f.n_channels) + c0 + j) * 2;
          ok = a[0] == b[0] && a[1] == b[1];
        }
    if (ok) return g;
  }
  return 1;
}

// What a frame contributes to the batch-wide launches.
struct Prepared {
  rc::UploadArgs up{};
  bool recheck = false;
  rc::Range64Args r6{};
  bool raw_in = true;
  rc::RangeArgs ra{};
  rc::PairArgs pa{};
  rc::TableArgs ta{};
  rc::BpFrame bf{};
  int chg = 1;
  int sums = 1;  // 3: a continuous-SAR sub-aperture under the Hann window
};

// Host part of a frame: geometry in local units through pinned staging (and,
// with the recheck on, the double-precision spectrum), and the argument
// blocks of its range compression, pixel tables and back-projection, which
// the batch launches for many frames at once.  A continuous-SAR sub-aperture
// (sl != nullptr) has an unwindowed table, per-row window-phase weights and
// writes its sums to its ring slot.
rc_status prepare_frame(Plan* p, Slot& s, const rc_frame& f, const Slide* sl, hipStream_t st, Prepared* out) {
  const rc_plan_desc& d = p->d;
  const double c = d.radar.c > 0 ? d.radar.c : 299792458.0;
  const double mu = d.radar.bandwidth / d.radar.t_chirp;
  const double df = f.fs / f.n_fft;
  const double a1 = mu / (c * df);
  const double kd = d.radar.f0 / (c * df);
  const int64_t rows = (int64_t)f.n_chirps * f.n_channels;
  const int64_t n_pix = (int64_t)f.n_rows * f.n_cols;

  // geometry in aperture-local wavelength units (origin: mean of all antenna
  // positions) as per-row uniforms (-2 q, |q|^2) for the RX of every (m, ch)
  // and the TX of every channel group; means and bounding boxes on the way
  const int chg = tx_group(f);
  double st_x = 0, st_y = 0, sr_x = 0, sr_y = 0;
  for (int64_t r = 0; r < rows; ++r) {
    const double tx = f.q_tx[2 * r], ty = f.q_tx[2 * r + 1];
    const double rx = f.q_rx[2 * r], ry = f.q_rx[2 * r + 1];
    st_x += tx; st_y += ty; sr_x += rx; sr_y += ry;
  }
  const double cen_x = (st_x + sr_x) / (2.0 * rows), cen_y = (st_y + sr_y) / (2.0 * rows);
  const double lam = c / d.radar.f0, inv_lam = d.radar.f0 / c;
  float tlx = INFINITY, tly = INFINITY, thx = -INFINITY, thy = -INFINITY;
  float rlx = INFINITY, rly = INFINITY, rhx = -INFINITY, rhy = -INFINITY;
  float* g = s.staging;
  float4* rowq = reinterpret_cast<float4*>(g);
  float4* grpq = rowq + rows;
  auto local = [&](const float* q, float& x, float& y) {
    x = (float)((q[0] - cen_x) * inv_lam);
    y = (float)((q[1] - cen_y) * inv_lam);
  };
  const bool exact = d.doppler == RC_DOPPLER_EXACT || d.doppler == RC_DOPPLER_EXACT_DIRECT;
  const bool direct = d.doppler == RC_DOPPLER_EXACT_DIRECT;
  double vmax = 0;
  double q_max = 0;  // largest antenna distance from the aperture centre, wavelengths
  for (int64_t r = 0; r < rows; ++r) {
    float x, y;
    // exact form: positions and kd v(m) (bins per unit radial speed)
    const int64_t m = r / f.n_channels;
    // the direct form keeps metres and m/s (Alg. 1 as stated)
    const double vs = direct ? 1.0 : kd;
    const float kvx = (float)(vs * f.vel[2 * m]), kvy = (float)(vs * f.vel[2 * m + 1]);
    local(f.q_rx + 2 * r, x, y);
    rowq[r] = direct  ? make_float4((float)(f.q_rx[2 * r] - cen_x), (float)(f.q_rx[2 * r + 1] - cen_y), kvx, kvy)
              : exact ? make_float4(x, y, kvx, kvy)
                      : make_float4(-2.f * x, -2.f * y, (float)((double)x * x + (double)y * y), 0.f);
    rlx = std::min(rlx, x); rly = std::min(rly, y); rhx = std::max(rhx, x); rhy = std::max(rhy, y);
    q_max = std::max(q_max, std::hypot((double)x, (double)y));
    local(f.q_tx + 2 * r, x, y);
    q_max = std::max(q_max, std::hypot((double)x, (double)y));
    if (r % chg == 0)
      grpq[r / chg] = direct ? make_float4((float)(f.q_tx[2 * r] - cen_x), (float)(f.q_tx[2 * r + 1] - cen_y), kvx, kvy)
                      : exact ? make_float4(x, y, kvx, kvy)
                              : make_float4(-2.f * x, -2.f * y, (float)((double)x * x + (double)y * y), 0.f);
    tlx = std::min(tlx, x); tly = std::min(tly, y); thx = std::max(thx, x); thy = std::max(thy, y);
    vmax = std::max(vmax, std::hypot((double)f.vel[2 * m], (double)f.vel[2 * m + 1]));
  }
  double vx = 0, vy = 0;
  for (int m = 0; m < f.n_chirps; ++m) {
    vx += f.vel[2 * m];
    vy += f.vel[2 * m + 1];
  }
  vx /= f.n_chirps;
  vy /= f.n_chirps;
  const bool recheck = d.max_rechecks > 0 && !sl;
  const int n_s = f.input_kind == RC_INPUT_RAW ? f.n_samples : 0;
  // the recheck's geometry or a sub-aperture's window-phase weights
  const int64_t metres = recheck ? (int64_t)recheck_floats(rows, f.n_chirps, n_s) : sl ? 2 * rows : 0;
  float4* geo_m = rowq + 2 * rows;
  float2* vel_m = reinterpret_cast<float2*>(geo_m + rows);
  double* w_sar64 = reinterpret_cast<double*>(vel_m + f.n_chirps);
  double* w_range64 = w_sar64 + f.n_chirps;
  if (recheck) {
    for (int64_t r = 0; r < rows; ++r)
      geo_m[r] = make_float4(f.q_tx[2 * r], f.q_tx[2 * r + 1], f.q_rx[2 * r], f.q_rx[2 * r + 1]);
    for (int m = 0; m < f.n_chirps; ++m) vel_m[m] = make_float2(f.vel[2 * m], f.vel[2 * m + 1]);
    if (f.w_sar)
      for (int m = 0; m < f.n_chirps; ++m) w_sar64[m] = f.w_sar[m];
    else
      make_window(d.sar_window, d.sar_kaiser_beta, f.n_chirps, w_sar64);
    make_window(d.range_window, d.range_kaiser_beta, n_s, w_range64);
  }
  if (sl) {
    // chirp m of sub-aperture b is chirp b S + m of the stream; its window
    // phase is 2 pi ((b S + m) mod (N - 1)) / (N - 1), N = K S (exact in integers)
    float2* roww = reinterpret_cast<float2*>(geo_m);
    const int64_t period = (int64_t)d.sliding_subapertures * f.n_chirps - 1;
    for (int m = 0; m < f.n_chirps; ++m) {
      float2 w = make_float2(1.f, 0.f);
      if (period > 0) {
        const double th = 2.0 * kPi * (double)((sl->block * f.n_chirps + m) % period) / (double)period;
        w = make_float2((float)std::cos(th), (float)std::sin(th));
      }
      roww[m] = w;
    }
  }
  float* w_sar = g + 8 * rows + metres;
  // a sub-aperture's table is unwindowed: the window enters when the
  // aperture is formed from the sums
  if (f.w_sar)
    std::memcpy(w_sar, f.w_sar, (size_t)f.n_chirps * sizeof(float));
  else
    make_window(sl ? RC_WIN_RECT : d.sar_window, d.sar_kaiser_beta, f.n_chirps, w_sar);
  float* w_range = w_sar + f.n_chirps;
  make_window(d.range_window, d.range_kaiser_beta, n_s, w_range);
  const size_t geo_bytes = (size_t)(8 * rows + metres + f.n_chirps + n_s) * sizeof(float);
  out->up = rc::UploadArgs{s.rowgeo, s.staging_dev, (int64_t)((geo_bytes + 15) / 16)};
  const float4* d_rowq = s.rowgeo;
  const float4* d_grpq = s.rowgeo + rows;
  const float* d_wsar = reinterpret_cast<const float*>(s.rowgeo) + 8 * rows + metres;
  const float* d_wrange = d_wsar + f.n_chirps;

  // 1. beat spectrum -> interpolation table (launched batch-wide)
  out->raw_in = f.input_kind == RC_INPUT_RAW;
  if (out->raw_in) {
    rc::RangeArgs& ra = out->ra;
    ra.raw = static_cast<const float2*>(f.data);
    ra.w_range = d_wrange;
    ra.w_sar = d_wsar;
    ra.pairs = s.pairs;
    ra.spectrum = static_cast<float2*>(f.spectrum_out);
    ra.rows = rows;
    ra.n_s = f.n_samples;
    ra.n_fft = f.n_fft;
    ra.log2n = ilog2(f.n_fft);
    ra.n_bins = f.n_bins;
    ra.n_ch = f.n_channels;
  } else {
    out->pa = rc::PairArgs{static_cast<const float2*>(f.data), d_wsar, s.pairs, rows, f.n_bins, f.n_channels};
  }

  if (recheck) {
    // the recheck's beat spectrum in double (same input, double arithmetic);
    // the double windows follow the velocities in the geometry region
    const double* d_wsar64 = reinterpret_cast<const double*>(reinterpret_cast<const float2*>(s.rowgeo + 3 * rows) + f.n_chirps);
    const bool raw_in = f.input_kind == RC_INPUT_RAW;
    rc::Range64Args r6{};
    r6.raw = raw_in ? static_cast<const float2*>(f.data) : nullptr;
    r6.spectrum_in = raw_in ? nullptr : static_cast<const float2*>(f.data);
    r6.w_range = d_wsar64 + f.n_chirps;
    r6.twiddle = p->twiddle64;
    r6.tw_log2 = p->tw_log2;
    r6.spec = s.spec64;
    r6.rows = rows;
    r6.n_s = n_s;
    r6.n_fft = raw_in ? f.n_fft : 0;
    r6.log2n = raw_in ? ilog2(f.n_fft) : 0;
    r6.n_bins = f.n_bins;
    out->recheck = true;
    out->r6 = r6;
  }

  // 2. per-frame tables: Doppler (Sec. III-D) and local pixel coordinates
  const float2* pix = reinterpret_cast<const float2*>(f.pixels);
  rc::TableArgs& ta = out->ta;
  ta.pix = pix;
  ta.n_pix = n_pix;
  ta.qt_x = st_x / rows; ta.qt_y = st_y / rows;
  ta.qr_x = sr_x / rows; ta.qr_y = sr_y / rows;
  ta.v_x = vx; ta.v_y = vy;
  ta.kd = kd;
  ta.c_x = cen_x; ta.c_y = cen_y;
  ta.inv_lam = inv_lam;
  ta.fd = s.fd;
  ta.pixc = s.pixc;
  ta.split = split_phase(d);
  ta.exact = direct ? 2 : exact ? 1 : 0;
  ta.a1 = a1 * lam;
  ta.fbase = s.fbase;
  ta.height = f.height;
  ta.fd_in = f.f_doppler;

  // back-projection descriptor (Alg. 2), launched batch-wide by the caller
  float2* img = f.image_out ? static_cast<float2*>(f.image_out) : s.image;
  const int n_kb = frame_chirp_blocks(p, f);
  const int planes = sl ? p->planes : 1;
  rc::BpFrame& ba = out->bf;
  ba = rc::BpFrame{};
  ba.pixc = s.pixc;
  ba.fidx = split_phase(d) ? s.fbase : s.fd;
  ba.pairs = s.pairs;
  ba.rowq = exact ? nullptr : d_rowq;
  ba.grpq = exact ? nullptr : d_grpq;
  ba.rowv = exact ? d_rowq : nullptr;
  ba.grpv = exact ? d_grpq : nullptr;
  // each leg's Doppler index shift is at most kd |v|
  ba.f_slack = exact ? (float)(2.0 * kd * vmax * (1.0 + 1e-6)) : 0.f;
  ba.roww = sl && planes == 3 ? reinterpret_cast<const float2*>(s.rowgeo + 2 * rows) : nullptr;
  ba.out = n_kb > 1 ? s.partials : sl ? sl->dst : img;
  ba.n_chirps = f.n_chirps;
  ba.n_ch = f.n_channels;
  ba.n_bins = f.n_bins;
  ba.n_rows = f.n_rows;
  ba.n_cols = f.n_cols;
  ba.n_kb = n_kb;
  ba.kb0 = 0;
  ba.kb_count = n_kb;
  rc::bp_tiles(f.n_rows, f.n_cols, &ba.tiles_x, &ba.n_tiles);
  ba.a1 = (float)(a1 * lam);
  ba.tx_lo_x = tlx; ba.tx_lo_y = tly; ba.tx_hi_x = thx; ba.tx_hi_y = thy;
  ba.rx_lo_x = rlx; ba.rx_lo_y = rly; ba.rx_hi_x = rhx; ba.rx_hi_y = rhy;
  // single-precision error of an index a1 d_hyp + f_doppler <= n_bins is a few
  // ulps of n_bins; the margin keeps such waves on the range-tested path
  ba.f_margin = (float)(1e-3 + 64.0 * f.n_bins * std::ldexp(1.0, -24));
  ba.h2 = (float)(f.height * inv_lam * f.height * inv_lam);
  ba.q_max = (float)(q_max * (1.0 + 1e-6));
  ba.lit_c = (float)c;
  ba.lit_mu = (float)mu;
  ba.lit_f0 = (float)d.radar.f0;
  ba.lit_df = (float)df;
  if (n_kb > 1 && (int64_t)n_kb * planes * n_pix > s.partial_cap)
    return fail(RC_EINVAL, "frame %lld: %d chirp blocks of %lld pixels exceed the slot's partial buffer",
                (long long)f.frame_id, n_kb, (long long)n_pix);
  // geometry of the double-precision recheck (metres, Alg. 2 or Alg. 1)
  rc::RecheckArgs& rk = s.rk;
  rk = rc::RecheckArgs{};
  if (recheck) {
    rk.pix = pix;
    rk.geo = s.rowgeo + 2 * rows;
    rk.vel = reinterpret_cast<const float2*>(s.rowgeo + 3 * rows);
    rk.spec = s.spec64;
    rk.w_sar = reinterpret_cast<const double*>(rk.vel + f.n_chirps);
    rk.n_chirps = f.n_chirps;
    rk.n_ch = f.n_channels;
    rk.n_bins = f.n_bins;
    rk.exact = exact;
    rk.a1 = a1;
    rk.kd = kd;
    rk.inv_lam = inv_lam;
    rk.qt_x = ta.qt_x; rk.qt_y = ta.qt_y;
    rk.qr_x = ta.qr_x; rk.qr_y = ta.qr_y;
    rk.v_x = vx; rk.v_y = vy;
    rk.height = f.height;
    rk.fd_in = f.f_doppler;
  }
  out->chg = chg;
  out->sums = planes;
  s.busy = true;
  s.frame_id = f.frame_id;
  s.n_rows = f.n_rows;
  s.n_cols = f.n_cols;
  s.sensor = sl ? sl->sensor : -1;
  s.image_used = img;
  return RC_OK;
}

// Step 4 of a batch: CA-CFAR of every frame, the double-precision recheck of
// near-threshold cells (if on), ordered compaction, then per frame the
// asynchronous read-back and its completion event.
rc_status finish_batch(Plan* p, const std::vector<Slot*>& slot, const rc_frame* frames, int n, hipStream_t st) {
  const rc_plan_desc& d = p->d;
  const bool timed = d.stage_timing != 0;
  const int h = d.cfar_guard + d.cfar_train;
  const int n_train = (2 * h + 1) * (2 * h + 1) - (2 * d.cfar_guard + 1) * (2 * d.cfar_guard + 1);
  const double alpha = n_train * (std::pow(d.cfar_pfa, -1.0 / n_train) - 1.0);
  // continuous-SAR apertures are not rechecked (their sub-apertures' spectra
  // are gone by the time a cell is listed)
  auto rechecked = [&](int i) { return d.max_rechecks > 0 && frames[i].sliding == RC_SLIDE_OFF; };
  auto wpr = [&](int i) { return (frames[i].n_cols + 63) / 64; };
  for (int i = 0; i < n; ++i)
    if (rechecked(i)) RC_HIP(rc::launch_clear_count(slot[i]->n_listed, st));
  for (int i0 = 0; i0 < n; i0 += rc::CfarMulti::kMax) {
    rc::CfarMulti m;
    for (int i = i0; i < n && m.n_frames < rc::CfarMulti::kMax; ++i) {
      Slot& s = *slot[i];
      m.f[m.n_frames++] = rc::CfarArgs{s.image_used, frames[i].n_rows, frames[i].n_cols, d.cfar_guard,
                                       d.cfar_train, alpha / n_train, d.cfar_margin_rel, s.mask, wpr(i),
                                       s.det_cell, s.listed, s.n_listed, rechecked(i) ? d.max_rechecks : 0};
    }
    RC_HIP(rc::launch_cfar(m, st));
  }
  {
    for (int i = 0; i < n; ++i) {
      if (!rechecked(i)) continue;
      Slot& s = *slot[i];
      rc::RecheckArgs rk = s.rk;
      rk.listed = s.listed;
      rk.n_listed = s.n_listed;
      rk.cap = d.max_rechecks;
      rk.n_rows = frames[i].n_rows;
      rk.n_cols = frames[i].n_cols;
      rk.half = h;
      rk.guard = d.cfar_guard;
      rk.alpha_over_n = alpha / n_train;
      rk.power = s.rpower;
      rk.need = s.need;
      rk.plist = s.plist;
      rk.map = s.pmap;
      rk.n_need = s.n_need;
      rk.mask = s.mask;
      rk.words_per_row = wpr(i);
      rk.det_cell = s.det_cell;
      RC_HIP(rc::launch_recheck(rk, st));
    }
  }
  for (int i0 = 0; i0 < n; i0 += rc::CompactMulti::kMax) {
    rc::CompactMulti m;
    for (int i = i0; i < n && m.n_frames < rc::CompactMulti::kMax; ++i) {
      Slot& s = *slot[i];
      // the count and the first records go straight to the slot's mapped
      // pinned memory: no copy per frame
      m.f[m.n_frames++] = rc::CompactArgs{s.mask, s.det_cell, frames[i].n_rows, frames[i].n_cols, wpr(i),
                                          s.det_out, det_capacity(d, frames[i]), s.det_count, s.h_count_dev,
                                          s.h_det_dev, std::min<int64_t>(kDetPrefix, det_capacity(d, frames[i]))};
    }
    RC_HIP(rc::launch_compact(m, st));
  }
  for (int i = 0; i < n; ++i) {
    Slot& s = *slot[i];
    if (timed) RC_HIP(hipEventRecord(s.stage_ev[4], st));
    RC_HIP(hipEventRecord(s.done, st));
  }
  return RC_OK;
}

// ---------------------------------------------------------------------------
// One frame without a plan and without allocating: every intermediate of the
// pipeline (interpolation table, geometry rows, pixel tables, partial images,
// CFAR mask and per-cell records) lives in `scratch`, a file-scope device
// array of RC_STATIC_SCRATCH_BYTES that each GPU holds from the library's load
// to the end of the process.  Its device address comes from
// hipGetSymbolAddress, once per device; host code uses only that address.
// ---------------------------------------------------------------------------
constexpr int64_t kStaticMaxRows = 16384;  // chirps x channels of one static frame
constexpr int kStaticMaxDevices = 64;
std::mutex g_static_mu;                    // guards the two tables below
void* g_static_scratch[kStaticMaxDevices] = {};
// host staging of one frame's geometry rows (pageable: the copy reads it
// before hipMemcpyAsync returns)
float g_static_geo[8 * kStaticMaxRows + kStaticMaxRows + 4096 + 4];

}  // namespace

static __device__ __align__(256) unsigned char scratch[RC_STATIC_SCRATCH_BYTES];

namespace {

struct StaticLayout {
  size_t pairs, geo, fd, pixc, fbase, partials, mask, det_cell, total;
};

StaticLayout static_layout(const rc_plan_desc& d, const rc_frame& f, int n_kb) {
  StaticLayout l{};
  const size_t rows = (size_t)f.n_chirps * f.n_channels;
  const size_t n_pix = (size_t)f.n_rows * f.n_cols;
  const size_t n_s = f.input_kind == RC_INPUT_RAW ? (size_t)f.n_samples : 0;
  l.pairs = round_up(rows * f.n_bins * sizeof(float4));
  l.geo = round_up(((8 * rows + f.n_chirps + n_s + 3) & ~size_t(3)) * sizeof(float));
  l.fd = round_up(n_pix * sizeof(float));
  l.pixc = round_up(n_pix * sizeof(float4));
  l.fbase = split_phase(d) ? round_up(n_pix * sizeof(float)) : 0;
  l.partials = n_kb > 1 ? round_up((size_t)n_kb * n_pix * sizeof(float2)) : 0;
  l.mask = round_up((size_t)f.n_rows * ((f.n_cols + 63) / 64) * sizeof(unsigned long long));
  l.det_cell = round_up(n_pix * sizeof(rc_detection));
  l.total = l.pairs + l.geo + l.fd + l.pixc + l.fbase + l.partials + l.mask + l.det_cell;
  return l;
}

}  // namespace

extern "C" {

rc_status rc_process_frame_static(const rc_plan_desc* desc, const rc_frame* frame, rc_detection* detections,
                                  int64_t det_cap, int64_t* n_det, void* stream) {
  g_err.clear();
  rc_status st = validate_desc(desc);
  if (st != RC_OK) return st;
  if (!frame) return fail(RC_EINVAL, "frame is NULL");
  const rc_frame& f = *frame;
  if (desc->max_rechecks != 0 || desc->sliding_sensors != 0 || f.sliding != RC_SLIDE_OFF)
    return fail(RC_EINVAL, "the static entry point has no double-precision recheck and no continuous SAR");
  if (f.data_host || !f.data) return fail(RC_EINVAL, "the static entry point takes its input on the device (data)");
  if (!f.image_out) return fail(RC_EINVAL, "frame %lld: image_out is required", (long long)f.frame_id);
  if (!n_det || det_cap < 0 || (det_cap > 0 && !detections))
    return fail(RC_EINVAL, "detections, det_cap and n_det must describe a device buffer and a device count");
  Plan shape;  // the descriptor only: no slot, nothing allocated
  shape.d = *desc;
  shape.d.stage_timing = 0;
  st = validate_frame(&shape, f);
  if (st != RC_OK) return st;
  const int64_t rows = (int64_t)f.n_chirps * f.n_channels;
  if (rows > kStaticMaxRows)
    return fail(RC_EINVAL, "frame %lld: %lld chirp x channel rows, the static entry point takes at most %lld",
                (long long)f.frame_id, (long long)rows, (long long)kStaticMaxRows);
  const int n_kb = frame_chirp_blocks(&shape, f);
  const StaticLayout L = static_layout(shape.d, f, n_kb);
  if (L.total > (size_t)RC_STATIC_SCRATCH_BYTES)
    return fail(RC_EINVAL, "frame %lld needs %zu bytes of scratch; the static scratch holds %lld",
                (long long)f.frame_id, L.total, (long long)RC_STATIC_SCRATCH_BYTES);
  int dev = 0;
  RC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kStaticMaxDevices) return fail(RC_EINVAL, "device %d beyond the static table", dev);
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_scratch[dev]) {
    void* ptr = nullptr;
    RC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_static_scratch[dev] = ptr;
  }
  char* base = static_cast<char*>(g_static_scratch[dev]);
  const int64_t n_pix = (int64_t)f.n_rows * f.n_cols;
  Slot s;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    void* q = bytes ? base + off : nullptr;
    off += bytes;
    return q;
  };
  s.pairs = static_cast<float4*>(carve(L.pairs));
  s.rowgeo = static_cast<float4*>(carve(L.geo));
  s.fd = static_cast<float*>(carve(L.fd));
  s.pixc = static_cast<float4*>(carve(L.pixc));
  s.fbase = static_cast<float*>(carve(L.fbase));
  s.partials = static_cast<float2*>(carve(L.partials));
  s.partial_cap = n_kb > 1 ? (int64_t)n_kb * n_pix : 0;
  s.mask = static_cast<unsigned long long*>(carve(L.mask));
  s.det_cell = static_cast<rc_detection*>(carve(L.det_cell));
  s.staging = g_static_geo;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  Prepared prep;
  st = prepare_frame(&shape, s, f, nullptr, hs, &prep);
  if (st != RC_OK) return st;
  // 0: geometry rows from the host staging
  RC_HIP(hipMemcpyAsync(s.rowgeo, g_static_geo, (size_t)prep.up.n16 * 16, hipMemcpyHostToDevice, hs));
  // 1: range compression (or the given spectrum) into the interpolation table
  if (prep.raw_in) {
    rc::RangeMulti m;
    m.f[m.n_frames++] = prep.ra;
    RC_HIP(mfma_spectrum(shape.d) ? rc::launch_range_mfma(m, shape.d.precision == RC_PREC_BF16, hs)
                                  : rc::launch_range_compress(m, hs));
  } else {
    rc::PairMulti m;
    m.f[m.n_frames++] = prep.pa;
    RC_HIP(rc::launch_spectrum_pairs(m, hs));
  }
  // 2: pixel tables
  {
    rc::TableMulti m;
    m.f[m.n_frames++] = prep.ta;
    RC_HIP(rc::launch_pixel_tables(m, hs));
  }
  if (f.doppler_out)
    RC_HIP(hipMemcpyAsync(f.doppler_out, s.fd, (size_t)n_pix * sizeof(float), hipMemcpyDeviceToDevice, hs));
  // 3: back-projection, and the sum of the chirp blocks' partial images
  {
    rc::BpBatch b{};
    b.chg = prep.chg;
    b.sums = 1;
    b.form = shape.d.doppler == RC_DOPPLER_EXACT_DIRECT ? rc::kBpDirect
             : shape.d.doppler == RC_DOPPLER_EXACT ? rc::kBpExact
             : split_phase(shape.d) ? rc::kBpSplit : rc::kBpPlain;
    rc::BpFrame bf = prep.bf;
    bf.chunk = (bf.kb_count * bf.n_tiles + 7) / 8;
    bf.slot_base = 0;
    b.f[b.n_frames++] = bf;
    b.n_slots = bf.chunk;
    RC_HIP(rc::launch_backproject(b, hs));
    if (bf.n_kb > 1) {
      rc::ReduceBatch rb{};
      rb.f[rb.n_frames++] = rc::ReduceFrame{bf.out, s.image_used, n_pix, bf.n_kb};
      RC_HIP(rc::launch_reduce_partials(rb, hs));
    }
  }
  // 4: CA-CFAR and ordered compaction into the caller's buffers
  const rc_plan_desc& d = shape.d;
  const int h = d.cfar_guard + d.cfar_train;
  const int n_train = (2 * h + 1) * (2 * h + 1) - (2 * d.cfar_guard + 1) * (2 * d.cfar_guard + 1);
  const double alpha = n_train * (std::pow(d.cfar_pfa, -1.0 / n_train) - 1.0);
  const int wpr = (f.n_cols + 63) / 64;
  {
    rc::CfarMulti m;
    m.f[m.n_frames++] = rc::CfarArgs{s.image_used, f.n_rows, f.n_cols, d.cfar_guard, d.cfar_train,
                                     alpha / n_train, d.cfar_margin_rel, s.mask, wpr, s.det_cell, nullptr,
                                     nullptr, 0};
    RC_HIP(rc::launch_cfar(m, hs));
  }
  {
    rc::CompactMulti m;
    m.f[m.n_frames++] = rc::CompactArgs{s.mask, s.det_cell, f.n_rows, f.n_cols, wpr, detections, det_cap, n_det,
                                        nullptr, nullptr, 0};
    RC_HIP(rc::launch_compact(m, hs));
  }
  return RC_OK;
}

rc_status rc_plan_slot_bytes(const rc_plan_desc* desc, int64_t* bytes) {
  rc_status st = validate_desc(desc);
  if (st != RC_OK) return st;
  if (!bytes) return fail(RC_EINVAL, "bytes is NULL");
  *bytes = (int64_t)slot_sizes(*desc).total();
  return RC_OK;
}

rc_status rc_frame_bytes(const rc_plan_desc* desc, const rc_frame* frame, int64_t* bytes) {
  g_err.clear();
  rc_status st = validate_desc(desc);
  if (st != RC_OK) return st;
  if (!frame || !bytes) return fail(RC_EINVAL, "frame and bytes are required");
  Plan shape;  // the descriptor's limits only: nothing is allocated
  shape.d = *desc;
  shape.planes = desc->sliding_sensors > 0 ? sliding_planes(*desc) : 0;
  st = validate_frame(&shape, *frame);
  if (st != RC_OK) return st;
  const int planes = frame->sliding != RC_SLIDE_OFF ? shape.planes : 1;
  *bytes = (int64_t)round_up(frame_sizes(*desc, *frame, frame_chirp_blocks(&shape, *frame), planes).total());
  return RC_OK;
}

rc_status rc_frame_validate(const rc_plan_desc* desc, const rc_frame* frame) {
  g_err.clear();
  rc_status st = validate_desc(desc);
  if (st != RC_OK) return st;
  if (!frame) return fail(RC_EINVAL, "frame is NULL");
  Plan shape;  // the descriptor's limits only: nothing is allocated
  shape.d = *desc;
  shape.planes = desc->sliding_sensors > 0 ? sliding_planes(*desc) : 0;
  return validate_frame(&shape, *frame);
}

rc_status rc_plan_create(const rc_plan_desc* desc, void** out) {
  g_err.clear();
  if (!out) return fail(RC_EINVAL, "out is NULL");
  *out = nullptr;
  rc_status st = validate_desc(desc);
  if (st != RC_OK) return st;
  const SlotSizes sz = slot_sizes(*desc);
  const size_t per_slot = sz.total();
  const size_t tw64_bytes = desc->max_rechecks > 0 ? (size_t)desc->n_fft_max / 2 * sizeof(double2) : 0;
  const size_t need = desc->frame_memory == RC_MEMORY_BUDGET
                          ? tw64_bytes + ring_bytes(*desc) + 256
                          : per_slot * desc->max_frames_in_flight + tw64_bytes + ring_bytes(*desc);
  if (desc->hbm_budget_bytes > 0 && need > (size_t)desc->hbm_budget_bytes)
    return fail(RC_ENOMEM, "plan needs %zu bytes of device memory, budget is %lld", need,
                (long long)desc->hbm_budget_bytes);

  Plan* p = new (std::nothrow) Plan();
  if (!p) return fail(RC_ENOMEM, "host allocation failed");
  p->d = *desc;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return fail(RC_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  }
  // double twiddles over the half circle of n_fft_max (for the recheck)
  p->tw_log2 = ilog2(desc->n_fft_max);
  if (desc->max_rechecks > 0) {
    std::vector<double2> tw64(desc->n_fft_max / 2);
    for (size_t k = 0; k < tw64.size(); ++k) {
      const double a = -2.0 * kPi * (double)k / desc->n_fft_max;
      tw64[k] = make_double2(std::cos(a), std::sin(a));
    }
    e = hipMalloc(&p->twiddle64, tw64_bytes);
    if (e == hipSuccess) e = hipMemcpy(p->twiddle64, tw64.data(), tw64_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      free_plan(p);
      return fail(e == hipErrorOutOfMemory ? RC_ENOMEM : RC_EHIP, "twiddle table: %s", hipGetErrorString(e));
    }
  }
  if (desc->sliding_sensors > 0) {
    p->n_ring = sliding_ring(*desc);
    p->planes = sliding_planes(*desc);
    p->ring_stride = (int64_t)p->planes * desc->n_pix_max;
    e = hipMalloc(&p->ring, ring_bytes(*desc));
    if (e != hipSuccess) {
      free_plan(p);
      return fail(RC_ENOMEM, "continuous-SAR ring of %zu bytes: %s", ring_bytes(*desc), hipGetErrorString(e));
    }
    p->sensors.resize(desc->sliding_sensors);
    for (Sensor& sn : p->sensors) {
      e = hipEventCreateWithFlags(&sn.done, hipEventDisableTiming);
      if (e != hipSuccess) {
        free_plan(p);
        return fail(RC_EHIP, "event creation failed: %s", hipGetErrorString(e));
      }
    }
  }
  p->slots.resize(desc->max_frames_in_flight);
  const size_t geo_bytes = geo_floats(*desc) * sizeof(float);
  const bool budget_mode = desc->frame_memory == RC_MEMORY_BUDGET;
  if (budget_mode) {
    // one arena: what the budget leaves after the recheck's twiddles and the
    // continuous-SAR ring
    p->arena_bytes = (size_t)desc->hbm_budget_bytes - tw64_bytes - ring_bytes(*desc);
    e = hipMalloc(&p->arena, p->arena_bytes);
    if (e != hipSuccess) {
      free_plan(p);
      return fail(RC_ENOMEM, "device arena of %zu bytes: %s", p->arena_bytes, hipGetErrorString(e));
    }
    p->free_list.emplace(0, p->arena_bytes);
    e = hipStreamCreateWithFlags(&p->copy_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->copied, hipEventDisableTiming);
    for (hipEvent_t& ev : p->pieces)
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      free_plan(p);
      return fail(RC_EHIP, "copy stream: %s", hipGetErrorString(e));
    }
  }
  for (Slot& s : p->slots) {
    if (!budget_mode) {
      char* base = nullptr;
      e = hipMalloc(&base, per_slot);
      if (e != hipSuccess) {
        free_plan(p);
        return fail(RC_ENOMEM, "device allocation of %zu bytes per slot failed: %s", per_slot,
                    hipGetErrorString(e));
      }
      carve_slot(s, base, sz);
      s.partial_cap = partial_capacity(*desc);
    }
    e = hipHostMalloc(reinterpret_cast<void**>(&s.staging), geo_bytes, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
      void* dev = nullptr;
      e = hipHostGetDevicePointer(&dev, s.staging, 0);
      s.staging_dev = static_cast<const float4*>(dev);
    }
    if (e == hipSuccess) {
      const size_t hb = 64 + (size_t)std::min(kDetPrefix, desc->max_detections) * sizeof(rc_detection);
      e = hipHostMalloc(reinterpret_cast<void**>(&s.h_count), hb, hipHostMallocMapped | hipHostMallocCoherent);
      if (e == hipSuccess) {
        s.h_det = reinterpret_cast<rc_detection*>(reinterpret_cast<char*>(s.h_count) + 64);
        void* dev = nullptr;
        e = hipHostGetDevicePointer(&dev, s.h_count, 0);
        s.h_count_dev = static_cast<int64_t*>(dev);
        s.h_det_dev = reinterpret_cast<rc_detection*>(static_cast<char*>(dev) + 64);
      }
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    if (desc->stage_timing)
      for (hipEvent_t& ev : s.stage_ev)
        if (e == hipSuccess) e = hipEventCreate(&ev);
    if (e != hipSuccess) {
      free_plan(p);
      return fail(RC_ENOMEM, "pinned host allocation / event creation failed: %s", hipGetErrorString(e));
    }
  }
  *out = p;
  return RC_OK;
}

rc_status rc_process_batch(void* plan, const rc_frame* frames, int32_t n_frames, void* stream) {
  g_err.clear();
  Plan* p = static_cast<Plan*>(plan);
  if (!p) return fail(RC_EINVAL, "plan is NULL");
  if (n_frames < 0 || (n_frames > 0 && !frames)) return fail(RC_EINVAL, "bad frame array");
  int free_slots = 0;
  for (const Slot& s : p->slots) free_slots += !s.busy;
  if (n_frames > free_slots)
    return fail(RC_ENOTREADY, "%d frames but only %d free slots", n_frames, free_slots);
  for (int i = 0; i < n_frames; ++i) {
    rc_status st = validate_frame(p, frames[i]);
    if (st != RC_OK) return st;
    if (find_slot(p, frames[i].frame_id))
      return fail(RC_EINVAL, "frame id %lld is already in flight", (long long)frames[i].frame_id);
    for (int j = 0; j < i; ++j)
      if (frames[j].frame_id == frames[i].frame_id)
        return fail(RC_EINVAL, "frame id %lld repeated in the batch", (long long)frames[i].frame_id);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  // continuous SAR: each sub-aperture's place in its stream, in batch order,
  // on a copy of the sensors' state that the batch commits when it succeeds
  std::vector<Slide> slide(n_frames);
  std::vector<Sensor> sensors = p->sensors;
  {
    std::vector<int> in_flight(p->sensors.size(), 0);
    for (const Slot& s : p->slots)
      if (s.busy && s.sensor >= 0) ++in_flight[s.sensor];
    for (int i = 0; i < n_frames; ++i) {
      const rc_frame& f = frames[i];
      if (f.sliding == RC_SLIDE_OFF) continue;
      Sensor& sn = sensors[f.sensor_id];
      if (f.sliding == RC_SLIDE_START) {
        sn.started = true;
        sn.next = 0;
        sn.n_chirps = f.n_chirps;
        sn.n_channels = f.n_channels;
        sn.n_rows = f.n_rows;
        sn.n_cols = f.n_cols;
        sn.pixels = f.pixels;
        sn.height = f.height;
      } else if (!sn.started) {
        return fail(RC_EINVAL, "frame %lld: sensor %d has no stream (start one with RC_SLIDE_START)",
                    (long long)f.frame_id, f.sensor_id);
      } else if (f.n_chirps != sn.n_chirps || f.n_channels != sn.n_channels || f.n_rows != sn.n_rows ||
                 f.n_cols != sn.n_cols || f.pixels != sn.pixels || f.height != sn.height) {
        return fail(RC_EINVAL, "frame %lld: sub-aperture of sensor %d unlike its stream (chirps, channels, "
                    "lattice, pixels and height must stay)", (long long)f.frame_id, f.sensor_id);
      }
      if (++in_flight[f.sensor_id] > p->d.sliding_depth)
        return fail(RC_ENOTREADY, "frame %lld: more than %d sub-apertures of sensor %d in flight",
                    (long long)f.frame_id, p->d.sliding_depth, f.sensor_id);
      Slide& sl = slide[i];
      sl.sensor = f.sensor_id;
      sl.block = sn.next;
      sl.ring_slot = (int)(sn.stored % p->n_ring);
      sl.n_blk = (int)std::min<int64_t>(sn.next + 1, p->d.sliding_subapertures);
      sl.first_slot = (int)((sn.stored - (sl.n_blk - 1)) % p->n_ring);
      sl.dst = p->ring + ((int64_t)f.sensor_id * p->n_ring + sl.ring_slot) * p->ring_stride;
      ++sn.next;
      ++sn.stored;
    }
  }
  std::vector<Slot*> slot(n_frames, nullptr);
  std::vector<Prepared> prep(n_frames);
  // RC_MEMORY_BUDGET: every frame's own bytes from the arena, or nothing at all
  const bool budget = p->arena != nullptr;
  std::vector<std::pair<size_t, size_t>> taken;  // (offset, length) per frame
  std::vector<SlotSizes> fsz(budget ? n_frames : 0);
  if (budget) {
    size_t wanted = 0;
    for (int i = 0; i < n_frames; ++i) {
      const int planes = frames[i].sliding != RC_SLIDE_OFF ? p->planes : 1;
      fsz[i] = frame_sizes(p->d, frames[i], frame_chirp_blocks(p, frames[i]), planes);
      const size_t len = round_up(fsz[i].total());
      if (len > p->arena_bytes) {  // would never fit, however many frames complete
        for (const auto& t : taken) arena_free(p, t.first, t.second);
        return fail(RC_ENOMEM, "frame %lld needs %zu bytes, more than the plan's whole arena of %zu",
                    (long long)frames[i].frame_id, len, p->arena_bytes);
      }
      wanted += len;
      const size_t off = arena_alloc(p, len);
      if (off == SIZE_MAX) {
        for (const auto& t : taken) arena_free(p, t.first, t.second);
        return fail(RC_ENOTREADY, "the batch needs %zu bytes of the HBM budget (frame %lld: %zu), more than is free",
                    wanted, (long long)frames[i].frame_id, len);
      }
      taken.emplace_back(off, len);
    }
  }
  auto undo = [&](rc_status r) {  // a failed batch leaves no slot busy and no stream advanced
    (void)hipStreamSynchronize(st);
    if (p->copy_stream) (void)hipStreamSynchronize(p->copy_stream);  // no copy still writes a freed range
    for (Slot* q : slot)
      if (q) { q->busy = false; q->frame_id = -1; q->sensor = -1; q->arena_len = 0; q->input = nullptr; }
    for (const auto& t : taken) arena_free(p, t.first, t.second);
    return r;
  };
#define RC_BATCH(call)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return undo(fail(RC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)));        \
  } while (0)
  const bool timed = p->d.stage_timing != 0;
  // host part of every frame: geometry upload, argument blocks
  for (int i = 0; i < n_frames; ++i) {
    for (Slot& c : p->slots)
      if (!c.busy) { slot[i] = &c; break; }
    rc_frame f = frames[i];
    if (budget) {
      Slot& q = *slot[i];
      carve_slot(q, p->arena + taken[i].first, fsz[i]);
      q.arena_off = taken[i].first;
      q.arena_len = taken[i].second;
      const int planes = f.sliding != RC_SLIDE_OFF ? p->planes : 1;
      q.partial_cap = (int64_t)frame_chirp_blocks(p, f) * planes * f.n_rows * f.n_cols;
      if (f.data_host) f.data = q.input;  // the plan's copy of the input
    }
    rc_status r = prepare_frame(p, *slot[i], f, slide[i].sensor >= 0 ? &slide[i] : nullptr, st, &prep[i]);
    if (r != RC_OK) return undo(r);
  }
  // inputs handed over in pinned host memory: copied into the frames' arena
  // shares on the plan's copy stream (the paper's pinned Load), which the
  // batch's stream waits for before its kernels.  A share is taken only from
  // ranges whose frames have completed, so no earlier work on any stream
  // still reads it.
  // A lone frame whose back-projection has several chirp blocks is copied in
  // pieces of those blocks' rows: each block's range compression and
  // back-projection wait only for its own piece, so all but the first piece's
  // copy overlap the frame's own compute (the results are those of the whole
  // launches: the same kernels over the same rows and blocks).
  const bool piped = n_frames == 1 && frames[0].data_host && prep[0].raw_in && !prep[0].recheck &&
                     slide[0].sensor < 0 && prep[0].bf.n_kb > 1 && prep[0].bf.n_kb <= 16 && p->pieces[0];
  auto block_rows = [&](int k, int64_t* r0, int64_t* r1) {  // the kernel's split of the chirps
    const rc::BpFrame& b = prep[0].bf;
    *r0 = (int64_t)(((int64_t)k * b.n_chirps) / b.n_kb) * b.n_ch;
    *r1 = (int64_t)(((int64_t)(k + 1) * b.n_chirps) / b.n_kb) * b.n_ch;
  };
  bool any_host = false;
  if (piped) {
    const size_t row_bytes = (size_t)frames[0].n_samples * sizeof(float2);
    for (int k = 0; k < prep[0].bf.n_kb; ++k) {
      int64_t r0, r1;
      block_rows(k, &r0, &r1);
      RC_BATCH(hipMemcpyAsync(static_cast<char*>(slot[0]->input) + r0 * row_bytes,
                              static_cast<const char*>(frames[0].data_host) + r0 * row_bytes,
                              (size_t)(r1 - r0) * row_bytes, hipMemcpyHostToDevice, p->copy_stream));
      RC_BATCH(hipEventRecord(p->pieces[k], p->copy_stream));
    }
  } else {
    for (int i = 0; i < n_frames; ++i)
      if (frames[i].data_host) {
        RC_BATCH(hipMemcpyAsync(slot[i]->input, frames[i].data_host, fsz[i].input, hipMemcpyHostToDevice,
                                p->copy_stream));
        any_host = true;
      }
  }
  if (any_host) {
    RC_BATCH(hipEventRecord(p->copied, p->copy_stream));
    RC_BATCH(hipStreamWaitEvent(st, p->copied, 0));
  }
  // 0: every frame's geometry from its staging buffer, one launch per 32 frames
  for (int i0 = 0; i0 < n_frames; i0 += rc::UploadMulti::kMax) {
    rc::UploadMulti m;
    for (int i = i0; i < n_frames && m.n_frames < rc::UploadMulti::kMax; ++i) m.f[m.n_frames++] = prep[i].up;
    RC_BATCH(rc::launch_upload(m, st));
  }
  if (timed)
    for (Slot* q : slot) RC_BATCH(hipEventRecord(q->stage_ev[0], st));
  // the recheck's beat spectra in double
  for (int i = 0; i < n_frames; ++i)
    if (prep[i].recheck) RC_BATCH(rc::launch_range64(prep[i].r6, st));
  // 1: range compression, one launch per DFT length and 32 frames
  {
    std::vector<char> done(n_frames, 0);
    for (int i = 0; i < n_frames; ++i) {
      if (done[i] || !prep[i].raw_in || piped) continue;
      rc::RangeMulti m;
      for (int j = i; j < n_frames && m.n_frames < rc::RangeMulti::kMax; ++j)
        if (!done[j] && prep[j].raw_in && prep[j].ra.log2n == prep[i].ra.log2n) {
          m.f[m.n_frames++] = prep[j].ra;
          done[j] = 1;
        }
      RC_BATCH(mfma_spectrum(p->d) ? rc::launch_range_mfma(m, p->d.precision == RC_PREC_BF16, st)
                                   : rc::launch_range_compress(m, st));
    }
    rc::PairMulti m;
    for (int i = 0; i < n_frames; ++i) {
      if (prep[i].raw_in) continue;
      m.f[m.n_frames++] = prep[i].pa;
      if (m.n_frames == rc::PairMulti::kMax) {
        RC_BATCH(rc::launch_spectrum_pairs(m, st));
        m.n_frames = 0;
      }
    }
    if (m.n_frames) RC_BATCH(rc::launch_spectrum_pairs(m, st));
  }
  if (timed)
    for (Slot* q : slot) RC_BATCH(hipEventRecord(q->stage_ev[1], st));
  // 2: pixel tables, one launch per 16 frames
  for (int i0 = 0; i0 < n_frames; i0 += rc::TableMulti::kMax) {
    rc::TableMulti m;
    for (int i = i0; i < n_frames && m.n_frames < rc::TableMulti::kMax; ++i) m.f[m.n_frames++] = prep[i].ta;
    RC_BATCH(rc::launch_pixel_tables(m, st));
  }
  for (int i = 0; i < n_frames; ++i)
    if (frames[i].doppler_out)
      RC_BATCH(hipMemcpyAsync(frames[i].doppler_out, slot[i]->fd,
                              (size_t)frames[i].n_rows * frames[i].n_cols * sizeof(float), hipMemcpyDeviceToDevice, st));
  if (timed)
    for (Slot* q : slot) RC_BATCH(hipEventRecord(q->stage_ev[2], st));
  // 3: back-projection, one launch per TX-group width and per 16 frames; the
  // frames of a launch go most expensive work item first (fewest short items
  // in the tail)
  std::vector<int> order(n_frames);
  for (int i = 0; i < n_frames; ++i) order[i] = i;
  auto item_cost = [&](int i) {
    const rc::BpFrame& b = prep[i].bf;
    return (int64_t)((b.n_chirps + b.n_kb - 1) / b.n_kb) * b.n_ch;
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return item_cost(x) > item_cost(y); });
  std::vector<char> done(n_frames, 0);
  if (piped) {
    // per chirp block: wait for its piece, then its range compression and
    // its back-projection
    for (int k = 0; k < prep[0].bf.n_kb; ++k) {
      int64_t r0, r1;
      block_rows(k, &r0, &r1);
      RC_BATCH(hipStreamWaitEvent(st, p->pieces[k], 0));
      rc::RangeMulti m;
      rc::RangeArgs ra = prep[0].ra;
      ra.raw += r0 * ra.n_s;
      ra.w_sar += r0 / ra.n_ch;
      ra.pairs += r0 * ra.n_bins;
      if (ra.spectrum) ra.spectrum += r0 * ra.n_bins;
      ra.rows = r1 - r0;
      m.f[m.n_frames++] = ra;
      RC_BATCH(mfma_spectrum(p->d) ? rc::launch_range_mfma(m, p->d.precision == RC_PREC_BF16, st)
                                   : rc::launch_range_compress(m, st));
      rc::BpBatch b{};
      b.chg = prep[0].chg;
      b.sums = prep[0].sums;
      b.form = p->d.doppler == RC_DOPPLER_EXACT_DIRECT ? rc::kBpDirect
               : p->d.doppler == RC_DOPPLER_EXACT ? rc::kBpExact
               : split_phase(p->d) ? rc::kBpSplit : rc::kBpPlain;
      rc::BpFrame bf = prep[0].bf;
      bf.kb0 = k;
      bf.kb_count = 1;
      bf.chunk = (bf.n_tiles + 7) / 8;
      bf.slot_base = 0;
      b.f[b.n_frames++] = bf;
      b.n_slots = bf.chunk;
      RC_BATCH(rc::launch_backproject(b, st));
    }
    done[0] = 1;
  }
  for (int oi = 0; oi < n_frames; ++oi) {
    const int i = order[oi];
    if (done[i]) continue;
    rc::BpBatch b{};
    b.chg = prep[i].chg;
    b.sums = prep[i].sums;
    b.form = p->d.doppler == RC_DOPPLER_EXACT_DIRECT ? rc::kBpDirect
             : p->d.doppler == RC_DOPPLER_EXACT ? rc::kBpExact
             : split_phase(p->d) ? rc::kBpSplit : rc::kBpPlain;
    for (int oj = oi; oj < n_frames && b.n_frames < rc::kBpMaxFrames; ++oj) {
      const int j = order[oj];
      if (done[j] || prep[j].chg != prep[i].chg || prep[j].sums != prep[i].sums) continue;
      rc::BpFrame fj = prep[j].bf;
      fj.chunk = (fj.kb_count * fj.n_tiles + 7) / 8;
      fj.slot_base = b.n_slots;
      b.f[b.n_frames++] = fj;
      b.n_slots += fj.chunk;
      done[j] = 1;
    }
    RC_BATCH(rc::launch_backproject(b, st));
  }
  rc::ReduceBatch rb{};
  for (int i = 0; i < n_frames; ++i) {
    if (prep[i].bf.n_kb == 1) continue;
    // a sub-aperture's [planes][n_pix] sums reduce like one image of planes n_pix pixels
    float2* dst = slide[i].sensor >= 0 ? slide[i].dst : slot[i]->image_used;
    rb.f[rb.n_frames++] = rc::ReduceFrame{prep[i].bf.out, dst,
                                          (int64_t)prep[i].sums * frames[i].n_rows * frames[i].n_cols,
                                          prep[i].bf.n_kb};
    if (rb.n_frames == rc::kReduceMaxFrames) {
      RC_BATCH(rc::launch_reduce_partials(rb, st));
      rb.n_frames = 0;
    }
  }
  if (rb.n_frames) RC_BATCH(rc::launch_reduce_partials(rb, st));
  // a sensor's apertures read the partial images of its earlier
  // sub-apertures: wait for the aperture the sensor formed last, whichever
  // stream formed it (on the same stream the wait is implied; a handle equal
  // to the last one may still name a new stream, so it is always recorded).
  // Back-projection before this point only writes the sub-apertures' own
  // ring slots, which no pending aperture reads (the ring holds K + depth - 1)
  for (size_t k = 0; k < sensors.size(); ++k) {
    bool used = false;
    for (int i = 0; i < n_frames && !used; ++i) used = slide[i].sensor == (int)k;
    if (used && p->sensors[k].recorded) RC_BATCH(hipStreamWaitEvent(st, p->sensors[k].done, 0));
  }
  // continuous SAR: each sub-aperture's aperture from the ring.  The window
  // over the aperture's N = K S chirps starts at chirp a = (b - K + 1) S of the
  // stream: w(m) = 1/2 - 1/2 cos(theta_m - phi), phi = 2 pi (a mod (N - 1)) / (N - 1)
  rc::CombineBatch cb{};
  for (int i = 0; i < n_frames; ++i) {
    const Slide& sl = slide[i];
    if (sl.sensor < 0) continue;
    rc::CombineFrame& c = cb.f[cb.n_frames++];
    c = rc::CombineFrame{};
    c.ring = p->ring + (int64_t)sl.sensor * p->n_ring * p->ring_stride;
    c.stride = p->ring_stride;
    c.n_ring = p->n_ring;
    c.first = sl.first_slot;
    c.n_blk = sl.n_blk;
    c.planes = p->planes;
    c.c0 = 1.f;
    if (p->planes == 3) {
      const int64_t period = (int64_t)p->d.sliding_subapertures * frames[i].n_chirps - 1;
      if (period > 0) {
        const int64_t a = (sl.block - p->d.sliding_subapertures + 1) * frames[i].n_chirps;
        const double phi = 2.0 * kPi * (double)(((a % period) + period) % period) / (double)period;
        c.c0 = 0.5f;
        c.cc = (float)(-0.5 * std::cos(phi));
        c.cs = (float)(-0.5 * std::sin(phi));
      }
    }
    c.out = slot[i]->image_used;
    c.n_pix = (int64_t)frames[i].n_rows * frames[i].n_cols;
    if (cb.n_frames == rc::kCombineMaxFrames) {
      RC_BATCH(rc::launch_combine(cb, st));
      cb.n_frames = 0;
    }
  }
  if (cb.n_frames) RC_BATCH(rc::launch_combine(cb, st));
  for (size_t k = 0; k < sensors.size(); ++k) {
    bool used = false;
    for (int i = 0; i < n_frames && !used; ++i) used = slide[i].sensor == (int)k;
    if (!used) continue;
    RC_BATCH(hipEventRecord(sensors[k].done, st));
    sensors[k].recorded = true;
  }
  if (timed)
    for (Slot* q : slot) RC_BATCH(hipEventRecord(q->stage_ev[3], st));
#undef RC_BATCH
  // 4: detection and read-back
  rc_status r = finish_batch(p, slot, frames, n_frames, st);
  if (r != RC_OK) return undo(r);
  p->sensors = sensors;
  return RC_OK;
}

rc_status rc_poll(void* plan, int64_t frame_id) {
  Plan* p = static_cast<Plan*>(plan);
  if (!p) return fail(RC_EINVAL, "plan is NULL");
  Slot* s = find_slot(p, frame_id);
  if (!s) return fail(RC_ENOTFOUND, "frame %lld is not in flight", (long long)frame_id);
  hipError_t e = hipEventQuery(s->done);
  if (e == hipSuccess) return RC_OK;
  if (e == hipErrorNotReady) return RC_ENOTREADY;
  return fail(RC_EHIP, "hipEventQuery: %s", hipGetErrorString(e));
}

rc_status rc_detections(void* plan, int64_t frame_id, rc_detection* dst, int64_t cap, int64_t* n_out) {
  Plan* p = static_cast<Plan*>(plan);
  if (!p || !n_out || cap < 0 || (cap > 0 && !dst)) return fail(RC_EINVAL, "bad arguments");
  Slot* s = find_slot(p, frame_id);
  if (!s) return fail(RC_ENOTFOUND, "frame %lld is not in flight", (long long)frame_id);
  RC_HIP(hipEventSynchronize(s->done));
  const int64_t n = *s->h_count;
  *n_out = n;
  const int64_t avail = std::min<int64_t>(n, p->d.max_detections);
  const int64_t ncopy = std::min<int64_t>(avail, cap);
  const int64_t pre = std::min<int64_t>(ncopy, std::min(kDetPrefix, p->d.max_detections));
  if (pre > 0) std::memcpy(dst, s->h_det, pre * sizeof(rc_detection));
  if (ncopy > pre)
    RC_HIP(hipMemcpy(dst + pre, s->det_out + pre, (ncopy - pre) * sizeof(rc_detection), hipMemcpyDeviceToHost));
  if (ncopy < n)
    return fail(RC_ETRUNC, "frame %lld has %lld detections, %lld copied", (long long)frame_id,
                (long long)n, (long long)ncopy);
  return RC_OK;
}

rc_status rc_image(void* plan, int64_t frame_id, void* dst, int64_t cap_pixels, void* stream) {
  Plan* p = static_cast<Plan*>(plan);
  if (!p || !dst) return fail(RC_EINVAL, "bad arguments");
  Slot* s = find_slot(p, frame_id);
  if (!s) return fail(RC_ENOTFOUND, "frame %lld is not in flight", (long long)frame_id);
  const int64_t n = (int64_t)s->n_rows * s->n_cols;
  if (cap_pixels < n) return fail(RC_ETRUNC, "image has %lld pixels, capacity %lld", (long long)n, (long long)cap_pixels);
  hipStream_t st = static_cast<hipStream_t>(stream);
  RC_HIP(hipStreamWaitEvent(st, s->done, 0));
  if (dst != s->image_used)
    RC_HIP(hipMemcpyAsync(dst, s->image_used, n * sizeof(float2), hipMemcpyDeviceToDevice, st));
  return RC_OK;
}

rc_status rc_stage_times(void* plan, int64_t frame_id, float* ms4) {
  Plan* p = static_cast<Plan*>(plan);
  if (!p || !ms4) return fail(RC_EINVAL, "bad arguments");
  if (!p->d.stage_timing) return fail(RC_EINVAL, "plan was created without stage_timing");
  Slot* s = find_slot(p, frame_id);
  if (!s) return fail(RC_ENOTFOUND, "frame %lld is not in flight", (long long)frame_id);
  RC_HIP(hipEventSynchronize(s->done));
  for (int i = 0; i < 4; ++i) RC_HIP(hipEventElapsedTime(&ms4[i], s->stage_ev[i], s->stage_ev[i + 1]));
  return RC_OK;
}

rc_status rc_frame_release(void* plan, int64_t frame_id) {
  Plan* p = static_cast<Plan*>(plan);
  if (!p) return fail(RC_EINVAL, "plan is NULL");
  Slot* s = find_slot(p, frame_id);
  if (!s) return fail(RC_ENOTFOUND, "frame %lld is not in flight", (long long)frame_id);
  RC_HIP(hipEventSynchronize(s->done));
  s->busy = false;
  s->frame_id = -1;
  s->sensor = -1;
  if (p->arena) {
    arena_free(p, s->arena_off, s->arena_len);
    s->arena_len = 0;
    s->input = nullptr;
  }
  return RC_OK;
}

// A tuned block count for a class must be one the kernels and the slots take.
rc_status check_tuning_entry(const Plan* p, const rc_tuning_entry& e) {
  const rc_plan_desc& d = p->d;
  if (e.n_rows < 1 || e.n_cols < 1 || (int64_t)e.n_rows * e.n_cols > d.n_pix_max || e.n_chirps < 1 ||
      e.n_chirps > d.n_chirps_max || e.n_channels < 1 || e.n_channels > d.n_channels_max)
    return fail(RC_EINVAL, "tuning entry %d x %d pixels, %d chirps, %d channels is outside the plan's limits",
                e.n_rows, e.n_cols, e.n_chirps, e.n_channels);
  const int most = std::min(16, e.n_chirps);
  if (e.chirp_blocks < 1 || e.chirp_blocks > most)
    return fail(RC_EINVAL, "tuning entry: %d chirp blocks outside [1, %d]", e.chirp_blocks, most);
  if (e.chirp_blocks > 1 && (int64_t)e.chirp_blocks * e.n_rows * e.n_cols > partial_capacity(d))
    return fail(RC_EINVAL, "tuning entry: %d chirp blocks exceed the partial-image buffer", e.chirp_blocks);
  return RC_OK;
}

rc_status rc_plan_set_tuning(void* plan, const rc_tuning_entry* entries, int32_t n) {
  g_err.clear();
  Plan* p = static_cast<Plan*>(plan);
  if (!p) return fail(RC_EINVAL, "plan is NULL");
  if (n < 0 || (n > 0 && !entries)) return fail(RC_EINVAL, "bad tuning table");
  std::map<std::array<int32_t, 4>, int> table;
  for (int i = 0; i < n; ++i) {
    const rc_status st = check_tuning_entry(p, entries[i]);
    if (st != RC_OK) return st;
    table[{entries[i].n_rows, entries[i].n_cols, entries[i].n_chirps, entries[i].n_channels}] = entries[i].chirp_blocks;
  }
  p->tuned = std::move(table);
  return RC_OK;
}

rc_status rc_plan_tune(void* plan, const rc_frame* frames, int32_t n_frames, void* stream, rc_tuning_entry* out,
                       int32_t cap, int32_t* n_out) {
  g_err.clear();
  Plan* p = static_cast<Plan*>(plan);
  if (!p) return fail(RC_EINVAL, "plan is NULL");
  if (n_frames < 0 || (n_frames > 0 && !frames) || cap < 0 || (cap > 0 && !out) || !n_out)
    return fail(RC_EINVAL, "bad frame array or output table");
  // the classes, each probed with its first frame
  std::vector<std::pair<std::array<int32_t, 4>, int>> classes;
  for (int i = 0; i < n_frames; ++i) {
    if (frames[i].sliding != RC_SLIDE_OFF)
      return fail(RC_EINVAL, "frame %lld: sub-apertures keep the rule's chirp split", (long long)frames[i].frame_id);
    const rc_status st = validate_frame(p, frames[i]);
    if (st != RC_OK) return st;
    const auto key = size_class(frames[i]);
    if (std::none_of(classes.begin(), classes.end(), [&](const auto& c) { return c.first == key; }))
      classes.emplace_back(key, i);
  }
  *n_out = (int32_t)classes.size();
  if ((int64_t)classes.size() > cap)
    return fail(RC_ETRUNC, "%zu size classes, room for %d entries", classes.size(), cap);
  if (classes.empty()) return RC_OK;
  // each measurement is a batch of `copies` copies of the class's frame (the
  // first one with the caller's outputs, the others into their slots), so
  // that the split is chosen for frames that share the GPU with others
  const int free_slots = (int)std::count_if(p->slots.begin(), p->slots.end(), [](const Slot& s) { return !s.busy; });
  if (free_slots < 1) return fail(RC_ENOTREADY, "the plan has no free slot to tune with");
  const int copies = std::min(4, free_slots);
  int64_t ids[4];
  int64_t next_id = INT64_MIN;
  for (int k = 0; k < copies; ++k) {
    while (find_slot(p, next_id)) ++next_id;
    ids[k] = next_id++;
  }
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  RC_HIP(hipEventCreate(&ev.a));
  RC_HIP(hipEventCreate(&ev.b));
  hipStream_t hs = static_cast<hipStream_t>(stream);
  for (size_t c = 0; c < classes.size(); ++c) {
    const auto key = classes[c].first;
    rc_frame f[4];
    for (int k = 0; k < copies; ++k) {
      f[k] = frames[classes[c].second];
      f[k].frame_id = ids[k];
      if (k > 0) {
        f[k].image_out = nullptr;
        f[k].doppler_out = nullptr;
        f[k].spectrum_out = nullptr;
      }
    }
    p->tuned.erase(key);
    const int k0 = frame_chirp_blocks(p, f[0]);
    std::vector<int> cand{k0};
    for (const int k : {k0 / 4, k0 / 2, 2 * k0, 4 * k0}) {
      rc_tuning_entry e{key[0], key[1], key[2], key[3], k, k0, 0.f, 0.f};
      if (k >= 1 && std::find(cand.begin(), cand.end(), k) == cand.end() && check_tuning_entry(p, e) == RC_OK)
        cand.push_back(k);
    }
    g_err.clear();
    // most blocks (most partial-image bytes) first: under an HBM budget the
    // batch shrinks there until it fits, and every later candidate fits too
    std::sort(cand.begin(), cand.end(), [](int x, int y) { return x > y; });
    int n = copies;
    std::vector<float> med(cand.size());
    for (size_t j = 0; j < cand.size(); ++j) {
      p->tuned[key] = cand[j];
      float t[3];
      for (int run = 0; run < 4; ++run) {
        const hipError_t e0 = hipEventRecord(ev.a, hs);
        rc_status st = e0 == hipSuccess ? rc_process_batch(p, f, n, stream)
                                        : fail(RC_EHIP, "tuning: %s", hipGetErrorString(e0));
        if (st == RC_ENOTREADY && n > 1 && j == 0 && run == 0) {  // nothing was enqueued
          g_err.clear();
          --n;
          --run;
          continue;
        }
        if (st == RC_OK) {
          hipError_t e = hipEventRecord(ev.b, hs);
          if (e == hipSuccess) e = hipEventSynchronize(ev.b);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.a, ev.b);
          for (int k = 0; k < n; ++k) {
            const rc_status rel = rc_frame_release(p, ids[k]);
            if (st == RC_OK) st = rel;
          }
          if (e != hipSuccess) st = fail(RC_EHIP, "tuning: %s", hipGetErrorString(e));
          if (run > 0) t[run - 1] = ms / n;
        }
        if (st != RC_OK) {
          p->tuned.erase(key);
          return st;
        }
      }
      std::sort(t, t + 3);
      med[j] = t[1];
    }
    const size_t i0 = (size_t)(std::find(cand.begin(), cand.end(), k0) - cand.begin());
    size_t best = i0;
    for (size_t j = 0; j < cand.size(); ++j)
      if (med[j] < 0.98f * med[i0] && med[j] < med[best]) best = j;
    p->tuned[key] = cand[best];
    out[c] = rc_tuning_entry{key[0], key[1], key[2], key[3], cand[best], k0, med[i0], med[best]};
  }
  return RC_OK;
}

rc_status rc_plan_destroy(void* plan) {
  Plan* p = static_cast<Plan*>(plan);
  if (!p) return fail(RC_EINVAL, "plan is NULL");
  for (Slot& s : p->slots)
    if (s.busy && s.done) (void)hipEventSynchronize(s.done);
  free_plan(p);
  return RC_OK;
}

const char* rc_last_error(void) { return g_err.c_str(); }

rc_status rc_grid_cartesian(double x0, double dx, int32_t nx, double y0, double dy, int32_t ny, float* xy) {
  if (nx < 1 || ny < 1 || !xy) return fail(RC_EINVAL, "bad grid arguments");
  for (int32_t iy = 0; iy < ny; ++iy)
    for (int32_t ix = 0; ix < nx; ++ix) {
      const size_t i = (size_t)iy * nx + ix;
      xy[2 * i] = (float)(x0 + ix * dx);
      xy[2 * i + 1] = (float)(y0 + iy * dy);
    }
  return RC_OK;
}

rc_status rc_grid_polar_params(const rc_radar* radar, double x0, double x1, double y0, double y1,
                               double ox, double oy, double aperture_len, double factor, double* out6) {
  if (!radar || !out6 || !(x1 >= x0) || !(y1 >= y0) || !(y0 > oy) || !(aperture_len > 0) || !(factor > 0) ||
      !(radar->bandwidth > 0) || !(radar->f0 > 0))
    return fail(RC_EINVAL, "bad polar grid arguments");
  const double c = radar->c > 0 ? radar->c : 299792458.0;
  const double lam = c / radar->f0;
  const double dr = c / (2.0 * radar->bandwidth) / factor;
  const double dth = lam / (2.0 * aperture_len) / factor;
  const double xs[2] = {x0 - ox, x1 - ox}, ys[2] = {y0 - oy, y1 - oy};
  const double cx = std::min(std::max(0.0, xs[0]), xs[1]);
  const double r_min = std::hypot(cx, ys[0]);
  double r_max = 0, th_min = INFINITY, th_max = -INFINITY;
  for (double x : xs)
    for (double y : ys) {
      r_max = std::max(r_max, std::hypot(x, y));
      const double th = std::atan2(x, y);
      th_min = std::min(th_min, th);
      th_max = std::max(th_max, th);
    }
  out6[0] = r_min;
  out6[1] = dr;
  out6[2] = th_min;
  out6[3] = dth;
  out6[4] = std::floor((r_max - r_min) / dr) + 1;
  out6[5] = std::floor((th_max - th_min) / dth) + 1;
  return RC_OK;
}

rc_status rc_grid_polar(double ox, double oy, double r0, double dr, int32_t nr, double th0, double dth,
                        int32_t nth, float* xy) {
  if (nr < 1 || nth < 1 || !xy) return fail(RC_EINVAL, "bad grid arguments");
  for (int32_t it = 0; it < nth; ++it) {
    const double th = th0 + it * dth;
    const double s = std::sin(th), c = std::cos(th);
    for (int32_t ir = 0; ir < nr; ++ir) {
      const double r = r0 + ir * dr;
      const size_t i = (size_t)it * nr + ir;
      xy[2 * i] = (float)(ox + r * s);
      xy[2 * i + 1] = (float)(oy + r * c);
    }
  }
  return RC_OK;
}

rc_status rc_resample_polar(const void* polar_image, int32_t nth, int32_t nr, double ox, double oy,
                            double r0, double dr, double th0, double dth, const void* points,
                            int64_t n_points, void* out, void* stream) {
  if (n_points < 0) return fail(RC_EINVAL, "n_points must be >= 0");
  if (n_points == 0) return RC_OK;
  if (!polar_image || !points || !out) return fail(RC_EINVAL, "image, points and out are required");
  if (nth < 1 || nr < 1) return fail(RC_EINVAL, "need nth >= 1 and nr >= 1");
  if (!(dr > 0) || !(dth > 0) || !std::isfinite(dr) || !std::isfinite(dth) || !std::isfinite(r0) ||
      !std::isfinite(th0) || !std::isfinite(ox) || !std::isfinite(oy))
    return fail(RC_EINVAL, "lattice parameters must be finite with dr, dth > 0");
  rc::ResampleArgs a{static_cast<const float2*>(polar_image), nth, nr, ox, oy, r0, dr, th0, dth,
                     static_cast<const float2*>(points), n_points, static_cast<float*>(out)};
  RC_HIP(rc::launch_resample_polar(a, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

}  // extern "C"
