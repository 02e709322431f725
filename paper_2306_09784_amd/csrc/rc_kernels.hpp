// Internal interface between the C-ABI runtime (runtime.hip) and the HIP
// kernels of librc.so.  Plain structs of device pointers and sizes; each
// launch_* function checks the launch shape it derives against the buffers
// described by its argument struct and returns a hipError_t.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rc.h"

namespace rc {

// Many frames in one launch: the launcher lays the workgroups of frame i out
// as [begin[i], begin[i + 1]) and each workgroup finds its frame by a scan over
// these (uniform) bounds, then reads that frame's arguments by value.
template <class A, int MAXF>
struct Multi {
  static constexpr int kMax = MAXF;
  int n_frames = 0;
  int begin[MAXF + 1] = {};
  A f[MAXF];
};

template <class M>
__device__ __forceinline__ int multi_frame(const M& m, int w) {
  int fi = 0;
  while (fi + 1 < m.n_frames && w >= m.begin[fi + 1]) ++fi;
  return __builtin_amdgcn_readfirstlane(fi);
}

// Entry k of back-projection's interpolation table (one row: one chirp and
// channel).  On the segment from bin k to k + 1 the windowed spectrum is
// w s[k] + (f - k) w (s[k+1] - s[k]) = A + f D with D = w (s[k+1] - s[k]) and
// A = w s[k] - k D, so a term at fractional bin index f in [k, k + 1] costs
// one FMA per component with f itself: no fraction of f is formed.  The last
// kept bin has D = 0.  A is rounded once (from w s[k] and k D); its error,
// half an ulp of about k |D|, is of the size of the rounding that f already
// carries at bin k.
__device__ __forceinline__ float4 table_entry(float w, float2 s, float2 d, int k) {
  const float dx = w * d.x, dy = w * d.y, kf = (float)k;
  return make_float4(fmaf(-kf, dx, w * s.x), fmaf(-kf, dy, w * s.y), dx, dy);
}

// Per-frame geometry from mapped pinned host memory (src, the device address
// of the staging buffer) to device memory, n16 16-byte units.
struct UploadArgs {
  float4* dst;
  const float4* src;
  int64_t n16;
};
using UploadMulti = Multi<UploadArgs, 32>;
hipError_t launch_upload(const UploadMulti& m, hipStream_t s);

// Range compression (beat signal -> beat spectrum): windowed, zero-padded
// radix-2 decimation-in-time FFT per (chirp, channel) row in LDS, cropped to
// n_bins.  Writes the interpolation table of back-projection (table_entry
// below); optionally also the plain spectrum s.
struct RangeArgs {
  const float2* raw;      // [rows][n_s]
  const float* w_range;   // [n_s]
  const float* w_sar;     // [n_chirps]
  float4* pairs;          // [rows][n_bins]
  float2* spectrum;       // [rows][n_bins] or nullptr
  int64_t rows;
  int n_s, n_fft, log2n, n_bins, n_ch;
};
// every frame of one launch has the same n_fft
using RangeMulti = Multi<RangeArgs, 32>;
hipError_t launch_range_compress(const RangeMulti& m, hipStream_t s);

// The same table from range compression on the matrix cores (FP16 or BF16
// operands, FP32 accumulation, split twiddles; range_mfma.hip).  Takes DFT
// lengths kRangeMfmaMinFft .. kRangeMfmaMaxFft with n_s <= n_fft / 2.
constexpr int kRangeMfmaMinFft = 256;
constexpr int kRangeMfmaMaxFft = 4096;
bool range_mfma_supported(int n_fft, int n_s);
hipError_t launch_range_mfma(const RangeMulti& m, bool bf16, hipStream_t s);

// Caller-supplied spectrum -> interpolation table (same layout as above).
struct PairArgs {
  const float2* spec;     // [rows][n_bins]
  const float* w_sar;     // [n_chirps]
  float4* pairs;          // [rows][n_bins]
  int64_t rows;
  int n_bins, n_ch;
};
using PairMulti = Multi<PairArgs, 32>;
hipError_t launch_spectrum_pairs(const PairMulti& m, hipStream_t s);

// Per-pixel tables, evaluated in double and rounded once (h: the antenna
// height above the pixel plane in wavelengths, 0 for planar geometry; R^2 =
// |P|^2 + h^2 the squared distance to the aperture centre):
//  * f_doppler(p) in bins from the mean velocity at the aperture centre;
//  * the pixel in aperture-local wavelength units, P = (p - c) / lambda, as
//    float4 (P'.x, P'.y, pp, corr) with P' = float(P), pp = float(R^2) and
//    corr = (R^2 - pp) / R, the first-order path correction (in turns) for
//    the rounding of pp that back-projection adds to every two-way path;
//  * exact-Doppler form: (P'.x, P'.y, h^2, corr) with corr = 2 <P, P - P'> / R,
//    the first-order correction for the rounding of P itself; the direct form
//    (exact == 2) the same in metres.
struct TableArgs {
  const float2* pix;
  int64_t n_pix;
  double qt_x, qt_y, qr_x, qr_y;  // mean TX / RX positions
  double v_x, v_y;                // mean velocity
  double kd;                      // f0 / (c df): bins per m/s of radial speed
  double c_x, c_y;                // aperture centre (origin of the local frame)
  double inv_lam;                 // 1 / lambda
  float* fd;                      // [n_pix]
  float4* pixc;                   // [n_pix]
  // split-phase form: pixc = (P'.x, P'.y, R, frac(2R)) with R = |P| and
  // fbase = a1 * 2R + f_doppler (the index of the reference path 2R)
  int split;
  int exact;                      // 1: exact-Doppler form, 2: direct form (metres)
  double a1;                      // bins per wavelength of path
  float* fbase;                   // [n_pix] (split only)
  double height;                  // antennas above the pixel plane, metres
  const float* fd_in;             // [n_pix] caller's f_doppler (bins) or nullptr
};
using TableMulti = Multi<TableArgs, 16>;
hipError_t launch_pixel_tables(const TableMulti& m, hipStream_t s);

// Back-projection (Alg. 2).  One lane per pixel; a wave covers an 8 x 8 block
// of the lattice (or 1 x 64 for single-row lattices); channels that share a
// TX position in every chirp form groups of chg channels whose d_tx is
// evaluated once.  Distances are in wavelengths (a path of d_hyp wavelengths
// has the carrier phase -2 pi d_hyp), squared distances are formed as
// |P|^2 + |q|^2 - 2 P.q from per-row uniforms.
//
// A launch processes a batch of frames that share chg and the precision form.
// Work items are (frame, chirp block, 16 x 16 pixel tile); every frame is
// spread over all eight XCDs, each XCD taking a contiguous eighth of its
// items (so one frame's neighbouring tiles share that XCD's L2 while the
// frames of a batch stay balanced over the XCDs); a frame too small
// to fill the GPU splits its chirp sum into n_kb blocks whose partial images
// are summed afterwards in block order (reduce_partials), so every frame's
// result depends only on its own sizes, never on the rest of the batch.
struct BpFrame {
  const float4* pixc;     // [n_pix]: (P.x, P.y, |P|^2, corr) or split (P.x, P.y, R, frac 2R)
  const float* fidx;      // [n_pix]: f_doppler (plain) or index of the path 2R (split)
  const float4* pairs;    // [n_chirps * n_ch][n_bins]
  const float4* rowq;     // [n_chirps * n_ch]: (-2 q_rx.x, -2 q_rx.y, |q_rx|^2, 0)
  const float4* grpq;     // [n_chirps * n_ch / chg]: (-2 q_tx.x, -2 q_tx.y, |q_tx|^2, 0)
  // exact-Doppler form (Alg. 1): per row (q_rx.x, q_rx.y, kd v.x, kd v.y) and
  // per TX group (q_tx.x, q_tx.y, kd v.x, kd v.y); kd v in bins per unit radial
  // speed, so <P - q, kd v> / |P - q| is the Doppler index shift of one leg
  const float4* rowv;
  const float4* grpv;
  // sub-aperture form (sums == 3): per chirp (cos, sin) of its window phase;
  // the launch accumulates the plain sum and the two weighted sums
  const float2* roww;     // [n_chirps]
  float2* out;            // [n_kb][sums][n_pix]: image(s) (n_kb == 1) or partial images
  int n_chirps, n_ch, n_bins;
  int n_rows, n_cols;
  int n_kb;               // chirp blocks
  int kb0, kb_count;      // the blocks this launch evaluates: [kb0, kb0 + kb_count)
  int tiles_x, n_tiles;   // workgroup tiles per chirp block
  // each XCD takes a contiguous chunk of ceil(kb_count n_tiles / 8) of the
  // frame's items; slot_base is the frame's first per-XCD slot in the launch
  int chunk, slot_base;
  float a1;               // bins per wavelength of two-way path
  // bounding boxes of all TX / RX positions (wavelengths, local frame) and
  // the index margin that lets a wave skip the per-term range test when every
  // term is provably in range
  float tx_lo_x, tx_lo_y, tx_hi_x, tx_hi_y;
  float rx_lo_x, rx_lo_y, rx_hi_x, rx_hi_y;
  float f_margin;
  float f_slack;          // largest |Doppler index| a term can carry (exact form)
  float h2;               // (antenna height / wavelength)^2 (0: planar geometry)
  float q_max;            // largest antenna distance from the aperture centre (wavelengths)
  // direct form (Alg. 1 as stated): rows and pixels in metres, velocities in
  // m/s, and the constants it divides by and multiplies with
  float lit_c, lit_mu, lit_f0, lit_df;
};

constexpr int kBpMaxFrames = 16;  // frames per launch (descriptors travel as kernel arguments)

enum BpForm { kBpPlain = 0, kBpSplit = 1, kBpExact = 2, kBpDirect = 3 };

struct BpBatch {
  int chg, form, n_frames, n_slots;  // n_slots: per-XCD slots (grid = 8 n_slots)
  int sums;                          // 1, or 3 for sub-apertures under a Hann window
  BpFrame f[kBpMaxFrames];
};
hipError_t launch_backproject(const BpBatch& b, hipStream_t s);

// Chirp blocks a frame of n_rows x n_cols pixels, n_chirps chirps and n_ch
// channels, whose blocks write `planes` partial images each, is split into,
// so that a launch of it alone has enough waves to fill the GPU: about
// kBpTargetGenerations x 8192 waves (the resident waves of the chip), at most
// 16 blocks and at least planes x kBpMinBlockRows rows (chirps x channels) per
// block where one generation stays filled, so k blocks of W waves each
// satisfy k <= min(16, ceil(T 8192 / W)).
constexpr int kBpTargetGenerations = 10;
constexpr int kBpMinBlockRows = 512;
int bp_chirp_blocks(int64_t n_rows, int64_t n_cols, int n_chirps, int n_ch, int planes);
// Number of work items (workgroups) of one chirp block of a frame.
void bp_tiles(int n_rows, int n_cols, int* tiles_x, int* n_tiles);

struct ReduceFrame {
  const float2* partial;  // [n_kb][n_pix]
  float2* out;            // [n_pix]
  int64_t n_pix;
  int n_kb;
};
constexpr int kReduceMaxFrames = 32;
struct ReduceBatch {
  int n_frames;
  ReduceFrame f[kReduceMaxFrames];
};
hipError_t launch_reduce_partials(const ReduceBatch& b, hipStream_t s);

// Aperture image of a continuous-SAR stream from the partial images of its
// last n_blk sub-apertures, kept in a ring of n_ring slots of
// [planes][n_pix] complex64 each (slot stride `stride` elements), oldest
// first from slot `first`:
//   out = sum_t (c0 S0_t + cc Sc_t + cs Ss_t)   (planes == 3)
//   out = sum_t S0_t                            (planes == 1)
struct CombineFrame {
  const float2* ring;
  int64_t stride;
  int n_ring, first, n_blk, planes;
  float c0, cc, cs;
  float2* out;
  int64_t n_pix;
};
constexpr int kCombineMaxFrames = 32;
struct CombineBatch {
  int n_frames;
  CombineFrame f[kCombineMaxFrames];
};
hipError_t launch_combine(const CombineBatch& b, hipStream_t s);

// 2-D CA-CFAR on |P|^2 (double) over the lattice.  mask holds one 64-bit word
// per 64 columns of a row; det_cell receives the record of every detection at
// its cell index.
struct CfarArgs {
  const float2* img;      // [n_rows][n_cols]
  int n_rows, n_cols, guard, train;
  double alpha_over_n;    // alpha / N_train
  double margin_rel;
  unsigned long long* mask;  // [n_rows][words_per_row]
  int words_per_row;
  rc_detection* det_cell;    // [n_rows * n_cols]
  // near-threshold cells are appended to listed[0, recheck_cap) (count in
  // *n_listed, which may exceed the capacity) for the double-precision
  // recheck; recheck_cap == 0 only flags them RC_DET_NEAR_THRESHOLD
  int* listed;
  int* n_listed;
  int recheck_cap;
};
using CfarMulti = Multi<CfarArgs, 16>;
hipError_t launch_cfar(const CfarMulti& m, hipStream_t s);

// Double-precision recheck of the listed cells (see recheck.hip).
struct RecheckArgs {
  const int* listed;
  const int* n_listed;
  int cap;
  int n_rows, n_cols, half, guard;   // half = guard + train
  double alpha_over_n;
  const float2* pix;        // pixel positions (metres)
  const float4* geo;        // [rows]: (q_tx.x, q_tx.y, q_rx.x, q_rx.y), metres
  const float2* vel;        // [n_chirps] velocity (exact form)
  const double2* spec;      // [rows][n_bins] beat spectrum in double
  const double* w_sar;      // [n_chirps] chirp window in double
  int n_chirps, n_ch, n_bins, exact;
  double a1;                // bins per metre of two-way path
  double kd;                // bins per m/s of radial speed
  double inv_lam;           // turns per metre of path
  double qt_x, qt_y, qr_x, qr_y, v_x, v_y;  // mean TX and RX positions and mean velocity (Doppler table)
  double height;            // antennas above the pixel plane, metres
  const float* fd_in;       // [n_pix] caller's f_doppler (bins) or nullptr
  // the pixels the listed windows need, each formed once: a bitmap in the
  // mask's layout, the list of needed pixels (ascending), and per pixel its
  // place in that list
  unsigned long long* need;  // [n_rows][words_per_row]
  int* plist;               // [cap * (2 half + 1)^2]
  int* map;                 // [n_rows * n_cols]
  int* n_need;
  double* power;            // [cap * (2 half + 1)^2]: power of plist[i]
  unsigned long long* mask;
  int words_per_row;
  rc_detection* det_cell;
};
hipError_t launch_recheck(const RecheckArgs& a, hipStream_t s);

// Beat spectrum in double for the recheck: from the raw cube by a double FFT
// (raw != nullptr) or widened from a complex64 spectrum input.
struct Range64Args {
  const float2* raw;          // [rows][n_s] or nullptr
  const float2* spectrum_in;  // [rows][n_bins] when raw == nullptr
  const double* w_range;      // [n_s]
  const double2* twiddle;     // exp(-2 pi i k / 2^tw_log2), k < 2^(tw_log2 - 1)
  int tw_log2;
  double2* spec;              // [rows][n_bins]
  int64_t rows;
  int n_s, n_fft, log2n, n_bins;
};
hipError_t launch_range64(const Range64Args& a, hipStream_t s);
// *count = 0 by a one-lane kernel (stream-ordered, capturable)
hipError_t launch_clear_count(int* count, hipStream_t s);

// Ordered compaction of the detection mask into det_out[0, cap) and count.
struct CompactArgs {
  const unsigned long long* mask;
  const rc_detection* det_cell;
  int n_rows, n_cols, words_per_row;
  rc_detection* det_out;
  int64_t cap;
  int64_t* count;
  // optional: the count and the first host_cap records also go straight to
  // mapped, coherent pinned host memory (device addresses), so no copy is
  // needed to read them on the host
  int64_t* host_count;
  rc_detection* host_out;
  int64_t host_cap;
};
using CompactMulti = Multi<CompactArgs, 32>;
hipError_t launch_compact(const CompactMulti& m, hipStream_t s);

// Magnitude of a polar-grid image [nth][nr] at n points (metres), bilinear
// in (theta, r); zero outside the lattice.
struct ResampleArgs {
  const float2* img;
  int nth, nr;
  double ox, oy, r0, dr, th0, dth;
  const float2* pts;
  int64_t n;
  float* out;
};
hipError_t launch_resample_polar(const ResampleArgs& a, hipStream_t s);

}  // namespace rc
