// Internal interface between the C-ABI runtime (runtime.hip) and the HIP
// kernels of librc.so.  Plain structs of device pointers and sizes; each
// launch_* function checks the launch shape it derives against the buffers
// described by its argument struct and returns a hipError_t.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rc.h"

namespace rc {

// Range compression (beat signal -> beat spectrum): windowed, zero-padded
// radix-2 decimation-in-time FFT per (chirp, channel) row in LDS, cropped to
// n_bins.  Writes the interpolation table of back-projection: for bin k the
// float4 (w s[k], w (s[k+1] - s[k])) with w = w_sar[row / n_ch] and a zero
// slope for the last kept bin; optionally also the plain spectrum s.
struct RangeArgs {
  const float2* raw;      // [rows][n_s]
  const float* w_range;   // [n_s]
  const float* w_sar;     // [n_chirps]
  const float2* twiddle;  // [n_fft_max / 2], exp(-2 pi i k / n_fft_max)
  int tw_log2;            // log2(n_fft_max)
  float4* pairs;          // [rows][n_bins]
  float2* spectrum;       // [rows][n_bins] or nullptr
  int64_t rows;
  int n_s, n_fft, log2n, n_bins, n_ch;
};
hipError_t launch_range_compress(const RangeArgs& a, hipStream_t s);

// Caller-supplied spectrum -> interpolation table (same layout as above).
struct PairArgs {
  const float2* spec;     // [rows][n_bins]
  const float* w_sar;     // [n_chirps]
  float4* pairs;          // [rows][n_bins]
  int64_t rows;
  int n_bins, n_ch;
};
hipError_t launch_spectrum_pairs(const PairArgs& a, hipStream_t s);

// Per-pixel tables, evaluated in double and rounded once:
//  * f_doppler(p) in bins from the mean velocity at the aperture centre;
//  * the pixel in aperture-local wavelength units, P = (p - c) / lambda, as
//    float4 (P'.x, P'.y, pp, corr) with P' = float(P), pp = float(|P|^2) and
//    corr = (|P|^2 - pp) / |P|, the first-order path correction (in turns) for
//    the rounding of pp that back-projection adds to every two-way path.
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
  double a1;                      // bins per wavelength of path
  float* fbase;                   // [n_pix] (split only)
};
hipError_t launch_pixel_tables(const TableArgs& a, hipStream_t s);

// Back-projection (Alg. 2).  One lane per pixel; a wave covers an 8 x 8 block
// of the lattice (or 1 x 64 for single-row lattices); channels that share a
// TX position in every chirp form groups of chg channels whose d_tx is
// evaluated once.  Distances are in wavelengths (a path of d_hyp wavelengths
// has the carrier phase -2 pi d_hyp), squared distances are formed as
// pp + |q|^2 - 2 P.q from per-row uniforms.
struct BpArgs {
  const float4* pixc;     // [n_rows * n_cols]: (P.x, P.y, |P|^2, corr), wavelengths
  const float* fd;        // [n_rows * n_cols], bins
  const float4* pairs;    // [n_chirps * n_ch][n_bins]
  const float4* rowq;     // [n_chirps * n_ch]: (-2 q_rx.x, -2 q_rx.y, |q_rx|^2, 0)
  const float4* grpq;     // [n_chirps * n_ch / chg]: (-2 q_tx.x, -2 q_tx.y, |q_tx|^2, 0)
  float2* out;            // [n_rows * n_cols]
  const float* fbase;     // split form: [n_rows * n_cols] index of the reference path
  int split;              // 0: plain single precision; 1: split phase (see tables)
  int n_chirps, n_ch, n_bins, chg;
  int n_rows, n_cols;
  float a1;               // bins per wavelength of two-way path
  // bounding boxes of all TX / RX positions (wavelengths, local frame) and
  // the index margin that lets a wave skip the per-term range test when every
  // term is provably in range
  float tx_lo_x, tx_lo_y, tx_hi_x, tx_hi_y;
  float rx_lo_x, rx_lo_y, rx_hi_x, rx_hi_y;
  float f_margin;
};
hipError_t launch_backproject(const BpArgs& a, hipStream_t s);

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
};
hipError_t launch_cfar(const CfarArgs& a, hipStream_t s);

// Ordered compaction of the detection mask into det_out[0, cap) and count.
struct CompactArgs {
  const unsigned long long* mask;
  const rc_detection* det_cell;
  int n_rows, n_cols, words_per_row;
  rc_detection* det_out;
  int64_t cap;
  int64_t* count;
};
hipError_t launch_compact(const CompactArgs& a, hipStream_t s);

}  // namespace rc
