// Double-precision recheck of near-threshold CFAR decisions.
//
// The detector compares |P|^2 with alpha / N times the training sum.  A cell
// whose single-precision statistic lies within the plan's margin of the
// threshold is listed by cfar_kernel; here its own pixel and every training
// pixel of its window are formed again by back-projection in double
// (Alg. 2, or Alg. 1 for exact-Doppler plans) from the antenna positions and
// pixel coordinates as given, the threshold is recomputed and the decision
// replaces the single-precision one.  Every input of that evaluation is
// double: the beat spectrum of the frame is formed again by a double-precision
// FFT (range64_kernel; a spectrum input is widened exactly), and the windows
// come from the host in double.
//
// Listed cells cluster around targets and their windows overlap, so every
// pixel some window needs is formed once: need_mark_kernel marks them in a
// bitmap, need_gather_kernel lists them in ascending order (and records each
// one's place), recheck_pixels_kernel forms one listed pixel per workgroup —
// the terms (chirp, channel) split over the 256 lanes and summed by a fixed
// tree, so every recomputed power is deterministic — and
// recheck_decide_kernel (one lane per listed cell) sums its window through
// the map in a fixed order.
#include <algorithm>

#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;

// distance from the antenna at q (h2 = squared height above the pixel plane)
// to the pixel, and the radial speed of a horizontal velocity along it
__device__ __forceinline__ double radial(double px, double py, double qx, double qy, double vx, double vy,
                                         double h2, double* d) {
  const double rx = px - qx, ry = py - qy;
  *d = sqrt(rx * rx + ry * ry + h2);
  return *d > 0.0 ? (rx * vx + ry * vy) / *d : 0.0;
}

// zeroes the need bitmap and the count of needed pixels
__global__ __launch_bounds__(kThreads) void need_clear_kernel(RecheckArgs a) {
  const int64_t n_words = (int64_t)a.n_rows * a.words_per_row;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n_words; i += (int64_t)gridDim.x * kThreads)
    a.need[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.n_need = 0;
}

// marks the cell and the training pixels of every listed cell's window
__global__ __launch_bounds__(kThreads) void need_mark_kernel(RecheckArgs a) {
  const int win = 2 * a.half + 1;
  const int n_off = win * win;
  const int count = min(*a.n_listed, a.cap);
  const int64_t n_work = (int64_t)count * n_off;
  for (int64_t wi = (int64_t)blockIdx.x * kThreads + threadIdx.x; wi < n_work; wi += (int64_t)gridDim.x * kThreads) {
    const int slot = (int)(wi / n_off);
    const int o = (int)(wi - (int64_t)slot * n_off);
    const int dr = o / win - a.half, dc = o % win - a.half;
    if ((dr >= -a.guard && dr <= a.guard && dc >= -a.guard && dc <= a.guard) && (dr || dc)) continue;
    const int cell = a.listed[slot];
    const int r = cell / a.n_cols + dr, c = cell % a.n_cols + dc;  // inside: tested cells have full windows
    atomicOr(a.need + (int64_t)r * a.words_per_row + c / 64, 1ull << (c % 64));
  }
}

// lists the marked pixels in ascending order (one workgroup: sweeps of 256 x 8
// words, a wave scan of the threads' counts and a scan of the four wave totals)
constexpr int kGatherWords = 8;
__global__ __launch_bounds__(kThreads) void need_gather_kernel(RecheckArgs a) {
  __shared__ int wave_sum[kThreads / 64];
  __shared__ int base_sh;
  const int64_t n_words = (int64_t)a.n_rows * a.words_per_row;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) base_sh = 0;
  __syncthreads();
  for (int64_t w0 = 0; w0 < n_words; w0 += (int64_t)kThreads * kGatherWords) {
    const int64_t wt = w0 + (int64_t)threadIdx.x * kGatherWords;
    unsigned long long word[kGatherWords];
    int total = 0;
#pragma unroll
    for (int k = 0; k < kGatherWords; ++k) {
      word[k] = wt + k < n_words ? a.need[wt + k] : 0ull;
      total += __popcll(word[k]);
    }
    int incl = total;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wave_sum[wave] = incl;
    __syncthreads();
    int pos = base_sh + incl - total;
    for (int k = 0; k < wave; ++k) pos += wave_sum[k];
#pragma unroll
    for (int k = 0; k < kGatherWords; ++k) {
      unsigned long long bits = word[k];
      if (!bits) continue;
      const int64_t w = wt + k;
      const int64_t r = w / a.words_per_row;
      const int64_t cb = (w - r * a.words_per_row) * 64;
      while (bits) {
        const int b = __ffsll((long long)bits) - 1;
        bits &= bits - 1;
        const int pixel = (int)(r * a.n_cols + cb + b);
        a.plist[pos] = pixel;
        a.map[pixel] = pos;
        ++pos;
      }
    }
    __syncthreads();
    if (threadIdx.x == kThreads - 1) base_sh = pos;
    __syncthreads();
  }
  if (threadIdx.x == 0) *a.n_need = base_sh;
}

__global__ __launch_bounds__(kThreads) void recheck_pixels_kernel(RecheckArgs a) {
  __shared__ double red_re[kThreads];
  __shared__ double red_im[kThreads];
  const int n_need = *a.n_need;
  const int rows = a.n_chirps * a.n_ch;
  for (int wi = blockIdx.x; wi < n_need; wi += gridDim.x) {
    const int pixel = a.plist[wi];
    const float2 pf = a.pix[pixel];
    const double px = pf.x, py = pf.y;
    const double h2 = a.height * a.height;
    double fd = 0.0;
    if (a.fd_in) {
      fd = (double)a.fd_in[pixel];
    } else if (!a.exact) {
      double d0;
      fd = a.kd * (radial(px, py, a.qt_x, a.qt_y, a.v_x, a.v_y, h2, &d0) +
                   radial(px, py, a.qr_x, a.qr_y, a.v_x, a.v_y, h2, &d0));
    }
    double acc_re = 0.0, acc_im = 0.0;
    for (int t = threadIdx.x; t < rows; t += kThreads) {
      const float4 q = a.geo[t];
      const int m = t / a.n_ch;
      const double w = a.w_sar[m];
      double d_tx, d_rx, f;
      if (a.exact) {
        const float2 v = a.vel[m];
        const double vt = radial(px, py, q.x, q.y, v.x, v.y, h2, &d_tx);
        const double vr = radial(px, py, q.z, q.w, v.x, v.y, h2, &d_rx);
        f = a.a1 * (d_tx + d_rx) + a.kd * (vt + vr);
      } else {
        const double tx = px - q.x, ty = py - q.y, rx = px - q.z, ry = py - q.w;
        d_tx = sqrt(tx * tx + ty * ty + h2);
        d_rx = sqrt(rx * rx + ry * ry + h2);
        f = a.a1 * (d_tx + d_rx) + fd;
      }
      if (!(f >= 0.0 && f <= (double)(a.n_bins - 1))) continue;
      // linear interpolation on the bin index; f = n_bins - 1 takes the last bin
      const double fl = floor(f);
      const int i = (int)fl;
      const double phi = f - fl;
      const double2* row = a.spec + (int64_t)t * a.n_bins;
      const double2 lo = row[i], hi = row[min(i + 1, a.n_bins - 1)];
      const double vre = w * ((1.0 - phi) * lo.x + phi * hi.x);
      const double vim = w * ((1.0 - phi) * lo.y + phi * hi.y);
      const double turns = (d_tx + d_rx) * a.inv_lam;
      double sn, cs;
      sincospi(2.0 * (turns - floor(turns)), &sn, &cs);
      acc_re += cs * vre + sn * vim;
      acc_im += cs * vim - sn * vre;
    }
    red_re[threadIdx.x] = acc_re;
    red_im[threadIdx.x] = acc_im;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        red_re[threadIdx.x] += red_re[threadIdx.x + s];
        red_im[threadIdx.x] += red_im[threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) a.power[wi] = red_re[0] * red_re[0] + red_im[0] * red_im[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void recheck_decide_kernel(RecheckArgs a) {
  const int win = 2 * a.half + 1;
  const int n_off = win * win;
  const int count = min(*a.n_listed, a.cap);
  for (int slot = blockIdx.x * kThreads + threadIdx.x; slot < count; slot += gridDim.x * kThreads) {
    const int cell = a.listed[slot];
    const int r = cell / a.n_cols, c = cell % a.n_cols;
    double train = 0.0;
    for (int o = 0; o < n_off; ++o) {
      const int dr = o / win - a.half, dc = o % win - a.half;
      if (dr >= -a.guard && dr <= a.guard && dc >= -a.guard && dc <= a.guard) continue;
      train += a.power[a.map[(int64_t)(r + dr) * a.n_cols + (c + dc)]];
    }
    const double thr = a.alpha_over_n * train;
    const double p = a.power[a.map[cell]];
    unsigned long long* word = a.mask + (int64_t)r * a.words_per_row + c / 64;
    const unsigned long long bit = 1ull << (c % 64);
    if (p > thr) {
      atomicOr(word, bit);
      rc_detection d;
      d.pixel = cell;
      d.power = (float)p;
      d.threshold = (float)thr;
      d.flags = RC_DET_RECHECKED;
      a.det_cell[cell] = d;
    } else {
      atomicAnd(word, ~bit);
    }
  }
}

constexpr int kFftThreads = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Windowed, zero-padded forward DFT of one (chirp, channel) row in double,
// first n_bins bins kept: radix-2 decimation in time in LDS after a
// bit-reversed scatter; twiddles exp(-2 pi i k / n_fft_max) from a table the
// host evaluates in double.
__global__ __launch_bounds__(kFftThreads) void range64_kernel(Range64Args a) {
  extern __shared__ double2 buf[];
  const int64_t row = blockIdx.x;
  const float2* x = a.raw + row * a.n_s;
  const int n = a.n_fft;
  for (int t = threadIdx.x; t < n; t += kFftThreads) {
    double2 v = make_double2(0.0, 0.0);
    if (t < a.n_s) {
      const float2 z = x[t];
      const double w = a.w_range[t];
      v = make_double2(w * z.x, w * z.y);
    }
    buf[__brev((unsigned)t) >> (32 - a.log2n)] = v;
  }
  __syncthreads();
  for (int lg = 1; lg <= a.log2n; ++lg) {
    const int half = 1 << (lg - 1);
    for (int j = threadIdx.x; j < n / 2; j += kFftThreads) {
      const int k = j & (half - 1);
      const int i0 = ((j >> (lg - 1)) << lg) + k, i1 = i0 + half;
      const double2 tw = a.twiddle[k << (a.tw_log2 - lg)];
      const double2 b = cmul(tw, buf[i1]);
      const double2 c = buf[i0];
      buf[i0] = make_double2(c.x + b.x, c.y + b.y);
      buf[i1] = make_double2(c.x - b.x, c.y - b.y);
    }
    __syncthreads();
  }
  double2* out = a.spec + row * a.n_bins;
  for (int k = threadIdx.x; k < a.n_bins; k += kFftThreads) out[k] = buf[k];
}

// Spectrum input: the complex64 samples widened to double.
__global__ void widen_kernel(const float2* in, double2* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float2 z = in[i];
    out[i] = make_double2(z.x, z.y);
  }
}

__global__ void clear_count_kernel(int* count) {
  if (threadIdx.x == 0) *count = 0;
}

}  // namespace

hipError_t launch_range64(const Range64Args& a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  if (a.n_bins < 1 || a.rows > 0x7fffffff) return hipErrorInvalidValue;
  if (a.raw) {
    if (a.log2n < 2 || a.log2n > 12 || a.n_fft != (1 << a.log2n) || a.log2n > a.tw_log2 || a.n_s < 1 ||
        a.n_s > a.n_fft || a.n_bins > a.n_fft)
      return hipErrorInvalidValue;
    hipLaunchKernelGGL(range64_kernel, dim3((unsigned)a.rows), dim3(kFftThreads),
                       (size_t)a.n_fft * sizeof(double2), s, a);
  } else {
    const int64_t n = a.rows * a.n_bins;
    const int64_t g = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(widen_kernel, dim3((unsigned)g), dim3(256), 0, s, a.spectrum_in, a.spec, n);
  }
  return hipGetLastError();
}

hipError_t launch_clear_count(int* count, hipStream_t s) {
  hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(64), 0, s, count);
  return hipGetLastError();
}

hipError_t launch_recheck(const RecheckArgs& a, hipStream_t s) {
  if (a.cap <= 0) return hipSuccess;
  if (a.half < 1 || a.half > 16 || a.guard < 0 || a.guard >= a.half || a.n_chirps < 1 || a.n_ch < 1 ||
      a.n_bins < 2 || a.n_cols < 1)
    return hipErrorInvalidValue;
  if (!a.need || !a.plist || !a.map || !a.n_need || !a.power || a.words_per_row != (a.n_cols + 63) / 64)
    return hipErrorInvalidValue;
  const int win = 2 * a.half + 1;
  const int64_t n_words = (int64_t)a.n_rows * a.words_per_row;
  const int64_t g0 = std::max<int64_t>(1, std::min<int64_t>((n_words + kThreads - 1) / kThreads, 1024));
  hipLaunchKernelGGL(need_clear_kernel, dim3((unsigned)g0), dim3(kThreads), 0, s, a);
  const int64_t g1 = std::min<int64_t>(((int64_t)a.cap * win * win + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(need_mark_kernel, dim3((unsigned)g1), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(need_gather_kernel, dim3(1), dim3(kThreads), 0, s, a);
  // grid-stride over the needed pixels (count known on the device only)
  int64_t grid = (int64_t)a.cap * win * win;
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(recheck_pixels_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t g2 = (a.cap + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(recheck_decide_kernel, dim3((unsigned)g2), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace rc
