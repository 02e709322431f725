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
// recheck_pixels_kernel: one workgroup per (listed cell, window offset), the
// terms (chirp, channel) split over the 256 lanes and summed by a fixed tree,
// so every recomputed power is deterministic.  recheck_decide_kernel: one lane
// per listed cell.
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

__global__ __launch_bounds__(kThreads) void recheck_pixels_kernel(RecheckArgs a) {
  __shared__ double red_re[kThreads];
  __shared__ double red_im[kThreads];
  const int win = 2 * a.half + 1;
  const int n_off = win * win;
  const int count = min(*a.n_listed, a.cap);
  const int64_t n_work = (int64_t)count * n_off;
  const int rows = a.n_chirps * a.n_ch;
  for (int64_t wi = blockIdx.x; wi < n_work; wi += gridDim.x) {
    const int slot = (int)(wi / n_off);
    const int o = (int)(wi - (int64_t)slot * n_off);
    const int dr = o / win - a.half, dc = o % win - a.half;
    const bool guard = (dr >= -a.guard && dr <= a.guard && dc >= -a.guard && dc <= a.guard) && (dr || dc);
    if (guard) continue;  // uniform over the workgroup
    const int cell = a.listed[slot];
    const int r = cell / a.n_cols + dr, c = cell % a.n_cols + dc;  // inside: tested cells have full windows
    const float2 pf = a.pix[(int64_t)r * a.n_cols + c];
    const double px = pf.x, py = pf.y;
    const double h2 = a.height * a.height;
    double fd = 0.0;
    if (a.fd_in) {
      fd = (double)a.fd_in[(int64_t)r * a.n_cols + c];
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
    if (threadIdx.x == 0) a.power[(int64_t)slot * n_off + o] = red_re[0] * red_re[0] + red_im[0] * red_im[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void recheck_decide_kernel(RecheckArgs a) {
  const int win = 2 * a.half + 1;
  const int n_off = win * win;
  const int count = min(*a.n_listed, a.cap);
  for (int slot = blockIdx.x * kThreads + threadIdx.x; slot < count; slot += gridDim.x * kThreads) {
    const double* pw = a.power + (int64_t)slot * n_off;
    double train = 0.0;
    for (int o = 0; o < n_off; ++o) {
      const int dr = o / win - a.half, dc = o % win - a.half;
      if (dr >= -a.guard && dr <= a.guard && dc >= -a.guard && dc <= a.guard) continue;
      train += pw[o];
    }
    const double thr = a.alpha_over_n * train;
    const double p = pw[a.half * win + a.half];
    const int cell = a.listed[slot];
    const int r = cell / a.n_cols, c = cell % a.n_cols;
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
  const int win = 2 * a.half + 1;
  int64_t grid = (int64_t)a.cap * win * win;
  if (grid > 8192) grid = 8192;  // grid-stride over the listed cells (count known on the device only)
  hipLaunchKernelGGL(recheck_pixels_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t g2 = (a.cap + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(recheck_decide_kernel, dim3((unsigned)g2), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace rc
