// Range compression: beat signal -> equidistant beat spectrum s (the input
// that Alg. 1 and Alg. 2 interpolate; Sec. III-C of the paper).
//
// s[row][k] = sum_{t < n_s} w_range[t] raw[row][t] exp(-2 pi i k t / n_fft),
// k < n_bins, computed as an n_fft-point FFT of the zero-padded row.
//
// Design (HBM-bound stage): each row is read once with coalesced loads,
// windowed on the fly and scattered in bit-reversed order into LDS; the
// decimation-in-time butterflies run in LDS two radix-2 stages at a time
// (four elements per thread, one barrier per pair of stages); only the n_bins
// kept bins are written, directly in the interleaved (value, slope) layout
// that back-projection gathers with one 16-byte load per term, with the chirp
// window w_sar[m] folded in.  Rows shorter than a wave share a workgroup.
#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }

__global__ __launch_bounds__(kThreads) void range_compress_kernel(RangeArgs a, int tpr) {
  extern __shared__ float2 lds[];
  const int n = a.n_fft;
  const int rows_per_wg = kThreads / tpr;
  const int lrow = threadIdx.x / tpr;
  const int t = threadIdx.x - lrow * tpr;
  const int64_t row = (int64_t)blockIdx.x * rows_per_wg + lrow;
  const bool live = row < a.rows;
  float2* buf = lds + (size_t)lrow * n;

  // zero-padding: clear the row buffer, then scatter the windowed samples to
  // their bit-reversed positions
  for (int k = t; k < n; k += tpr) buf[k] = make_float2(0.f, 0.f);
  __syncthreads();
  if (live) {
    const float2* src = a.raw + row * a.n_s;
    const int sh = 32 - a.log2n;
    for (int k = t; k < a.n_s; k += tpr) {
      const float2 x = src[k];
      const float w = a.w_range[k];
      buf[__builtin_bitreverse32((unsigned)k) >> sh] = make_float2(x.x * w, x.y * w);
    }
  }
  __syncthreads();

  // odd log2(n): one size-2 stage (twiddle 1)
  int h = 1;
  if (a.log2n & 1) {
    for (int g = t; g < n / 2; g += tpr) {
      const float2 u = buf[2 * g], v = buf[2 * g + 1];
      buf[2 * g] = cadd(u, v);
      buf[2 * g + 1] = csub(u, v);
    }
    h = 2;
    __syncthreads();
  }
  // pairs of stages: sizes 2h (half h) and 4h (half 2h)
  for (; h < n; h *= 4) {
    const int shA = a.tw_log2 - __builtin_ctz(2 * h);  // W_{2h}^j = tw[j << shA]
    const int shB = a.tw_log2 - __builtin_ctz(4 * h);  // W_{4h}^j = tw[j << shB]
    for (int g = t; g < n / 4; g += tpr) {
      const int j = g & (h - 1);
      const int base = (g - j) * 4 + j;
      const float2 wA = a.twiddle[j << shA];
      const float2 wB = a.twiddle[j << shB];
      const float2 x0 = buf[base], x1 = buf[base + h], x2 = buf[base + 2 * h], x3 = buf[base + 3 * h];
      const float2 t1 = cmul(wA, x1), t3 = cmul(wA, x3);
      const float2 b0 = cadd(x0, t1), b1 = csub(x0, t1);
      const float2 b2 = cadd(x2, t3), b3 = csub(x2, t3);
      const float2 u2 = cmul(wB, b2);
      const float2 u3 = cmul_mi(cmul(wB, b3));            // W_{4h}^{j+h} = -i W_{4h}^j
      buf[base] = cadd(b0, u2);
      buf[base + 2 * h] = csub(b0, u2);
      buf[base + h] = cadd(b1, u3);
      buf[base + 3 * h] = csub(b1, u3);
    }
    __syncthreads();
  }

  if (!live) return;
  const float w = a.w_sar[row / a.n_ch];
  float4* dst = a.pairs + row * a.n_bins;
  float2* spec = a.spectrum ? a.spectrum + row * a.n_bins : nullptr;
  const int last = a.n_bins - 1;
  for (int k = t; k < a.n_bins; k += tpr) {
    const float2 x = buf[k];
    const float2 d = (k < last) ? csub(buf[k + 1], x) : make_float2(0.f, 0.f);
    dst[k] = make_float4(w * x.x, w * x.y, w * d.x, w * d.y);
    if (spec) spec[k] = x;
  }
}

__global__ __launch_bounds__(kThreads) void spectrum_pairs_kernel(PairArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t total = a.rows * a.n_bins;
  if (i >= total) return;
  const int64_t row = i / a.n_bins;
  const int k = (int)(i - row * a.n_bins);
  const float w = a.w_sar[row / a.n_ch];
  const float2 x = a.spec[i];
  const float2 d = (k < a.n_bins - 1) ? csub(a.spec[i + 1], x) : make_float2(0.f, 0.f);
  a.pairs[i] = make_float4(w * x.x, w * x.y, w * d.x, w * d.y);
}

}  // namespace

hipError_t launch_range_compress(const RangeArgs& a, hipStream_t s) {
  if (a.rows <= 0) return hipSuccess;
  if (a.n_fft < 4 || (a.n_fft & (a.n_fft - 1)) || (1 << a.log2n) != a.n_fft || a.n_fft > 4096 ||
      a.n_s < 1 || a.n_s > a.n_fft || a.n_bins < 1 || a.n_bins > a.n_fft || a.n_ch < 1 ||
      a.tw_log2 < a.log2n || a.tw_log2 > 12)
    return hipErrorInvalidValue;
  int tpr = a.n_fft / 4;
  if (tpr > kThreads) tpr = kThreads;
  const int rows_per_wg = kThreads / tpr;
  const int64_t grid = (a.rows + rows_per_wg - 1) / rows_per_wg;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = (size_t)rows_per_wg * a.n_fft * sizeof(float2);
  hipLaunchKernelGGL(range_compress_kernel, dim3((unsigned)grid), dim3(kThreads), lds, s, a, tpr);
  return hipGetLastError();
}

hipError_t launch_spectrum_pairs(const PairArgs& a, hipStream_t s) {
  const int64_t total = a.rows * a.n_bins;
  if (total <= 0) return hipSuccess;
  if (a.n_ch < 1) return hipErrorInvalidValue;
  const int64_t grid = (total + kThreads - 1) / kThreads;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(spectrum_pairs_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace rc
