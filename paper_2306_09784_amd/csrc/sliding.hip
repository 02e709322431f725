// Continuous SAR: the aperture image of a sensor's stream from the partial
// images of its last sub-apertures (the conclusion of the paper, Sec. V,
// argues that a continuous measurement can be imaged as it arrives).
//
// The chirp window of an aperture of N chirps starting at chirp a is
// w(m) = a0 - a1 cos(2 pi (m - a) / (N - 1)) (Hann: a0 = a1 = 1/2, Sec. III-B).
// With theta_m = 2 pi (m mod (N - 1)) / (N - 1) and phi = 2 pi (a mod (N - 1)) /
// (N - 1), cos(theta_m - phi) = cos theta_m cos phi + sin theta_m sin phi, so
//   sum_m w(m) c_m = a0 S0 - a1 cos(phi) Sc - a1 sin(phi) Ss
// with S0 = sum c_m, Sc = sum cos(theta_m) c_m, Ss = sum sin(theta_m) c_m,
// sums that back-projection forms once per sub-aperture, whatever aperture
// the sub-aperture later belongs to.  This kernel evaluates that combination
// for the sub-apertures of one aperture, oldest first.  It is bound by HBM:
// per pixel it reads n_blk * planes complex values and writes one.
#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void combine_kernel(CombineBatch b) {
  const CombineFrame& f = b.f[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < f.n_pix;
       i += (int64_t)gridDim.x * kThreads) {
    float re = 0.f, im = 0.f;
    int slot = f.first;
    for (int t = 0; t < f.n_blk; ++t) {
      const float2* s = f.ring + (int64_t)slot * f.stride;
      const float2 v0 = s[i];
      if (f.planes == 3) {
        const float2 vc = s[f.n_pix + i];
        const float2 vs = s[2 * f.n_pix + i];
        re += fmaf(f.c0, v0.x, fmaf(f.cc, vc.x, f.cs * vs.x));
        im += fmaf(f.c0, v0.y, fmaf(f.cc, vc.y, f.cs * vs.y));
      } else {
        re += v0.x;
        im += v0.y;
      }
      slot = slot + 1 == f.n_ring ? 0 : slot + 1;
    }
    f.out[i] = make_float2(re, im);
  }
}

}  // namespace

hipError_t launch_combine(const CombineBatch& b, hipStream_t s) {
  if (b.n_frames < 0 || b.n_frames > kCombineMaxFrames) return hipErrorInvalidValue;
  if (b.n_frames == 0) return hipSuccess;
  int64_t most = 0;
  for (int i = 0; i < b.n_frames; ++i) {
    const CombineFrame& f = b.f[i];
    if (!f.ring || !f.out || f.n_pix < 0 || f.n_ring < 1 || f.first < 0 || f.first >= f.n_ring ||
        f.n_blk < 1 || f.n_blk > f.n_ring || (f.planes != 1 && f.planes != 3) || f.stride < f.planes * f.n_pix)
      return hipErrorInvalidValue;
    most = f.n_pix > most ? f.n_pix : most;
  }
  int64_t bx = (most + kThreads - 1) / kThreads;
  if (bx > 4096) bx = 4096;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(combine_kernel, dim3((unsigned)bx, b.n_frames), dim3(kThreads), 0, s, b);
  return hipGetLastError();
}

}  // namespace rc
