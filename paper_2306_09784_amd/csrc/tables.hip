// Per-frame pixel tables.
//
// Doppler simplification (Sec. III-D of the paper): the velocity is taken as
// constant over the chirp sequence, so the radial-velocity Doppler term of
// Alg. 1 is evaluated once per pixel, at the aperture centre and with the mean
// velocity, and stored in bins:
//   f_doppler(p) = kd (<p - qt, v>/|p - qt| + <p - qr, v>/|p - qr|),
// kd = f0 / (c df).  A velocity towards the pixel gives a positive shift.
// Evaluated in double (the table is O(pixels), the cost is negligible) and
// rounded once to float.
#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double radial(double px, double py, double qx, double qy, double vx,
                                         double vy) {
  const double rx = px - qx, ry = py - qy;
  const double d = sqrt(rx * rx + ry * ry);
  return d > 0.0 ? (rx * vx + ry * vy) / d : 0.0;
}

__global__ __launch_bounds__(kThreads) void doppler_table_kernel(TableArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= a.n_pix) return;
  const float2 p = a.pix[i];
  const double px = p.x, py = p.y;
  const double r = radial(px, py, a.qt_x, a.qt_y, a.v_x, a.v_y) +
                   radial(px, py, a.qr_x, a.qr_y, a.v_x, a.v_y);
  a.fd[i] = (float)(a.kd * r);
}

}  // namespace

hipError_t launch_doppler_table(const TableArgs& a, hipStream_t s) {
  if (a.n_pix <= 0) return hipSuccess;
  const int64_t grid = (a.n_pix + kThreads - 1) / kThreads;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(doppler_table_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace rc
