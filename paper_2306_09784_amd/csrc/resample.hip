// Polar-grid image -> magnitude at arbitrary points.
//
// Sec. III-E forms the image on a polar lattice around the aperture centre;
// showing it on the Cartesian reference grid (the comparison of Fig. 3) needs
// its magnitude at Cartesian points.  A point's range r and azimuth theta
// (measured from +y towards +x) give fractional lattice indices
// u = (r - r0) / dr and v = (theta - th0) / dth, and |P| is interpolated
// bilinearly in (v, u): an index equal to the last one takes that sample,
// outside [0, n - 1] the result is 0.  The magnitude is interpolated, not the
// complex value, whose phase turns once per half wavelength of range.
//
// One lane per point; coordinates and weights in double (the stage is bound
// by its gathers, not by arithmetic), the result rounded once to float.
#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double mag(float2 z) { return sqrt((double)z.x * z.x + (double)z.y * z.y); }

__global__ __launch_bounds__(kThreads) void resample_polar_kernel(ResampleArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kThreads) {
    const float2 p = a.pts[i];
    const double dx = (double)p.x - a.ox, dy = (double)p.y - a.oy;
    const double u = (sqrt(dx * dx + dy * dy) - a.r0) / a.dr;
    const double v = (atan2(dx, dy) - a.th0) / a.dth;
    float out = 0.f;
    if (u >= 0.0 && u <= (double)(a.nr - 1) && v >= 0.0 && v <= (double)(a.nth - 1)) {
      const int iu = min((int)floor(u), a.nr - 1), iv = min((int)floor(v), a.nth - 1);
      const int iu1 = min(iu + 1, a.nr - 1), iv1 = min(iv + 1, a.nth - 1);
      const double fu = u - iu, fv = v - iv;
      const float2* r0 = a.img + (int64_t)iv * a.nr;
      const float2* r1 = a.img + (int64_t)iv1 * a.nr;
      const double lo = (1.0 - fu) * mag(r0[iu]) + fu * mag(r0[iu1]);
      const double hi = (1.0 - fu) * mag(r1[iu]) + fu * mag(r1[iu1]);
      out = (float)((1.0 - fv) * lo + fv * hi);
    }
    a.out[i] = out;
  }
}

}  // namespace

hipError_t launch_resample_polar(const ResampleArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.nth < 1 || a.nr < 1 || !(a.dr > 0.0) || !(a.dth > 0.0) || !a.img || !a.pts || !a.out)
    return hipErrorInvalidValue;
  int64_t grid = (a.n + kThreads - 1) / kThreads;
  if (grid > 65536) grid = 65536;  // grid-stride beyond
  hipLaunchKernelGGL(resample_polar_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace rc
