// Per-frame pixel tables.
//
// Doppler simplification (Sec. III-D of the paper): the velocity is taken as
// constant over the chirp sequence, so the radial-velocity Doppler term of
// Alg. 1 is evaluated once per pixel, at the aperture centre and with the mean
// velocity, and stored in bins:
//   f_doppler(p) = kd (<p - qt, v>/|p - qt| + <p - qr, v>/|p - qr|),
// kd = f0 / (c df).  A velocity towards the pixel gives a positive shift.
//
// Back-projection works in aperture-local wavelength units P = (p - c) / lambda
// so that the carrier phase of a path is its length in turns.  The table holds
// P rounded to float, |P|^2 rounded to float, and the correction (in turns)
// that restores the rounding of |P|^2 to first order: back-projection forms
// d^2 = |P|^2 + |q|^2 - 2 P.q, so a rounding delta of |P|^2 shortens each of
// the two distances of a path by delta / (2 d) ~ delta / (2 |P|).
// Everything is evaluated in double (O(pixels) work) and rounded once.  A
// caller-supplied Doppler table replaces the computed one (and enters the
// split form's reference index).
//
// Split-phase form: a two-way path is written 2R + delta_tx + delta_rx with
// R = |P| (the path via the aperture centre) and delta = |P - q| - R, a
// quantity no larger than the antenna's offset from the centre.  The table
// then holds R and frac(2R) (the reference carrier phase in turns, exact to
// float rounding) and the index a1 2R + f_doppler of the reference path, so
// back-projection only ever rounds the small differences.
#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;

// radial speed towards the pixel of a (horizontal) velocity at q, the antenna
// h2 = height^2 above the pixel plane
__device__ __forceinline__ double radial(double px, double py, double qx, double qy, double vx,
                                         double vy, double h2) {
  const double rx = px - qx, ry = py - qy;
  const double d = sqrt(rx * rx + ry * ry + h2);
  return d > 0.0 ? (rx * vx + ry * vy) / d : 0.0;
}

__global__ __launch_bounds__(kThreads) void pixel_tables_kernel(TableMulti m) {
  const int fi = multi_frame(m, blockIdx.x);
  const TableArgs a = m.f[fi];
  const int64_t i = (int64_t)(blockIdx.x - m.begin[fi]) * kThreads + threadIdx.x;
  if (i >= a.n_pix) return;
  const float2 p = a.pix[i];
  const double px = p.x, py = p.y;
  const double h2m = a.height * a.height;
  const double fdop = a.fd_in ? (double)a.fd_in[i]
                              : a.kd * (radial(px, py, a.qt_x, a.qt_y, a.v_x, a.v_y, h2m) +
                                        radial(px, py, a.qr_x, a.qr_y, a.v_x, a.v_y, h2m));
  a.fd[i] = (float)fdop;
  const double lx = (px - a.c_x) * a.inv_lam, ly = (py - a.c_y) * a.inv_lam;
  const double hl = a.height * a.inv_lam;
  // |P|^2 + h^2: the squared distance to the aperture centre, which carries the
  // antenna height into every distance back-projection forms
  const double pp = lx * lx + ly * ly + hl * hl;
  const float ppf = (float)pp;
  const double R = sqrt(pp);
  if (a.exact) {
    // exact form: wavelengths; direct form (exact == 2): metres
    const double u = a.exact == 2 ? 1.0 / a.inv_lam : 1.0;
    const double mx = lx * u, my = ly * u, mr = R * u, mh = hl * u;
    const float fx = (float)mx, fy = (float)my;
    const double corr = mr > 0.0 ? 2.0 * (mx * (mx - fx) + my * (my - fy)) / mr : 0.0;
    a.pixc[i] = make_float4(fx, fy, (float)(mh * mh), (float)corr);
  } else if (a.split) {
    const double two_r = 2.0 * R;
    a.pixc[i] = make_float4((float)lx, (float)ly, (float)R, (float)(two_r - floor(two_r)));
    a.fbase[i] = (float)(a.a1 * two_r + fdop);
  } else {
    const double corr = R > 0.0 ? (pp - (double)ppf) / R : 0.0;
    a.pixc[i] = make_float4((float)lx, (float)ly, ppf, (float)corr);
  }
}

}  // namespace

hipError_t launch_pixel_tables(const TableMulti& m0, hipStream_t s) {
  if (m0.n_frames < 1 || m0.n_frames > TableMulti::kMax) return hipErrorInvalidValue;
  TableMulti m = m0;
  int64_t grid = 0;
  for (int i = 0; i < m.n_frames; ++i) {
    if (m.f[i].n_pix < 0) return hipErrorInvalidValue;
    m.begin[i] = (int)grid;
    grid += (m.f[i].n_pix + kThreads - 1) / kThreads;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
  }
  m.begin[m.n_frames] = (int)grid;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(pixel_tables_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, m);
  return hipGetLastError();
}

}  // namespace rc
