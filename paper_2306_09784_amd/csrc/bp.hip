// Back-projection core: Alg. 2 of the paper (Sec. IV), single precision.
//
// For every pixel p the lane evaluates, for each chirp m and channel ch,
//   d_hyp = |p - q_tx(m,ch)| + |p - q_rx(m,ch)|,
//   f_ind = a1 d_hyp + f_doppler(p)                 (index of s, Sec. III-C),
//   s_hyp = exp(a2 d_hyp) = exp(-2 pi i d_hyp f0/c)  (carrier phase),
//   P(p) += s_hyp * w_sar[m] * lerp(s[m,ch,:], f_ind),
// and writes P(p) once.  The chirp window w_sar[m] (Sec. III-B) is folded into
// the interpolation table by range compression.
//
// gfx950 mapping.  The loop is VALU/transcendental bound (three quarter-rate
// ops per term: sqrt, sin, cos), so the design minimises VALU slots per term:
//  * per-(m, ch) geometry is wave-uniform and is read with scalar loads;
//  * channels sharing a TX position evaluate d_tx once per group;
//  * the phase is reduced to a fraction of a turn (v_fract) and fed to the
//    hardware sin/cos, which take their argument in turns;
//  * the table holds (s[k], s[k+1] - s[k]) so one 16-byte buffer load and two
//    FMAs interpolate a term; loads go through a per-row buffer descriptor, so
//    an index outside the row reads zeros instead of faulting;
//  * a wave first bounds the index range of all its terms from the bounding
//    boxes of the antenna positions; if every term is provably inside
//    [0, n_bins - 1] it runs the loop without the per-term range test.
// A wave covers an 8 x 8 pixel block of the lattice so its gathers of one
// (m, ch) row touch a handful of neighbouring bins.
#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)

__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

template <int CHG, bool CHECKED>
__device__ __forceinline__ void bp_terms(const BpArgs& a, float px, float py, float fdp,
                                         float& acc_re, float& acc_im) {
  const float nbm1 = (float)(a.n_bins - 1);
  const unsigned row_bytes = (unsigned)a.n_bins * 16u;
  for (int m = 0; m < a.n_chirps; ++m) {
    const int row_m = m * a.n_ch;
    for (int g = 0; g < a.n_ch; g += CHG) {
      const int row0 = row_m + g;
      const float4 q0 = a.rowgeo[row0];
      const float tx = px - q0.x, ty = py - q0.y;
      const float d_tx = hw_sqrt(fmaf(tx, tx, ty * ty));
#pragma unroll
      for (int j = 0; j < CHG; ++j) {
        const float4 q = a.rowgeo[row0 + j];
        const float rx = px - q.z, ry = py - q.w;
        const float d_hyp = d_tx + hw_sqrt(fmaf(rx, rx, ry * ry));
        const float f = fmaf(a.a1, d_hyp, fdp);
        int i;
        float phi;
        if (CHECKED) {
          const float fl = floorf(f);
          phi = f - fl;
          i = (f >= 0.f && f <= nbm1) ? (int)fl : -1;  // -1: out of the descriptor -> zeros
        } else {
          i = (int)f;                                  // f >= 0 here: truncation is floor
          phi = __builtin_amdgcn_fractf(f);
        }
        const float turn = __builtin_amdgcn_fractf(d_hyp * a.inv_lam);
        const float sn = __builtin_amdgcn_sinf(turn);   // sin(2 pi turn)
        const float cs = __builtin_amdgcn_cosf(turn);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(a.pairs + (size_t)(row0 + j) * a.n_bins), (short)0, (int)row_bytes, kRsrcWord3);
        const u32x4 e = __builtin_amdgcn_raw_buffer_load_b128(rs, (unsigned)i * 16u, 0, 0);
        const float vr = fmaf(phi, __uint_as_float(e.z), __uint_as_float(e.x));
        const float vi = fmaf(phi, __uint_as_float(e.w), __uint_as_float(e.y));
        // (cs - i sn) (vr + i vi)
        acc_re = fmaf(cs, vr, acc_re);
        acc_re = fmaf(sn, vi, acc_re);
        acc_im = fmaf(cs, vi, acc_im);
        acc_im = fmaf(-sn, vr, acc_im);
      }
    }
  }
}

__device__ __forceinline__ float box_min_dist(float px, float py, float lx, float ly, float hx, float hy) {
  const float dx = fmaxf(fmaxf(lx - px, px - hx), 0.f);
  const float dy = fmaxf(fmaxf(ly - py, py - hy), 0.f);
  return sqrtf(dx * dx + dy * dy);
}
__device__ __forceinline__ float box_max_dist(float px, float py, float lx, float ly, float hx, float hy) {
  const float dx = fmaxf(fabsf(px - lx), fabsf(px - hx));
  const float dy = fmaxf(fabsf(py - ly), fabsf(py - hy));
  return sqrtf(dx * dx + dy * dy);
}

template <int CHG>
__global__ __launch_bounds__(kThreads) void bp_kernel(BpArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int r, c;
  if (a.n_rows >= 8) {  // 16 x 16 workgroup tile of four 8 x 8 wave blocks
    r = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
    c = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
  } else {              // 1 x 256 workgroup tile of four 1 x 64 wave rows
    r = blockIdx.y;
    c = blockIdx.x * kThreads + threadIdx.x;
  }
  const bool live = r < a.n_rows && c < a.n_cols;
  // lanes outside the lattice replay its last pixel and store nothing, so the
  // wave stays converged
  const int rr = r < a.n_rows ? r : a.n_rows - 1;
  const int cc = c < a.n_cols ? c : a.n_cols - 1;
  const int64_t idx = (int64_t)rr * a.n_cols + cc;
  const float2 p = a.pix[idx];
  const float fdp = a.fd[idx];

  const float dlo = box_min_dist(p.x, p.y, a.tx_lo_x, a.tx_lo_y, a.tx_hi_x, a.tx_hi_y) +
                    box_min_dist(p.x, p.y, a.rx_lo_x, a.rx_lo_y, a.rx_hi_x, a.rx_hi_y);
  const float dhi = box_max_dist(p.x, p.y, a.tx_lo_x, a.tx_lo_y, a.tx_hi_x, a.tx_hi_y) +
                    box_max_dist(p.x, p.y, a.rx_lo_x, a.rx_lo_y, a.rx_hi_x, a.rx_hi_y);
  const float flo = fmaf(a.a1, dlo, fdp), fhi = fmaf(a.a1, dhi, fdp);
  const bool inside = flo >= a.f_margin && fhi <= (float)(a.n_bins - 1) - a.f_margin;

  float acc_re = 0.f, acc_im = 0.f;
  if (__all(inside))
    bp_terms<CHG, false>(a, p.x, p.y, fdp, acc_re, acc_im);
  else
    bp_terms<CHG, true>(a, p.x, p.y, fdp, acc_re, acc_im);
  if (live) a.out[idx] = make_float2(acc_re, acc_im);
}

}  // namespace

hipError_t launch_backproject(const BpArgs& a, hipStream_t s) {
  if (a.n_rows <= 0 || a.n_cols <= 0) return hipSuccess;
  if (a.n_chirps < 1 || a.n_ch < 1 || a.n_bins < 2 || a.chg < 1 || a.n_ch % a.chg != 0 ||
      (int64_t)a.n_bins * 16 >= (int64_t)1 << 31 || (int64_t)a.n_chirps * a.n_ch >= (int64_t)1 << 31)
    return hipErrorInvalidValue;
  dim3 grid;
  if (a.n_rows >= 8)
    grid = dim3((a.n_cols + 15) / 16, (a.n_rows + 15) / 16);
  else
    grid = dim3((a.n_cols + kThreads - 1) / kThreads, a.n_rows);
  switch (a.chg) {
    case 16: hipLaunchKernelGGL(bp_kernel<16>, grid, dim3(kThreads), 0, s, a); break;
    case 8: hipLaunchKernelGGL(bp_kernel<8>, grid, dim3(kThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL(bp_kernel<4>, grid, dim3(kThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL(bp_kernel<2>, grid, dim3(kThreads), 0, s, a); break;
    case 1: hipLaunchKernelGGL(bp_kernel<1>, grid, dim3(kThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rc
