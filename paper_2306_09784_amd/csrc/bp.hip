// Back-projection core: Alg. 2 of the paper (Sec. IV), single precision; the
// exact-Doppler form evaluates Alg. 1 (Sec. II) for the ablation of Sec. III-D,
// and the direct form evaluates Alg. 1 as the paper states it, before the
// constants of Sec. III-C are folded (the reference of Tab. II's "Opt." row).
//
// For every pixel p the lane evaluates, for each chirp m and channel ch,
//   d_hyp = |p - q_tx(m,ch)| + |p - q_rx(m,ch)|,
//   f_ind = a1 d_hyp + f_doppler(p)                 (index of s, Sec. III-C),
//   s_hyp = exp(a2 d_hyp) = exp(-2 pi i d_hyp / lambda)  (carrier phase),
//   P(p) += s_hyp * w_sar[m] * lerp(s[m,ch,:], f_ind),
// and writes P(p) once.  The chirp window w_sar[m] (Sec. III-B) is folded into
// the interpolation table by range compression.
//
// gfx950 mapping.  The loop is bound by VALU issue (three quarter-rate
// transcendentals per term: sqrt, sin, cos; the half-rate index conversion;
// eleven full-rate adds and FMAs), so the design minimises instructions per
// term:
//  * geometry is in aperture-local wavelength units, so a path length is its
//    carrier phase in turns and goes straight into the hardware sin/cos
//    (which take turns);
//  * a squared distance is |P|^2 + |q|^2 - 2 P.q: two FMAs and an add with the
//    per-row uniforms (-2 q, |q|^2), read with scalar loads;
//  * channels sharing a TX position evaluate d_tx once per group;
//  * the table holds each segment's intercept and slope in the bin index f
//    (A = s[k] - k D, D = s[k+1] - s[k]), so one 16-byte buffer load and two
//    FMAs with f itself interpolate a term, with no fraction of f; loads go
//    through a per-row buffer descriptor, so
//    an index outside the row reads zeros instead of faulting, and where the
//    index is proven in range the load takes the bin index itself (the
//    descriptor's 16-byte stride scales it: no shift per term);
//  * a wave first bounds the index range of all its terms from the bounding
//    boxes of the antenna positions; if every term is provably inside
//    [0, n_bins - 1] it runs the loop without the per-term range test;
//  * even and odd channels accumulate into separate registers to shorten the
//    dependency chains of the multiply-accumulates.
// A wave covers an 8 x 8 pixel block of the lattice so its gathers of one
// (m, ch) row touch a handful of neighbouring bins.
//
// Sub-apertures of a continuous stream (SUMS = 3): the table carries no chirp
// window; the lane keeps the plain sum of the terms and the sums weighted by
// cos and sin of each chirp's window phase, from which the runtime forms the
// windowed aperture, instead of back-projecting every chirp once per
// aperture it belongs to.  All channels of a chirp share its weights, so the
// terms of a chirp accumulate as usual and their sum enters the three sums
// once per chirp (a dozen instructions per chirp and pixel).  The three sums
// live in the lane's own LDS slot between chirps, which keeps the register
// count, and so the occupancy, of the single-sum kernel.
//
// Work distribution: one launch covers a batch of frames; its work items are
// (frame, chirp block, 16 x 16 tile).  Workgroups are dispatched to the eight
// XCDs round robin, so workgroup w runs on XCD k = w % 8 as its slot w / 8.
// The slots of an XCD walk the frames in order (the caller sorts them by
// cost, largest first) and, within a frame, the k-th contiguous eighth of its
// items: neighbouring tiles of one chirp block, whose gathers hit the same
// table rows in that XCD's L2, while every frame is spread over all XCDs.
#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)

// Indexed ("structured") buffer load of one 16-byte record: the hardware
// forms base + vindex x stride from the descriptor's stride, so the caller
// passes the record index instead of a byte offset.  Declared by its LLVM
// intrinsic name (the compiler has no builtin for it; the backend emits
// buffer_load_dwordx4 ... idxen and tracks the load like any other).
__device__ u32x4 struct_buffer_load_b128(__amdgpu_buffer_rsrc_t rsrc, int vindex, int voffset, int soffset,
                                         int aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.v4i32");

// Per-form geometry of one term.  Plain (Alg. 2): d = sqrt(|P|^2 + |q|^2 -
// 2 P.q) from the per-row uniforms (-2 q, |q|^2) and the pixel's |P|^2 split
// into a float and a correction.  Split-phase: d = R + delta with
// N = |P - q|^2 - R^2 = |q|^2 - 2 P.q (two FMAs) and delta = N / (d + R),
// d = sqrt(R^2 + N); only delta (|delta| <= |q|) and the reference phase
// frac(2R) enter the phase, so its rounding error scales with the aperture
// size, not with the range.  Exact (Alg. 1): each leg also contributes its own
// Doppler index shift <P - q, kd v(m)> / |P - q| from the chirp's velocity.
template <int FORM>
struct Leg {
  float d;    // plain: distance (TX leg: + correction); split: delta; exact: distance
  float dop;  // exact only: Doppler index shift of the leg
};

// Per-pixel coefficients of the split form's series in N (below).
struct PixAux {
  float c[5];
};

// Split-phase offset by series.  With u = N / R^2,
//   delta = sqrt(R^2 + N) - R = (N / (2R)) (1 + u G(u)),
//   G(u) = -1/4 + u/8 - 5u^2/64 + 7u^3/128 - ...
// (the binomial series of sqrt(1 + u)).  G is taken as the cubic that
// interpolates it at the four Chebyshev nodes of [-kSeriesU, kSeriesU]
// (kSeriesU = 0.1): with the coefficients rounded to float, 1 + u G(u) is off
// by at most 5.7e-8 of itself there (the Taylor cubic: 4.5e-7).  Multiplied
// out, delta is a quintic in N with no constant term whose coefficients
// depend on the pixel only: c1 = 1/(2R), c(i+2) = G_i / (2R^(2i+3)), so a leg
// costs four FMAs and a multiply (Horner in N) once per pixel has formed the
// five; its rounding matches the nested form's (2.0e-7 of delta at most, over
// R in [0.5, 60] and the whole u range).  Far from the aperture (R above ~20
// times the antennas' spread) this replaces a square root and a reciprocal,
// both quarter-rate; waves with any pixel closer take the exact form.
constexpr float kSeriesU = 0.1f;
constexpr float kG0 = -0.24999947845935822f, kG1 = 0.12499959766864777f, kG2 = -0.0785374641418457f,
                kG3 = 0.05501168593764305f;

template <int FORM, bool SERIES>
__device__ __forceinline__ Leg<FORM> leg(const float4 q, const float4 p, const PixAux x_) {
  Leg<FORM> l;
  if constexpr (FORM == kBpExact) {
    const float x = p.x - q.x, y = p.y - q.y;
    l.d = __builtin_amdgcn_sqrtf(fmaf(x, x, fmaf(y, y, p.z)));  // p.z: squared antenna height
    l.dop = fmaf(x, q.z, y * q.w) * __builtin_amdgcn_rcpf(l.d);
  } else if constexpr (FORM == kBpDirect) {
    // metres and metres per second: the distance and the radial speed
    // <p - q, v> / d (a division, as Alg. 1 writes it)
    const float x = p.x - q.x, y = p.y - q.y;
    l.d = sqrtf(fmaf(x, x, fmaf(y, y, p.z)));
    l.dop = fmaf(x, q.z, y * q.w) / l.d;
  } else if constexpr (FORM == kBpSplit) {
    const float n = fmaf(q.x, p.x, fmaf(q.y, p.y, q.z));
    if constexpr (SERIES) {
      float t = fmaf(x_.c[4], n, x_.c[3]);
      t = fmaf(t, n, x_.c[2]);
      t = fmaf(t, n, x_.c[1]);
      t = fmaf(t, n, x_.c[0]);
      l.d = t * n;
    } else {
      l.d = n * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(fmaf(p.z, p.z, n)) + p.z);
    }
    l.dop = 0.f;
  } else {
    l.d = __builtin_amdgcn_sqrtf(fmaf(q.x, p.x, fmaf(q.y, p.y, p.z)) + q.z);
    l.dop = 0.f;
  }
  return l;
}

// One pipeline stage: U terms whose table loads are in flight.
template <int U>
struct Stage {
  u32x4 e[U];
  float f[U];  // fractional bin index of the term
  float turn[U];
};

// The terms of rows [row_begin, row_end) for one pixel, software-pipelined:
// the table loads of the next U rows are issued before the phases and
// multiply-accumulates of the current U rows, so their latency overlaps the
// transcendentals.  U = min(CHG, 4) rows per stage; the TX leg is evaluated
// once per group of CHG rows.
template <int CHG, int FORM, bool CHECKED, int SUMS, bool SERIES = false>
__device__ __forceinline__ void bp_terms(const BpFrame& a, int row_begin, int row_end, const float4 p,
                                         const float fidx, float (&out_re)[SUMS], float (&out_im)[SUMS]) {
  constexpr bool EXACT = FORM == kBpExact || FORM == kBpDirect;
  constexpr int U = CHG < 4 ? CHG : 4;
  constexpr int UPG = CHG / U;  // stages per TX group
  const float nbm1 = (float)(a.n_bins - 1);
  const int row_bytes = a.n_bins * 16;
  const float4* rq = (EXACT ? a.rowv : a.rowq) + row_begin;
  const float4* gq = (EXACT ? a.grpv : a.grpq) + row_begin / CHG;
  const float4* tab = a.pairs + (size_t)row_begin * a.n_bins;
  // SUMS == 3: the chirps' window-phase weights (cos, sin), one per chirp
  const float2* wp = SUMS == 3 ? a.roww + row_begin / a.n_ch : nullptr;
  const float2* wend = SUMS == 3 ? a.roww + row_end / a.n_ch : nullptr;
  const int n = row_end - row_begin;  // a multiple of CHG
  // per-pixel index base: plain f_doppler; split the index of the reference
  // path, less a1 frac(2R): the split form's TX leg carries the reference
  // phase frac(2R), so a term's phase and index both come from one sum
  const float fb = FORM == kBpSplit ? fmaf(-a.a1, p.w, fidx) : fidx;
  // split form's series coefficients from 1 / (2R) and 1 / R^2 (p.z = R)
  PixAux aux{};
  if constexpr (FORM == kBpSplit && SERIES) {
    const float ir = __builtin_amdgcn_rcpf(p.z);
    const float h = 0.5f * ir, k = ir * ir;
    const float hk = h * k, hk2 = hk * k, hk3 = hk2 * k;
    aux.c[0] = h;
    aux.c[1] = hk * kG0;
    aux.c[2] = hk2 * kG1;
    aux.c[3] = hk3 * kG2;
    aux.c[4] = (hk3 * k) * kG3;
  }
  float re0 = 0.f, im0 = 0.f, re1 = 0.f, im1 = 0.f;
  // SUMS == 3: the plain, cos- and sin-weighted sums over the chirps done,
  // in this lane's LDS slot my[0] = (re: plain, cos, sin), my[1] = (im: ...)
  __shared__ float3 sums[SUMS == 3 ? 2 * kThreads : 1];
  float3* my = sums + (SUMS == 3 ? 2 * threadIdx.x : 0);
  if constexpr (SUMS == 3) {
    my[0] = make_float3(0.f, 0.f, 0.f);
    my[1] = make_float3(0.f, 0.f, 0.f);
  }
  float2 wcur = SUMS == 3 ? wp[0] : make_float2(0.f, 0.f);
  int chirp_rows = 0;  // rows of the current chirp consumed (wave-uniform)
  Leg<FORM> tx;

  auto tx_leg = [&](int r) {
    tx = leg<FORM, SERIES>(gq[r / CHG], p, aux);
    tx.d += p.w;  // plain, exact: the pixel's rounding correction; split: frac(2R)
  };
  auto issue = [&](int r, Stage<U>& st) {
    // the stage's row uniforms as one vector, so they arrive in one scalar load
    typedef float uvec __attribute__((ext_vector_type(4 * U)));
    const uvec u = *reinterpret_cast<const uvec*>(rq + r);
    float4 q[U];
#pragma unroll
    for (int j = 0; j < U; ++j) q[j] = make_float4(u[4 * j], u[4 * j + 1], u[4 * j + 2], u[4 * j + 3]);
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const Leg<FORM> rx = leg<FORM, SERIES>(q[j], p, aux);
      float f, turn;
      if constexpr (FORM == kBpSplit) {
        turn = tx.d + rx.d;  // frac(2R) + delta_tx + delta_rx
        f = fmaf(a.a1, turn, fb);
      } else if constexpr (FORM == kBpExact) {
        const float d_hyp = tx.d + rx.d;
        f = fmaf(a.a1, d_hyp, tx.dop + rx.dop);
        turn = d_hyp;
      } else if constexpr (FORM == kBpDirect) {
        // Alg. 1: tau = (d_tx + d_rx) / c, f_hyp = mu tau + f0 v / c in Hz, its
        // bin f_hyp / df, and the carrier phase f0 tau in turns
        const float tau = (tx.d + rx.d) / a.lit_c;
        const float f_hyp = fmaf(a.lit_mu, tau, a.lit_f0 * (tx.dop + rx.dop) / a.lit_c);
        f = f_hyp / a.lit_df;
        turn = a.lit_f0 * tau;
      } else {
        const float d_hyp = tx.d + rx.d;
        f = fmaf(a.a1, d_hyp, fb);
        turn = d_hyp;
      }
      int i;
      if (CHECKED)
        i = (f >= 0.f && f <= nbm1) ? (int)f : -1;  // -1: outside the descriptor -> zeros
      else
        i = (int)f;                                  // f >= 0 here: truncation is floor
      st.f[j] = f;
      st.turn[j] = turn;
      if (CHECKED) {
        // i = -1 reads past the descriptor's range: zeros, no access
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(tab + (size_t)(r + j) * a.n_bins), (short)0, row_bytes, kRsrcWord3);
        st.e[j] = __builtin_amdgcn_raw_buffer_load_b128(rs, (unsigned)i * 16u, 0, 0);
      } else {
        // 0 <= i <= n_bins - 1 by the wave's range proof: the record index
        // goes to the load, which scales it by the 16-byte stride (no shift
        // per term).  With a non-zero stride the range check counts records,
        // so the descriptor's bound is n_bins: an index past the row would
        // read zeros, never the next row.
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(tab + (size_t)(r + j) * a.n_bins), (short)16, a.n_bins, kRsrcWord3);
        st.e[j] = struct_buffer_load_b128(rs, i, 0, 0, 0);
      }
    }
  };
  // PAR selects the accumulator pair of a single-row stage
  auto consume = [&](const Stage<U>& st, int par) {
#pragma unroll
    for (int j = 0; j < U; ++j) {
      // the hardware sin/cos take turns and reduce any argument exactly (checked
      // to 2^16 turns: error 1.1e-7, as for arguments below one turn), so the
      // path length in wavelengths goes in without a fraction
      const float sn = __builtin_amdgcn_sinf(st.turn[j]);  // sin(2 pi turn)
      const float cs = __builtin_amdgcn_cosf(st.turn[j]);
      // the segment's intercept + f x slope (zeros outside the row: 0)
      const float vr = fmaf(st.f[j], __uint_as_float(st.e[j].z), __uint_as_float(st.e[j].x));
      const float vi = fmaf(st.f[j], __uint_as_float(st.e[j].w), __uint_as_float(st.e[j].y));
      // (cs - i sn) (vr + i vi); the sub-aperture form keeps one accumulator pair
      if (SUMS == 1 && (((U == 1) ? par : j) & 1)) {
        re1 = fmaf(cs, vr, re1);
        re1 = fmaf(sn, vi, re1);
        im1 = fmaf(cs, vi, im1);
        im1 = fmaf(-sn, vr, im1);
      } else {
        re0 = fmaf(cs, vr, re0);
        re0 = fmaf(sn, vi, re0);
        im0 = fmaf(cs, vi, im0);
        im0 = fmaf(-sn, vr, im0);
      }
    }
    if constexpr (SUMS == 3) {
      // U divides the channels of a chirp: at the end of a chirp its sum joins
      // the three sums with the chirp's weights and the accumulators restart
      chirp_rows += U;
      if (chirp_rows == a.n_ch) {
        chirp_rows = 0;
        float3 sr = my[0], si = my[1];
        sr.x += re0;
        si.x += im0;
        sr.y = fmaf(wcur.x, re0, sr.y);
        si.y = fmaf(wcur.x, im0, si.y);
        sr.z = fmaf(wcur.y, re0, sr.z);
        si.z = fmaf(wcur.y, im0, si.z);
        my[0] = sr;
        my[1] = si;
        re0 = im0 = 0.f;
        if (++wp < wend) wcur = *wp;
      }
    }
  };
  auto step = [&](int r, Stage<U>& st) {
    if (UPG == 1 || ((r / U) & (UPG - 1)) == 0) tx_leg(r);
    issue(r, st);
  };

  Stage<U> sa, sb;
  step(0, sa);
  int r = U;
  for (; r + U < n; r += 2 * U) {
    step(r, sb);
    consume(sa, 0);
    step(r + U, sa);
    consume(sb, 1);
  }
  if (r < n) {
    step(r, sb);
    consume(sa, 0);
    consume(sb, 1);
  } else {
    consume(sa, 0);
  }
  if constexpr (SUMS == 3) {
    const float3 sr = my[0], si = my[1];
    out_re[0] = sr.x;
    out_im[0] = si.x;
    out_re[1] = sr.y;
    out_im[1] = si.y;
    out_re[2] = sr.z;
    out_im[2] = si.z;
  } else {
    out_re[0] = re0 + re1;
    out_im[0] = im0 + im1;
  }
}

// nearest and farthest distance from the pixel to an antenna in a box, with
// the antennas h2 (squared height) above the pixel plane
__device__ __forceinline__ float box_min_dist(float px, float py, float lx, float ly, float hx, float hy,
                                              float h2) {
  const float dx = fmaxf(fmaxf(lx - px, px - hx), 0.f);
  const float dy = fmaxf(fmaxf(ly - py, py - hy), 0.f);
  return sqrtf(dx * dx + dy * dy + h2);
}
__device__ __forceinline__ float box_max_dist(float px, float py, float lx, float ly, float hx, float hy,
                                              float h2) {
  const float dx = fmaxf(fabsf(px - lx), fabsf(px - hx));
  const float dy = fmaxf(fabsf(py - ly), fabsf(py - hy));
  return sqrtf(dx * dx + dy * dy + h2);
}

template <int CHG, int FORM, int SUMS>
__global__ __launch_bounds__(kThreads) void bp_kernel(BpBatch b) {
  constexpr bool SPLIT = FORM == kBpSplit;
  constexpr bool EXACT = FORM == kBpExact || FORM == kBpDirect;
  const int w = blockIdx.x;
  const int xcd = w & 7;
  const int slot = w >> 3;
  if (slot >= b.n_slots) return;
  int fi = 0;
  while (fi + 1 < b.n_frames && slot >= b.f[fi + 1].slot_base) ++fi;
  // a by-value copy read before any lane-dependent branch keeps every
  // descriptor field in scalar registers
  const BpFrame a = b.f[__builtin_amdgcn_readfirstlane(fi)];
  // the integer divisions below run on the VALU; readfirstlane hands their
  // (workgroup-uniform) results back to scalar registers so that the table
  // descriptors derived from them stay scalar
  const int local = xcd * a.chunk + (slot - a.slot_base);
  if (local >= a.kb_count * a.n_tiles) return;
  const int kb_local = __builtin_amdgcn_readfirstlane(local / a.n_tiles);
  const int tile = local - kb_local * a.n_tiles;
  const int kb = a.kb0 + kb_local;
  const int ty = __builtin_amdgcn_readfirstlane(tile / a.tiles_x);
  const int tx = tile - ty * a.tiles_x;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int r, c;
  if (a.n_rows >= 8) {  // 16 x 16 workgroup tile of four 8 x 8 wave blocks
    r = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
    c = tx * 16 + (wave & 1) * 8 + (lane & 7);
  } else {              // 1 x 256 workgroup tile of four 1 x 64 wave rows
    r = ty;
    c = tx * kThreads + threadIdx.x;
  }
  const bool live = r < a.n_rows && c < a.n_cols;
  // lanes outside the lattice replay its last pixel and store nothing, so the
  // wave stays converged
  const int rr = r < a.n_rows ? r : a.n_rows - 1;
  const int cc = c < a.n_cols ? c : a.n_cols - 1;
  const int64_t idx = (int64_t)rr * a.n_cols + cc;
  const float4 p = a.pixc[idx];
  const float fi_p = a.fidx[idx];
  // f_doppler of the pixel (split form: from the index of the reference path;
  // exact form: per term, bounded by f_slack)
  const float fdp = EXACT ? 0.f : (SPLIT ? fi_p - a.a1 * 2.f * p.z : fi_p);

  const float dlo = box_min_dist(p.x, p.y, a.tx_lo_x, a.tx_lo_y, a.tx_hi_x, a.tx_hi_y, a.h2) +
                    box_min_dist(p.x, p.y, a.rx_lo_x, a.rx_lo_y, a.rx_hi_x, a.rx_hi_y, a.h2);
  const float dhi = box_max_dist(p.x, p.y, a.tx_lo_x, a.tx_lo_y, a.tx_hi_x, a.tx_hi_y, a.h2) +
                    box_max_dist(p.x, p.y, a.rx_lo_x, a.rx_lo_y, a.rx_hi_x, a.rx_hi_y, a.h2);
  const float flo = fmaf(a.a1, dlo, fdp), fhi = fmaf(a.a1, dhi, fdp);
  const float mg = a.f_margin + a.f_slack;
  // (the direct form keeps metres and runs the range-tested loop throughout)
  const bool inside = FORM != kBpDirect && (flo >= mg) & (fhi <= (float)(a.n_bins - 1) - mg);

  // chirp block kb covers chirps [m0, m1), i.e. rows [m0 n_ch, m1 n_ch)
  const int m0 = __builtin_amdgcn_readfirstlane((int)(((int64_t)kb * a.n_chirps) / a.n_kb));
  const int m1 = __builtin_amdgcn_readfirstlane((int)(((int64_t)(kb + 1) * a.n_chirps) / a.n_kb));
  const int row_begin = m0 * a.n_ch, row_end = m1 * a.n_ch;

  float re[SUMS], im[SUMS];
  const float fb = SPLIT ? fi_p : fdp;
  if constexpr (SPLIT) {
    // the series of the split-phase offset holds where |N| / R^2 <= kSeriesU
    // for every antenna: |N| <= 2 R Q + Q^2, Q the antennas' largest distance
    // from the aperture centre
    const float qr = a.q_max / p.z;
    const bool series = p.z > 0.f && fmaf(qr, qr, 2.f * qr) <= kSeriesU;
    if (__all(series)) {
      if (__all(inside))
        bp_terms<CHG, FORM, false, SUMS, true>(a, row_begin, row_end, p, fb, re, im);
      else
        bp_terms<CHG, FORM, true, SUMS, true>(a, row_begin, row_end, p, fb, re, im);
    } else {
      if (__all(inside))
        bp_terms<CHG, FORM, false, SUMS>(a, row_begin, row_end, p, fb, re, im);
      else
        bp_terms<CHG, FORM, true, SUMS>(a, row_begin, row_end, p, fb, re, im);
    }
  } else {
    if (__all(inside))
      bp_terms<CHG, FORM, false, SUMS>(a, row_begin, row_end, p, fb, re, im);
    else
      bp_terms<CHG, FORM, true, SUMS>(a, row_begin, row_end, p, fb, re, im);
  }
  if (live) {
    const int64_t n_pix = (int64_t)a.n_rows * a.n_cols;
#pragma unroll
    for (int k = 0; k < SUMS; ++k) a.out[((int64_t)kb * SUMS + k) * n_pix + idx] = make_float2(re[k], im[k]);
  }
}

// Sum of the chirp-block partial images in block order.
__global__ __launch_bounds__(kThreads) void reduce_partials_kernel(ReduceBatch b) {
  const ReduceFrame& f = b.f[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < f.n_pix;
       i += (int64_t)gridDim.x * kThreads) {
    float re = 0.f, im = 0.f;
    for (int k = 0; k < f.n_kb; ++k) {
      const float2 v = f.partial[(int64_t)k * f.n_pix + i];
      re += v.x;
      im += v.y;
    }
    f.out[i] = make_float2(re, im);
  }
}

template <int CHG, int SUMS>
void launch_form(const BpBatch& b, dim3 grid, hipStream_t s) {
  if (b.form == kBpSplit) {
    hipLaunchKernelGGL((bp_kernel<CHG, kBpSplit, SUMS>), grid, dim3(kThreads), 0, s, b);
  } else if (b.form == kBpExact) {
    hipLaunchKernelGGL((bp_kernel<CHG, kBpExact, SUMS>), grid, dim3(kThreads), 0, s, b);
  } else if (b.form == kBpDirect) {
    // (launch_backproject admits the direct form with single sums only)
    if constexpr (SUMS == 1) hipLaunchKernelGGL((bp_kernel<CHG, kBpDirect, 1>), grid, dim3(kThreads), 0, s, b);
  } else {
    hipLaunchKernelGGL((bp_kernel<CHG, kBpPlain, SUMS>), grid, dim3(kThreads), 0, s, b);
  }
}

template <int CHG>
void launch_chg(const BpBatch& b, dim3 grid, hipStream_t s) {
  if (b.sums == 3)
    launch_form<CHG, 3>(b, grid, s);
  else
    launch_form<CHG, 1>(b, grid, s);
}

}  // namespace

void bp_tiles(int n_rows, int n_cols, int* tiles_x, int* n_tiles) {
  if (n_rows >= 8) {
    *tiles_x = (n_cols + 15) / 16;
    *n_tiles = *tiles_x * ((n_rows + 15) / 16);
  } else {
    *tiles_x = (n_cols + kThreads - 1) / kThreads;
    *n_tiles = *tiles_x * n_rows;
  }
}

int bp_chirp_blocks(int64_t n_rows, int64_t n_cols, int n_chirps, int n_ch, int planes) {
  // 256 CUs x 4 SIMDs x 8 waves = 8192 wave slots (the plain kernel's 65
  // VGPRs leave 7 per SIMD resident: 7168; the split below is measured, not
  // exact in that unit).  Aim at ten
  // generations of waves: the ragged end of the launch then idles a small
  // share of it (measured, a lone frame's time stops falling from about ten
  // generations on).  But each block also adds a wave's fixed work (pixel
  // tables, range proof, stores) and `planes` partial images to write and
  // reduce, which frames batched together, or streamed two at a time, pay
  // without needing the extra waves: so at least planes x kBpMinBlockRows rows
  // (chirps x channels) per block, unless fewer blocks would leave a lone
  // frame short of one generation.  At most 16 blocks and at least one chirp
  // per block.
  int tx, nt;
  bp_tiles((int)n_rows, (int)n_cols, &tx, &nt);
  const int64_t waves = (int64_t)nt * (kThreads / 64);
  int64_t k = (kBpTargetGenerations * 8192 + waves - 1) / waves;
  const int64_t by_rows = (int64_t)n_chirps * n_ch / ((int64_t)planes * kBpMinBlockRows);
  const int64_t fill = (8192 + waves - 1) / waves;
  if (k > by_rows) k = by_rows > fill ? by_rows : fill;
  if (k > 16) k = 16;
  if (k > n_chirps) k = n_chirps;
  return k < 1 ? 1 : (int)k;
}

hipError_t launch_backproject(const BpBatch& b, hipStream_t s) {
  if (b.n_frames < 1 || b.n_frames > kBpMaxFrames || b.n_slots < 1 || b.chg < 1 || b.form < kBpPlain ||
      b.form > kBpDirect || (b.sums != 1 && b.sums != 3) || (b.form == kBpDirect && b.sums != 1))
    return hipErrorInvalidValue;
  int slots = 0;
  for (int i = 0; i < b.n_frames; ++i) {
    const BpFrame& f = b.f[i];
    int tx, nt;
    bp_tiles(f.n_rows, f.n_cols, &tx, &nt);
    if (f.n_rows < 1 || f.n_cols < 1 || f.n_chirps < 1 || f.n_ch < 1 || f.n_bins < 2 || f.n_ch % b.chg != 0 ||
        ((b.form == kBpExact || b.form == kBpDirect) && (!f.rowv || !f.grpv)) ||
        (b.form != kBpExact && b.form != kBpDirect && (!f.rowq || !f.grpq)) ||
        (b.sums == 3 && (!f.roww || (reinterpret_cast<uintptr_t>(f.roww) & 7))) || !f.out ||
        f.n_kb < 1 || f.n_kb > f.n_chirps || f.kb0 < 0 || f.kb_count < 1 || f.kb0 + f.kb_count > f.n_kb ||
        f.tiles_x != tx || f.n_tiles != nt || f.slot_base != slots || f.chunk != (f.kb_count * nt + 7) / 8 ||
        (f.n_rows >= 8 && (f.n_rows + 15) / 16 > 0x7fffffff / 16) ||
        (int64_t)f.n_bins * 16 >= (int64_t)1 << 31 || (int64_t)f.n_chirps * f.n_ch >= (int64_t)1 << 31)
      return hipErrorInvalidValue;
    slots += f.chunk;
  }
  if (slots != b.n_slots) return hipErrorInvalidValue;
  const int64_t blocks = (int64_t)b.n_slots * 8;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  switch (b.chg) {
    case 16: launch_chg<16>(b, grid, s); break;
    case 8: launch_chg<8>(b, grid, s); break;
    case 4: launch_chg<4>(b, grid, s); break;
    case 2: launch_chg<2>(b, grid, s); break;
    case 1: launch_chg<1>(b, grid, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const ReduceBatch& b, hipStream_t s) {
  if (b.n_frames < 0 || b.n_frames > kReduceMaxFrames) return hipErrorInvalidValue;
  if (b.n_frames == 0) return hipSuccess;
  int64_t most = 0;
  for (int i = 0; i < b.n_frames; ++i) {
    if (b.f[i].n_kb < 1 || b.f[i].n_pix < 0) return hipErrorInvalidValue;
    most = b.f[i].n_pix > most ? b.f[i].n_pix : most;
  }
  int64_t bx = (most + kThreads - 1) / kThreads;
  if (bx > 4096) bx = 4096;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)bx, b.n_frames), dim3(kThreads), 0, s, b);
  return hipGetLastError();
}

}  // namespace rc
