// Range compression: beat signal -> equidistant beat spectrum s (the input
// that Alg. 1 and Alg. 2 interpolate; Sec. III-C of the paper).
//
// s[row][k] = sum_{t < n_s} w_range[t] raw[row][t] exp(-2 pi i k t / n_fft),
// k < n_bins, computed as an n_fft-point FFT of the zero-padded row.
//
// Design (HBM-bound stage): a self-sorting (Stockham) FFT whose passes are
// radix-16 butterflies held in registers, 16 samples per lane, so a 2048-point
// row takes three passes and two exchanges through LDS instead of eleven
// radix-2 stages.  The first pass reads the windowed samples straight from
// HBM (coalesced: lane j of a row reads samples j + r n/16) and treats the
// zero padding as zeros without loading it; the last pass keeps only the
// n_bins bins that are written, directly in the interleaved (intercept,
// slope) layout that back-projection gathers with one 16-byte load per term,
// with the chirp window w_sar[m] folded in.  Pass p of radix R at stride Ns
// multiplies input r of butterfly b by W_{Ns R}^{(b mod Ns) r} (evaluated by the
// hardware sine and cosine, which take their argument in turns: the argument
// (b mod Ns) r / (Ns R) is exact in single precision, so each twiddle carries
// only the unit's own rounding, about 1e-7, and costs no memory access) and
// writes output r to (b / Ns) Ns R + (b mod Ns) + r Ns.  When every
// row of a launch has at most n_fft / 2 samples (zero padding by two or more,
// the usual case), the upper half of every first-pass butterfly's inputs is
// zero at compile time: neither loaded nor computed.  LDS rows are padded by one element
// per 16, which keeps the stride-16 writes of the first passes free of bank
// conflicts.  Rows shorter than 16 x 64 samples share a workgroup.  Samples
// and the range window are read through buffer descriptors: the
// zero padding and the rows past the frame read past the descriptor's range,
// which returns zeros without a branch.
#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// x * exp(-2 pi i q / 16), q in [0, 8)
template <int Q>
__device__ __forceinline__ float2 rot16(float2 x) {
  constexpr float c1 = 0.92387953251128674f;  // cos(pi / 8)
  constexpr float s1 = 0.38268343236508978f;  // sin(pi / 8)
  constexpr float h = 0.70710678118654752f;   // sqrt(1/2)
  if constexpr (Q == 0) return x;
  else if constexpr (Q == 4) return make_float2(x.y, -x.x);
  else if constexpr (Q == 2) return make_float2(h * (x.x + x.y), h * (x.y - x.x));
  else if constexpr (Q == 6) return make_float2(h * (x.y - x.x), -h * (x.x + x.y));
  else {
    constexpr float c = Q == 1 ? c1 : Q == 3 ? s1 : Q == 5 ? -s1 : -c1;
    constexpr float s = Q == 1 ? s1 : Q == 3 ? c1 : Q == 5 ? c1 : s1;
    return make_float2(fmaf(x.x, c, x.y * s), fmaf(x.y, c, -x.x * s));
  }
}

template <int R>
constexpr int bitrev(int r) {
  int o = 0;
  for (int b = 1; b < R; b <<= 1) o = (o << 1) | ((r & b) ? 1 : 0);
  return o;
}

// In-register DFT of R = 2^q points: radix-2 decimation-in-frequency stages
// on natural-order input; X[r] ends in v[bitrev(r)] (callers index through
// bitrev, so the permutation costs nothing).
template <int R, int S>
__device__ __forceinline__ void dif_stage(float2* v) {
#pragma unroll
  for (int blk = 0; blk < R; blk += 2 * S) {
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const float2 a = v[blk + k], b = v[blk + k + S];
      v[blk + k] = cadd(a, b);
      const float2 d = csub(a, b);
      // W_{2S}^k = W_16^{k 16 / (2S)}
      constexpr int step = 16 / (2 * S);
      switch (k * step) {
        case 0: v[blk + k + S] = d; break;
        case 1: v[blk + k + S] = rot16<1>(d); break;
        case 2: v[blk + k + S] = rot16<2>(d); break;
        case 3: v[blk + k + S] = rot16<3>(d); break;
        case 4: v[blk + k + S] = rot16<4>(d); break;
        case 5: v[blk + k + S] = rot16<5>(d); break;
        case 6: v[blk + k + S] = rot16<6>(d); break;
        default: v[blk + k + S] = rot16<7>(d); break;
      }
    }
  }
}

template <int R>
__device__ __forceinline__ void dft_br(float2* v) {
  if constexpr (R >= 16) dif_stage<R, 8>(v);
  if constexpr (R >= 8) dif_stage<R, 4>(v);
  if constexpr (R >= 4) dif_stage<R, 2>(v);
  if constexpr (R >= 2) dif_stage<R, 1>(v);
}

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

template <int LOG2N>
struct Fft {
  static constexpr int N = 1 << LOG2N;
  static constexpr int E = N < 16 ? N : 16;  // samples per lane
  static constexpr int T = N / E;            // lanes per row
  static constexpr int RPW = kThreads / T;   // rows per workgroup
  static constexpr int PADN = N + N / 16;    // padded LDS row
};

struct RowIo {
  __amdgpu_buffer_rsrc_t raw;   // the frame's samples
  __amdgpu_buffer_rsrc_t win;   // w_range; an index past n_s reads 0
  unsigned row_off;             // byte offset of this lane's row in raw
  bool live;
};

// One Stockham pass of radix R at stride NS over the E samples of this lane
// (E / R butterflies b = j + T u).  HALF (first pass only): inputs r >= R / 2
// lie at or beyond n_fft / 2 >= n_s, i.e. in the zero padding.
template <int LOG2N, int R, int NS, bool FIRST, bool LAST, bool HALF = false>
__device__ __forceinline__ void fft_pass(const RangeArgs& a, const RowIo& io, float2* buf, int j) {
  using F = Fft<LOG2N>;
  constexpr int N = F::N, E = F::E, T = F::T, B = E / R;
  float2 v[E];
  float2 w[E];
  if constexpr (NS > 1) {
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int b = j + T * u;
      // W_{NS R}^{(b mod NS) r} = exp(-2 pi i t), t = (b mod NS) r / (NS R) turns
      const float q = (float)(b & (NS - 1)) * (1.0f / (float)(NS * R));
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float t = q * (float)r;
        w[u * R + r] = make_float2(__builtin_amdgcn_cosf(t), -__builtin_amdgcn_sinf(t));
      }
    }
  }
#pragma unroll
  for (int u = 0; u < B; ++u) {
    const int b = j + T * u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = b + r * (N / R);
      if constexpr (FIRST && HALF) {
        if (r >= R / 2) {
          v[u * R + r] = make_float2(0.f, 0.f);
          continue;
        }
      }
      if constexpr (FIRST) {
        // zero padding and dead rows read past the descriptor, which returns zeros
        const unsigned off = (io.live && i < a.n_s) ? io.row_off + (unsigned)i * 8u : 0xfffffff0u;
        const u32x2 z = __builtin_amdgcn_raw_buffer_load_b64(io.raw, off, 0, 0);
        const float wr = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(io.win, (unsigned)i * 4u, 0, 0));
        v[u * R + r] = make_float2(__uint_as_float(z.x) * wr, __uint_as_float(z.y) * wr);
      } else {
        v[u * R + r] = buf[pad(i)];
      }
    }
  }
  if constexpr (!FIRST) __syncthreads();  // every read of this pass precedes its writes
#pragma unroll
  for (int u = 0; u < B; ++u) {
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[u * R + r] = cmul(v[u * R + r], w[u * R + r]);
    }
    dft_br<R>(v + u * R);
  }
#pragma unroll
  for (int u = 0; u < B; ++u) {
    const int b = j + T * u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float2 x = v[u * R + bitrev<R>(r)];
      if constexpr (LAST) {
        // natural order after the last pass; only the kept bins are stored
        if (r * NS < a.n_bins) {
          const int k = b + r * NS;
          if (k < a.n_bins) buf[pad(k)] = x;
        }
      } else {
        const int i = (b / NS) * NS * R + (b & (NS - 1)) + r * NS;
        buf[pad(i)] = x;
      }
    }
  }
  __syncthreads();
}

template <int LOG2N, bool HALF>
__global__ __launch_bounds__(kThreads) void range_compress_kernel(RangeMulti m) {
  using F = Fft<LOG2N>;
  __shared__ float2 lds[F::RPW * F::PADN];
  const int fi = multi_frame(m, blockIdx.x);
  const RangeArgs a = m.f[fi];
  const int lrow = threadIdx.x / F::T;
  const int j = threadIdx.x - lrow * F::T;
  const int64_t row = (int64_t)(blockIdx.x - m.begin[fi]) * F::RPW + lrow;
  const bool live = row < a.rows;
  float2* buf = lds + lrow * F::PADN;
  RowIo io;
  io.raw = __builtin_amdgcn_make_buffer_rsrc((void*)a.raw, (short)0, (int)(a.rows * a.n_s * 8), kRsrcWord3);
  io.row_off = (unsigned)(row * a.n_s) * 8u;
  io.live = live;
  io.win = __builtin_amdgcn_make_buffer_rsrc((void*)a.w_range, (short)0, a.n_s * 4, kRsrcWord3);

  if constexpr (LOG2N < 4) {
    fft_pass<LOG2N, F::N, 1, true, true, HALF>(a, io, buf, j);
  } else {
    constexpr int P16 = LOG2N / 4, REM = LOG2N % 4;
    fft_pass<LOG2N, 16, 1, true, P16 == 1 && REM == 0, HALF>(a, io, buf, j);
    if constexpr (P16 >= 2) fft_pass<LOG2N, 16, 16, false, P16 == 2 && REM == 0>(a, io, buf, j);
    if constexpr (P16 >= 3) fft_pass<LOG2N, 16, 256, false, REM == 0>(a, io, buf, j);
    if constexpr (REM > 0) fft_pass<LOG2N, (1 << REM), (1 << (4 * P16)), false, true>(a, io, buf, j);
  }

  if (!live) return;
  const float w = a.w_sar[row / a.n_ch];
  float4* dst = a.pairs + row * a.n_bins;
  float2* spec = a.spectrum ? a.spectrum + row * a.n_bins : nullptr;
  const int last = a.n_bins - 1;
  for (int k = j; k < a.n_bins; k += F::T) {
    const float2 x = buf[pad(k)];
    const float2 d = (k < last) ? csub(buf[pad(k + 1)], x) : make_float2(0.f, 0.f);
    dst[k] = table_entry(w, x, d, k);
    if (spec) spec[k] = x;
  }
}

template <int LOG2N>
hipError_t launch_fft(RangeMulti m, hipStream_t s) {
  using F = Fft<LOG2N>;
  int64_t grid = 0;
  bool half = true;
  for (int i = 0; i < m.n_frames; ++i) {
    m.begin[i] = (int)grid;
    grid += (m.f[i].rows + F::RPW - 1) / F::RPW;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    half = half && 2 * m.f[i].n_s <= F::N;
  }
  m.begin[m.n_frames] = (int)grid;
  if (grid == 0) return hipSuccess;
  if (half)
    hipLaunchKernelGGL((range_compress_kernel<LOG2N, true>), dim3((unsigned)grid), dim3(kThreads), 0, s, m);
  else
    hipLaunchKernelGGL((range_compress_kernel<LOG2N, false>), dim3((unsigned)grid), dim3(kThreads), 0, s, m);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void spectrum_pairs_kernel(PairMulti m) {
  const int fi = multi_frame(m, blockIdx.x);
  const PairArgs a = m.f[fi];
  const int64_t i = (int64_t)(blockIdx.x - m.begin[fi]) * kThreads + threadIdx.x;
  const int64_t total = a.rows * a.n_bins;
  if (i >= total) return;
  const int64_t row = i / a.n_bins;
  const int k = (int)(i - row * a.n_bins);
  const float w = a.w_sar[row / a.n_ch];
  const float2 x = a.spec[i];
  const float2 d = (k < a.n_bins - 1) ? csub(a.spec[i + 1], x) : make_float2(0.f, 0.f);
  a.pairs[i] = table_entry(w, x, d, k);
}

}  // namespace

hipError_t launch_range_compress(const RangeMulti& m, hipStream_t s) {
  if (m.n_frames < 1 || m.n_frames > RangeMulti::kMax) return hipErrorInvalidValue;
  const int log2n = m.f[0].log2n;
  for (int i = 0; i < m.n_frames; ++i) {
    const RangeArgs& a = m.f[i];
    if (a.rows < 0 || a.n_fft < 4 || (a.n_fft & (a.n_fft - 1)) || (1 << a.log2n) != a.n_fft ||
        a.n_fft > 4096 || a.log2n != log2n || a.n_s < 1 || a.n_s > a.n_fft || a.n_bins < 1 ||
        a.n_bins > a.n_fft || a.n_ch < 1 || a.rows * a.n_s * 8 >= (int64_t(1) << 31))
      return hipErrorInvalidValue;
  }
  switch (log2n) {
    case 2: return launch_fft<2>(m, s);
    case 3: return launch_fft<3>(m, s);
    case 4: return launch_fft<4>(m, s);
    case 5: return launch_fft<5>(m, s);
    case 6: return launch_fft<6>(m, s);
    case 7: return launch_fft<7>(m, s);
    case 8: return launch_fft<8>(m, s);
    case 9: return launch_fft<9>(m, s);
    case 10: return launch_fft<10>(m, s);
    case 11: return launch_fft<11>(m, s);
    default: return launch_fft<12>(m, s);
  }
}

hipError_t launch_spectrum_pairs(const PairMulti& m0, hipStream_t s) {
  if (m0.n_frames < 1 || m0.n_frames > PairMulti::kMax) return hipErrorInvalidValue;
  PairMulti m = m0;
  int64_t grid = 0;
  for (int i = 0; i < m.n_frames; ++i) {
    const PairArgs& a = m.f[i];
    if (a.n_ch < 1 || a.rows < 0 || a.n_bins < 1) return hipErrorInvalidValue;
    m.begin[i] = (int)grid;
    grid += (a.rows * a.n_bins + kThreads - 1) / kThreads;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
  }
  m.begin[m.n_frames] = (int)grid;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(spectrum_pairs_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, m);
  return hipGetLastError();
}

}  // namespace rc
