// Range compression on the matrix cores (the reduced-precision spectrum form):
// the same windowed, zero-padded DFT of every (chirp, channel) row as the
// single-precision FFT (the beat spectrum Alg. 1 and Alg. 2 interpolate,
// Sec. III-C), computed as two small complex matrix products of a
// Cooley-Tukey split of the N-point DFT into N1 = 32 and N2 = N / 32 points:
//   t = t1 + 32 t2,  k = k2 + N2 k1,
//   Y[t1][k2]      = sum_{t2} x[t1 + 32 t2] W_N2^(t2 k2)            (stage 1)
//   s[k2 + N2 k1]  = sum_{t1} W_32^(k1 t1) (W_N^(t1 k2) Y[t1][k2])  (stage 2)
// with W_n = exp(-2 pi i / n).  The zero padding (n_s <= N / 2) halves the t2
// range, and only the k1 rows that reach the n_bins kept bins are formed.
//
// A complex product runs as a real one in which every complex entry is a 2 x 2
// real block, on MFMA with FP16 or BF16 operands and FP32 accumulation
// (stage 1: v_mfma_f32_32x32x16, the 32 rows t1 of one row's data against a
// 16-wide slab of k2; stage 2: v_mfma_f32_16x16x32, the k1 rows against a
// 16-wide slab of k2).  The twiddles of both stages are constant operands and
// enter split into a high and a low part (hi + lo carries ~22 significant
// bits, as much as the single-precision sine and cosine they come from), so
// the data operand is the only one rounded to the 16-bit type: once on entry
// and once between the stages.  BF16 (8-bit mantissa) also splits the data
// operand and forms hi*hi + hi*lo + lo*hi; FP16 (11 bits) forms data*hi +
// data*lo.  FP16's range is kept by scaling each row by a power of two from
// its largest sample (exact, undone on output).  The twiddle between the
// stages and everything after stage 2 run in single precision.
//
// Work distribution: one workgroup per row at a time, max(1, N2 / 16) waves,
// wave w owning k2 in [16 w, 16 w + 16) in both stages; the row's data are read
// by every wave (the L1 and L2 serve the repeats); Y crosses to the stage-2
// layout through LDS; the kept bins go through LDS once more to be written as
// the interpolation table of back-projection (intercept and slope of the
// segment from bin k to k + 1, the chirp window folded in), 16 bytes per
// bin, coalesced.  Workgroups stay resident and
// loop over the rows of the launch, loading each row one trip ahead; the
// twiddle operands are formed where they are used (from the hardware sine and
// cosine), which costs a few transcendentals per output and keeps the
// register count, and so the rows in flight per CU, up.
#include "rc_kernels.hpp"

namespace rc {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)

template <bool BF>
struct Op;
template <>
struct Op<false> {
  using T = _Float16;
  using V = h8;
  static __device__ __forceinline__ f16v mma32(V a, V b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ f4v mma16(V a, V b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Op<true> {
  using T = __bf16;
  using V = b8;
  static __device__ __forceinline__ f16v mma32(V a, V b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ f4v mma16(V a, V b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// element j of a hi and a lo operand vector: v split into the 16-bit type
// (hi) and the 16-bit rounding of what hi misses (lo)
template <bool BF>
__device__ __forceinline__ void put(float v, typename Op<BF>::V& hi, typename Op<BF>::V& lo, int j) {
  using T = typename Op<BF>::T;
  const T h = (T)v;
  hi[j] = h;
  lo[j] = (T)(v - (float)h);
}

// exp(-2 pi i num / den) for integers 0 <= num < den (den a power of two): the
// argument in turns is exact in single precision and the hardware sine and
// cosine take turns
__device__ __forceinline__ float2 twiddle(int num, int den) {
  const float t = (float)num / (float)den;
  return make_float2(__builtin_amdgcn_cosf(t), -__builtin_amdgcn_sinf(t));
}

constexpr int kN1 = 32;

// v, hidden from the compiler's loop-invariant code motion: values formed
// from it inside a loop are formed on every trip instead of being kept live
// in registers across the loop
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

template <int LOG2N>
struct Mfft {
  static constexpr int N = 1 << LOG2N;
  static constexpr int N2 = N / kN1;
  static constexpr int W = N2 >= 16 ? N2 / 16 : 1;  // waves per workgroup
  static constexpr int S1 = N2 >= 16 ? N2 / 16 : 1;  // stage-1 K steps (8 complex t2 each, t2 < N2 / 2)
  static constexpr int ZROW = kN1 * 2 + 8;          // LDS halves per k2 row of Y (t1, re/im; padded)
  static constexpr int K2R = W * 16;                // k2 rows held (>= N2)
};

template <int LOG2N, bool BF, int MT>
__global__ __launch_bounds__(64 * Mfft<LOG2N>::W) void range_mfma_kernel(RangeMulti m, int64_t total_rows) {
  using F = Mfft<LOG2N>;
  using O = Op<BF>;
  using T = typename O::T;
  using V = typename O::V;
  constexpr int N = F::N, N2 = F::N2, S1 = F::S1;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* zh = reinterpret_cast<T*>(lds_raw);                       // [K2R][ZROW]: Y after the twiddle (hi)
  T* zl = zh + F::K2R * F::ZROW;                               // (lo, BF16 only)
  float2* sb = reinterpret_cast<float2*>(lds_raw + (BF ? 2 : 1) * F::K2R * F::ZROW * sizeof(T));

  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int h32 = lane >> 5;           // 32x32x16 operand layout: which 8 of the 16 K
  const int h16 = lane >> 4;           // 16x16x32 operand layout: which 8 of the 32 K

  // ---- per-wave constants ----
  // this lane's stage-1 output column 32 w + (lane & 31) = (k2, c)
  const int col1 = 32 * w + (lane & 31);
  const int k2s1 = col1 >> 1, c1 = col1 & 1;
  // k2 rows of the LDS slab beyond N2 (N2 = 8) stay zero
  if constexpr (N2 < 16) {
    for (int i = threadIdx.x; i < (BF ? 2 : 1) * F::K2R * F::ZROW; i += 64 * F::W) zh[i] = (T)0.f;
    __syncthreads();
  }

  // the samples of a row for this lane's K steps: t = (lane & 31) + 32 t2,
  // t2 = 8 s + 4 h32 + q, through a buffer descriptor (a sample past the row
  // reads past the descriptor's range: zero, no branch).  Rows are loaded one
  // trip ahead, so a row's loads are in flight while the previous row is
  // transformed; the window values of the current row are requested before
  // that prefetch, so waiting for them does not wait for it.
  // (a row past the launch's last reads zeros: the loads are issued on every
  // trip, so the compiler's wait counts stay exact and the prefetch is never
  // waited for early)
  auto load_row = [&](int64_t gr, float2 (&dst)[S1][4]) {
    const bool live = gr < total_rows;
    int fj = 0;
    while (fj + 1 < m.n_frames && gr >= m.begin[fj + 1]) ++fj;
    fj = __builtin_amdgcn_readfirstlane(fj);
    const RangeArgs& b = m.f[fj];
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)b.raw, (short)0, (int)(b.rows * b.n_s * 8), kRsrcWord3);
    const unsigned base = (unsigned)((gr - m.begin[fj]) * b.n_s) * 8u;
#pragma unroll
    for (int s = 0; s < S1; ++s) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t = (lane & 31) + kN1 * (8 * s + 4 * h32 + q);
        const unsigned off = live && t < b.n_s ? base + (unsigned)t * 8u : 0xfffffff0u;
        const u32x2 z = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
        dst[s][q] = make_float2(__uint_as_float(z.x), __uint_as_float(z.y));
      }
    }
  };
  float2 xn[S1][4];
  if (blockIdx.x < total_rows) load_row(blockIdx.x, xn);

  for (int64_t g = blockIdx.x; g < total_rows; g += gridDim.x) {
    int fi = 0;
    while (fi + 1 < m.n_frames && g >= m.begin[fi + 1]) ++fi;
    fi = __builtin_amdgcn_readfirstlane(fi);
    const RangeArgs& a = m.f[fi];
    const int64_t r = g - m.begin[fi];

    // ---- stage 1 ----
    const __amdgpu_buffer_rsrc_t wrs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)a.w_range, (short)0, a.n_s * 4, kRsrcWord3);
    float wr[S1][4];
#pragma unroll
    for (int s = 0; s < S1; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t = (lane & 31) + kN1 * (8 * s + 4 * h32 + q);
        wr[s][q] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(wrs, (unsigned)t * 4u, 0, 0));
      }
    float2 x[S1][4];
#pragma unroll
    for (int s = 0; s < S1; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q) x[s][q] = xn[s][q];
    load_row(g + gridDim.x, xn);
    float amax = 0.f;
#pragma unroll
    for (int s = 0; s < S1; ++s) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x[s][q] = make_float2(x[s][q].x * wr[s][q], x[s][q].y * wr[s][q]);
        amax = fmaxf(amax, fmaxf(fabsf(x[s][q].x), fabsf(x[s][q].y)));
      }
    }
    // FP16: scale the row by 2^e so that its largest windowed sample is below
    // 2^8 (a real stage-1 output sums at most 2 (N2 / 2) <= 128 such values:
    // below 2^15, inside FP16's range)
    float scale = 1.f, unscale = 1.f;
    if constexpr (!BF) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
      if (amax > 0.f) {
        const int e = 8 - ilogbf(amax) - 1;  // amax 2^e < 2^8
        scale = ldexpf(1.f, e);
        unscale = ldexpf(1.f, -e);
      }
    }
    f16v acc = {};
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      if (8 * s * kN1 >= a.n_s) break;  // the rest of the rows' samples are zero padding
      V ah, al;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        put<BF>(x[s][q].x * scale, ah, al, 2 * q);
        put<BF>(x[s][q].y * scale, ah, al, 2 * q + 1);
      }
      // B operand of K step s: rows (t2, d), column (k2, c) of the 2 x 2 real
      // block of W_N2^(t2 k2) (re of the product takes (Wr, -Wi) against
      // (xr, xi), im takes (Wi, Wr)); formed per step, which keeps the
      // register count down
      V bh, bl;
      const int k2o = opaque(k2s1);
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        const int t2 = 8 * s + 4 * h32 + (j >> 1);
        float2 W2 = make_float2(0.f, 0.f);
        if (k2o < N2) W2 = twiddle((t2 * k2o) & (N2 - 1), N2);
        put<BF>(c1 == 0 ? W2.x : W2.y, bh, bl, j);
        put<BF>(c1 == 0 ? -W2.y : W2.x, bh, bl, j + 1);
      }
      acc = O::mma32(ah, bh, acc);
      acc = O::mma32(ah, bl, acc);
      if constexpr (BF) acc = O::mma32(al, bh, acc);
    }

    // ---- twiddle, then Y to the stage-2 layout through LDS ----
    // lane pairs (c = 0, 1) hold the re and im of the same (t1, k2); this
    // lane's outputs are rows t1 = 8 (a / 4) + 4 h32 + a % 4 of column (k2, c),
    // each multiplied by W_N^(t1 k2) (formed per row, as the stage-1 operand)
    float z[16];
    const int k2t = opaque(k2s1);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int t1 = 8 * (i >> 2) + 4 * h32 + (i & 3);
      const float2 W = twiddle((t1 * k2t) & (N - 1), N);
      const float own = acc[i];
      const float other = __shfl_xor(own, 1, 64);
      // Zr = Yr Wr - Yi Wi, Zi = Yi Wr + Yr Wi
      z[i] = fmaf(other, c1 == 0 ? -W.y : W.y, own * W.x);
    }
    // the c = 0 lane writes rows t1 of groups 0, 1 (a < 8), the c = 1 lane of
    // groups 2, 3, each group four consecutive t1 as (re, im) pairs
#pragma unroll
    for (int gsel = 0; gsel < 2; ++gsel) {
      float zo[4], zp[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i0 = 4 * gsel + q;       // group gsel (c = 0 lane)
        const int i1 = 4 * (gsel + 2) + q; // group gsel + 2 (c = 1 lane)
        const float mine = c1 == 0 ? z[i0] : z[i1];
        const float send = c1 == 0 ? z[i1] : z[i0];
        zo[q] = mine;
        zp[q] = __shfl_xor(send, 1, 64);
      }
      const int grp = c1 == 0 ? gsel : gsel + 2;
      const int t1 = 8 * grp + 4 * h32;
      if (k2s1 < N2) {
        V hv, lv;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float re = c1 == 0 ? zo[q] : zp[q];
          const float im = c1 == 0 ? zp[q] : zo[q];
          put<BF>(re, hv, lv, 2 * q);
          put<BF>(im, hv, lv, 2 * q + 1);
        }
        *reinterpret_cast<V*>(zh + k2s1 * F::ZROW + 2 * t1) = hv;
        if constexpr (BF) *reinterpret_cast<V*>(zl + k2s1 * F::ZROW + 2 * t1) = lv;
      }
    }
    __syncthreads();

    // ---- stage 2 ----
    const int n_k1 = (a.n_bins + N2 - 1) / N2;      // k1 rows reaching the kept bins
    const int k2b = 16 * w + (lane & 15);
    const int row2 = opaque(lane & 15);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      if (16 * mt >= 2 * n_k1) break;
      f4v acc2 = {};
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        // A operand: rows (k1, c) of M tile mt, columns (t1, d) of K step s2:
        // the 2 x 2 real block of W_32^(k1 t1)
        V ah, al;
        const int k1 = 8 * mt + (row2 >> 1), c = row2 & 1;
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          const int t1 = 16 * s2 + 4 * h16 + (j >> 1);
          const float2 W1 = twiddle((k1 * t1) & (kN1 - 1), kN1);
          put<BF>(c == 0 ? W1.x : W1.y, ah, al, j);
          put<BF>(c == 0 ? -W1.y : W1.x, ah, al, j + 1);
        }
        const int t1 = 16 * s2 + 4 * h16;
        const V bh = *reinterpret_cast<const V*>(zh + k2b * F::ZROW + 2 * t1);
        acc2 = O::mma16(ah, bh, acc2);
        acc2 = O::mma16(al, bh, acc2);
        if constexpr (BF) {
          const V bl = *reinterpret_cast<const V*>(zl + k2b * F::ZROW + 2 * t1);
          acc2 = O::mma16(ah, bl, acc2);
        }
      }
      // rows 4 h16 + i = (k1, c): k1 = 8 mt + 2 h16 + i / 2
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int k1 = 8 * mt + 2 * h16 + p;
        const int k = k2b + N2 * k1;
        if (k2b < N2 && k < a.n_bins) sb[k] = make_float2(acc2[2 * p] * unscale, acc2[2 * p + 1] * unscale);
      }
    }
    __syncthreads();

    // ---- the interpolation table ----
    const float wv = a.w_sar[r / a.n_ch];
    float4* dst = a.pairs + r * a.n_bins;
    float2* spec = a.spectrum ? a.spectrum + r * a.n_bins : nullptr;
    const int last = a.n_bins - 1;
    for (int k = threadIdx.x; k < a.n_bins; k += 64 * F::W) {
      const float2 v = sb[k];
      const float2 d = k < last ? make_float2(sb[k + 1].x - v.x, sb[k + 1].y - v.y) : make_float2(0.f, 0.f);
      dst[k] = table_entry(wv, v, d, k);
      if (spec) spec[k] = v;
    }
    __syncthreads();
  }
}

template <int LOG2N, bool BF>
hipError_t launch_mt(RangeMulti m, int max_bins, hipStream_t s) {
  using F = Mfft<LOG2N>;
  int64_t total = 0;
  for (int i = 0; i < m.n_frames; ++i) {
    m.begin[i] = (int)total;
    total += m.f[i].rows;
    if (total > 0x7fffffff) return hipErrorInvalidValue;
  }
  m.begin[m.n_frames] = (int)total;
  if (total == 0) return hipSuccess;
  const int n_k1 = (max_bins + F::N2 - 1) / F::N2;
  const int mt = (2 * n_k1 + 15) / 16;
  const size_t lds = (BF ? 2 : 1) * F::K2R * F::ZROW * sizeof(typename Op<BF>::T) + (size_t)max_bins * sizeof(float2);
  const dim3 block(64 * F::W);
  auto go = [&](auto kernel) {
    // more than 64 KiB of dynamic LDS (4096-point rows keeping most bins) needs the attribute
    if (lds > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    // as many workgroups as stay resident, each looping over its share of the rows
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), (int)block.x,
                                                       lds);
    if (e != hipSuccess) return e;
    const int64_t blocks = std::min<int64_t>(total, (int64_t)std::max(1, cus) * std::max(1, per_cu));
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), block, lds, s, m, total);
    return hipGetLastError();
  };
  if (mt <= 1) return go(range_mfma_kernel<LOG2N, BF, 1>);
  if (mt <= 2) return go(range_mfma_kernel<LOG2N, BF, 2>);
  return go(range_mfma_kernel<LOG2N, BF, 4>);
}

template <bool BF>
hipError_t launch_kind(const RangeMulti& m, int log2n, int max_bins, hipStream_t s) {
  switch (log2n) {
    case 8: return launch_mt<8, BF>(m, max_bins, s);
    case 9: return launch_mt<9, BF>(m, max_bins, s);
    case 10: return launch_mt<10, BF>(m, max_bins, s);
    case 11: return launch_mt<11, BF>(m, max_bins, s);
    case 12: return launch_mt<12, BF>(m, max_bins, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool range_mfma_supported(int n_fft, int n_s) {
  return n_fft >= kRangeMfmaMinFft && n_fft <= kRangeMfmaMaxFft && (n_fft & (n_fft - 1)) == 0 && 2 * n_s <= n_fft;
}

hipError_t launch_range_mfma(const RangeMulti& m, bool bf16, hipStream_t s) {
  if (m.n_frames < 1 || m.n_frames > RangeMulti::kMax) return hipErrorInvalidValue;
  const int log2n = m.f[0].log2n;
  int max_bins = 1;
  for (int i = 0; i < m.n_frames; ++i) {
    const RangeArgs& a = m.f[i];
    if (a.rows < 0 || a.log2n != log2n || (1 << a.log2n) != a.n_fft || !range_mfma_supported(a.n_fft, a.n_s) ||
        a.n_s < 1 || a.n_bins < 1 || a.n_bins > a.n_fft || a.n_ch < 1 ||
        a.rows * a.n_s * 8 >= (int64_t(1) << 31))
      return hipErrorInvalidValue;
    max_bins = a.n_bins > max_bins ? a.n_bins : max_bins;
  }
  return bf16 ? launch_kind<true>(m, log2n, max_bins, s) : launch_kind<false>(m, log2n, max_bins, s);
}

}  // namespace rc
