// Detection stage on the SAR image (not part of the paper): 2-D square-law
// cell-averaging CFAR over the pixel lattice, then ordered compaction.
//
// For a cell with its whole window inside the lattice the training set is the
// (2h+1)^2 square (h = guard + train) minus the (2g+1)^2 guard square; the cell
// is a detection iff |P|^2 > alpha / N * sum(training).  Powers and box sums
// are formed in double, so the decision differs from an exact evaluation only
// through the image itself.
//
// A 256-thread workgroup produces 16 rows x 64 columns of decisions (each
// wave four row segments, whose ballots are those segments' 64-bit mask
// words).  The (16 + 2h) x (64 + 2h) power halo is staged in LDS (sized for
// the launch's h), box sums are separable: vertical sums per halo column
// first, then horizontal sums per cell, each summed directly in double.
#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;
constexpr int kTileRows = 16;
constexpr int kTileCols = 64;
constexpr int kMaxHalf = 16;  // guard + train <= 16

__host__ __device__ constexpr size_t cfar_lds_bytes(int h) {
  return sizeof(double) * (size_t)(kTileCols + 2 * h) * ((kTileRows + 2 * h) + 2 * kTileRows);
}

__global__ __launch_bounds__(kThreads) void cfar_kernel(CfarMulti m) {
  extern __shared__ double smem[];
  const int fi = multi_frame(m, blockIdx.x);
  const CfarArgs a = m.f[fi];
  const int tile = blockIdx.x - m.begin[fi];
  const int bx = tile % a.words_per_row, by = tile / a.words_per_row;  // one mask word per 64 columns
  const int h = a.guard + a.train;
  const int g = a.guard;
  const int r0 = by * kTileRows;
  const int c0 = bx * kTileCols;
  const int hr = kTileRows + 2 * h, hc = kTileCols + 2 * h;
  double* pw = smem;                  // [hr][hc]
  double* vo = pw + hr * hc;          // [kTileRows][hc]
  double* vi = vo + kTileRows * hc;   // [kTileRows][hc]

  for (int e = threadIdx.x; e < hr * hc; e += kThreads) {
    const int i = e / hc, j = e - i * hc;
    const int r = r0 - h + i, c = c0 - h + j;
    double v = 0.0;
    if (r >= 0 && r < a.n_rows && c >= 0 && c < a.n_cols) {
      const float2 z = a.img[(int64_t)r * a.n_cols + c];
      v = (double)z.x * z.x + (double)z.y * z.y;
    }
    pw[e] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kTileRows * hc; e += kThreads) {
    const int i = e / hc, j = e - i * hc;
    double so = 0.0, si = 0.0;
    for (int d = 0; d <= 2 * h; ++d) so += pw[(i + d) * hc + j];
    for (int d = h - g; d <= h + g; ++d) si += pw[(i + d) * hc + j];
    vo[e] = so;
    vi[e] = si;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  for (int i = threadIdx.x >> 6; i < kTileRows; i += kThreads / 64) {  // tile row of this wave
    const int r = r0 + i, c = c0 + lane;
    double so = 0.0, si = 0.0;
    for (int d = 0; d <= 2 * h; ++d) so += vo[i * hc + lane + d];
    for (int d = h - g; d <= h + g; ++d) si += vi[i * hc + lane + d];
    const double thr = a.alpha_over_n * (so - si);
    const double p = pw[(i + h) * hc + lane + h];
    const bool tested = r >= h && r < a.n_rows - h && c >= h && c < a.n_cols - h;
    const bool det = tested && p > thr;
    const unsigned long long word = __ballot(det);
    if (r < a.n_rows && lane == 0)
      a.mask[(int64_t)r * a.words_per_row + bx] = word;
    const bool near = tested && fabs(p - thr) <= a.margin_rel * thr;
    bool listed = false;
    if (near && a.recheck_cap > 0) {
      const int pos = atomicAdd(a.n_listed, 1);
      if (pos < a.recheck_cap) {
        a.listed[pos] = r * a.n_cols + c;
        listed = true;
      }
    }
    if (det) {
      const int64_t cell = (int64_t)r * a.n_cols + c;
      rc_detection d;
      d.pixel = (int32_t)cell;
      d.power = (float)p;
      d.threshold = (float)thr;
      d.flags = (near && !listed) ? RC_DET_NEAR_THRESHOLD : 0u;
      a.det_cell[cell] = d;
    }
  }
}

constexpr int kCompactWords = 8;  // mask words per thread per sweep
// A frame whose mask fits in this many sweeps of a 256-thread workgroup is
// compacted by one: while another stream's back-projection holds the CUs, a
// workgroup of four waves finds room as soon as one of its workgroups ends,
// where one of sixteen waves may wait for a CU to drain.
constexpr int kCompactSmallSweeps = 4;

// Inclusive prefix sum over the 64 lanes of a wave (shuffles, no barrier).
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

// Ordered compaction of one frame's detection mask: each sweep covers
// THREADS x 8 consecutive mask words; a thread counts its eight words, the
// workgroup scans the thread totals (wave scans, then a scan of the wave
// totals), every thread writes the cell index of each set bit of its words
// to its output slot, and then all threads copy the sweep's records from
// those cells in parallel (detections cluster, so a thread may own many set
// bits: copying them one by one would chain that many memory latencies).
// Output order is ascending pixel index.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void compact_kernel(CompactMulti m) {
  const CompactArgs a = m.f[__builtin_amdgcn_readfirstlane((int)blockIdx.x)];  // one workgroup per frame
  __shared__ int wave_sum[THREADS / 64];
  __shared__ int64_t base_sh;
  const int64_t n_words = (int64_t)a.n_rows * a.words_per_row;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) base_sh = 0;
  __syncthreads();
  for (int64_t w0 = 0; w0 < n_words; w0 += (int64_t)THREADS * kCompactWords) {
    const int64_t wt = w0 + (int64_t)threadIdx.x * kCompactWords;
    unsigned long long word[kCompactWords];
    int total = 0;
#pragma unroll
    for (int k = 0; k < kCompactWords; ++k) {
      word[k] = (wt + k < n_words) ? a.mask[wt + k] : 0ull;
      total += __popcll(word[k]);
    }
    const int incl = wave_inclusive_scan(total);
    if (lane == 63) wave_sum[wave] = incl;
    __syncthreads();
    if (wave == 0) {
      const int ws = lane < THREADS / 64 ? wave_sum[lane] : 0;
      const int wincl = wave_inclusive_scan(ws);
      if (lane < THREADS / 64) wave_sum[lane] = wincl - ws;  // exclusive
    }
    __syncthreads();
    const int64_t base = base_sh;
    int64_t pos = base + wave_sum[wave] + incl - total;
    if (total) {
#pragma unroll
      for (int k = 0; k < kCompactWords; ++k) {
        unsigned long long bits = word[k];
        if (!bits) continue;
        const int64_t w = wt + k;
        const int64_t r = w / a.words_per_row;
        const int64_t cb = (w - r * a.words_per_row) * 64;
        while (bits) {
          const int b = __ffsll((long long)bits) - 1;
          bits &= bits - 1;
          if (pos < a.cap) a.det_out[pos].pixel = (int)(r * a.n_cols + cb + b);
          ++pos;
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == THREADS - 1) base_sh = pos;  // the last thread ends the sweep
    __syncthreads();
    const int64_t end = base_sh < a.cap ? base_sh : a.cap;
    const int64_t hend = base_sh < a.host_cap ? base_sh : a.host_cap;
    for (int64_t i = base + threadIdx.x; i < end; i += THREADS) {
      const rc_detection d = a.det_cell[a.det_out[i].pixel];
      a.det_out[i] = d;
      if (i < hend) a.host_out[i] = d;
    }
  }
  if (threadIdx.x == 0) {
    *a.count = base_sh;
    if (a.host_count) *a.host_count = base_sh;
  }
}

}  // namespace

hipError_t launch_cfar(const CfarMulti& m0, hipStream_t s) {
  if (m0.n_frames < 1 || m0.n_frames > CfarMulti::kMax) return hipErrorInvalidValue;
  CfarMulti m = m0;
  int64_t grid = 0;
  const int h = m.f[0].guard + m.f[0].train;
  for (int i = 0; i < m.n_frames; ++i) {
    const CfarArgs& a = m.f[i];
    if (a.guard + a.train != h) return hipErrorInvalidValue;  // one halo size per launch
    if (a.n_rows < 0 || a.n_cols < 0 || a.guard < 0 || a.train < 1 || a.guard + a.train > kMaxHalf ||
        a.words_per_row != (a.n_cols + kTileCols - 1) / kTileCols || (a.recheck_cap > 0 && (!a.listed || !a.n_listed)))
      return hipErrorInvalidValue;
    m.begin[i] = (int)grid;
    grid += (int64_t)a.words_per_row * ((a.n_rows + kTileRows - 1) / kTileRows);
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
  }
  m.begin[m.n_frames] = (int)grid;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(cfar_kernel, dim3((unsigned)grid), dim3(kThreads), cfar_lds_bytes(h), s, m);
  return hipGetLastError();
}

hipError_t launch_compact(const CompactMulti& m, hipStream_t s) {
  if (m.n_frames < 1 || m.n_frames > CompactMulti::kMax) return hipErrorInvalidValue;
  for (int i = 0; i < m.n_frames; ++i) {
    const CompactArgs& a = m.f[i];
    if (a.words_per_row != (a.n_cols + kTileCols - 1) / kTileCols || a.n_rows < 0 || a.cap < 0 ||
        a.host_cap < 0 || a.host_cap > a.cap || (a.host_cap > 0 && !a.host_out))
      return hipErrorInvalidValue;
  }
  int64_t words = 0;
  for (int i = 0; i < m.n_frames; ++i)
    words = std::max<int64_t>(words, (int64_t)m.f[i].n_rows * m.f[i].words_per_row);
  if (words <= (int64_t)kCompactSmallSweeps * 256 * kCompactWords)
    hipLaunchKernelGGL(compact_kernel<256>, dim3((unsigned)m.n_frames), dim3(256), 0, s, m);
  else
    hipLaunchKernelGGL(compact_kernel<1024>, dim3((unsigned)m.n_frames), dim3(1024), 0, s, m);
  return hipGetLastError();
}

}  // namespace rc
