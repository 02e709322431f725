// Detection stage on the SAR image (not part of the paper): 2-D square-law
// cell-averaging CFAR over the pixel lattice, then ordered compaction.
//
// For a cell with its whole window inside the lattice the training set is the
// (2h+1)^2 square (h = guard + train) minus the (2g+1)^2 guard square; the cell
// is a detection iff |P|^2 > alpha / N * sum(training).  Powers and box sums
// are formed in double, so the decision differs from an exact evaluation only
// through the image itself.
//
// A 256-thread workgroup produces 4 rows x 64 columns of decisions (one wave
// per row segment, whose ballot is that segment's 64-bit mask word).  The
// (4 + 2h) x (64 + 2h) power halo is staged in LDS, box sums are separable:
// vertical sums per halo column first, then horizontal sums per cell.
#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;
constexpr int kTileRows = 4;
constexpr int kTileCols = 64;
constexpr int kMaxHalf = 16;  // guard + train <= 16
constexpr int kHaloCols = kTileCols + 2 * kMaxHalf;
constexpr int kHaloRows = kTileRows + 2 * kMaxHalf;

__global__ __launch_bounds__(kThreads) void cfar_kernel(CfarMulti m) {
  __shared__ double pw[kHaloRows][kHaloCols];
  __shared__ double vo[kTileRows][kHaloCols];
  __shared__ double vi[kTileRows][kHaloCols];
  const int fi = multi_frame(m, blockIdx.x);
  const CfarArgs a = m.f[fi];
  const int tile = blockIdx.x - m.begin[fi];
  const int bx = tile % a.words_per_row, by = tile / a.words_per_row;  // one mask word per 64 columns
  const int h = a.guard + a.train;
  const int g = a.guard;
  const int r0 = by * kTileRows;
  const int c0 = bx * kTileCols;
  const int hr = kTileRows + 2 * h, hc = kTileCols + 2 * h;

  for (int e = threadIdx.x; e < hr * hc; e += kThreads) {
    const int i = e / hc, j = e - i * hc;
    const int r = r0 - h + i, c = c0 - h + j;
    double v = 0.0;
    if (r >= 0 && r < a.n_rows && c >= 0 && c < a.n_cols) {
      const float2 z = a.img[(int64_t)r * a.n_cols + c];
      v = (double)z.x * z.x + (double)z.y * z.y;
    }
    pw[i][j] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kTileRows * hc; e += kThreads) {
    const int i = e / hc, j = e - i * hc;
    double so = 0.0, si = 0.0;
    for (int d = 0; d <= 2 * h; ++d) so += pw[i + d][j];
    for (int d = h - g; d <= h + g; ++d) si += pw[i + d][j];
    vo[i][j] = so;
    vi[i][j] = si;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int i = threadIdx.x >> 6;  // tile row of this wave
  const int r = r0 + i, c = c0 + lane;
  double so = 0.0, si = 0.0;
  for (int d = 0; d <= 2 * h; ++d) so += vo[i][lane + d];
  for (int d = h - g; d <= h + g; ++d) si += vi[i][lane + d];
  const double thr = a.alpha_over_n * (so - si);
  const double p = pw[i + h][lane + h];
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

constexpr int kCompactThreads = 1024;

__global__ __launch_bounds__(kCompactThreads) void compact_kernel(CompactMulti m) {
  const CompactArgs a = m.f[__builtin_amdgcn_readfirstlane((int)blockIdx.x)];  // one workgroup per frame
  __shared__ int64_t scan[kCompactThreads];
  __shared__ int64_t base_sh;
  const int64_t n_words = (int64_t)a.n_rows * a.words_per_row;
  if (threadIdx.x == 0) base_sh = 0;
  __syncthreads();
  for (int64_t w0 = 0; w0 < n_words; w0 += kCompactThreads) {
    const int64_t w = w0 + threadIdx.x;
    const unsigned long long word = (w < n_words) ? a.mask[w] : 0ull;
    const int cnt = __popcll(word);
    scan[threadIdx.x] = cnt;
    __syncthreads();
    // inclusive Hillis-Steele scan over the block
    for (int off = 1; off < kCompactThreads; off <<= 1) {
      const int64_t add = (threadIdx.x >= off) ? scan[threadIdx.x - off] : 0;
      __syncthreads();
      scan[threadIdx.x] += add;
      __syncthreads();
    }
    const int64_t base = base_sh;
    int64_t pos = base + scan[threadIdx.x] - cnt;
    if (cnt) {
      const int64_t r = w / a.words_per_row;
      const int64_t cb = (w - r * a.words_per_row) * 64;
      unsigned long long bits = word;
      while (bits) {
        const int b = __ffsll((long long)bits) - 1;
        bits &= bits - 1;
        const int64_t cell = r * a.n_cols + cb + b;
        if (pos < a.cap) a.det_out[pos] = a.det_cell[cell];
        ++pos;
      }
    }
    __syncthreads();
    if (threadIdx.x == kCompactThreads - 1) base_sh = base + scan[kCompactThreads - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) *a.count = base_sh;
}

}  // namespace

hipError_t launch_cfar(const CfarMulti& m0, hipStream_t s) {
  if (m0.n_frames < 1 || m0.n_frames > CfarMulti::kMax) return hipErrorInvalidValue;
  CfarMulti m = m0;
  int64_t grid = 0;
  for (int i = 0; i < m.n_frames; ++i) {
    const CfarArgs& a = m.f[i];
    if (a.n_rows < 0 || a.n_cols < 0 || a.guard < 0 || a.train < 1 || a.guard + a.train > kMaxHalf ||
        a.words_per_row != (a.n_cols + kTileCols - 1) / kTileCols || (a.recheck_cap > 0 && (!a.listed || !a.n_listed)))
      return hipErrorInvalidValue;
    m.begin[i] = (int)grid;
    grid += (int64_t)a.words_per_row * ((a.n_rows + kTileRows - 1) / kTileRows);
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
  }
  m.begin[m.n_frames] = (int)grid;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(cfar_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, m);
  return hipGetLastError();
}

hipError_t launch_compact(const CompactMulti& m, hipStream_t s) {
  if (m.n_frames < 1 || m.n_frames > CompactMulti::kMax) return hipErrorInvalidValue;
  for (int i = 0; i < m.n_frames; ++i) {
    const CompactArgs& a = m.f[i];
    if (a.words_per_row != (a.n_cols + kTileCols - 1) / kTileCols || a.n_rows < 0 || a.cap < 0)
      return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)m.n_frames), dim3(kCompactThreads), 0, s, m);
  return hipGetLastError();
}

}  // namespace rc
