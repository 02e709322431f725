// Upload of per-frame geometry (antenna uniforms, windows) from the pinned,
// mapped host staging buffers to the frame slots, as a compute kernel on the
// frame's stream: the kernel reads host memory over the bus and writes device
// memory, so the stream never waits for a copy engine between frames (a
// copy-engine transfer of a few hundred kB stalled the stream for ~0.14 ms).
#include "rc_kernels.hpp"

namespace rc {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void upload_kernel(UploadMulti m) {
  const int fi = multi_frame(m, blockIdx.x);
  const UploadArgs a = m.f[fi];
  const int64_t i = (int64_t)(blockIdx.x - m.begin[fi]) * kThreads + threadIdx.x;
  if (i < a.n16) a.dst[i] = a.src[i];
}

}  // namespace

hipError_t launch_upload(const UploadMulti& m0, hipStream_t s) {
  if (m0.n_frames < 1 || m0.n_frames > UploadMulti::kMax) return hipErrorInvalidValue;
  UploadMulti m = m0;
  int64_t grid = 0;
  for (int i = 0; i < m.n_frames; ++i) {
    if (m.f[i].n16 < 0 || (m.f[i].n16 > 0 && (!m.f[i].dst || !m.f[i].src))) return hipErrorInvalidValue;
    m.begin[i] = (int)grid;
    grid += (m.f[i].n16 + kThreads - 1) / kThreads;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
  }
  m.begin[m.n_frames] = (int)grid;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(upload_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, m);
  return hipGetLastError();
}

}  // namespace rc
