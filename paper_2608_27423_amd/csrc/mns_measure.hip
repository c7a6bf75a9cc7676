// Measurement helper: the practical HBM rate of a read-dominated stream on
// this device, for the roofline figures (the Jacobian reads about six bytes
// for every byte it writes).  The source is seen as `ratio` contiguous blocks
// of 32-byte words; word o of the destination is the sum of word o of every
// block, so each load instruction of a wavefront reads consecutive words and
// the kernel moves `read_bytes` of reads and read_bytes / ratio of writes
// (the sums keep the loads alive).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "mns_internal.hpp"

namespace mns {

// U outputs per thread and step, so that U * ratio loads are in flight
template <int U>
__global__ __launch_bounds__(256) void k_stream(const double4* __restrict__ src, long long nwords,
                                                 double4* __restrict__ dst, int ratio) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long nout = nwords / ratio;
  for (long long o0 = (long long)blockIdx.x * blockDim.x + threadIdx.x; o0 < nout; o0 += U * stride) {
    double4 acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long o = o0 + u * stride;
      acc[u] = o < nout ? src[o] : double4{0, 0, 0, 0};
    }
    for (int j = 1; j < ratio; ++j) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long o = o0 + u * stride;
        if (o < nout) {
          const double4 v = src[(long long)j * nout + o];
          acc[u].x += v.x;
          acc[u].y += v.y;
          acc[u].z += v.z;
          acc[u].w += v.w;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long o = o0 + u * stride;
      if (o < nout) dst[o] = acc[u];
    }
  }
}

}  // namespace mns

// best rate over a few launch shapes (grid of 1,024 to 8,192 blocks of 256
// threads, one or two outputs per thread and step)
extern "C" int mns_stream_bandwidth(const void* src, void* dst, int64_t read_bytes, int ratio, int reps,
                                     void* stream, double* gbs) {
  using namespace mns;
  if (!src || !dst || !gbs || read_bytes < (1 << 20) || ratio < 1 || ratio > 64 || reps < 1 || reps > 1000 ||
      ((uintptr_t)src % 32) || ((uintptr_t)dst % 32))
    return MNS_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const long long nwords = read_bytes / 32;
  const long long nout = nwords / ratio;
  const double moved = (double)(nout * ratio) * 32.0 + (double)nout * 32.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MNS_ERR_HIP;
  double best = 0;
  hipError_t e = hipSuccess;
  for (int u = 1; u <= 2 && e == hipSuccess; ++u) {
    for (unsigned blocks = 1024; blocks <= 8192 && e == hipSuccess; blocks *= 2) {
      auto launch = [&]() {
        if (u == 1)
          hipLaunchKernelGGL(k_stream<1>, dim3(blocks), dim3(256), 0, s, (const double4*)src, nwords, (double4*)dst,
                             ratio);
        else
          hipLaunchKernelGGL(k_stream<2>, dim3(blocks), dim3(256), 0, s, (const double4*)src, nwords, (double4*)dst,
                             ratio);
      };
      launch();
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r) launch();
      (void)hipEventRecord(e1, s);
      e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && ms > 0) best = std::max(best, moved * reps / (ms * 1e-3) / 1e9);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess || !(best > 0)) return MNS_ERR_HIP;
  *gbs = best;
  return MNS_OK;
}
