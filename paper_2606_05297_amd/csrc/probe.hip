// Streaming-bandwidth probe: the measured HBM ceiling that the kernel rooflines
// are read against (the published 8 TB/s is a peak no kernel reaches).  Three
// grid-stride kernels over caller buffers with 16-byte accesses: copy (read a,
// write b), read (sum of a, one store per workgroup) and in-place update (read
// and write b, the access pattern of an in-place gate).  The caller picks the
// grid; timed with HIP events on the caller's stream.
#include "fock_internal.h"

namespace fock {
namespace {

constexpr int kProbeThreads = 256;

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const float4 *__restrict__ a, float4 *__restrict__ b,
                                                              size_t n) {
  const size_t st = (size_t)gridDim.x * kProbeThreads;
  for (size_t i = blockIdx.x * (size_t)kProbeThreads + threadIdx.x; i < n; i += st) b[i] = a[i];
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const float4 *__restrict__ a, float *__restrict__ out,
                                                              size_t n) {
  const size_t st = (size_t)gridDim.x * kProbeThreads;
  float s = 0.f;
  for (size_t i = blockIdx.x * (size_t)kProbeThreads + threadIdx.x; i < n; i += st) {
    const float4 v = a[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  __shared__ float red[kProbeThreads];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kProbeThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_update(float4 *__restrict__ b, size_t n) {
  const size_t st = (size_t)gridDim.x * kProbeThreads;
  for (size_t i = blockIdx.x * (size_t)kProbeThreads + threadIdx.x; i < n; i += st) {
    const float4 v = b[i];
    b[i] = make_float4(-v.y, v.x, -v.w, v.z);  // multiply each complex amplitude by i
  }
}

}  // namespace
}  // namespace fock

using namespace fock;

extern "C" int fock_stream_probe(int kind, const void *a, void *b, size_t bytes, int grid, int iters, double *ms,
                                 fock_stream_t stream) {
  if (kind < 0 || kind > 2) return set_error(FOCK_ERR_ARG, "kind must be 0 (copy), 1 (read) or 2 (update)");
  if (!ms || iters < 1 || grid < 1 || grid > (1 << 20)) return set_error(FOCK_ERR_ARG, "bad ms/iters/grid");
  if (bytes == 0 || bytes % 16 != 0) return set_error(FOCK_ERR_ARG, "bytes must be a positive multiple of 16");
  if (kind != 2 && !a) return set_error(FOCK_ERR_ARG, "a is NULL");
  if (!b) return set_error(FOCK_ERR_ARG, "b is NULL");
  if ((((uintptr_t)a) | ((uintptr_t)b)) & 15) return set_error(FOCK_ERR_ARG, "buffers must be 16-byte aligned");
  if (kind == 1 && bytes < sizeof(float) * (size_t)grid)
    return set_error(FOCK_ERR_ARG, "read probe writes one float per workgroup into b: b too small");
  hipStream_t s = (hipStream_t)stream;
  const size_t n = bytes / 16;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  FOCK_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_error(FOCK_ERR_HIP, "hipEventCreate failed");
  }
  int rc = FOCK_OK;
  auto launch = [&]() {
    if (kind == 0)
      hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(kProbeThreads), 0, s, (const float4 *)a, (float4 *)b, n);
    else if (kind == 1)
      hipLaunchKernelGGL(k_probe_read, dim3(grid), dim3(kProbeThreads), 0, s, (const float4 *)a, (float *)b, n);
    else
      hipLaunchKernelGGL(k_probe_update, dim3(grid), dim3(kProbeThreads), 0, s, (float4 *)b, n);
  };
  launch();  // warm-up
  if (hipEventRecord(e0, s) != hipSuccess) rc = set_error(FOCK_ERR_HIP, "hipEventRecord failed");
  for (int k = 0; k < iters && !rc; ++k) launch();
  if (!rc && hipGetLastError() != hipSuccess) rc = set_error(FOCK_ERR_HIP, "probe launch failed");
  float t = 0.f;
  if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&t, e0, e1) != hipSuccess))
    rc = set_error(FOCK_ERR_HIP, "event timing failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!rc) *ms = (double)t / iters;
  return rc;
}
