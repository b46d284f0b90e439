// Measurement aid: a plain coalesced streaming read of the input points, the
// bandwidth reference for the tile kernel (which reads the same bytes).  It
// computes nothing of the hull; it lives in its own translation unit so that
// the hull kernels' source is untouched by it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wagener_hull.h"

namespace {

constexpr int READ_BLOCK = 256;
constexpr int READ_UNROLL = 4;  // 16-byte loads in flight per lane

// Each workgroup reads READ_BLOCK * READ_UNROLL float4 (2 points each); the
// sum only keeps the loads alive.
__global__ __launch_bounds__(READ_BLOCK) void read_kernel(const float4 *__restrict__ a,
                                                          int64_t n4, float *sink) {
  const int64_t base = (int64_t)blockIdx.x * (READ_BLOCK * READ_UNROLL) + threadIdx.x;
  float4 v[READ_UNROLL];
#pragma unroll
  for (int u = 0; u < READ_UNROLL; ++u) {
    const int64_t i = base + (int64_t)READ_BLOCK * u;
    v[u] = i < n4 ? a[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  float acc = 0.0f;
#pragma unroll
  for (int u = 0; u < READ_UNROLL; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  if (acc == 0x1p120f) sink[threadIdx.x] = acc;  // practically never taken
}

}  // namespace

extern "C" int upper_hull_read_reference(const float *points, int64_t n, int32_t reps, float *ms,
                                         hipStream_t stream) {
  if (!points || n < 2 || reps < 1 || reps > 1000 || !ms || ((uintptr_t)points & 15u))
    return UH_ERR_ARG;
  const int64_t n4 = n / 2;  // whole 16-byte pairs of points
  const int64_t nb = (n4 + READ_BLOCK * READ_UNROLL - 1) / (READ_BLOCK * READ_UNROLL);
  if (nb > INT32_MAX) return UH_ERR_ARG;
  float *sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = UH_OK;
  if (hipMalloc((void **)&sink, READ_BLOCK * sizeof(float)) != hipSuccess) {
    sink = nullptr;
    rc = UH_ERR_ALLOC;
  }
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = UH_ERR_HIP;
  float t = 0.0f;
  if (!rc) {
    hipLaunchKernelGGL(read_kernel, dim3((unsigned)nb), dim3(READ_BLOCK), 0, stream,
                       (const float4 *)points, n4, sink);  // untimed
    if (hipGetLastError() != hipSuccess || hipEventRecord(e0, stream) != hipSuccess) rc = UH_ERR_HIP;
    for (int r = 0; r < reps && !rc; ++r)
      hipLaunchKernelGGL(read_kernel, dim3((unsigned)nb), dim3(READ_BLOCK), 0, stream,
                         (const float4 *)points, n4, sink);
    if (!rc && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      rc = UH_ERR_HIP;
  }
  *ms = rc ? 0.0f : t / (float)reps;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (sink) (void)hipFree(sink);
  return rc;
}
