// Streaming-read probe: the HBM read bandwidth a plain kernel reaches on this device, the
// practical ceiling next to the datasheet figure for the bandwidth-bound kernels.
#include "kernels.hpp"

namespace fde {

static constexpr int PR_NT = 256;

// out[block] = sum of the block's values (keeps the loads live); 4 independent 16-byte loads in
// flight per thread and iteration, grid-stride over n float4 values.
__global__ __launch_bounds__(PR_NT) void k_read_probe(const float4 *__restrict__ x, size_t n,
                                                      float *__restrict__ out) {
  const size_t stride = (size_t)gridDim.x * PR_NT;
  size_t i = (size_t)blockIdx.x * PR_NT + threadIdx.x;
  float acc = 0.0f;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const float4 a = x[i], b = x[i + stride], c = x[i + 2 * stride], d = x[i + 3 * stride];
    acc += (a.x + b.x) + (c.x + d.x) + (a.w + b.w) + (c.w + d.w);
  }
  for (; i < n; i += stride) acc += x[i].x;
  if (acc == 1.0f) out[blockIdx.x] = acc;  // practically never taken; the loads are not dead
}

hipError_t launch_read_probe(const void *x, size_t bytes, float *out, int blocks, hipStream_t st) {
  if (bytes < 16 || blocks <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_read_probe, dim3(blocks), dim3(PR_NT), 0, st, (const float4 *)x, bytes / 16,
                     out);
  return hipGetLastError();
}

}  // namespace fde
