// Measurement probes: the HBM read bandwidth a plain streaming kernel reaches on this device,
// and the rate of back-to-back MFMA products (the instructions the LU uses), the practical
// ceilings next to the datasheet figures.
#include "common.hpp"
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

// Each wavefront issues `iters` rounds of PR_ACC independent 16x16x4 MFMAs
// (v_mfma_f64_16x16x4f64 or v_mfma_f32_16x16x4f32) on register operands, 2 * 16 * 16 * 4
// flops each; PR_ACC accumulators keep dependent products far enough apart for the pipeline.
static constexpr int PR_ACC = 8;

template <typename T>
__global__ __launch_bounds__(PR_NT) void k_mfma_probe(int iters, float *__restrict__ out) {
  acc_t<T> c[PR_ACC];
#pragma unroll
  for (int q = 0; q < PR_ACC; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) c[q][v] = (T)0;
  const T a = (T)(threadIdx.x & 7) * (T)1e-3, b = (T)1e-3;
  // sixteen rounds per trip, so that the register-class copies the compiler places at the loop
  // edge are rare (iters is a multiple of 16)
  for (int i = 0; i < iters; i += 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int q = 0; q < PR_ACC; ++q) c[q] = mfma16((q & 1) ? a : b, (q & 2) ? a : b, c[q]);
  }
  T t = (T)0;
#pragma unroll
  for (int q = 0; q < PR_ACC; ++q) t += c[q][q & 3];
  if (t == (T)-1) out[blockIdx.x] = (float)t;  // never taken for these operands; keeps the chains live
}

hipError_t launch_mfma_probe(int fp64, int iters, float *out, int blocks, hipStream_t st) {
  if (iters < 16 || iters % 16 != 0 || blocks <= 0) return hipErrorInvalidValue;
  if (fp64)
    hipLaunchKernelGGL(k_mfma_probe<double>, dim3(blocks), dim3(PR_NT), 0, st, iters, out);
  else
    hipLaunchKernelGGL(k_mfma_probe<float>, dim3(blocks), dim3(PR_NT), 0, st, iters, out);
  return hipGetLastError();
}

double mfma_probe_flops(int iters, int blocks) {
  return (double)blocks * (PR_NT / 64) * iters * (double)PR_ACC * (2.0 * 16 * 16 * 4);
}

}  // namespace fde
