// FP64 Krylov vector kernels for GMRES: modified Gram-Schmidt as a chain of launches
// (launch i subtracts the projection on v_{i-1} and accumulates the dot with v_i, so the
// MGS order is kept exactly), normalisation, residual, solution update.  Every
// reduction has a fixed order (block partials summed in index order), so results are
// bitwise reproducible run to run.
#include "common.hpp"
#include "kernels.hpp"

namespace fde {

static constexpr int KR_NT = 256;

int krylov_blocks(size_t n) {
  size_t b = (n + 1023) / 1024;
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int nblk, double *red) {
  double t = 0.0;
  for (int q = threadIdx.x; q < nblk; q += KR_NT) t += part[q];
  return block_sum<KR_NT>(t, red);
}

// i = 0..j+1.  i > 0: h_{i-1} = <v_{i-1}, w> from part_in; w -= h_{i-1} v_{i-1}.
// i <= j: partial <v_i, w>;  i == j+1: partial <w, w>.
__global__ __launch_bounds__(KR_NT) void k_mgs_step(int i, int j, const double *__restrict__ V,
                                                    double *__restrict__ w, size_t n,
                                                    const double *__restrict__ part_in,
                                                    double *__restrict__ part_out, int nblk,
                                                    double *__restrict__ Hcol) {
  __shared__ double red[KR_NT / 64];
  double h = 0.0;
  if (i > 0) {
    h = sum_partials(part_in, nblk, red);
    if (blockIdx.x == 0 && threadIdx.x == 0) Hcol[i - 1] = h;
  }
  const size_t chunk = (n + nblk - 1) / nblk;
  const size_t begin = (size_t)blockIdx.x * chunk;
  const size_t end = begin + chunk < n ? begin + chunk : n;
  const double *vp = (i > 0) ? V + (size_t)(i - 1) * n : V;
  const double *vc = (i <= j) ? V + (size_t)i * n : V;
  double acc = 0.0;
  for (size_t e = begin + threadIdx.x; e < end; e += KR_NT) {
    double we = w[e];
    if (i > 0) {
      we = fma(-h, vp[e], we);
      w[e] = we;
    }
    acc = (i <= j) ? fma(vc[e], we, acc) : fma(we, we, acc);
  }
  acc = block_sum<KR_NT>(acc, red);
  if (threadIdx.x == 0) part_out[blockIdx.x] = acc;
}

// nrm = sqrt(sum part); dst = src / nrm (0 if nrm == 0); *out_norm = nrm.
__global__ __launch_bounds__(KR_NT) void k_normalize(const double *__restrict__ src,
                                                     double *__restrict__ dst, size_t n,
                                                     const double *__restrict__ part, int nblk,
                                                     double *__restrict__ out_norm) {
  __shared__ double red[KR_NT / 64];
  const double nrm = sqrt(sum_partials(part, nblk, red));
  if (blockIdx.x == 0 && threadIdx.x == 0) *out_norm = nrm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (size_t e = (size_t)blockIdx.x * KR_NT + threadIdx.x; e < n; e += (size_t)gridDim.x * KR_NT)
    dst[e] = src[e] * inv;
}

__global__ __launch_bounds__(KR_NT) void k_residual(const double *__restrict__ b,
                                                    const double *__restrict__ Mx,
                                                    double *__restrict__ r, size_t n,
                                                    double *__restrict__ part, int nblk) {
  __shared__ double red[KR_NT / 64];
  const size_t chunk = (n + nblk - 1) / nblk;
  const size_t begin = (size_t)blockIdx.x * chunk;
  const size_t end = begin + chunk < n ? begin + chunk : n;
  double acc = 0.0;
  for (size_t e = begin + threadIdx.x; e < end; e += KR_NT) {
    const double re = b[e] - Mx[e];
    r[e] = re;
    acc = fma(re, re, acc);
  }
  acc = block_sum<KR_NT>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(KR_NT) void k_dot_partial(const double *__restrict__ x,
                                                       const double *__restrict__ y, size_t n,
                                                       double *__restrict__ part, int nblk) {
  __shared__ double red[KR_NT / 64];
  const size_t chunk = (n + nblk - 1) / nblk;
  const size_t begin = (size_t)blockIdx.x * chunk;
  const size_t end = begin + chunk < n ? begin + chunk : n;
  double acc = 0.0;
  for (size_t e = begin + threadIdx.x; e < end; e += KR_NT) acc = fma(x[e], y[e], acc);
  acc = block_sum<KR_NT>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(KR_NT) void k_update_x(double *__restrict__ x,
                                                    const double *__restrict__ Z,
                                                    const double *__restrict__ y, int k, size_t n) {
  for (size_t e = (size_t)blockIdx.x * KR_NT + threadIdx.x; e < n; e += (size_t)gridDim.x * KR_NT) {
    double acc = x[e];
    for (int j = 0; j < k; ++j) acc = fma(y[j], Z[(size_t)j * n + e], acc);
    x[e] = acc;
  }
}

static int grid_for(size_t n) {
  size_t g = (n + KR_NT - 1) / KR_NT;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_mgs_step(int i, int j, double *V, double *w, size_t n, const double *part_in,
                           double *part_out, int nblk, double *Hcol, hipStream_t st) {
  hipLaunchKernelGGL(k_mgs_step, dim3(nblk), dim3(KR_NT), 0, st, i, j, V, w, n, part_in, part_out,
                     nblk, Hcol);
  return hipGetLastError();
}

hipError_t launch_normalize(const double *src, double *dst, size_t n, const double *part, int nblk,
                            double *out_norm, hipStream_t st) {
  hipLaunchKernelGGL(k_normalize, dim3(grid_for(n)), dim3(KR_NT), 0, st, src, dst, n, part, nblk,
                     out_norm);
  return hipGetLastError();
}

hipError_t launch_residual(const double *b, const double *Mx, double *r, size_t n, double *part,
                           int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_residual, dim3(nblk), dim3(KR_NT), 0, st, b, Mx, r, n, part, nblk);
  return hipGetLastError();
}

hipError_t launch_dot_partial(const double *x, const double *y, size_t n, double *part, int nblk,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial, dim3(nblk), dim3(KR_NT), 0, st, x, y, n, part, nblk);
  return hipGetLastError();
}

hipError_t launch_update_x(double *x, const double *Z, const double *y, int k, size_t n,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_update_x, dim3(grid_for(n)), dim3(KR_NT), 0, st, x, Z, y, k, n);
  return hipGetLastError();
}

}  // namespace fde
