// FP64 Krylov vector kernels for GMRES, batched over instances (item = (instance, chunk)):
// modified Gram-Schmidt as a chain of launches (launch i subtracts the projection on v_{i-1}
// and accumulates the dot with v_i, so the MGS order is kept exactly), normalisation,
// residual, solution update.  Every reduction has a fixed order (chunk partials summed in
// index order), so results are bitwise reproducible run to run.
#include "batch.hpp"
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

struct Chunk {
  const InstDesc *d;
  int b;
  size_t begin, end, n;
};

// c.d is null if the item's instance is gated off (uniform per workgroup).
__device__ __forceinline__ Chunk chunk_of(const InstDesc *__restrict__ D, const ItemMap &map) {
  const int q = item_slot(map, blockIdx.x);
  Chunk c;
  if (item_gated(map, q)) {
    c.d = nullptr;
    return c;
  }
  c.d = &D[map.ids[q]];
  c.b = blockIdx.x - map.pre[q];
  c.n = (size_t)c.d->s * c.d->m;
  const size_t len = (c.n + c.d->nblk - 1) / c.d->nblk;
  c.begin = (size_t)c.b * len;
  c.end = c.begin + len < c.n ? c.begin + len : c.n;
  return c;
}

// i = 0..j+1.  i > 0: h_{i-1} = <v_{i-1}, w> from the partials of launch i-1; w -= h v_{i-1}.
// i <= j: partial <v_i, w>;  i == j+1: partial <w, w>.  Launch i reads part[(i+1)&1] and
// writes part[i&1].
__global__ __launch_bounds__(KR_NT) void k_mgs_step(const InstDesc *__restrict__ D, ItemMap map,
                                                    int i, int j) {
  __shared__ double red[KR_NT / 64];
  const Chunk c = chunk_of(D, map);
  if (!c.d) return;
  const InstDesc &d = *c.d;
  const double *pin = (i & 1) ? d.part0 : d.part1;
  double *pout = (i & 1) ? d.part1 : d.part0;
  double h = 0.0;
  if (i > 0) {
    h = sum_partials(pin, d.nblk, red);
    if (c.b == 0 && threadIdx.x == 0) d.H[i - 1] = h;
  }
  const double *vp = d.V + (size_t)(i > 0 ? i - 1 : 0) * c.n;
  const double *vc = d.V + (size_t)(i <= j ? i : 0) * c.n;
  double *w = d.w;
  double acc = 0.0;
  for (size_t e = c.begin + threadIdx.x; e < c.end; e += KR_NT) {
    double we = w[e];
    if (i > 0) {
      we = fma(-h, vp[e], we);
      w[e] = we;
    }
    acc = (i <= j) ? fma(vc[e], we, acc) : fma(we, we, acc);
  }
  acc = block_sum<KR_NT>(acc, red);
  if (threadIdx.x == 0) pout[c.b] = acc;
}

// nrm = sqrt(sum of part[psel]); dst = src / nrm (0 if nrm == 0).  The norm is stored in
// H[hidx] if hidx >= 0, else in nrm[0].
__global__ __launch_bounds__(KR_NT) void k_normalize(const InstDesc *__restrict__ D, ItemMap map,
                                                     int src_sel, int src_j, int dst_sel, int dst_j,
                                                     int psel, int hidx) {
  __shared__ double red[KR_NT / 64];
  const Chunk c = chunk_of(D, map);
  if (!c.d) return;
  const InstDesc &d = *c.d;
  const double nrm = sqrt(sum_partials(psel ? d.part1 : d.part0, d.nblk, red));
  if (c.b == 0 && threadIdx.x == 0) {
    if (hidx >= 0) d.H[hidx] = nrm;
    else d.nrm[0] = nrm;
  }
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  const double *src = vsel(d, src_sel, src_j);
  double *dst = vsel(d, dst_sel, dst_j);
  for (size_t e = c.begin + threadIdx.x; e < c.end; e += KR_NT) dst[e] = src[e] * inv;
}

// v_0 = b - tmp (tmp = M x), partial <v_0, v_0> into part0.
__global__ __launch_bounds__(KR_NT) void k_residual(const InstDesc *__restrict__ D, ItemMap map) {
  __shared__ double red[KR_NT / 64];
  const Chunk c = chunk_of(D, map);
  if (!c.d) return;
  const InstDesc &d = *c.d;
  double acc = 0.0;
  for (size_t e = c.begin + threadIdx.x; e < c.end; e += KR_NT) {
    const double re = d.b[e] - d.tmp[e];
    d.V[e] = re;
    acc = fma(re, re, acc);
  }
  acc = block_sum<KR_NT>(acc, red);
  if (threadIdx.x == 0) d.part0[c.b] = acc;
}

__global__ __launch_bounds__(KR_NT) void k_dot_partial(const InstDesc *__restrict__ D, ItemMap map,
                                                       int xsel, int ysel, int psel) {
  __shared__ double red[KR_NT / 64];
  const Chunk c = chunk_of(D, map);
  if (!c.d) return;
  const InstDesc &d = *c.d;
  const double *x = vsel(d, xsel, 0), *y = vsel(d, ysel, 0);
  double acc = 0.0;
  for (size_t e = c.begin + threadIdx.x; e < c.end; e += KR_NT) acc = fma(x[e], y[e], acc);
  acc = block_sum<KR_NT>(acc, red);
  if (threadIdx.x == 0) (psel ? d.part1 : d.part0)[c.b] = acc;
}

// dst += a * src (vector selectors)
__global__ __launch_bounds__(KR_NT) void k_axpy(const InstDesc *__restrict__ D, ItemMap map,
                                                int dst_sel, int src_sel, double a) {
  const Chunk c = chunk_of(D, map);
  if (!c.d) return;
  const InstDesc &d = *c.d;
  double *dst = vsel(d, dst_sel, 0);
  const double *src = vsel(d, src_sel, 0);
  for (size_t e = c.begin + threadIdx.x; e < c.end; e += KR_NT) dst[e] = fma(a, src[e], dst[e]);
}

hipError_t launch_axpy(const InstDesc *D, const ItemMap &map, int items, int dst_sel, int src_sel,
                       double a, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3(items), dim3(KR_NT), 0, st, D, map, dst_sel, src_sel, a);
  return hipGetLastError();
}

// x *= y[0]  (per-instance factor)
__global__ __launch_bounds__(KR_NT) void k_scale_x(const InstDesc *__restrict__ D, ItemMap map) {
  const Chunk c = chunk_of(D, map);
  if (!c.d) return;
  const InstDesc &d = *c.d;
  const double g = d.y[0];
  for (size_t e = c.begin + threadIdx.x; e < c.end; e += KR_NT) d.x[e] *= g;
}

// x += sum_{j<k} y[1+j] Q_j with k = (int) y[0]; Q = Z (right preconditioning) or V (left).
__global__ __launch_bounds__(KR_NT) void k_update_x(const InstDesc *__restrict__ D, ItemMap map,
                                                    int basis_sel) {
  const Chunk c = chunk_of(D, map);
  if (!c.d) return;
  const InstDesc &d = *c.d;
  const int k = (int)d.y[0];
  const double *Q = basis_sel == VS_V ? d.V : d.Z;
  for (size_t e = c.begin + threadIdx.x; e < c.end; e += KR_NT) {
    double acc = d.x[e];
    for (int j = 0; j < k; ++j) acc = fma(d.y[1 + j], Q[(size_t)j * c.n + e], acc);
    d.x[e] = acc;
  }
}

// dst = src (vector selectors with basis index)
__global__ __launch_bounds__(KR_NT) void k_copy(const InstDesc *__restrict__ D, ItemMap map,
                                                int src_sel, int src_j, int dst_sel, int dst_j) {
  const Chunk c = chunk_of(D, map);
  if (!c.d) return;
  const InstDesc &d = *c.d;
  const double *src = vsel(d, src_sel, src_j);
  double *dst = vsel(d, dst_sel, dst_j);
  for (size_t e = c.begin + threadIdx.x; e < c.end; e += KR_NT) dst[e] = src[e];
}

hipError_t launch_copy(const InstDesc *D, const ItemMap &map, int items, int src_sel, int src_j,
                       int dst_sel, int dst_j, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(items), dim3(KR_NT), 0, st, D, map, src_sel, src_j, dst_sel, dst_j);
  return hipGetLastError();
}

hipError_t launch_mgs_step(const InstDesc *D, const ItemMap &map, int items, int i, int j,
                           hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mgs_step, dim3(items), dim3(KR_NT), 0, st, D, map, i, j);
  return hipGetLastError();
}

hipError_t launch_normalize(const InstDesc *D, const ItemMap &map, int items, int src_sel,
                            int src_j, int dst_sel, int dst_j, int psel, int hidx, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_normalize, dim3(items), dim3(KR_NT), 0, st, D, map, src_sel, src_j, dst_sel,
                     dst_j, psel, hidx);
  return hipGetLastError();
}

hipError_t launch_residual(const InstDesc *D, const ItemMap &map, int items, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual, dim3(items), dim3(KR_NT), 0, st, D, map);
  return hipGetLastError();
}

hipError_t launch_dot_partial(const InstDesc *D, const ItemMap &map, int items, int xsel, int ysel,
                              int psel, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dot_partial, dim3(items), dim3(KR_NT), 0, st, D, map, xsel, ysel, psel);
  return hipGetLastError();
}

hipError_t launch_scale_x(const InstDesc *D, const ItemMap &map, int items, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_x, dim3(items), dim3(KR_NT), 0, st, D, map);
  return hipGetLastError();
}

hipError_t launch_update_x(const InstDesc *D, const ItemMap &map, int items, int basis_sel,
                           hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_update_x, dim3(items), dim3(KR_NT), 0, st, D, map, basis_sel);
  return hipGetLastError();
}

}  // namespace fde
