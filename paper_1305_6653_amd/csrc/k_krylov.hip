// FP64 Krylov vector kernels for GMRES, batched over instances (item = (instance, chunk)):
// Gram-Schmidt orthogonalisation of the new Arnoldi vector, normalisation, residual, solution
// update.  Every reduction has a fixed order (chunk partials summed in index order), so results
// are bitwise reproducible run to run.
//
// Orthogonalisation, two forms selected per solve:
// * modified Gram-Schmidt (the default) as a chain of launches: launch i subtracts the
//   projection on v_{i-1} and accumulates the dot with v_i, so the MGS order is kept exactly;
// * classical Gram-Schmidt applied twice (CGS2), h = V^T w, w -= V h, then
// h' = V^T w, w -= V h', column = h + h'.  In exact arithmetic it equals modified Gram-Schmidt;
// in floating point the second pass makes the basis orthogonal to working precision, as MGS
// does for GMRES.  It takes three launches per Arnoldi step whatever j (projection partials;
// update + second partials; update + norm partial) instead of the j + 2 dependent launches of
// MGS: the chunk that finishes last in a launch sums every chunk's partials (index order) and
// writes the coefficients, so no separate reduction launch is needed.  Partials go through
// agent-coherent stores and loads, and a chunk counts itself done only after its stores have
// completed.
#include "batch.hpp"
#include "common.hpp"
#include "gmres_step.hpp"
#include "kernels.hpp"

namespace fde {

static constexpr int KR_NT = 256;
// Vectors of up to KR_ONE_MAX entries form one chunk (one workgroup per reduction), which
// lets a whole Arnoldi step run in one launch (k_arnoldi1).  Larger vectors keep chunks of
// 1024 entries: one workgroup streaming a longer vector through a chain launch (a batch that
// mixes sizes) would become the launch's tail.
static constexpr size_t KR_ONE_MAX = 4096;

size_t krylov_one_max() { return KR_ONE_MAX; }

int krylov_blocks(size_t n) {
  if (n <= KR_ONE_MAX) return 1;
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

__device__ __forceinline__ void st_coh1(double *p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                     (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh1(const double *p) {
  return __longlong_as_double((long long)__hip_atomic_load(
      reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Partial sums over chunk b of V_i . w, i = 0..j, into partm[i][b]: up to 16 dot products per
// pass accumulated together (w is read once per pass), wave sums by DPP, one barrier per pass.
static constexpr int CG_G = 16;

__device__ __forceinline__ void cgs_partials(const InstDesc &d, const Chunk &c, int j, double *red) {
  const double *w = d.w;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i0 = 0; i0 <= j; i0 += CG_G) {
    const int ng = j + 1 - i0 < CG_G ? j + 1 - i0 : CG_G;
    double acc[CG_G];
#pragma unroll
    for (int t = 0; t < CG_G; ++t) acc[t] = 0.0;
    for (size_t e = c.begin + threadIdx.x; e < c.end; e += KR_NT) {
      const double we = w[e];
#pragma unroll
      for (int t = 0; t < CG_G; ++t)
        if (t < ng) acc[t] = fma(d.V[(size_t)(i0 + t) * c.n + e], we, acc[t]);
    }
#pragma unroll
    for (int t = 0; t < CG_G; ++t) {
      if (t < ng) {
        const double s = wave_sum_dpp(acc[t]);
        if (lane == 0) red[wv * CG_G + t] = s;
      }
    }
    __syncthreads();
    if (threadIdx.x < ng) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < KR_NT / 64; ++q) s += red[q * CG_G + threadIdx.x];
      st_coh1(d.partm + (size_t)(i0 + threadIdx.x) * d.nblk + c.b, s);
    }
    __syncthreads();
  }
}

// After this chunk's partials are stored: returns true in the chunk that finishes last (every
// thread), which then owns the sums.  The counter is reset for the next launch.
__device__ __forceinline__ bool cgs_last_chunk(const InstDesc &d, int *sh) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's partial stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned done = __hip_atomic_fetch_add(d.gctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int last = done == (unsigned)d.nblk - 1;
    if (last) __hip_atomic_store(d.gctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *sh = last;
  }
  __syncthreads();
  return *sh != 0;
}

// In the last chunk: h_i = sum_b partm[i][b] (index order; one wavefront per coefficient, DPP
// wave sum).  pass 0: H[i] = h_i; pass 1: h2[i] = h_i and H[i] += h_i.
__device__ __forceinline__ void cgs_sums(const InstDesc &d, int j, int pass) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = wv; i <= j; i += KR_NT / 64) {
    const double *p = d.partm + (size_t)i * d.nblk;
    double t = 0.0;
    for (int b = lane; b < d.nblk; b += 64) t += ld_coh1(p + b);
    const double h = wave_sum_dpp(t);
    if (lane == 0) {
      if (pass == 0) {
        d.H[i] = h;
      } else {
        d.h2[i] = h;
        d.H[i] += h;
      }
    }
  }
}

__global__ __launch_bounds__(KR_NT) void k_cgs_dot(const InstDesc *__restrict__ D, ItemMap map, int j) {
  __shared__ double red[(KR_NT / 64) * CG_G];
  __shared__ int sh;
  const Chunk c = chunk_of(D, map);
  if (!c.d) return;
  cgs_partials(*c.d, c, j, red);
  if (cgs_last_chunk(*c.d, &sh)) cgs_sums(*c.d, j, 0);
}

// w -= sum_{i<=j} c_i V_i with c = H (pass 0) or h2 (pass 1), in i order for every element;
// then pass 0: the partials of the second projection V^T w and, in the last chunk, h2 and
// H += h2; pass 1: the partial of w . w into part[(j+1) & 1] (read by the normalisation).
__global__ __launch_bounds__(KR_NT) void k_cgs_update(const InstDesc *__restrict__ D, ItemMap map, int j,
                                                      int pass) {
  __shared__ double red[(KR_NT / 64) * CG_G];
  __shared__ double cf[GM_RMAX + 1];
  __shared__ int sh;
  const Chunk c = chunk_of(D, map);
  if (!c.d) return;
  const InstDesc &d = *c.d;
  const double *co = pass == 0 ? d.H : d.h2;
  for (int i = threadIdx.x; i <= j; i += KR_NT) cf[i] = co[i];
  __syncthreads();
  double *w = d.w;
  double nn = 0.0;
  for (size_t e = c.begin + threadIdx.x; e < c.end; e += KR_NT) {
    double we = w[e];
    for (int i = 0; i <= j; ++i) we = fma(-cf[i], d.V[(size_t)i * c.n + e], we);
    w[e] = we;
    nn = fma(we, we, nn);
  }
  if (pass == 0) {
    __syncthreads();
    cgs_partials(d, c, j, red);
    if (cgs_last_chunk(d, &sh)) cgs_sums(d, j, 1);
  } else {
    nn = block_sum<KR_NT>(nn, red);
    if (threadIdx.x == 0) (((j + 1) & 1) ? d.part1 : d.part0)[c.b] = nn;
  }
}

hipError_t launch_cgs_dot(const InstDesc *D, const ItemMap &map, int items, int j, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cgs_dot, dim3(items), dim3(KR_NT), 0, st, D, map, j);
  return hipGetLastError();
}

hipError_t launch_cgs_update(const InstDesc *D, const ItemMap &map, int items, int j, int pass,
                             hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cgs_update, dim3(items), dim3(KR_NT), 0, st, D, map, j, pass);
  return hipGetLastError();
}

// i = 0..j+1.  i > 0: h_{i-1} = <v_{i-1}, w> from the partials of launch i-1; w -= h v_{i-1}.
// i <= j: partial <v_i, w>;  i == j+1: partial <w, w>.  Launch i reads part[(i+1)&1] and
// writes part[i&1].
static constexpr int MGS_U = 4;

__device__ __forceinline__ void mgs_load(const double *w, const double *vp, const double *vc,
                                         size_t e0, size_t end, int i, int j, double (&we)[MGS_U],
                                         double (&pe)[MGS_U], double (&ce)[MGS_U]) {
#pragma unroll
  for (int u = 0; u < MGS_U; ++u) {
    const size_t e = e0 + (size_t)u * KR_NT;
    we[u] = pe[u] = ce[u] = 0.0;
    if (e < end) {
      we[u] = w[e];
      if (i > 0) pe[u] = vp[e];
      if (i <= j) ce[u] = vc[e];
    }
  }
}

__global__ __launch_bounds__(KR_NT) void k_mgs_step(const InstDesc *__restrict__ D, ItemMap map,
                                                    int i, int j) {
  __shared__ double red[KR_NT / 64];
  const Chunk c = chunk_of(D, map);
  if (!c.d) return;
  const InstDesc &d = *c.d;
  const double *pin = (i & 1) ? d.part0 : d.part1;
  double *pout = (i & 1) ? d.part1 : d.part0;
  const double *vp = d.V + (size_t)(i > 0 ? i - 1 : 0) * c.n;
  const double *vc = d.V + (size_t)(i <= j ? i : 0) * c.n;
  double *w = d.w;
  // MGS_U elements per thread and pass, all loaded before any is stored (the stores to w could
  // alias the loads for the compiler, which would otherwise serialise the passes); the first
  // pass is loaded before the coefficient of the previous projection is summed.
  double we[MGS_U], pe[MGS_U], ce[MGS_U];
  size_t e0 = c.begin + threadIdx.x;
  mgs_load(w, vp, vc, e0, c.end, i, j, we, pe, ce);
  double h = 0.0;
  if (i > 0) {
    h = sum_partials(pin, d.nblk, red);
    if (c.b == 0 && threadIdx.x == 0) d.H[i - 1] = h;
  }
  double acc = 0.0;
  for (;;) {
    // out-of-range elements were loaded as zeros and add nothing; the stores come last so that
    // no wait for a store's completion lands between them
#pragma unroll
    for (int u = 0; u < MGS_U; ++u) {
      const double x = i > 0 ? fma(-h, pe[u], we[u]) : we[u];
      acc = fma(i <= j ? ce[u] : x, x, acc);
      we[u] = x;
    }
    if (i > 0) {
#pragma unroll
      for (int u = 0; u < MGS_U; ++u) {
        const size_t e = e0 + (size_t)u * KR_NT;
        if (e < c.end) w[e] = we[u];
      }
    }
    e0 += (size_t)MGS_U * KR_NT;
    if (e0 >= c.end) break;
    mgs_load(w, vp, vc, e0, c.end, i, j, we, pe, ce);
  }
  acc = block_sum<KR_NT>(acc, red);
  if (threadIdx.x == 0) pout[c.b] = acc;
}

// Arnoldi step j of instances whose vectors are one chunk (nblk = 1): the modified
// Gram-Schmidt projections on v_0 .. v_j, the norm of the remainder, v_{j+1} and the Givens
// update of the control record, in one launch of one workgroup per instance instead of the
// j + 4 launches of the chain (k_mgs_step i = 0 .. j+1, k_normalize, k_gm_givens).  Each
// thread takes the elements it takes in the chain (e = t + KR_NT u) in the same order; w stays
// in registers between projections, and each basis vector is read once (v_{i-1} is kept from
// the projection before).  The reductions are the chain's: block_sum, then the one-chunk
// partial sum 0 + p (sum_partials over a single partial), so the H column, w, v_{j+1} and the
// control record equal the chain's to the bit.  U = elements per thread (n <= KR_NT U).
template <int U>
__global__ __launch_bounds__(KR_NT) void k_arnoldi1(const InstDesc *__restrict__ D, ItemMap map,
                                                    int j, GmresCtl *__restrict__ ctl,
                                                    GmresWork *__restrict__ work,
                                                    int *__restrict__ gates, int count, int R) {
  __shared__ double red[KR_NT / 64];
  __shared__ double hcol[GM_RMAX + 2], csl[GM_RMAX], snl[GM_RMAX], gjs;
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const int inst = map.ids[q];
  const InstDesc &d = D[inst];
  const size_t n = (size_t)d.s * d.m;
  const int t = threadIdx.x;
  // the Givens update's other inputs (previous rotations, g[j]) copied into LDS now, while the
  // projections run (the first reduction's barriers publish them)
  for (int r = t; r < j; r += KR_NT) {
    csl[r] = work[inst].cs[r];
    snl[r] = work[inst].sn[r];
  }
  if (t == 0) gjs = work[inst].g[j];
  double w[U], cv[U], pv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const size_t e = (size_t)t + (size_t)u * KR_NT;
    w[u] = e < n ? d.w[e] : 0.0;
    cv[u] = e < n ? d.V[e] : 0.0;
    pv[u] = 0.0;
  }
  double h = 0.0;
  for (int i = 0; i <= j + 1; ++i) {
    // i <= j: w -= h_{i-1} v_{i-1} (i > 0), partial <v_i, w>;  i = j + 1: the last
    // subtraction and <w, w>
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if ((size_t)t + (size_t)u * KR_NT < n) {
        const double x = i > 0 ? fma(-h, pv[u], w[u]) : w[u];
        acc = fma(i <= j ? cv[u] : x, x, acc);
        w[u] = x;
      }
    }
    if (i <= j) {  // the next pass needs v_i and v_{i+1}; the loads fly during the reduction
      const double *vn = d.V + (size_t)(i + 1) * n;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t e = (size_t)t + (size_t)u * KR_NT;
        pv[u] = cv[u];
        cv[u] = (i + 1 <= j && e < n) ? vn[e] : 0.0;
      }
    }
    acc = block_sum<KR_NT>(acc, red);
    h = 0.0 + acc;
    if (t == 0 && i <= j) {
      d.H[i] = h;
      hcol[i] = h;
    }
  }
  const double nrm = sqrt(h);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  double *vj1 = d.V + (size_t)(j + 1) * n;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const size_t e = (size_t)t + (size_t)u * KR_NT;
    if (e < n) {
      d.w[e] = w[u];
      vj1[e] = w[u] * inv;
    }
  }
  if (t == 0) {
    d.H[j + 1] = nrm;
    hcol[j + 1] = nrm;
    gm_givens_core(hcol, csl, snl, gjs, ctl[inst], work[inst], gates, count, inst, j, R);
  }
}

hipError_t launch_arnoldi1(const InstDesc *D, const ItemMap &map, int items, size_t max_n, int j,
                           GmresCtl *ctl, GmresWork *work, int *gates, int count, int R,
                           hipStream_t st) {
  if (items <= 0) return hipSuccess;
  static_assert(KR_ONE_MAX == (size_t)KR_NT * 16, "one-chunk limit");
  if (max_n > KR_ONE_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_arnoldi1<16>, dim3(items), dim3(KR_NT), 0, st, D, map, j, ctl, work, gates, count, R);
  return hipGetLastError();
}

// The restart step's tail for one-chunk instances: v_0 = (b - tmp) / ||b - tmp|| with the norm
// into nrm[0] (k_residual, then k_normalize) for live instances, then the restart decision
// (k_gm_restart) for every instance, in one launch; the same bits as those three launches.
// Item = instance (the Krylov map without its gate).
template <int U>
__global__ __launch_bounds__(KR_NT) void k_restart1(const InstDesc *__restrict__ D, ItemMap map,
                                                    GmresCtl *__restrict__ ctl,
                                                    GmresWork *__restrict__ work,
                                                    int *__restrict__ gates, int count) {
  __shared__ double red[KR_NT / 64];
  const int inst = map.ids[item_slot(map, blockIdx.x)];
  const InstDesc &d = D[inst];
  const int t = threadIdx.x;
  if (gates[GATE_LIVE * count + inst]) {
    const size_t n = (size_t)d.s * d.m;
    double r[U];
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t e = (size_t)t + (size_t)u * KR_NT;
      r[u] = 0.0;
      if (e < n) {
        r[u] = d.b[e] - d.tmp[e];
        acc = fma(r[u], r[u], acc);
      }
    }
    acc = block_sum<KR_NT>(acc, red);
    const double nrm = sqrt(0.0 + acc);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t e = (size_t)t + (size_t)u * KR_NT;
      if (e < n) d.V[e] = r[u] * inv;
    }
    if (t == 0) d.nrm[0] = nrm;
  }
  if (t == 0) gm_restart_one(d, ctl[inst], work[inst], gates, count, inst);
}

// The end of a cycle for one-chunk instances: y = H^{-1} g (k_gm_backsolve) for every
// instance, then x += sum_{j<k} y_j Q_j (k_update_x) for live instances, in one launch; the
// same bits (no reduction: each element's sum is formed in j order whatever the thread
// mapping, so FN_NT threads share the elements).  x and Q_0 are loaded while H is staged and
// the back substitution runs.  Item = instance (the Krylov map without its gate).
static constexpr int FN_NT = 1024;

template <int U>
__global__ __launch_bounds__(FN_NT) void k_finish1(const InstDesc *__restrict__ D, ItemMap map,
                                                   GmresCtl *__restrict__ ctl,
                                                   const GmresWork *__restrict__ work,
                                                   const int *__restrict__ gates, int count,
                                                   int basis_sel) {
  __shared__ double ys[GM_RMAX + 1];
  __shared__ double Hs[GM_RMAX][GM_RMAX + 1], gs[GM_RMAX];
  const int inst = map.ids[item_slot(map, blockIdx.x)];
  const InstDesc &d = D[inst];
  const int t = threadIdx.x;
  const size_t n = (size_t)d.s * d.m;
  const double *Q = basis_sel == VS_V ? d.V : d.Z;
  // the k x k triangle of H and g staged in LDS by every thread (independent loads), so the
  // back substitution (one thread) runs on LDS instead of a chain of dependent global loads
  const int kk = ctl[inst].k;
  double acc[U], q0[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const size_t e = (size_t)t + (size_t)u * FN_NT;
    acc[u] = e < n ? d.x[e] : 0.0;
    q0[u] = (kk > 0 && e < n) ? Q[e] : 0.0;
  }
  for (int e = t; e < kk * kk; e += FN_NT) {
    const int r = e / kk, q = e % kk;
    if (q >= r) Hs[r][q] = work[inst].H[r][q];
  }
  for (int r = t; r < kk; r += FN_NT) gs[r] = work[inst].g[r];
  __syncthreads();
  if (t == 0) {
    gm_backsolve_lds(ctl[inst], Hs, gs, ys);
    for (int q = 0; q <= kk; ++q) d.y[q] = ys[q];
  }
  __syncthreads();
  if (!gates[GATE_LIVE * count + inst]) return;
  const int k = (int)ys[0];
  for (int j = 0; j < k; ++j) {
    const double yj = ys[1 + j];
    const double *Qj = Q + (size_t)j * n;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t e = (size_t)t + (size_t)u * FN_NT;
      if (e < n) acc[u] = fma(yj, j == 0 ? q0[u] : Qj[e], acc[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const size_t e = (size_t)t + (size_t)u * FN_NT;
    if (e < n) d.x[e] = acc[u];
  }
}

hipError_t launch_restart1(const InstDesc *D, const ItemMap &map, int items, size_t max_n,
                           GmresCtl *ctl, GmresWork *work, int *gates, int count, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  ItemMap all = map;
  all.gate = nullptr;
  if (max_n > KR_ONE_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_restart1<16>, dim3(items), dim3(KR_NT), 0, st, D, all, ctl, work, gates, count);
  return hipGetLastError();
}

hipError_t launch_finish1(const InstDesc *D, const ItemMap &map, int items, size_t max_n,
                          GmresCtl *ctl, const GmresWork *work, const int *gates, int count,
                          int basis_sel, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  ItemMap all = map;
  all.gate = nullptr;
  static_assert(KR_ONE_MAX == (size_t)FN_NT * 4, "one-chunk limit");
  if (max_n > KR_ONE_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finish1<4>, dim3(items), dim3(FN_NT), 0, st, D, all, ctl, work, gates, count, basis_sel);
  return hipGetLastError();
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
  const double *src = vsel(d, src_sel, src_j);
  double *dst = vsel(d, dst_sel, dst_j);
  double x[MGS_U];  // the first pass is loaded before the norm is summed
  size_t e0 = c.begin + threadIdx.x;
#pragma unroll
  for (int u = 0; u < MGS_U; ++u) {
    const size_t e = e0 + (size_t)u * KR_NT;
    x[u] = e < c.end ? src[e] : 0.0;
  }
  const double nrm = sqrt(sum_partials(psel ? d.part1 : d.part0, d.nblk, red));
  if (c.b == 0 && threadIdx.x == 0) {
    if (hidx >= 0) d.H[hidx] = nrm;
    else d.nrm[0] = nrm;
  }
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (;;) {
#pragma unroll
    for (int u = 0; u < MGS_U; ++u) {
      const size_t e = e0 + (size_t)u * KR_NT;
      if (e < c.end) dst[e] = x[u] * inv;
    }
    e0 += (size_t)MGS_U * KR_NT;
    if (e0 >= c.end) break;
#pragma unroll
    for (int u = 0; u < MGS_U; ++u) {
      const size_t e = e0 + (size_t)u * KR_NT;
      x[u] = e < c.end ? src[e] : 0.0;
    }
  }
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
