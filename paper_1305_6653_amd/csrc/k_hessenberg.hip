// The blocks of the Strang preconditioner through one Hessenberg form of J.
//
// Every block K_k = lambda_k I - tau mu_k J (Section 3.2) is a shift of the same real matrix
// J.  With J = Q H Q^T (Q orthogonal, H upper Hessenberg, Householder reduction),
//     K_k^{-1} v = Q (lambda_k I - tau mu_k H)^{-1} Q^T v,
// and each shifted Hessenberg matrix C_k is factored in O(m^2) by Gaussian elimination with
// partial pivoting (in column i only rows i and i+1 are nonzero, so the pivot is the larger
// of two): C_k = P_0 L_0 ... P_{m-2} L_{m-2} U_k.  The factorization of all blocks costs one
// O(m^3) reduction plus O(nb m^2) instead of nb dense LUs, and the U factors are half the
// bytes of the LU factors, which the HBM-bound block solve reads at every apply.
//
// Kernels:
//   k_hess_reduce  cooperative; the columns of J live in registers across the grid
//                  (workgroup g owns columns g, g+G, ...; thread t rows t, t+256, ...).  Step k:
//                  the owner of column k builds the Householder vector v (x = A[k+1:, k],
//                  alpha = -sign(x_0)|x|, v = x - alpha e_1, beta = 2 / v^T v) and publishes it;
//                  every workgroup applies the left reflection to its columns (column sums are
//                  local), forms partial sums of A v and Q v over its columns; a grid barrier;
//                  each workgroup reduces a slice of rows; a grid barrier; every workgroup
//                  applies A -= beta (A v) v^T and Q -= beta (Q v) v^T (Q accumulates
//                  P_0 P_1 ... so that H = Q^T J Q).  Writes H, Q and Q^T.
//   k_hess_lu      one workgroup per block: the pivoted elimination, U rows into the factor
//                  storage (row i of U is final after step i), multipliers and exchanges.
//   k_hess_lsolve  the exchanges and eliminations replayed on a right-hand side (a serial
//                  chain per block, staged in LDS).
//   k_qgemm        Y = X Q or X Q^T for the [nb][mp] complex frequency vectors (MFMA f64:
//                  the real and imaginary parts of X share the real operand).
// The U sweep of the block solve and the inverses of U's diagonal 64x64 tiles are in
// k_factor.hip (the same code as the LU route).
#include "batch.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace fde {

static constexpr int HR_NT = 256;
static constexpr int HR_CPW = 4;  // columns per workgroup
static constexpr int HR_SPIN_MAX = 1 << 21;

__device__ __forceinline__ void st_cd(double *p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                     (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_cd(const double *p) {
  return __longlong_as_double((long long)__hip_atomic_load(
      reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Waits (thread 0, bounded) until *word >= target; uniform result: false if abandoned.
__device__ __forceinline__ bool hr_wait(const unsigned *word, unsigned target, int *err, int *sh) {
  if (threadIdx.x == 0) {
    int ok = 1;
    if (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      for (int it = 0;; ++it) {
        __builtin_amdgcn_s_sleep(1);
        if (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
        if (it > HR_SPIN_MAX || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          atomicOr(err, 1);
          ok = 0;
          break;
        }
      }
    }
    *sh = ok;
  }
  __syncthreads();
  const bool ok = *sh != 0;
  __syncthreads();
  return ok;
}

// Grid barrier on a monotone counter: the n-th barrier of a launch waits for n * G arrivals.
// Every thread's coherent stores complete before its workgroup arrives.
__device__ __forceinline__ bool hr_barrier(unsigned *ctr, unsigned target, int *err, int *sh) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return hr_wait(ctr, target, err, sh);
}

// sums of CPW per-thread values over the workgroup (fixed order), result in every thread
__device__ __forceinline__ void hr_colsum(double (&v)[HR_CPW], double (*red)[HR_CPW]) {
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < HR_CPW; ++c) {
    v[c] = wave_sum(v[c]);
    if ((threadIdx.x & 63) == 0) red[w][c] = v[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < HR_CPW; ++c) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < HR_NT / 64; ++q) t += red[q][c];
    v[c] = t;
  }
  __syncthreads();
}

// Householder vector of column kk, by its owner (workgroup kk % G, register slot kk / G):
// publishes v (zero in rows <= kk) and beta, sets column kk to (.., alpha, 0, ..), raises the
// v flag to kk + 1.  With sigma = |x_1..|^2 = 0 no reflection is needed (beta = 0).
template <int RPT>
__device__ __forceinline__ void hr_make_v(double (&a)[RPT][HR_CPW], int kk, int G, int m, int mp,
                                          const HessWork &wk, double (*red)[HR_CPW], double *bc) {
  const int tid = threadIdx.x, cs = kk / G;
  double sv[HR_CPW];
#pragma unroll
  for (int c = 0; c < HR_CPW; ++c) sv[c] = 0.0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + HR_NT * r;
#pragma unroll
    for (int c = 0; c < HR_CPW; ++c) {
      if (c != cs) continue;
      if (i == kk + 1) bc[0] = a[r][c];
      if (i >= kk + 2 && i < m) sv[0] = fma(a[r][c], a[r][c], sv[0]);
    }
  }
  hr_colsum(sv, red);  // its barriers also publish bc[0]
  const double x0 = bc[0], sig = sv[0];
  double alpha = x0, beta = 0.0, v0 = 1.0;
  if (sig > 0.0) {
    const double nrm = sqrt(fma(x0, x0, sig));
    alpha = x0 >= 0.0 ? -nrm : nrm;
    v0 = x0 - alpha;
    beta = 1.0 / (alpha * (alpha - x0));
  }
  double *vb = wk.vbuf + (size_t)(kk & 1) * (mp + 1);
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + HR_NT * r;
    if (i < m) {
      double vi = 0.0;
#pragma unroll
      for (int c = 0; c < HR_CPW; ++c)
        if (c == cs) vi = (i == kk + 1) ? v0 : (i >= kk + 2 ? a[r][c] : 0.0);
      st_cd(vb + i, vi);
      if (beta != 0.0) {
#pragma unroll
        for (int c = 0; c < HR_CPW; ++c)
          if (c == cs && i >= kk + 1) a[r][c] = (i == kk + 1) ? alpha : 0.0;
      }
    }
  }
  if (tid == 0) st_cd(vb + mp, beta);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0)
    __hip_atomic_store(wk.sync + 1, (unsigned)(kk + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workspace of one reduction (HessWork in kernels.hpp): sync = {barrier counter, v flag},
// vbuf [2][mp + 1] (v, then beta), part [G][2][mp], ybuf [2][mp].
template <int RPT>
__global__ __launch_bounds__(HR_NT) void k_hess_reduce(const InstDesc *__restrict__ D, int inst,
                                                       HessWork wk, int G) {
  __shared__ double red[HR_NT / 64][HR_CPW];
  __shared__ int sh;
  __shared__ double bc[2];
  const InstDesc &d = D[inst];
  const int m = d.m, mp = d.mp, g = blockIdx.x, tid = threadIdx.x;
  unsigned *ctr = wk.sync, *vflag = wk.sync + 1;
  int *err = wk.err;
  double a[RPT][HR_CPW], q[RPT][HR_CPW];
  // J[i][j] = dx^{-alpha} (d+_i g_{i-j+1} + d-_i g_{j-i+1}), g_k = 0 outside 0..m
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + HR_NT * r;
#pragma unroll
    for (int c = 0; c < HR_CPW; ++c) {
      const int j = g + G * c;
      double v = 0.0;
      if (i < m && j < m) {
        const int k1 = i - j + 1, k2 = j - i + 1;
        const double gp = (k1 >= 0 && k1 <= m) ? d.g[k1] : 0.0;
        const double gm = (k2 >= 0 && k2 <= m) ? d.g[k2] : 0.0;
        v = d.scale * (d.dp[i] * gp + d.dm[i] * gm);
      }
      a[r][c] = v;
      q[r][c] = (i == j && i < m) ? 1.0 : 0.0;
    }
  }
  const int nsteps = m - 2;  // steps k = 0 .. m-3
  const int rpw = (m + G - 1) / G;  // rows reduced per workgroup
  unsigned nbar = 0;
  if (nsteps > 0 && g == 0) hr_make_v<RPT>(a, 0, G, m, mp, wk, red, bc);
  for (int k = 0; k < nsteps; ++k) {
    if (!hr_wait(vflag, (unsigned)(k + 1), err, &sh)) return;
    const double *vb = wk.vbuf + (size_t)(k & 1) * (mp + 1);
    const double beta = ld_cd(vb + mp);
    double vr[RPT], vc[HR_CPW];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + HR_NT * r;
      vr[r] = i < m ? ld_cd(vb + i) : 0.0;
    }
#pragma unroll
    for (int c = 0; c < HR_CPW; ++c) {
      const int j = g + G * c;
      vc[c] = j < m ? ld_cd(vb + j) : 0.0;
    }
    // left reflection on the columns j >= k+1 (column k was set by its owner)
    double w[HR_CPW];
#pragma unroll
    for (int c = 0; c < HR_CPW; ++c) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) t = fma(vr[r], a[r][c], t);
      w[c] = t;
    }
    hr_colsum(w, red);
#pragma unroll
    for (int c = 0; c < HR_CPW; ++c) {
      const int j = g + G * c;
      if (j >= k + 1 && j < m) {
        const double bw = beta * w[c];
#pragma unroll
        for (int r = 0; r < RPT; ++r) a[r][c] = fma(-bw, vr[r], a[r][c]);
      }
    }
    // partial sums of A v and Q v over this workgroup's columns (v_j = 0 for j <= k)
    double *pg = wk.part + (size_t)g * 2 * mp;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + HR_NT * r;
      if (i < m) {
        double pa = 0.0, pq = 0.0;
#pragma unroll
        for (int c = 0; c < HR_CPW; ++c) {
          pa = fma(a[r][c], vc[c], pa);
          pq = fma(q[r][c], vc[c], pq);
        }
        st_cd(pg + i, pa);
        st_cd(pg + mp + i, pq);
      }
    }
    if (!hr_barrier(ctr, (unsigned)G * ++nbar, err, &sh)) return;
    // rows g*rpw .. : y = A v, z = Q v summed over the workgroups in index order
    {
      const int wv = tid >> 6, lane = tid & 63;
      for (int rl = wv; rl < rpw; rl += HR_NT / 64) {
        const int i = g * rpw + rl;
        if (i >= m) break;
        double sa = 0.0, sq = 0.0;
        for (int gg = lane; gg < G; gg += 64) {
          sa += ld_cd(wk.part + (size_t)gg * 2 * mp + i);
          sq += ld_cd(wk.part + (size_t)gg * 2 * mp + mp + i);
        }
        sa = wave_sum(sa);
        sq = wave_sum(sq);
        if (lane == 0) {
          st_cd(wk.ybuf + i, sa);
          st_cd(wk.ybuf + mp + i, sq);
        }
      }
    }
    if (!hr_barrier(ctr, (unsigned)G * ++nbar, err, &sh)) return;
    // right reflection: A -= beta (A v) v^T, Q -= beta (Q v) v^T on this workgroup's columns
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + HR_NT * r;
      if (i < m) {
        const double by = beta * ld_cd(wk.ybuf + i), bz = beta * ld_cd(wk.ybuf + mp + i);
#pragma unroll
        for (int c = 0; c < HR_CPW; ++c) {
          a[r][c] = fma(-by, vc[c], a[r][c]);
          q[r][c] = fma(-bz, vc[c], q[r][c]);
        }
      }
    }
    if (k + 1 < nsteps && (k + 1) % G == g) hr_make_v<RPT>(a, k + 1, G, m, mp, wk, red, bc);
  }
  // H, Q and Q^T, row-major with leading dimension mp
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + HR_NT * r;
    if (i >= m) continue;
#pragma unroll
    for (int c = 0; c < HR_CPW; ++c) {
      const int j = g + G * c;
      if (j >= m) continue;
      wk.H[(size_t)i * mp + j] = a[r][c];
      wk.Q[(size_t)i * mp + j] = q[r][c];
      wk.Qt[(size_t)j * mp + i] = q[r][c];
    }
  }
}

__global__ void k_hess_init(HessWork wk) {
  if (threadIdx.x == 0) {
    wk.sync[0] = 0u;
    wk.sync[1] = 0u;
    *wk.err = 0;
  }
}

int hess_reduce_groups(int m) { return (m + HR_CPW - 1) / HR_CPW; }

static int hess_rpt(int m) {
  const int r = (m + HR_NT - 1) / HR_NT;
  return r <= 1 ? 1 : r <= 2 ? 2 : r <= 4 ? 4 : 0;
}

// Up to four rows per thread: with eight the register file holds one workgroup per CU, fewer
// than the m/4 workgroups a cooperative launch would need.
int hess_reduce_max_m() { return 4 * HR_NT; }

template <int RPT>
static hipError_t hess_launch(const InstDesc *D, int inst, const HessWork &wk, int G, hipStream_t st) {
  int per = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_hess_reduce<RPT>, HR_NT, 0) != hipSuccess)
    return hipErrorNotSupported;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorNotSupported;
  if ((long)per * cus < G) return hipErrorNotSupported;  // every workgroup must be resident
  HessWork w = wk;
  void *args[] = {(void *)&D, (void *)&inst, (void *)&w, (void *)&G};
  return hipLaunchCooperativeKernel((const void *)k_hess_reduce<RPT>, dim3(G), dim3(HR_NT), args, 0, st);
}

hipError_t launch_hess_reduce(const InstDesc *D, int inst, int m, const HessWork &wk, hipStream_t st) {
  const int G = hess_reduce_groups(m);
  hipLaunchKernelGGL(k_hess_init, dim3(1), dim3(64), 0, st, wk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (hess_rpt(m)) {
    case 1: return hess_launch<1>(D, inst, wk, G, st);
    case 2: return hess_launch<2>(D, inst, wk, G, st);
    case 4: return hess_launch<4>(D, inst, wk, G, st);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------------------------
// Shifted Hessenberg LU of C_k = lambda_k I - tau mu_k H, one workgroup per block.
// Thread t holds columns t, t+256, ... of the carried row (the row that is eliminated next)
// and of the incoming row i+1 of C; the pivot pair (column i of both) goes through LDS.
static constexpr int HL_NT = 256;

template <typename T, int CPT>
__global__ __launch_bounds__(HL_NT) void k_hess_lu(const InstDesc *__restrict__ Dd, ItemMap map,
                                                   int *__restrict__ flag) {
  __shared__ double2 pv[2][2];
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int blk = blockIdx.x - map.pre[q], tid = threadIdx.x;
  const int m = d.m, mp = d.mp;
  const double2 lam = d.lam[blk];
  const double2 sh = make_double2(-d.tau * d.mu[blk].x, -d.tau * d.mu[blk].y);  // -tau mu_k
  const double *H = d.hH;
  c_t<T> *U = (c_t<T> *)d.K + (size_t)blk * mp * mp;
  double2 *lo = d.hl + (size_t)blk * mp;
  int *pivo = d.hpiv + (size_t)blk * mp;
  // row r of C at column j
  auto crow = [&](int r, int j, double h) -> double2 {
    double2 v = make_double2(sh.x * h, sh.y * h);
    if (j == r) {
      v.x += lam.x;
      v.y += lam.y;
    }
    return v;
  };
  double2 cr[CPT], nr[CPT];
  double hn[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = tid + HL_NT * c;
    cr[c] = (j < m) ? crow(0, j, H[j]) : make_double2(0.0, 0.0);
    hn[c] = (m > 1 && j < m) ? H[(size_t)mp + j] : 0.0;
  }
  int bad = 0;
  for (int i = 0; i + 1 < m; ++i) {
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int j = tid + HL_NT * c;
      nr[c] = (j < m && j >= i) ? crow(i + 1, j, hn[c]) : make_double2(0.0, 0.0);
      // prefetch row i+2 of H (entries j >= i+1 are the only nonzero ones)
      hn[c] = (i + 2 < m && j < m && j >= i + 1) ? H[(size_t)(i + 2) * mp + j] : 0.0;
    }
    const int oc = i % HL_NT, os = i / HL_NT;
    if (tid == oc) {
#pragma unroll
      for (int c = 0; c < CPT; ++c)
        if (c == os) {
          pv[i & 1][0] = cr[c];
          pv[i & 1][1] = nr[c];
        }
    }
    __syncthreads();
    const double2 pa = pv[i & 1][0], pb = pv[i & 1][1];
    const double na = pa.x * pa.x + pa.y * pa.y, nb2 = pb.x * pb.x + pb.y * pb.y;
    const bool sw = nb2 > na;
    const double2 piv = sw ? pb : pa, oth = sw ? pa : pb;
    const double pn = sw ? nb2 : na;
    if (!(pn > 0.0) || !isfinite(pn)) bad = 1;
    const double ip = 1.0 / pn;
    const double2 l = make_double2((oth.x * piv.x + oth.y * piv.y) * ip,
                                   (oth.y * piv.x - oth.x * piv.y) * ip);  // oth / piv
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int j = tid + HL_NT * c;
      const double2 p = sw ? nr[c] : cr[c], o = sw ? cr[c] : nr[c];
      if (j >= i && j < mp) U[(size_t)i * mp + j] = mk<T>((T)p.x, (T)p.y);
      cr[c] = (j > i) ? make_double2(o.x - (l.x * p.x - l.y * p.y), o.y - (l.x * p.y + l.y * p.x))
                      : make_double2(0.0, 0.0);
    }
    if (tid == 0) {
      lo[i] = l;
      pivo[i] = sw ? 1 : 0;
    }
  }
  // last row of U, then the pad rows: unit diagonal
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int j = tid + HL_NT * c;
    if (j >= m - 1 && j < mp) U[(size_t)(m - 1) * mp + j] = mk<T>((T)cr[c].x, (T)cr[c].y);
  }
  for (int i = m; i < mp; ++i)
    for (int j = i + tid; j < mp; j += HL_NT) U[(size_t)i * mp + j] = mk<T>((T)(j == i ? 1 : 0), (T)0);
  // the last pivot
  {
    const int oc = (m - 1) % HL_NT, os = (m - 1) / HL_NT;
    if (tid == oc) {
#pragma unroll
      for (int c = 0; c < CPT; ++c)
        if (c == os) {
          const double n2 = cr[c].x * cr[c].x + cr[c].y * cr[c].y;
          if (!(n2 > 0.0) || !isfinite(n2)) bad = 1;
        }
    }
  }
  if (bad) atomicOr(flag, 1);
}

template <typename T>
hipError_t launch_hess_lu(const InstDesc *D, const ItemMap &map, int items, int max_mp, int *flag,
                          hipStream_t st) {
  if (items <= 0) return hipSuccess;
  const int cpt = (max_mp + HL_NT - 1) / HL_NT;
  if (cpt <= 1) hipLaunchKernelGGL((k_hess_lu<T, 1>), dim3(items), dim3(HL_NT), 0, st, D, map, flag);
  else if (cpt <= 2) hipLaunchKernelGGL((k_hess_lu<T, 2>), dim3(items), dim3(HL_NT), 0, st, D, map, flag);
  else if (cpt <= 4) hipLaunchKernelGGL((k_hess_lu<T, 4>), dim3(items), dim3(HL_NT), 0, st, D, map, flag);
  else if (cpt <= 8) hipLaunchKernelGGL((k_hess_lu<T, 8>), dim3(items), dim3(HL_NT), 0, st, D, map, flag);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Row exchanges and eliminations of the shifted Hessenberg LU applied to y (in place on
// Vts row k): a serial chain per block, run by one lane from LDS copies.
static constexpr int LS_NT = 64;

__global__ __launch_bounds__(LS_NT) void k_hess_lsolve(const InstDesc *__restrict__ Dd, ItemMap map) {
  extern __shared__ double2 lsm[];
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int blk = blockIdx.x - map.pre[q], m = d.m, mp = d.mp;
  double2 *z = lsm, *ll = lsm + mp;
  int *pp = reinterpret_cast<int *>(lsm + 2 * mp);
  double2 *v = d.Vts + (size_t)blk * mp;
  const double2 *lo = d.hl + (size_t)blk * mp;
  const int *pivo = d.hpiv + (size_t)blk * mp;
  for (int i = threadIdx.x; i < m; i += LS_NT) {
    z[i] = v[i];
    if (i + 1 < m) {
      ll[i] = lo[i];
      pp[i] = pivo[i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 carry = z[0];
    for (int i = 0; i + 1 < m; ++i) {
      const double2 nx = z[i + 1], l = ll[i];
      const bool sw = pp[i] != 0;
      const double2 out = sw ? nx : carry, oth = sw ? carry : nx;
      carry = make_double2(oth.x - (l.x * out.x - l.y * out.y), oth.y - (l.x * out.y + l.y * out.x));
      v[i] = out;
    }
    v[m - 1] = carry;
  }
}

hipError_t launch_hess_lsolve(const InstDesc *D, const ItemMap &map, int items, int max_mp,
                              hipStream_t st) {
  if (items <= 0) return hipSuccess;
  const size_t lds = (size_t)max_mp * (2 * sizeof(double2) + sizeof(int));
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)k_hess_lsolve,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_hess_lsolve, dim3(items), dim3(LS_NT), lds, st, D, map);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Y[k][j] = sum_{i<m} X[k][i] B[i][j] with B = Q (trans = 0) or Q^T (trans = 1), both stored
// row-major with leading dimension mp; X, Y are [nb][mp] complex; Y[k][j] = 0 for j >= m.
// Workgroup tile 32 (k) x 32 (j); wave w owns the 16x16 sub-tile (w / 2, w % 2) for the real
// and the imaginary part (two MFMA accumulators sharing the B operand).  Item = (instance,
// row tile, column tile).
static constexpr int QG_T = 32;

__global__ __launch_bounds__(256) void k_qgemm(const InstDesc *__restrict__ Dd, ItemMap map,
                                               int trans, int src2) {
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int local = blockIdx.x - map.pre[q];
  const int m = d.m, mp = d.mp, nb = d.nb;
  const int ncol = mp / QG_T;
  const int rt = local / ncol, ct = local % ncol;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = rt * QG_T + 16 * (wv >> 1), c0 = ct * QG_T + 16 * (wv & 1);
  const double2 *X = src2 ? d.Vts : d.Vh;
  double2 *Y = src2 ? d.Vh : d.Vts;
  const double *B = trans ? d.hQt : d.hQ;
  const int li = lane & 15, lk = lane >> 4;
  const int arow = r0 + li;  // A operand row of this lane
  const int bcol = c0 + li;  // B operand column of this lane
  const bool arow_ok = arow < nb;
  v4d cre = {0.0, 0.0, 0.0, 0.0}, cim = {0.0, 0.0, 0.0, 0.0};
  const double2 *Xr = X + (size_t)(arow_ok ? arow : 0) * mp;
  for (int k0 = 0; k0 < m; k0 += 16) {
    double2 xa[4];
    double bb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = k0 + 4 * s + lk;
      xa[s] = (arow_ok && kk < m) ? Xr[kk] : make_double2(0.0, 0.0);
      bb[s] = (kk < m && bcol < m) ? B[(size_t)kk * mp + bcol] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      cre = mfma16(xa[s].x, bb[s], cre);
      cim = mfma16(xa[s].y, bb[s], cim);
    }
  }
  // D element v of this lane: row lk + 4v, column li (FP64 layout)
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = r0 + mfma_row<double>(lk, v), col = c0 + li;
    if (row < nb && col < mp)
      Y[(size_t)row * mp + col] = col < m ? make_double2(cre[v], cim[v]) : make_double2(0.0, 0.0);
  }
}

int qgemm_items(int nb, int mp) { return ((nb + QG_T - 1) / QG_T) * (mp / QG_T); }

hipError_t launch_qgemm(const InstDesc *D, const ItemMap &map, int items, int trans, int src2,
                        hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_qgemm, dim3(items), dim3(256), 0, st, D, map, trans, src2);
  return hipGetLastError();
}

template hipError_t launch_hess_lu<double>(const InstDesc *, const ItemMap &, int, int, int *, hipStream_t);
template hipError_t launch_hess_lu<float>(const InstDesc *, const ItemMap &, int, int, int *, hipStream_t);

}  // namespace fde
