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
//                  (workgroup g owns columns g, g+G, ...; thread t rows t, t+512).  Step k:
//                  with the Householder vector v of column k (x = A[k+1:, k], alpha =
//                  -sign(x_0)|x|, v = x - alpha e_1, beta = 2 / v^T v), every workgroup applies
//                  the left reflection to its columns (column sums are local) and forms partial
//                  sums of A v and Q v over its columns; a grid barrier; each workgroup reduces
//                  a slice of rows; a grid barrier; every workgroup applies A -= beta (A v) v^T
//                  and Q -= beta (Q v) v^T (Q accumulates P_0 P_1 ... so that H = Q^T J Q) and
//                  computes the next v itself from a snapshot of column k+1.  Writes H, Q, Q^T.
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

static constexpr int HR_NT = 512;
static constexpr int HR_CPW = 8;  // columns per workgroup
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

// Grid barrier b (b = 1, 2, ... within a launch): workgroup g raises arrive[g] to b, then the
// first wavefront polls all G entries (one load per lane) until every one has reached b.  No
// atomic read-modify-write, so arrivals do not serialise.  Every thread's coherent stores
// complete before its workgroup arrives.  Bounded: after HR_SPIN_MAX polls, or once any
// workgroup has raised *err, the wait is abandoned (uniform false).
__device__ __forceinline__ bool hr_barrier(unsigned *arrive, int G, unsigned b, int *err, int *sh) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane == 0) __hip_atomic_store(arrive + blockIdx.x, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    for (int it = 0;; ++it) {
      bool done = true;
      for (int q = lane; q < G; q += 64)
        done = done && __hip_atomic_load(arrive + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= b;
      if (__all(done)) break;
      if (it > HR_SPIN_MAX || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        if (lane == 0) atomicOr(err, 1);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) *sh = ok;
  }
  __syncthreads();
  const bool ok = *sh != 0;
  __syncthreads();
  return ok;
}

// sums of CPW per-thread values over the workgroup (fixed order), result in every thread
template <int NV>
__device__ __forceinline__ void hr_sum(double (&v)[NV], double (*red)[HR_CPW]) {
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    v[c] = wave_sum_dpp(v[c]);
    if ((threadIdx.x & 63) == 0) red[w][c] = v[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < HR_NT / 64; ++q) t += red[q][c];
    v[c] = t;
  }
  __syncthreads();
}

// Householder vector of a column x (this thread's rows in c[]) for step kk: acts on rows
// >= kk+1; x0 = x[kk+1], sigma = |x[kk+2..]|^2; v = x - alpha e_{kk+1}, alpha = -sign(x0)|x|,
// beta = 2 / v^T v (beta = 0: nothing to eliminate).  Every workgroup computes it from the same
// data in the same order, so all hold bitwise-equal copies: vr (own rows) and vl (all rows, LDS).
template <int RPT>
__device__ __forceinline__ void hr_house(const double (&c)[RPT], int kk, int m, double (&vr)[RPT],
                                         double *vl, double (*red)[HR_CPW], double *bc,
                                         double &alpha, double &beta) {
  const int tid = threadIdx.x;
  double sv[1] = {0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + HR_NT * r;
    if (i == kk + 1) bc[0] = c[r];
    if (i >= kk + 2 && i < m) sv[0] = fma(c[r], c[r], sv[0]);
  }
  hr_sum<1>(sv, red);  // its barriers also publish bc[0]
  const double x0 = bc[0], sig = sv[0];
  alpha = x0;
  beta = 0.0;
  double v0 = 1.0;
  if (sig > 0.0) {
    const double nrm = sqrt(fma(x0, x0, sig));
    alpha = x0 >= 0.0 ? -nrm : nrm;
    v0 = x0 - alpha;
    beta = 1.0 / (alpha * (alpha - x0));
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + HR_NT * r;
    vr[r] = (i == kk + 1) ? v0 : ((i >= kk + 2 && i < m) ? c[r] : 0.0);
    vl[i] = vr[r];
  }
  __syncthreads();
}

// Workspace of one reduction (HessWork in kernels.hpp): sync = arrival flags [G], err;
// vbuf [mp] (the column snapshot), part [G][2][mp], ybuf [2][mp].
//
// Step k: (b) left reflection on the columns j >= k+1 (column sums are local), partial sums
// of A v and Q v over this workgroup's columns, and the owner of column k+1 publishes that
// column; barrier; (c) each workgroup sums a slice of rows over the workgroups; barrier;
// (d) right reflection A -= beta (A v) v^T, Q -= beta (Q v) v^T; every workgroup then forms
// column k+1 after step k from the snapshot and A v, and derives the next Householder vector
// itself (no wait on the owner).
template <int RPT>
__global__ __launch_bounds__(HR_NT) void k_hess_reduce(const InstDesc *__restrict__ D, int inst,
                                                       HessWork wk, int G) {
  __shared__ double red[HR_NT / 64][HR_CPW];
  __shared__ double vl[HR_NT * RPT];
  __shared__ double bc[2];
  __shared__ int sh;
  const InstDesc &d = D[inst];
  const int m = d.m, mp = d.mp, g = blockIdx.x, tid = threadIdx.x;
  unsigned *arrive = wk.sync;
  int *err = wk.err;
  double a[RPT][HR_CPW], q[RPT][HR_CPW], vr[RPT], col[RPT];
  // J[i][j] = dx^{-alpha} (d+_i g_{i-j+1} + d-_i g_{j-i+1}), g_k = 0 outside 0..m
  auto jent = [&](int i, int j) -> double {
    const int k1 = i - j + 1, k2 = j - i + 1;
    const double gp = (k1 >= 0 && k1 <= m) ? d.g[k1] : 0.0;
    const double gm = (k2 >= 0 && k2 <= m) ? d.g[k2] : 0.0;
    return d.scale * (d.dp[i] * gp + d.dm[i] * gm);
  };
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + HR_NT * r;
#pragma unroll
    for (int c = 0; c < HR_CPW; ++c) {
      const int j = g + G * c;
      a[r][c] = (i < m && j < m) ? jent(i, j) : 0.0;
      q[r][c] = (i == j && i < m) ? 1.0 : 0.0;
    }
    col[r] = i < m ? jent(i, 0) : 0.0;
  }
  const int nsteps = m - 2;  // steps k = 0 .. m-3
  const int rpw = (m + G - 1) / G;
  unsigned nbar = 0;
  double alpha = 0.0, beta = 0.0;
  if (nsteps > 0) {
    hr_house<RPT>(col, 0, m, vr, vl, red, bc, alpha, beta);
    if (g == 0 && beta != 0.0) {  // column 0 (slot 0 of workgroup 0) becomes (x, alpha, 0, ..)
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int i = tid + HR_NT * r;
        if (i >= 1) a[r][0] = (i == 1) ? alpha : 0.0;
      }
    }
  }
  for (int k = 0; k < nsteps; ++k) {
    double vc[HR_CPW];
#pragma unroll
    for (int c = 0; c < HR_CPW; ++c) {
      const int j = g + G * c;
      vc[c] = j < m ? vl[j] : 0.0;
    }
    // (b) left reflection on the columns j >= k+1
    double w[HR_CPW];
#pragma unroll
    for (int c = 0; c < HR_CPW; ++c) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) t = fma(vr[r], a[r][c], t);
      w[c] = t;
    }
    hr_sum<HR_CPW>(w, red);
#pragma unroll
    for (int c = 0; c < HR_CPW; ++c) {
      const int j = g + G * c;
      if (j >= k + 1 && j < m) {
        const double bw = beta * w[c];
#pragma unroll
        for (int r = 0; r < RPT; ++r) a[r][c] = fma(-bw, vr[r], a[r][c]);
      }
    }
    double *pg = wk.part + (size_t)g * 2 * mp;
    const int own1 = (k + 1) % G == g && k + 1 < nsteps, cs1 = (k + 1) / G;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + HR_NT * r;
      if (i < m) {
        double pa = 0.0, pq = 0.0;
#pragma unroll
        for (int c = 0; c < HR_CPW; ++c) {
          pa = fma(a[r][c], vc[c], pa);
          pq = fma(q[r][c], vc[c], pq);
          if (own1 && c == cs1) st_cd(wk.vbuf + i, a[r][c]);  // snapshot of column k+1
        }
        st_cd(pg + i, pa);
        st_cd(pg + mp + i, pq);
      }
    }
    if (!hr_barrier(arrive, G, ++nbar, err, &sh)) return;
    // (c) rows g*rpw ..: y = A v, z = Q v summed over the workgroups in index order
    {
      const int wv = tid >> 6, lane = tid & 63;
      for (int rl = wv; rl < rpw; rl += HR_NT / 64) {
        const int i = g * rpw + rl;
        if (i >= m) break;
        double sa = 0.0, sq = 0.0;
        for (int g0 = 0; g0 < G; g0 += 128) {  // four loads in flight per lane
          const int ga = g0 + lane, gb = g0 + 64 + lane;
          const double a0 = ga < G ? ld_cd(wk.part + (size_t)ga * 2 * mp + i) : 0.0;
          const double q0 = ga < G ? ld_cd(wk.part + (size_t)ga * 2 * mp + mp + i) : 0.0;
          const double a1 = gb < G ? ld_cd(wk.part + (size_t)gb * 2 * mp + i) : 0.0;
          const double q1 = gb < G ? ld_cd(wk.part + (size_t)gb * 2 * mp + mp + i) : 0.0;
          sa += a0 + a1;
          sq += q0 + q1;
        }
        sa = wave_sum_dpp(sa);
        sq = wave_sum_dpp(sq);
        if (lane == 0) {
          st_cd(wk.ybuf + i, sa);
          st_cd(wk.ybuf + mp + i, sq);
        }
      }
    }
    if (!hr_barrier(arrive, G, ++nbar, err, &sh)) return;
    // (d) right reflection, then the next Householder vector from column k+1
    const double vk1 = vl[k + 1 < m ? k + 1 : 0];  // v at row k+1 (read before vl is rewritten)
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + HR_NT * r;
      double by = 0.0;
      if (i < m) {
        by = beta * ld_cd(wk.ybuf + i);
        const double bz = beta * ld_cd(wk.ybuf + mp + i);
#pragma unroll
        for (int c = 0; c < HR_CPW; ++c) {
          a[r][c] = fma(-by, vc[c], a[r][c]);
          q[r][c] = fma(-bz, vc[c], q[r][c]);
        }
      }
      if (k + 1 < nsteps) col[r] = i < m ? fma(-by, vk1, ld_cd(wk.vbuf + i)) : 0.0;
    }
    if (k + 1 < nsteps) {
      __syncthreads();  // every thread has read vl (vc, vk1) before it is rewritten
      hr_house<RPT>(col, k + 1, m, vr, vl, red, bc, alpha, beta);
      if (own1 && beta != 0.0) {
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
          const int i = tid + HR_NT * r;
#pragma unroll
          for (int c = 0; c < HR_CPW; ++c)
            if (c == cs1 && i >= k + 2) a[r][c] = (i == k + 2) ? alpha : 0.0;
        }
      }
    }
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

// arrival flags and the error word (G + 1 words)
__global__ void k_hess_init(HessWork wk, int G) {
  for (int i = threadIdx.x; i < G; i += blockDim.x) wk.sync[i] = 0u;
  if (threadIdx.x == 0) *wk.err = 0;
}

int hess_reduce_groups(int m) { return (m + HR_CPW - 1) / HR_CPW; }

static int hess_rpt(int m) {
  const int r = (m + HR_NT - 1) / HR_NT;
  return r <= 1 ? 1 : r <= 2 ? 2 : 0;
}

// Up to two rows per thread (m <= 1024): the register-resident columns then keep two
// workgroups per CU, more than the m/8 workgroups the cooperative launch needs.
int hess_reduce_max_m() { return 2 * HR_NT; }

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
  hipLaunchKernelGGL(k_hess_init, dim3(1), dim3(256), 0, st, wk, G);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (hess_rpt(m)) {
    case 1: return hess_launch<1>(D, inst, wk, G, st);
    case 2: return hess_launch<2>(D, inst, wk, G, st);
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
// Row exchanges and eliminations of the shifted Hessenberg LU applied to y (in place on Vts
// row k).  Step i maps the carried value c (current entry i) to
//   no exchange: out_i = c,       c' = y_{i+1} - l_i c      (c' = -l_i c + y_{i+1})
//   exchange:    out_i = y_{i+1}, c' = c - l_i y_{i+1}      (c' =  1  c - l_i y_{i+1})
// an affine recurrence c' = A_i c + B_i with |A_i| <= 1.  One wavefront per block: lane t
// composes the maps of its segment of steps, an inclusive scan over the lanes (shuffles)
// gives every segment its incoming carry, and each lane replays its segment.
static constexpr int LS_NT = 64;

__device__ __forceinline__ double2 cm(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 shfl_up2(double2 v, int o) {
  return make_double2(__shfl_up(v.x, o, 64), __shfl_up(v.y, o, 64));
}

__global__ __launch_bounds__(LS_NT) void k_hess_lsolve(const InstDesc *__restrict__ Dd, ItemMap map) {
  extern __shared__ double2 lsm[];
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int blk = blockIdx.x - map.pre[q], m = d.m, mp = d.mp, lane = threadIdx.x;
  double2 *z = lsm, *ll = lsm + mp;
  int *pp = reinterpret_cast<int *>(lsm + 2 * mp);
  double2 *v = d.Vts + (size_t)blk * mp;
  const double2 *lo = d.hl + (size_t)blk * mp;
  const int *pivo = d.hpiv + (size_t)blk * mp;
  for (int i = lane; i < m; i += LS_NT) {
    z[i] = v[i];
    if (i + 1 < m) {
      ll[i] = lo[i];
      pp[i] = pivo[i];
    }
  }
  __syncthreads();
  const int nst = m - 1;  // steps 0 .. m-2
  const int seg = (nst + LS_NT - 1) / LS_NT;
  const int i0 = lane * seg, i1 = i0 + seg < nst ? i0 + seg : nst;
  // (A, B) of this lane's segment: c_out = A c_in + B
  double2 A = make_double2(1.0, 0.0), B = make_double2(0.0, 0.0);
  for (int i = i0; i < i1; ++i) {
    const double2 l = ll[i], y = z[i + 1];
    if (pp[i]) {
      B = make_double2(B.x - (l.x * y.x - l.y * y.y), B.y - (l.x * y.y + l.y * y.x));
    } else {
      const double2 nl = make_double2(-l.x, -l.y);
      A = cm(nl, A);
      B = make_double2(fma(nl.x, B.x, fma(-nl.y, B.y, y.x)), fma(nl.x, B.y, fma(nl.y, B.x, y.y)));
    }
  }
  // inclusive scan of the maps over the lanes: lane t ends with segments 0..t composed
#pragma unroll
  for (int o = 1; o < LS_NT; o <<= 1) {
    const double2 Ap = shfl_up2(A, o), Bp = shfl_up2(B, o);
    if (lane >= o) {  // (A, B) after (Ap, Bp): c -> A (Ap c + Bp) + B
      const double2 AB = cm(A, Bp);
      B = make_double2(AB.x + B.x, AB.y + B.y);
      A = cm(A, Ap);
    }
  }
  const double2 z0 = z[0];
  const double2 endc = make_double2(A.x * z0.x - A.y * z0.y + B.x, A.x * z0.y + A.y * z0.x + B.y);
  double2 c = shfl_up2(endc, 1);
  if (lane == 0) c = z0;
  __syncthreads();  // every lane has read z[0] and its segment's inputs
  // replay: out_i into a register list first (z[i + 1] of this segment is still needed)
  for (int i = i0; i < i1; ++i) {
    const double2 l = ll[i], y = z[i + 1];
    const bool sw = pp[i] != 0;
    const double2 out = sw ? y : c, oth = sw ? c : y;
    c = make_double2(oth.x - (l.x * out.x - l.y * out.y), oth.y - (l.x * out.y + l.y * out.x));
    v[i] = out;
  }
  if (i0 < i1 && i1 == nst) v[nst] = c;
  if (nst == 0 && lane == 0) v[0] = z0;
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
// As a real product its rows are the real and imaginary parts of the bins 1 .. s/2 - 1 and the
// real parts of bins 0 and s/2, paired in slot 0: the imaginary parts of those two bins never
// reach the preconditioner's result (the inverse time FFT of a real vector discards them), so
// they are not read and are written as 0.  That is s real rows.
// Workgroup tile: 32 slots (64 real rows) x 64 columns over the whole K range.  Four groups of
// four wavefronts take interleaved 16-deep K slices (group g the slices g, g + 4, ...), each
// wavefront a 32 x 32 quarter of the tile (2 x 2 FP64 MFMA 16x16x4 tiles), staged through LDS
// one slice ahead; the groups' partial tiles are summed at the end in group order.  Sixteen
// wavefronts per CU hide the slices' latency.  Consecutive workgroups run on different XCDs;
// the slot tiles of one column tile go to the same XCD, so its L2 serves their common B
// columns.  Item = (instance, slot tile, column tile).
static constexpr int QG_NG = 4, QG_NT = 256 * QG_NG, QG_KS = 16, QG_LD = 64 + 1;
static constexpr int QG_BUF = QG_KS * QG_LD;  // one staged slice of A or B

__global__ __launch_bounds__(QG_NT) void k_qgemm(const InstDesc *__restrict__ Dd, ItemMap map,
                                                 int trans, int src2) {
  // [group][buffer] A slices (k x real row) then B slices (k x column); reused for the partials
  __shared__ double sm[2 * QG_NG * 2 * QG_BUF];
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int local = blockIdx.x - map.pre[q];
  const int m = d.m, mp = d.mp, nb = d.nb, ns = nb - 1;
  const int ncol = mp / 64, nrt = (ns + 31) / 32;
  int rt, ct;
  if (ncol % 8 == 0) {
    ct = 8 * ((local / 8) / nrt) + local % 8;
    rt = (local / 8) % nrt;
  } else {
    rt = local / ncol;
    ct = local % ncol;
  }
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int kg = wv >> 2, wr = ((wv & 3) >> 1) * 32, wc = (wv & 1) * 32, ht = tid & 255;
  const double2 *X = src2 ? d.Vts : d.Vh;
  double2 *Y = src2 ? d.Vh : d.Vts;
  const double *B = trans ? d.hQt : d.hQ;
  const int s0 = rt * 32, c0 = ct * 64;
  double *Ag = sm + (size_t)kg * 2 * QG_BUF, *Bg = sm + (size_t)(QG_NG + kg) * 2 * QG_BUF;
  // loaders (per group): A slot ht / 8 at k 2 (ht % 8) .. + 1; B row ht / 16 at columns 4 (ht % 16) .. + 3
  const int as = ht >> 3, aslot = s0 + as, ak = (ht & 7) * 2, bk = ht >> 4, bc = (ht & 15) * 4;
  const bool aok = aslot < ns;
  const double2 *Xa = X + (size_t)(aok ? aslot : 0) * mp, *Xn = X + (size_t)ns * mp;
  // The global loads of a slice go to registers of their own (from in-range addresses only) and
  // the zeros and the slot-0 pairing are applied when the slice is staged, after the products:
  // nothing waits for the loads before then.
  double2 xa[2], xb[2];
  double xs[2];
  int kpend = 0;
  auto load = [&](int k0) {
    kpend = k0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int k = k0 + ak + u;
      const bool in = aok && k < m;
      xa[u] = gld(Xa + (in ? k : 0));
      // slot 0 pairs the real parts of bins 0 and s/2; loaded by every thread (no branch, so no
      // wait at its join), an L2 hit but for the first
      xs[u] = gld(&Xn[in ? k : 0].x);
    }
    const int k = k0 + bk;
    const double2 *pb = reinterpret_cast<const double2 *>(B + (size_t)(k < m ? k : 0) * mp + c0 + bc);
#pragma unroll
    for (int u = 0; u < 2; ++u) xb[u] = gld(pb + u);
  };
  auto stage = [&](int buf) {
    double *A_ = Ag + buf * QG_BUF, *B_ = Bg + buf * QG_BUF;
    const bool bin = kpend + bk < m;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const bool in = aok && kpend + ak + u < m;
      A_[(ak + u) * QG_LD + 2 * as] = in ? xa[u].x : 0.0;
      A_[(ak + u) * QG_LD + 2 * as + 1] = in ? (aslot == 0 ? xs[u] : xa[u].y) : 0.0;
      B_[bk * QG_LD + bc + 2 * u] = bin ? xb[u].x : 0.0;
      B_[bk * QG_LD + bc + 2 * u + 1] = bin ? xb[u].y : 0.0;
    }
  };
  v4d acc[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[r][c] = v4d{0.0, 0.0, 0.0, 0.0};
  const int nround = (m + QG_NG * QG_KS - 1) / (QG_NG * QG_KS);  // slice rounds covering K = m
  load(kg * QG_KS);
  stage(0);
  __syncthreads();
  for (int p = 0; p < nround; ++p) {
    const int buf = p & 1;
    if (p + 1 < nround) load(((p + 1) * QG_NG + kg) * QG_KS);
    __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of the products
    const double *A_ = Ag + buf * QG_BUF, *B_ = Bg + buf * QG_BUF;
#pragma unroll
    for (int kk = 0; kk < QG_KS; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) av[r] = A_[(kk + lk) * QG_LD + wr + 16 * r + li];
#pragma unroll
      for (int c = 0; c < 2; ++c) bv[c] = B_[(kk + lk) * QG_LD + wc + 16 * c + li];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[r][c] = mfma16(av[r], bv[c], acc[r][c]);
    }
    __builtin_amdgcn_sched_barrier(0);  // and the staging, which waits for them, after
    if (p + 1 < nround) stage(buf ^ 1);
    __syncthreads();
  }
  // groups 1 .. 3 hand their tiles to group 0 (the staging buffers reused as [3][64][64])
  if (kg > 0) {
    double *part = sm + (size_t)(kg - 1) * 64 * 64;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          part[(wr + 16 * r + mfma_row<double>(lk, v)) * 64 + wc + 16 * c + li] = acc[r][c][v];
  }
  __syncthreads();
  if (kg > 0) return;
  double *Yd = reinterpret_cast<double *>(Y);
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + 16 * r + mfma_row<double>(lk, v), col = c0 + wc + 16 * c + li;
        const int slot = s0 + (row >> 1), im = row & 1;
        if (slot >= ns) continue;
        double val = acc[r][c][v];
#pragma unroll
        for (int g = 0; g < QG_NG - 1; ++g) val += sm[(size_t)g * 64 * 64 + row * 64 + wc + 16 * c + li];
        if (col >= m) val = 0.0;
        if (slot == 0)
          Y[(size_t)(im ? ns : 0) * mp + col] = make_double2(val, 0.0);
        else
          Yd[((size_t)slot * mp + col) * 2 + im] = val;
      }
}

int qgemm_items(int nb, int mp) { return ((nb - 1 + 31) / 32) * (mp / 64); }

hipError_t launch_qgemm(const InstDesc *D, const ItemMap &map, int items, int trans, int src2,
                        hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_qgemm, dim3(items), dim3(QG_NT), 0, st, D, map, trans, src2);
  return hipGetLastError();
}

template hipError_t launch_hess_lu<double>(const InstDesc *, const ItemMap &, int, int, int *, hipStream_t);
template hipError_t launch_hess_lu<float>(const InstDesc *, const ItemMap &, int, int, int *, hipStream_t);

}  // namespace fde
