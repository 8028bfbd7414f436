// Preconditioner blocks K_k = lambda_k I - tau mu_k J (Section 3.2): assembly, batched
// pivot-free blocked LU on MFMA and the forward/back substitutions that apply K_k^{-1}.
//
// Storage (T = double for complex FP64, float for complex FP32, interleaved re/im):
//   K    [nb][mp][mp] row-major, mp = m rounded up to a multiple of 64; the pad carries a
//        unit diagonal so it factors exactly and leaves the solution untouched.
//   dinv [nb][mp/64][2][64][64]: inverses of the unit-lower and upper 64x64 diagonal
//        triangles of every panel (used by the panel update and by the solves).
//
// LU step p (panel width 64):  A11 = L11 U11 in LDS (one workgroup per block), then
//   L21 = A21 U11^{-1},  U12 = L11^{-1} A12   (k_lu_panel, 64x64x64 complex GEMMs)
//   A22 -= L21 U12                             (k_lu_update, 64x64 tiles, K = 64)
// Complex products use four real MFMAs on the re/im parts (gfx950 has no complex MFMA).
#include "common.hpp"
#include "kernels.hpp"

namespace fde {

static constexpr int PB = 64;  // panel width / tile size

// ------------------------------------------------------------------------------------
// Assembly: one workgroup per row i, covering blocks [k0, k0+kchunk).
// J[i][j] = dx^{-a} (d+_i g_{i-j+1} + d-_i g_{j-i+1}), g_k = 0 outside 0..m.
template <typename T>
__global__ __launch_bounds__(256) void k_assemble(c_t<T> *__restrict__ K, int m, int mp, int nb,
                                                  int kchunk, const double2 *__restrict__ lam,
                                                  const double2 *__restrict__ mu, double tau,
                                                  double scale, const double *__restrict__ g,
                                                  const double *__restrict__ dp,
                                                  const double *__restrict__ dm) {
  const int i = blockIdx.x;
  const int k0 = blockIdx.y * kchunk;
  const int k1 = min(nb, k0 + kchunk);
  for (int j = threadIdx.x; j < mp; j += 256) {
    double Jij = 0.0;
    if (i < m && j < m) {
      const int d = i - j;
      const double gp = (d >= -1 && d + 1 <= m) ? g[d + 1] : 0.0;
      const double gm = (d <= 1 && 1 - d <= m) ? g[1 - d] : 0.0;
      Jij = scale * fma(dp[i], gp, dm[i] * gm);
    }
    for (int k = k0; k < k1; ++k) {
      double re = -tau * mu[k].x * Jij, im = -tau * mu[k].y * Jij;
      if (i == j) {
        if (i < m) {
          re += lam[k].x;
          im += lam[k].y;
        } else {
          re = 1.0;
          im = 0.0;
        }
      }
      K[((size_t)k * mp + i) * mp + j] = mk<T>((T)re, (T)im);
    }
  }
}

// ------------------------------------------------------------------------------------
// Diagonal tile: LU without pivoting, then the two triangular inverses.  256 threads;
// thread t owns row t/4 and columns (t%4) + 4j, j = 0..15.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_diag(c_t<T> *__restrict__ K, int mp, int p,
                                                 c_t<T> *__restrict__ dinv, int *__restrict__ flag) {
  typedef c_t<T> C;
  __shared__ C a[PB][PB + 1];
  __shared__ C x[PB][PB + 1];
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int npan = mp / PB;
  C *A = K + (size_t)blk * mp * mp + (size_t)p * PB * mp + (size_t)p * PB;
  for (int e = tid; e < PB * PB; e += 256) a[e >> 6][e & 63] = A[(size_t)(e >> 6) * mp + (e & 63)];
  __syncthreads();
  const int r = tid >> 2, cq = tid & 3;
  int bad = 0;
  for (int k = 0; k < PB; ++k) {
    const C piv = a[k][k];
    const T pm = piv.x * piv.x + piv.y * piv.y;
    if (!(pm > (T)0) || !isfinite(pm)) bad = 1;
    const C ip = trecip<T>(piv);
    C l = mk<T>(0, 0);
    C nv[16];
    if (r > k) {
      l = tmul<T>(a[r][k], ip);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int c = cq + 4 * j;
        nv[j] = (c > k) ? tsub<T>(a[r][c], tmul<T>(l, a[k][c])) : a[r][c];
      }
    }
    __syncthreads();
    if (r > k) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int c = cq + 4 * j;
        if (c > k) a[r][c] = nv[j];
        else if (c == k) a[r][c] = l;
      }
    }
    __syncthreads();
  }
  if (bad && tid == 0) atomicOr(flag, 1);
  for (int e = tid; e < PB * PB; e += 256) A[(size_t)(e >> 6) * mp + (e & 63)] = a[e >> 6][e & 63];

  C *Dl = dinv + ((size_t)(blk * npan + p) * 2 + 0) * PB * PB;
  C *Du = Dl + PB * PB;
  // X = L11^{-1}: rows r > k receive -L[r][k] X[k][:], row k is final at step k.
  for (int e = tid; e < PB * PB; e += 256)
    x[e >> 6][e & 63] = mk<T>((e >> 6) == (e & 63) ? (T)1 : (T)0, (T)0);
  __syncthreads();
  for (int k = 0; k < PB - 1; ++k) {
    if (r > k) {
      const C lrk = a[r][k];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int c = cq + 4 * j;
        if (c <= k) x[r][c] = tsub<T>(x[r][c], tmul<T>(lrk, x[k][c]));
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < PB * PB; e += 256) Dl[e] = x[e >> 6][e & 63];
  __syncthreads();
  // X = U11^{-1}: for k = 63..0, scale row k by 1/U[k][k], then rows r < k receive -U[r][k] X[k][:].
  for (int e = tid; e < PB * PB; e += 256)
    x[e >> 6][e & 63] = mk<T>((e >> 6) == (e & 63) ? (T)1 : (T)0, (T)0);
  __syncthreads();
  for (int k = PB - 1; k >= 0; --k) {
    if (r == k) {
      const C iu = trecip<T>(a[k][k]);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int c = cq + 4 * j;
        if (c >= k) x[k][c] = tmul<T>(x[k][c], iu);
      }
    }
    __syncthreads();
    if (r < k) {
      const C u = a[r][k];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int c = cq + 4 * j;
        if (c >= k) x[r][c] = tsub<T>(x[r][c], tmul<T>(u, x[k][c]));
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < PB * PB; e += 256) Du[e] = x[e >> 6][e & 63];
}

// ------------------------------------------------------------------------------------
// One wavefront: acc (+/-)= A[32x64] * B[64x32] (complex), 2x2 MFMA 16x16 sub-tiles.
template <typename T, bool NEG>
__device__ __forceinline__ void wave_mma(const c_t<T> *__restrict__ A, int lda,
                                         const c_t<T> *__restrict__ B, int ldb,
                                         acc_t<T> (&cre)[2][2], acc_t<T> (&cim)[2][2]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int k0 = 0; k0 < PB; k0 += 4) {
    c_t<T> a[2], b[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) a[r] = A[(size_t)(r * 16 + li) * lda + k0 + lk];
#pragma unroll
    for (int c = 0; c < 2; ++c) b[c] = B[(size_t)(k0 + lk) * ldb + c * 16 + li];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const T ar = NEG ? -a[r].x : a[r].x;
      const T ai = NEG ? -a[r].y : a[r].y;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        cre[r][c] = mfma16(ar, b[c].x, cre[r][c]);
        cre[r][c] = mfma16(-ai, b[c].y, cre[r][c]);
        cim[r][c] = mfma16(ar, b[c].y, cim[r][c]);
        cim[r][c] = mfma16(ai, b[c].x, cim[r][c]);
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void tile_load(const c_t<T> *__restrict__ Cp, int ldc,
                                          acc_t<T> (&cre)[2][2], acc_t<T> (&cim)[2][2]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const c_t<T> z = Cp[(size_t)(r * 16 + mfma_row<T>(lk, v)) * ldc + c * 16 + li];
        cre[r][c][v] = z.x;
        cim[r][c][v] = z.y;
      }
}

template <typename T>
__device__ __forceinline__ void tile_store(c_t<T> *__restrict__ Cp, int ldc,
                                           const acc_t<T> (&cre)[2][2], const acc_t<T> (&cim)[2][2]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Cp[(size_t)(r * 16 + mfma_row<T>(lk, v)) * ldc + c * 16 + li] = mk<T>(cre[r][c][v], cim[r][c][v]);
}

template <typename T>
__device__ __forceinline__ void tile_zero(acc_t<T> (&cre)[2][2], acc_t<T> (&cim)[2][2]) {
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        cre[r][c][v] = (T)0;
        cim[r][c][v] = (T)0;
      }
}

// Panel: blockIdx.x < nrem -> L21 tile t = A21_t U11^{-1}; else U12 tile = L11^{-1} A12_t.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_panel(c_t<T> *__restrict__ K, int mp, int p,
                                                  const c_t<T> *__restrict__ dinv) {
  typedef c_t<T> C;
  const int npan = mp / PB, nrem = npan - p - 1;
  const int t = blockIdx.x, blk = blockIdx.y;
  C *Kb = K + (size_t)blk * mp * mp;
  const int wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  acc_t<T> cre[2][2], cim[2][2];
  tile_zero<T>(cre, cim);
  const C *Dl = dinv + ((size_t)(blk * npan + p) * 2 + 0) * PB * PB;
  const C *Du = Dl + PB * PB;
  C *Ct;
  if (t < nrem) {
    Ct = Kb + (size_t)(p + 1 + t) * PB * mp + (size_t)p * PB;
    wave_mma<T, false>(Ct + (size_t)wr * mp, mp, Du + wc, PB, cre, cim);
  } else {
    Ct = Kb + (size_t)p * PB * mp + (size_t)(p + 1 + t - nrem) * PB;
    wave_mma<T, false>(Dl + (size_t)wr * PB, PB, Ct + wc, mp, cre, cim);
  }
  __syncthreads();  // every wave has read its operands before the tile is overwritten
  tile_store<T>(Ct + (size_t)wr * mp + wc, mp, cre, cim);
}

// Trailing update: tile (ti, tj) of A22 -= L21_ti U12_tj.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_update(c_t<T> *__restrict__ K, int mp, int p) {
  typedef c_t<T> C;
  const int npan = mp / PB, nrem = npan - p - 1;
  const int ti = blockIdx.x / nrem, tj = blockIdx.x % nrem, blk = blockIdx.y;
  C *Kb = K + (size_t)blk * mp * mp;
  const int wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  C *Ct = Kb + (size_t)(p + 1 + ti) * PB * mp + (size_t)(p + 1 + tj) * PB + (size_t)wr * mp + wc;
  const C *A = Kb + (size_t)(p + 1 + ti) * PB * mp + (size_t)p * PB + (size_t)wr * mp;
  const C *B = Kb + (size_t)p * PB * mp + (size_t)(p + 1 + tj) * PB + wc;
  acc_t<T> cre[2][2], cim[2][2];
  tile_load<T>(Ct, mp, cre, cim);
  wave_mma<T, true>(A, mp, B, mp, cre, cim);
  tile_store<T>(Ct, mp, cre, cim);
}

// ------------------------------------------------------------------------------------
// Block solves K_k w = v in place on Vh[k] (FP64 vectors, factors of type T).
// One workgroup per block: per 64-row panel an off-diagonal GEMV streamed from HBM,
// then the 64x64 inverse of the diagonal triangle.
static constexpr int TS_NT = 1024;

template <typename T>
__global__ __launch_bounds__(TS_NT) void k_trsv(const c_t<T> *__restrict__ K,
                                                const c_t<T> *__restrict__ dinv,
                                                double2 *__restrict__ Vh, int mp) {
  extern __shared__ double2 sh[];
  double2 *y = sh;
  double2 *tmp = sh + mp;
  const int blk = blockIdx.x, npan = mp / PB;
  const c_t<T> *A = K + (size_t)blk * mp * mp;
  double2 *v = Vh + (size_t)blk * mp;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int NW = TS_NT / 64;
  for (int i = threadIdx.x; i < mp; i += TS_NT) y[i] = v[i];
  __syncthreads();
  for (int P = 0; P < npan; ++P) {
    const int p0 = P * PB;
    for (int rr = wave; rr < PB; rr += NW) {
      const c_t<T> *row = A + (size_t)(p0 + rr) * mp;
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll 8
      for (int c = lane; c < p0; c += 64) acc = cfma(widen(row[c]), y[c], acc);
      acc = wave_sum(acc);
      if (lane == 0) tmp[rr] = csub(y[p0 + rr], acc);
    }
    __syncthreads();
    const c_t<T> *Li = dinv + ((size_t)(blk * npan + P) * 2 + 0) * PB * PB;
    for (int rr = wave; rr < PB; rr += NW) {
      double2 acc = cfma(widen(Li[rr * PB + lane]), tmp[lane], make_double2(0.0, 0.0));
      acc = wave_sum(acc);
      if (lane == 0) y[p0 + rr] = acc;
    }
    __syncthreads();
  }
  for (int P = npan - 1; P >= 0; --P) {
    const int p0 = P * PB;
    for (int rr = wave; rr < PB; rr += NW) {
      const c_t<T> *row = A + (size_t)(p0 + rr) * mp;
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll 8
      for (int c = p0 + PB + lane; c < mp; c += 64) acc = cfma(widen(row[c]), y[c], acc);
      acc = wave_sum(acc);
      if (lane == 0) tmp[rr] = csub(y[p0 + rr], acc);
    }
    __syncthreads();
    const c_t<T> *Ui = dinv + ((size_t)(blk * npan + P) * 2 + 1) * PB * PB;
    for (int rr = wave; rr < PB; rr += NW) {
      double2 acc = cfma(widen(Ui[rr * PB + lane]), tmp[lane], make_double2(0.0, 0.0));
      acc = wave_sum(acc);
      if (lane == 0) y[p0 + rr] = acc;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < mp; i += TS_NT) v[i] = y[i];
}

// ------------------------------------------------------------------------------------
template <typename T>
hipError_t launch_assemble(void *K, int m, int mp, int nb, const double2 *lam, const double2 *mu,
                           double tau, double scale, const double *g, const double *dp,
                           const double *dm, hipStream_t st) {
  const int kchunk = 8;
  hipLaunchKernelGGL(k_assemble<T>, dim3(mp, (nb + kchunk - 1) / kchunk), dim3(256), 0, st,
                     (c_t<T> *)K, m, mp, nb, kchunk, lam, mu, tau, scale, g, dp, dm);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lu_diag(void *K, int mp, int nb, int p, void *dinv, int *flag, hipStream_t st) {
  hipLaunchKernelGGL(k_lu_diag<T>, dim3(nb), dim3(256), 0, st, (c_t<T> *)K, mp, p,
                     (c_t<T> *)dinv, flag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lu_panel(void *K, int mp, int nb, int p, const void *dinv, hipStream_t st) {
  const int nrem = mp / PB - p - 1;
  if (nrem <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lu_panel<T>, dim3(2 * nrem, nb), dim3(256), 0, st, (c_t<T> *)K, mp, p,
                     (const c_t<T> *)dinv);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lu_update(void *K, int mp, int nb, int p, hipStream_t st) {
  const int nrem = mp / PB - p - 1;
  if (nrem <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lu_update<T>, dim3(nrem * nrem, nb), dim3(256), 0, st, (c_t<T> *)K, mp, p);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_trsv(const void *K, const void *dinv, double2 *Vh, int mp, int nb,
                       hipStream_t st) {
  const size_t lds = sizeof(double2) * (mp + PB);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)k_trsv<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_trsv<T>, dim3(nb), dim3(TS_NT), lds, st, (const c_t<T> *)K,
                     (const c_t<T> *)dinv, Vh, mp);
  return hipGetLastError();
}

#define FDE_INST(T)                                                                              \
  template hipError_t launch_assemble<T>(void *, int, int, int, const double2 *, const double2 *, \
                                         double, double, const double *, const double *,         \
                                         const double *, hipStream_t);                           \
  template hipError_t launch_lu_diag<T>(void *, int, int, int, void *, int *, hipStream_t);      \
  template hipError_t launch_lu_panel<T>(void *, int, int, int, const void *, hipStream_t);      \
  template hipError_t launch_lu_update<T>(void *, int, int, int, hipStream_t);                   \
  template hipError_t launch_trsv<T>(const void *, const void *, double2 *, int, int, hipStream_t);
FDE_INST(double)
FDE_INST(float)
#undef FDE_INST

}  // namespace fde
