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
//   A22 -= L21 U12                             (k_lu_update, 64x64 tiles; steps are paired
//                                               so the bulk of the update runs with K = 128)
// Complex products use four real MFMAs on the re/im parts (gfx950 has no complex MFMA).
#include "batch.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace fde {

static constexpr int PB = 64;  // panel width / tile size

// ------------------------------------------------------------------------------------
// Assembly.  K_k[i][j] = lam_k delta_ij - tau mu_k J[i][j],
// J[i][j] = dx^{-a} (d+_i g_{i-j+1} + d-_i g_{j-i+1}), g_k = 0 outside 0..m; the pad rows and
// columns (i or j >= m) carry the unit diagonal.  Computed in FP64, rounded once to T.
struct EntryGen {  // the scalars of one block, read once (stores to K could alias them)
  double tau, scale;
  double2 mu, lam;
  int m;
  const double *g, *dp, *dm;
};
__device__ __forceinline__ EntryGen entry_gen(const InstDesc &d, int k) {
  EntryGen e;
  e.tau = d.tau;
  e.scale = d.scale;
  e.mu = d.mu[k];
  e.lam = d.lam[k];
  e.m = d.m;
  e.g = d.g;
  e.dp = d.dp;
  e.dm = d.dm;
  return e;
}

__device__ __forceinline__ double j_entry(const EntryGen &e, int i, int j) {
  if (i >= e.m || j >= e.m) return 0.0;
  const int dd = i - j, m = e.m;
  const double gp = (dd >= -1 && dd + 1 <= m) ? e.g[dd + 1] : 0.0;
  const double gm = (dd <= 1 && 1 - dd <= m) ? e.g[1 - dd] : 0.0;
  return e.scale * fma(e.dp[i], gp, e.dm[i] * gm);
}

template <typename T>
__device__ __forceinline__ c_t<T> block_entry(const EntryGen &e, int i, int j, double Jij) {
  double re = -e.tau * e.mu.x * Jij, im = -e.tau * e.mu.y * Jij;
  if (i == j) {
    if (i < e.m) {
      re += e.lam.x;
      im += e.lam.y;
    } else {
      re = 1.0;
      im = 0.0;
    }
  }
  return mk<T>((T)re, (T)im);
}

// The LU reads the entries of the first two block rows and columns (i or j < ASM_LEAD) before
// any update; the others are first read by the trailing update of the first pair of steps,
// which forms them itself (k_lu_update, p = 0).  So the assembly writes only the former.
// Item = (instance, row i, chunk of kchunk blocks).
static constexpr int ASM_LEAD = 2 * PB;

template <typename T>
__global__ __launch_bounds__(256) void k_assemble(const InstDesc *__restrict__ D, ItemMap map,
                                                  int kchunk) {
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = D[map.ids[q]];
  const int local = blockIdx.x - map.pre[q];
  const int mp = d.mp, nb = d.nb;
  const int nkc = (nb + kchunk - 1) / kchunk;
  const int i = local / nkc;
  const int k0 = (local % nkc) * kchunk;
  const int k1 = min(nb, k0 + kchunk);
  const int jend = i < ASM_LEAD ? mp : min(mp, ASM_LEAD);
  c_t<T> *K = (c_t<T> *)d.K;
  const EntryGen e0 = entry_gen(d, 0);
  for (int j = threadIdx.x; j < jend; j += 256) {
    const double Jij = j_entry(e0, i, j);
    for (int k = k0; k < k1; ++k) {
      EntryGen e = e0;
      e.mu = d.mu[k];
      e.lam = d.lam[k];
      K[((size_t)k * mp + i) * mp + j] = block_entry<T>(e, i, j, Jij);
    }
  }
}

// ------------------------------------------------------------------------------------
// Diagonal tile: LU without pivoting, then the inverses of its unit-lower and upper
// triangles.  NT threads: 1024 for FP32 factors, 512 for FP64 (whose registers would
// otherwise allow only one workgroup per CU).
//
// LU: thread t owns row r = t / (NT/64) and columns c = t % (NT/64) + (NT/64) j in registers.
// Step k needs the pivot row, the pivot column and the pivot's reciprocal; their owners
// publish them into double-buffered LDS vectors at the end of step k-1 (the reciprocal is
// computed once, by the pivot's owner), so a step costs one barrier, one batch of LDS reads
// and at most 64^2/NT complex multiply-adds per thread.
//
// Inverses: both triangles at once by recursive doubling (tri_inv_doubling), in the LDS copy
// of the factored tile.
template <typename T> struct DiagThreads { static constexpr int value = 1024; };
template <> struct DiagThreads<double> { static constexpr int value = 512; };

// cond ? a : b, component-wise (a select of the vector struct would be lowered through
// private memory)
template <typename T>
__device__ __forceinline__ c_t<T> csel(bool cond, c_t<T> a, c_t<T> b) {
  return mk<T>(cond ? a.x : b.x, cond ? a.y : b.y);
}

// 1/z = conj(z) / |z|^2 (one real division); `ok` is false for a zero or non-finite |z|^2.
template <typename T>
__device__ __forceinline__ c_t<T> recip_checked(c_t<T> z, bool &ok) {
  const T m2 = z.x * z.x + z.y * z.y;
  ok = (m2 > (T)0) && isfinite(m2);
  const T inv = (T)1 / m2;
  return mk<T>(z.x * inv, -z.y * inv);
}

// acc + a b in T
template <typename T>
__device__ __forceinline__ c_t<T> tfma(c_t<T> a, c_t<T> b, c_t<T> acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}

// Output e of a doubling level (b = 2^lb): side (lower / upper), block offset o and entry
// (i, j) of the b x b off-diagonal block; per side there are (32 / b) blocks of b^2 entries.
struct DblIdx {
  bool up;
  int o, i, j;
};
template <bool LOWER>
__device__ __forceinline__ DblIdx dbl_idx(int e, int lb) {
  const int per = 32 << lb;
  DblIdx x;
  x.up = !LOWER || e >= per;
  const int e2 = (LOWER && x.up) ? e - per : e;
  const int b = 1 << lb;
  x.o = (e2 >> (2 * lb)) << (lb + 1);
  x.i = (e2 >> lb) & (b - 1);
  x.j = e2 & (b - 1);
  return x;
}

// The inverses of both triangles of a 64x64 LU tile in a[][] (L strictly below the diagonal
// with an implicit unit diagonal; U on and above it, its diagonal already replaced by the
// reciprocals), in place, by recursive doubling.  At level b = 1, 2, ..., 32 every diagonal
// block of size 2b is inverted from its two inverted halves:
//   lower  [X1 0; L21 X2]^{-1}  has the off-diagonal block  -X2 (L21 X1),
//   upper  [Y1 U12; 0 Y2]^{-1}  has the off-diagonal block  -Y1 (U12 Y2);
// the product in parentheses is formed in registers and stored over L21 / U12, then the outer
// one replaces it.  Six levels of four barriers each, instead of two substitutions of 63
// barrier-separated steps.  LOWER = false: the upper triangle only.
template <typename T, int NT, bool LOWER>
__device__ __forceinline__ void tri_inv_doubling(c_t<T> (*a)[PB + 1]) {
  typedef c_t<T> C;
  constexpr int SIDES = LOWER ? 2 : 1;
  constexpr int NO = (SIDES * 32 * 32 + NT - 1) / NT;  // outputs per thread at b = 32
  const C zero = mk<T>((T)0, (T)0);
#pragma unroll 1
  for (int lb = 0; lb < 6; ++lb) {
    const int b = 1 << lb, tot = SIDES * (32 << lb);
    C t[NO];
#pragma unroll
    for (int u = 0; u < NO; ++u) {  // inner products
      const int e = threadIdx.x + NT * u;
      C acc = zero;
      if (e < tot) {
        const DblIdx x = dbl_idx<LOWER>(e, lb);
        const int o = x.o, i = x.i, j = x.j;
        if (!x.up) {  // (L21 X1)[i][j] = L21[i][j] + sum_{k > j} L21[i][k] X1[k][j]
          acc = a[o + b + i][o + j];
          for (int k = j + 1; k < b; ++k) acc = tfma<T>(a[o + b + i][o + k], a[o + k][o + j], acc);
        } else {  // (U12 Y2)[i][j] = sum_{k <= j} U12[i][k] Y2[k][j]
          for (int k = 0; k <= j; ++k) acc = tfma<T>(a[o + i][o + b + k], a[o + b + k][o + b + j], acc);
        }
      }
      t[u] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NO; ++u) {
      const int e = threadIdx.x + NT * u;
      if (e < tot) {
        const DblIdx x = dbl_idx<LOWER>(e, lb);
        if (!x.up) a[x.o + b + x.i][x.o + x.j] = t[u];
        else a[x.o + x.i][x.o + b + x.j] = t[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NO; ++u) {  // outer products, negated
      const int e = threadIdx.x + NT * u;
      C acc = zero;
      if (e < tot) {
        const DblIdx x = dbl_idx<LOWER>(e, lb);
        const int o = x.o, i = x.i, j = x.j;
        if (!x.up) {  // X21[i][j] = -(T[i][j] + sum_{k < i} X2[i][k] T[k][j])
          acc = a[o + b + i][o + j];
          for (int k = 0; k < i; ++k) acc = tfma<T>(a[o + b + i][o + b + k], a[o + b + k][o + j], acc);
        } else {  // Y12[i][j] = -sum_{k >= i} Y1[i][k] T[k][j]
          for (int k = i; k < b; ++k) acc = tfma<T>(a[o + i][o + k], a[o + k][o + b + j], acc);
        }
      }
      t[u] = mk<T>(-acc.x, -acc.y);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NO; ++u) {
      const int e = threadIdx.x + NT * u;
      if (e < tot) {
        const DblIdx x = dbl_idx<LOWER>(e, lb);
        if (!x.up) a[x.o + b + x.i][x.o + x.j] = t[u];
        else a[x.o + x.i][x.o + b + x.j] = t[u];
      }
    }
    __syncthreads();
  }
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_lu_diag(const InstDesc *__restrict__ Dd, ItemMap map, int p,
                                                int *__restrict__ flag) {
  typedef c_t<T> C;
  constexpr int TPR = NT / PB, NC = PB / TPR;  // LU: threads per row, columns per thread
  __shared__ C a[PB][PB + 1];
  __shared__ C prow[2][PB];
  __shared__ C pcol[2][PB];
  __shared__ C dgi[PB];  // reciprocals of U's diagonal
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int blk = blockIdx.x - map.pre[q], tid = threadIdx.x;
  const int mp = d.mp, npan = d.npan;
  C *K = (C *)d.K;
  C *dinv = (C *)d.dinv;
  C *A = K + (size_t)blk * mp * mp + (size_t)p * PB * mp + (size_t)p * PB;
  int bad = 0;
  {
    const int r = tid / TPR, cl = tid % TPR;
    C x[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) x[j] = A[(size_t)r * mp + cl + TPR * j];
    if (r == 0) {
#pragma unroll
      for (int j = 0; j < NC; ++j) prow[0][cl + TPR * j] = x[j];
    }
    if (cl == 0) pcol[0][r] = x[0];
    if (tid == 0) {
      bool ok;
      dgi[0] = recip_checked<T>(x[0], ok);
      bad |= ok ? 0 : 1;
    }
    __syncthreads();
    // k = TPR kk + ki; kk is unrolled so that every register index below is a constant
#pragma unroll
    for (int kk = 0; kk < NC; ++kk) {
#pragma unroll 1
      for (int ki = 0; ki < TPR; ++ki) {
        const int k = TPR * kk + ki, b = k & 1, nbuf = b ^ 1;
        if (r > k) {
          const C l = tmul<T>(pcol[b][r], dgi[k]);
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            const int c = cl + TPR * j;
            const C upd = tsub<T>(x[j], tmul<T>(l, prow[b][c]));
            x[j] = csel<T>(c > k, upd, csel<T>(c == k, l, x[j]));
          }
        }
        const int kc = k + 1;
        if (kc < PB) {
          if (r == kc) {
#pragma unroll
            for (int j = 0; j < NC; ++j) prow[nbuf][cl + TPR * j] = x[j];
          }
          if (cl == kc % TPR) {
            // column kc lives in register x[kc / TPR]: x[kk], or x[kk + 1] after the last ki
            const C xc = csel<T>(ki == TPR - 1, x[kk + 1 < NC ? kk + 1 : NC - 1], x[kk]);
            pcol[nbuf][r] = xc;
            if (r == kc) {
              bool ok;
              dgi[kc] = recip_checked<T>(xc, ok);
              bad |= ok ? 0 : 1;
            }
          }
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c = cl + TPR * j;
      A[(size_t)r * mp + c] = x[j];
      a[r][c] = csel<T>(c == r, dgi[r], x[j]);  // U's diagonal by its reciprocal
    }
  }
  if (bad) atomicOr(flag, 1);
  __syncthreads();  // a[][] complete
  tri_inv_doubling<T, NT, true>(a);
  C *Dl = dinv + ((size_t)(blk * npan + p) * 2 + 0) * PB * PB;
  C *Du = Dl + PB * PB;
  const C zero = mk<T>((T)0, (T)0), one = mk<T>((T)1, (T)0);
  for (int e = tid; e < PB * PB; e += NT) {
    const int r = e / PB, c = e % PB;
    const C v = a[r][c];
    Dl[e] = csel<T>(r > c, v, csel<T>(r == c, one, zero));
    Du[e] = csel<T>(r <= c, v, zero);
  }
}

// Inverse of the upper triangle of a diagonal 64x64 tile of U (the Hessenberg route: U comes
// from the shifted Hessenberg LU), by the same recursive doubling as the LU route.
// Item = (instance, block, panel); 512 threads.
template <typename T>
__global__ __launch_bounds__(512) void k_hess_uinv(const InstDesc *__restrict__ Dd, ItemMap map,
                                                   int *__restrict__ flag) {
  typedef c_t<T> C;
  __shared__ C a[PB][PB + 1];
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int local = blockIdx.x - map.pre[q], tid = threadIdx.x;
  const int mp = d.mp, npan = d.npan, blk = local / npan, p = local % npan;
  const C *A = (const C *)d.K + (size_t)blk * mp * mp + (size_t)p * PB * mp + (size_t)p * PB;
  const C zero = mk<T>((T)0, (T)0);
  int bad = 0;
  for (int e = tid; e < PB * PB; e += 512) {
    const int r = e / PB, c = e % PB;
    C v = zero;
    if (c >= r) v = A[(size_t)r * mp + c];
    if (c == r) {
      bool ok;
      v = recip_checked<T>(v, ok);
      bad |= ok ? 0 : 1;
    }
    a[r][c] = v;
  }
  __syncthreads();
  tri_inv_doubling<T, 512, false>(a);
  C *Du = (C *)d.dinv + ((size_t)(blk * npan + p) * 2 + 1) * PB * PB;
  for (int e = tid; e < PB * PB; e += 512) {
    const int r = e / PB, c = e % PB;
    Du[e] = csel<T>(r <= c, a[r][c], zero);
  }
  if (bad) atomicOr(flag, 1);
}

template <typename T>
hipError_t launch_hess_uinv(const InstDesc *D, const ItemMap &map, int items, int *flag,
                            hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hess_uinv<T>, dim3(items), dim3(512), 0, st, D, map, flag);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// 64x64 complex tiles on MFMA: each of the 4 wavefronts owns a 32x32 quarter as 2x2 16x16
// sub-tiles of real and imaginary accumulators.
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

// C += acc for this wave's 32x32 part of a tile (layout as tile_load)
template <typename T>
__device__ __forceinline__ void tile_add_store(c_t<T> *__restrict__ Cp, int ldc,
                                               const acc_t<T> (&cre)[2][2], const acc_t<T> (&cim)[2][2]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        c_t<T> *e = Cp + (size_t)(r * 16 + mfma_row<T>(lk, v)) * ldc + c * 16 + li;
        const c_t<T> z = *e;
        *e = mk<T>(z.x + cre[r][c][v], z.y + cim[r][c][v]);
      }
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

// 64x64 complex GEMM on one workgroup (4 wavefronts, 32x32 each): (cre, cim) = (+/-) A B
// with A 64 x (nsl US), B (nsl US) x 64.  The K dimension streams through LDS in slices of US,
// double-buffered: while the MFMAs of slice s read LDS, the registers already hold slice
// s + 1 (loaded once per workgroup, 16-byte coalesced), stored to the other buffer before the
// slice's barrier.  Every read of A and B completes before the function returns.
// Complex products take three real MFMAs instead of four (the 3M form of a complex GEMM):
//   P1 = Ar Br,  P2 = Ai Bi,  P3 = (Ar + Ai)(Br + Bi),   Re = P1 - P2,  Im = P3 - P1 - P2,
// with three accumulators; the operand sums cost two additions per LDS read.
static constexpr int US = 8;

template <typename T>
struct GemmLds {
  c_t<T> As[2][PB][US + 1];  // A slice: 64 rows x US
  c_t<T> Bs[2][US][PB + 1];  // B slice: US x 64 columns
};

// Load of a complex value through a global-address-space pointer (a global_load, counted in
// vmcnt only; a load through a generic pointer is a flat load, counted in lgkmcnt as well).
template <typename T>
__device__ __forceinline__ c_t<T> ld_global(const c_t<T> *p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  typedef __attribute__((address_space(1))) const v2 gv2;
  const v2 v = *(gv2 *)p;
  return mk<T>(v.x, v.y);
}

// Output layout of gemm64_lds: wave w holds the 16x16 sub-blocks (r, c), r, c < 2, at rows
// gemm_row0(w, r) and columns gemm_col0(w, c).  TRI = 0: the wave's 32x32 quadrant.  With a
// triangular operand the sub-blocks need different K ranges (16-wide group g: 2g + 2 of the
// 8 slices), so each wave takes the groups {0, 3} or {1, 2} of the triangular side, 10 of 16
// slice-groups per wave: TRI = 1, B upper triangular (column groups); TRI = 2, A lower
// triangular (row groups).
__device__ __forceinline__ int tri_pair(int h, int i) { return h == 0 ? 3 * i : 1 + i; }
template <int TRI>
__device__ __forceinline__ int gemm_row0(int wave, int r) {
  return TRI == 2 ? 16 * tri_pair(wave >> 1, r) : (wave >> 1) * 32 + 16 * r;
}
template <int TRI>
__device__ __forceinline__ int gemm_col0(int wave, int c) {
  return TRI == 1 ? 16 * tri_pair(wave & 1, c) : (wave & 1) * 32 + 16 * c;
}

template <typename T, bool NEG, int TRI = 0>
__device__ __forceinline__ void gemm64_lds(const c_t<T> *__restrict__ A, int lda,
                                           const c_t<T> *__restrict__ B, int ldb, int nsl,
                                           GemmLds<T> &sm, acc_t<T> (&cre)[2][2],
                                           acc_t<T> (&cim)[2][2]) {
  typedef c_t<T> C;
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  // (a triangular operand skips MFMAs per wave: the wave index is made scalar so that the
  // tests are scalar branches)
  const int wave = TRI ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  int row0[2], col0[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    row0[i] = gemm_row0<TRI>(wave, i);
    col0[i] = gemm_col0<TRI>(wave, i);
  }
  // staging: A slice thread -> row tid / 4, columns 2 (tid % 4) + {0, 1};
  //          B slice thread -> row tid / 32, columns 2 (tid % 32) + {0, 1}
  const int ar = tid >> 2, ac = (tid & 3) * 2, br = tid >> 5, bc = (tid & 31) * 2;
  const C *Ap = A + (size_t)ar * lda + ac;
  const C *Bp = B + (size_t)br * ldb + bc;
  acc_t<T> p1[2][2], p2[2][2], p3[2][2];
  tile_zero<T>(p1, p2);
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) p3[r][c][v] = (T)0;
  // the slices are staged with global (not flat) loads: a flat load also counts in lgkmcnt, so
  // the wait for a slice's first LDS read would wait for the next slice's loads as well
  C ra0 = ld_global<T>(Ap), ra1 = ld_global<T>(Ap + 1);  // slice 0
  C rb0 = ld_global<T>(Bp), rb1 = ld_global<T>(Bp + 1);
  sm.As[0][ar][ac] = ra0;
  sm.As[0][ar][ac + 1] = ra1;
  sm.Bs[0][br][bc] = rb0;
  sm.Bs[0][br][bc + 1] = rb1;
  __syncthreads();
#pragma unroll 1
  for (int sl = 0; sl < nsl; ++sl) {
    const int buf = sl & 1;
    const bool more = sl + 1 < nsl;
    if (more) {
      const int k1 = (sl + 1) * US;
      ra0 = ld_global<T>(Ap + k1);
      ra1 = ld_global<T>(Ap + k1 + 1);
      rb0 = ld_global<T>(Bp + (size_t)k1 * ldb);
      rb1 = ld_global<T>(Bp + (size_t)k1 * ldb + 1);
    }
#pragma unroll
    for (int kk = 0; kk < US; kk += 4) {
      C a[2], b[2];
      if constexpr (TRI == 0) {
#pragma unroll
        for (int r = 0; r < 2; ++r) a[r] = sm.As[buf][wr + r * 16 + li][kk + lk];
#pragma unroll
        for (int c = 0; c < 2; ++c) b[c] = sm.Bs[buf][kk + lk][wc + c * 16 + li];
      } else {
#pragma unroll
        for (int r = 0; r < 2; ++r) a[r] = sm.As[buf][row0[r] + li][kk + lk];
#pragma unroll
        for (int c = 0; c < 2; ++c) b[c] = sm.Bs[buf][kk + lk][col0[c] + li];
      }
      T bs[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) bs[c] = b[c].x + b[c].y;
      const int k0 = sl * US + kk;  // this step's K rows k0 .. k0+3
      (void)k0;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const T ar_ = NEG ? -a[r].x : a[r].x, ai_ = NEG ? -a[r].y : a[r].y;
        const T as_ = ar_ + ai_;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          // a triangular operand is zero in the whole step for this sub-block: skip it
          if constexpr (TRI == 1)
            if (k0 >= col0[c] + 16) continue;
          if constexpr (TRI == 2)
            if (k0 >= row0[r] + 16) continue;
          p1[r][c] = mfma16(ar_, b[c].x, p1[r][c]);
          p2[r][c] = mfma16(ai_, b[c].y, p2[r][c]);
          p3[r][c] = mfma16(as_, bs[c], p3[r][c]);
        }
      }
    }
    if (more) {
      sm.As[buf ^ 1][ar][ac] = ra0;
      sm.As[buf ^ 1][ar][ac + 1] = ra1;
      sm.Bs[buf ^ 1][br][bc] = rb0;
      sm.Bs[buf ^ 1][br][bc + 1] = rb1;
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        cre[r][c][v] = p1[r][c][v] - p2[r][c][v];
        cim[r][c][v] = p3[r][c][v] - p1[r][c][v] - p2[r][c][v];
      }
}

// Panel.  Item = (instance, block, t): t < nrem -> L21 tile t = A21_t U11^{-1};
// else U12 tile t-nrem = L11^{-1} A12_t.  In place: every read of the tile completes inside
// gemm64_lds before the result is stored.
template <typename T>
__global__ __launch_bounds__(256, 3) void k_lu_panel(const InstDesc *__restrict__ Dd, ItemMap map,
                                                     int p) {
  typedef c_t<T> C;
  __shared__ GemmLds<T> sm;
  const int item = xcd_item(blockIdx.x, gridDim.x);  // the tiles of a block share an L2
  const int q = item_slot(map, item);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int mp = d.mp, npan = d.npan, nrem = npan - p - 1;
  const int local = item - map.pre[q];
  const int blk = local / (2 * nrem), t = local % (2 * nrem);
  C *Kb = (C *)d.K + (size_t)blk * mp * mp;
  const int wave = threadIdx.x >> 6;
  acc_t<T> cre[2][2], cim[2][2];
  const C *Dl = (const C *)d.dinv + ((size_t)(blk * npan + p) * 2 + 0) * PB * PB;
  const C *Du = Dl + PB * PB;
  C *Ct;
  int row0[2], col0[2];
  if (t < nrem) {
    Ct = Kb + (size_t)(p + 1 + t) * PB * mp + (size_t)p * PB;
    gemm64_lds<T, false, 1>(Ct, mp, Du, PB, PB / US, sm, cre, cim);
    for (int i = 0; i < 2; ++i) {
      row0[i] = gemm_row0<1>(wave, i);
      col0[i] = gemm_col0<1>(wave, i);
    }
  } else {
    Ct = Kb + (size_t)p * PB * mp + (size_t)(p + 1 + t - nrem) * PB;
    gemm64_lds<T, false, 2>(Dl, PB, Ct, mp, PB / US, sm, cre, cim);
    for (int i = 0; i < 2; ++i) {
      row0[i] = gemm_row0<2>(wave, i);
      col0[i] = gemm_col0<2>(wave, i);
    }
  }
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Ct[(size_t)(row0[r] + mfma_row<T>(lk, v)) * mp + col0[c] + li] = mk<T>(cre[r][c][v], cim[r][c][v]);
}

// Trailing updates, in pairs of panel steps (p, p+1) so that the trailing matrix is read and
// written once per two steps.  Tiles are indexed (ti, tj) from panel p + 1, nrem = npan - p - 1.
//   mode 1 (band of step p): the tiles step p + 1 needs, its row and column (ti == 0 or
//          tj == 0): A[ti][tj] -= L[ti][p] U[p][tj]                 (2 nrem - 1 tiles per block)
//   mode 2 (rest of the pair): ti, tj >= 1:
//          A[ti][tj] -= L[ti][p] U[p][tj] + L[ti][p+1] U[p+1][tj]    ((nrem - 1)^2 tiles, K = 128)
//   mode 0 (single step p, no pairing): every tile, K = 64         (nrem^2 tiles)
__device__ __forceinline__ int update_tiles(int mode, int nrem) {
  return mode == 0 ? nrem * nrem : mode == 1 ? 2 * nrem - 1 : (nrem - 1) * (nrem - 1);
}

template <typename T>
__global__ __launch_bounds__(256, 3) void k_lu_update(const InstDesc *__restrict__ Dd, ItemMap map,
                                                      int p, int mode) {
  typedef c_t<T> C;
  __shared__ GemmLds<T> sm;
  const int item = xcd_item(blockIdx.x, gridDim.x);  // the tiles of a block share an L2
  const int q = item_slot(map, item);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int mp = d.mp, npan = d.npan, nrem = npan - p - 1;
  const int local = item - map.pre[q];
  const int per = update_tiles(mode, nrem);
  const int blk = local / per, t = local % per;
  int ti, tj;
  if (mode == 1) {
    ti = t < nrem ? 0 : t - nrem + 1;
    tj = t < nrem ? t : 0;
  } else if (mode == 2) {
    ti = 1 + t / (nrem - 1);
    tj = 1 + t % (nrem - 1);
  } else {
    ti = t / nrem;
    tj = t % nrem;
  }
  C *Kb = (C *)d.K + (size_t)blk * mp * mp;
  const int wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  C *Ct = Kb + (size_t)(p + 1 + ti) * PB * mp + (size_t)(p + 1 + tj) * PB + (size_t)wr * mp + wc;
  const C *A = Kb + (size_t)(p + 1 + ti) * PB * mp + (size_t)p * PB;  // 64 x K, row stride mp
  const C *B = Kb + (size_t)p * PB * mp + (size_t)(p + 1 + tj) * PB;  // K x 64, row stride mp
  // acc = -A B; C is added at the end (keeps the C tile out of the loop's registers)
  acc_t<T> cre[2][2], cim[2][2];
  gemm64_lds<T, true>(A, mp, B, mp, (mode == 2 ? 2 * PB : PB) / US, sm, cre, cim);
  if (mode == 2 && p == 0) {  // first touch of these tiles: C is formed here, not read
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int i0 = (p + 1 + ti) * PB + wr, j0 = (p + 1 + tj) * PB + wc;
    const EntryGen e = entry_gen(d, blk);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + r * 16 + mfma_row<T>(lk, v), j = j0 + c * 16 + li;
          const C z = block_entry<T>(e, i, j, j_entry(e, i, j));
          cre[r][c][v] += z.x;
          cim[r][c][v] += z.y;
        }
    tile_store<T>(Ct, mp, cre, cim);
  } else {
    tile_add_store<T>(Ct, mp, cre, cim);
  }
}

// ------------------------------------------------------------------------------------
// Block solves K_k w = v in place on Vts[k] (FP64 vectors, factors of type T): per 64-row
// panel an off-diagonal GEMV streamed from HBM, then the 64x64 inverse of the diagonal
// triangle (dinv).
//
// Several workgroups per block (cooperative launch, all workgroups
// co-resident).  Item (k, w), w < W, owns the 64-row panels P = w, w+W, ... of block k in
// both sweeps.  Panel P of the forward sweep needs y_Q for every Q < P: the owner streams
// L[P][Q] as soon as y_Q is published (flag[k][Q][0] == epoch), so the bulk of the bytes
// is read in parallel and only the last 64x64 chunk plus the diagonal inverse sit on the
// dependency chain.  The backward sweep mirrors it with U and flag[k][Q][1].
//
// Coherence across the XCDs' separate L2 caches: the published pieces y_Q and the flags
// are written and read with relaxed agent-scope atomics (sc1: write-through / re-fetch
// at the coherence point); the producer waits for its stores before raising the flag.
// This avoids agent-scope fences, which write back or invalidate a whole L2.
// Every wait is bounded: after TS_SPIN_MAX polls, or once any workgroup has raised the
// error flag, the workgroup sets the flag and returns, so the grid always drains.
static constexpr int TS_SPIN_MAX = 1 << 18;

__device__ __forceinline__ void st_coh(double2 *p, double2 v) {
  unsigned long long *q = reinterpret_cast<unsigned long long *>(p);
  __hip_atomic_store(q, (unsigned long long)__double_as_longlong(v.x), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, (unsigned long long)__double_as_longlong(v.y), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double2 ld_coh(const double2 *p) {
  const unsigned long long *q = reinterpret_cast<const unsigned long long *>(p);
  const unsigned long long a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_double2(__longlong_as_double((long long)a), __longlong_as_double((long long)b));
}

__device__ __forceinline__ void ts_publish(unsigned long long *flag, unsigned long long epoch) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's coherent stores have completed
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum over the 16 lanes that share lane/16 (xor 1, 2, 4, 8 stay inside the group).
__device__ __forceinline__ double2 sum16(double2 v) {
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

// This wave's part of a 64x64 chunk: 16 rows (4 groups of 4, row = base + 4g + lane/16) by
// 64 columns.  Lane column set: FP64, col = 16j + lane%16 (j < 4, one complex per load);
// FP32, col = 32(j/2) + 2(lane%16) + j%2 (two adjacent complex values per 16-byte load).
// chunk_col gives the column of register j; the caller supplies x[j] = x[chunk_col(j)].
template <typename T>
__device__ __forceinline__ int chunk_col(int j, int cs) {
  return sizeof(T) == 8 ? 16 * j + cs : 32 * (j >> 1) + 2 * cs + (j & 1);
}

template <typename T>
__device__ __forceinline__ void chunk_load(const c_t<T> *__restrict__ M, size_t ld,
                                           c_t<T> (&a)[4][4]) {
  const int lane = threadIdx.x & 63, rs = lane >> 4, cs = lane & 15;
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int j = 0; j < 4; ++j) a[g][j] = M[(size_t)(4 * g + rs) * ld + 16 * j + cs];
  } else {
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float4 v = *reinterpret_cast<const float4 *>(M + (size_t)(4 * g + rs) * ld + 32 * h + 2 * cs);
        a[g][2 * h] = mk<T>(v.x, v.y);
        a[g][2 * h + 1] = mk<T>(v.z, v.w);
      }
  }
}

// acc[g] += a[g][:] * x; x[j] is the value at column chunk_col(j).
template <typename T>
__device__ __forceinline__ void chunk_fma(const c_t<T> (&a)[4][4], const double2 (&x)[4],
                                          double2 (&acc)[4]) {
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[g] = cfma(widen(a[g][j]), x[j], acc[g]);
}

// FP64 chunk_load restricted to the column groups [glo, ghi] (register j of a lane holds a
// column of group j, 16 columns each): a triangular 64x64 tile is zero outside the groups that
// meet this wave's 16 rows, so those are not loaded and their registers hold zero.
template <typename T>
__device__ __forceinline__ void chunk_load_groups(const c_t<T> *__restrict__ M, size_t ld,
                                                  c_t<T> (&a)[4][4], int glo, int ghi) {
  static_assert(sizeof(T) == 8, "FP64 layout");
  const int lane = threadIdx.x & 63, rs = lane >> 4, cs = lane & 15;
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      a[g][j] = (j >= glo && j <= ghi) ? M[(size_t)(4 * g + rs) * ld + 16 * j + cs] : mk<T>(0.0, 0.0);
}

// 16-column groups of a 64x64 diagonal inverse that can be nonzero in rows r16 .. r16+15: the
// unit-lower inverse (forward sweep) has columns <= row, the upper one (backward) >= row.
__device__ __forceinline__ void tri_groups(int sweep, int r16, int &glo, int &ghi) {
  glo = sweep == 0 ? 0 : r16 / 16;
  ghi = sweep == 0 ? r16 / 16 : 3;
}

// Flags are raised in sweep order (each panel depends on the previous one), so the chunks
// t, t+1, ... of a sweep that are ready form a prefix.  Waits for chunk t, then counts with one
// probe per lane how many of the following chunks are ready as well; returns the first chunk
// not known ready (> t), or -1 if the wait was abandoned.  Uniform across the workgroup;
// *sh is a workgroup-shared slot (alternate two slots between consecutive calls).
__device__ __forceinline__ int ts_ready(const unsigned long long *fl, int sweep, int npan, int t,
                                        int nq, unsigned long long epoch, int *err, int *sh) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    auto flag = [&](int tt) -> const unsigned long long * {
      const int Q = sweep == 0 ? tt : npan - 1 - tt;
      return &fl[Q * 2 + sweep];
    };
    int ok = 1;
    if (lane == 0 && __hip_atomic_load(flag(t), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
      for (int it = 0;; ++it) {
        __builtin_amdgcn_s_sleep(1);
        if (__hip_atomic_load(flag(t), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) break;
        if (it > TS_SPIN_MAX || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          atomicOr(err, 1);
          ok = 0;
          break;
        }
      }
    }
    ok = __shfl(ok, 0, 64);
    const int tt = t + 1 + lane;
    const bool r = tt < nq &&
                   __hip_atomic_load(flag(tt < nq ? tt : t), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch;
    const unsigned long long m = __ballot(r);  // bit 63 is clear: nq - t - 1 < 64
    if (lane == 0) *sh = ok ? t + 1 + (__ffsll((long long)~m) - 1) : -1;
  }
  __syncthreads();
  return *sh;
}

// Waits until *flag holds the epoch (thread 0 polls; bounded like ts_ready); uniform result.
__device__ __forceinline__ bool ts_wait(const unsigned long long *flag, unsigned long long epoch,
                                        int *err, int *sh) {
  if (threadIdx.x == 0) {
    int ok = 1;
    if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
      for (int it = 0;; ++it) {
        __builtin_amdgcn_s_sleep(1);
        if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) break;
        if (it > TS_SPIN_MAX || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          atomicOr(err, 1);
          ok = 0;
          break;
        }
      }
    }
    *sh = ok;
  }
  __syncthreads();
  return *sh != 0;
}

// One 64-row panel P of block k in one sweep: stream the off-diagonal chunks as their pieces
// are published, subtract, multiply by the diagonal inverse, publish.  need_fwd (backward
// sweep, panels handed out dynamically): the forward result of this panel may come from
// another workgroup, so its flag is awaited before it is read.  Returns false if a wait was
// abandoned.  Every thread of the workgroup calls it.  SOLO: the workgroup owns the whole
// block, so every piece it reads was stored by itself before a barrier: no flag is read or
// raised (the arithmetic is the same, so the result is the same to the bit).
template <typename T, bool SOLO = false>
__device__ __forceinline__ bool trsv_panel(const InstDesc &d, int k, int P, int sweep,
                                           bool need_fwd, unsigned long long epoch, int *err,
                                           int *ready_slot, int &calls, double2 *tmp) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, rs = lane >> 4, cs = lane & 15;
  const int r16 = wave * 16;  // this wave's first row inside the panel
  const int mp = d.mp, npan = d.npan;
  const c_t<T> *dinv = (const c_t<T> *)d.dinv;
  const c_t<T> *A = (const c_t<T> *)d.K + (size_t)k * mp * mp;
  double2 *v = d.Vts + (size_t)k * mp;
  unsigned long long *fl = d.tsflags + (size_t)k * npan * 2;
  const int p0 = P * PB;
  const c_t<T> *Di = dinv + ((size_t)(k * npan + P) * 2 + sweep) * PB * PB;
  // FP32: touch every 128-byte line of the diagonal inverse now, so that its read after
  // the off-diagonal GEMV (on the dependency chain of the sweep) hits L2; the touched
  // values enter the result as x * 0 (they are finite), which keeps the loads.  (For FP64
  // factors the extra loads cost more than they save.)
  constexpr int TL = sizeof(T) == 4 ? 1 : 0;  // lines per thread
  double touch[TL > 0 ? TL : 1];
#pragma unroll
  for (int u = 0; u < TL; ++u)
    touch[u] = (double)reinterpret_cast<const T *>(Di)[(size_t)(threadIdx.x * TL + u) * (128 / sizeof(T))];
  double2 acc[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) acc[g] = make_double2(0.0, 0.0);
  // SOLO: the diagonal inverse depends on nothing, so its loads are issued first and fly
  // while the panel's right-hand side is formed
  int glo = 0, ghi = 3;
  if constexpr (sizeof(T) == 8) tri_groups(sweep, __builtin_amdgcn_readfirstlane(r16), glo, ghi);
  c_t<T> ad[4][4];
  if (SOLO) {
    if constexpr (sizeof(T) == 8)
      chunk_load_groups<T>(Di + (size_t)r16 * PB, PB, ad, glo, ghi);
    else
      chunk_load<T>(Di + (size_t)r16 * PB, PB, ad);
  }
  const int nq = sweep == 0 ? P : npan - 1 - P;
  int have = 0;  // chunks t < have are known to be published
  for (int t = 0; t < nq; ++t) {
    const int Q = sweep == 0 ? t : npan - 1 - t;
    // FP32 chunks are loaded before a possible wait, so the loads are in flight meanwhile
    // (FP64 chunks would need twice the registers and halve the co-resident workgroups)
    constexpr bool early = sizeof(T) == 4;
    c_t<T> a[4][4];
    if (early) chunk_load<T>(A + (size_t)(p0 + r16) * mp + (size_t)Q * PB, mp, a);
    if (!SOLO && t >= have) {
      have = ts_ready(fl, sweep, npan, t, nq, epoch, err, &ready_slot[calls++ & 1]);
      if (have < 0) return false;
    }
    if (!early) chunk_load<T>(A + (size_t)(p0 + r16) * mp + (size_t)Q * PB, mp, a);
    // the published piece y_Q: one coherent load per lane (entry `lane`), then each lane
    // takes its four entries from the wavefront by shuffles
    const double2 xl = ld_coh(&v[Q * PB + lane]);
    double2 x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int src = chunk_col<T>(j, cs);
      x[j] = make_double2(__shfl(xl.x, src, 64), __shfl(xl.y, src, 64));
    }
    chunk_fma<T>(a, x, acc);
  }
  if (!SOLO && need_fwd && !ts_wait(&fl[P * 2 + 0], epoch, err, &ready_slot[calls++ & 1])) return false;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    acc[g] = sum16(acc[g]);
    if (cs == 0) {
      const int rr = r16 + 4 * g + rs;
      tmp[rr] = csub(ld_coh(&v[p0 + rr]), acc[g]);
    }
  }
  __syncthreads();
  double2 x[4], b[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] = tmp[chunk_col<T>(j, cs)];
#pragma unroll
  for (int g = 0; g < 4; ++g) b[g] = make_double2(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < TL; ++u) b[0].x = fma(touch[u], 0.0, b[0].x);
  if (SOLO) {
    chunk_fma<T>(ad, x, b);
  } else {
    // FP64: only the column groups of the triangular inverse that meet this wave's rows are
    // read (5/8 of the tile on average).  (FP32 reads the whole tile: with its touched lines in
    // L2 the conditional loads cost more than they save.)
    c_t<T> a[4][4];
    if constexpr (sizeof(T) == 8)
      chunk_load_groups<T>(Di + (size_t)r16 * PB, PB, a, glo, ghi);
    else
      chunk_load<T>(Di + (size_t)r16 * PB, PB, a);
    chunk_fma<T>(a, x, b);
  }
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    b[g] = sum16(b[g]);
    if (cs == 0) st_coh(&v[p0 + r16 + 4 * g + rs], b[g]);
  }
  if (SOLO) {
    __builtin_amdgcn_s_waitcnt(0);  // the next panel reads these entries
    __syncthreads();
  } else {
    ts_publish(&fl[P * 2 + sweep], epoch);
  }
  return true;
}

// One workgroup per block, no flags (an ordinary launch): the panels of both sweeps (the U
// sweep only for first_sweep = 1) in order, by the cooperative kernel's panel code, so the
// result equals its result for any W.  The item map counts nb W items per instance; the
// workgroup of item k W solves block k, the others return.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_trsv(const InstDesc *__restrict__ Dd, ItemMap map,
                                              int first_sweep) {
  __shared__ double2 tmp[PB];
  __shared__ int ready_slot[2];
  int calls = 0;
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int local = blockIdx.x - map.pre[q];
  if (local % d.W != 0) return;
  const int k = local / d.W, npan = d.npan;
  for (int sweep = first_sweep; sweep < 2; ++sweep)
    for (int t = 0; t < npan; ++t)
      trsv_panel<T, true>(d, k, sweep == 0 ? t : npan - 1 - t, sweep, false, 0ull, nullptr, ready_slot,
                          calls, tmp);
}

// Two ways of handing out the panels.  Static (npan_u = 0): item (k, w), w < W, owns the panels
// P = w, w+W, ... of block k.  Dynamic (all instances of the plan have npan_u panels): each
// workgroup claims the next unit from a counter (reset by the time FFT that draws the epoch):
// units run through the forward sweep level by level (panel 0 of every block, then panel 1,
// ...), then the backward sweep from the last panel down, so a unit only waits on units
// claimed before it, all held by running workgroups; a workgroup that is slowed (a CU shared
// by more workgroups) simply claims fewer units, and the grid need not be a multiple of the
// block count.
template <typename T>
__global__ __launch_bounds__(256, 4) void k_trsv_coop(const InstDesc *__restrict__ Dd, ItemMap map,
                                                   int items,
                                                   const unsigned long long *__restrict__ epoch_p,
                                                   int *__restrict__ err, int first_sweep,
                                                   ItemMap blkmap, int nblk, int npan_u) {
  __shared__ double2 tmp[PB];
  __shared__ int ready_slot[2];
  __shared__ int claim;
  int calls = 0;
  const unsigned long long epoch =
      __hip_atomic_load(epoch_p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (npan_u > 0) {
    unsigned *ctr = reinterpret_cast<unsigned *>(const_cast<unsigned long long *>(epoch_p + 1));
    const int U = npan_u * nblk;  // units per sweep
    for (;;) {
      if (threadIdx.x == 0)
        claim = (int)__hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      const int u = claim + first_sweep * U;
      __syncthreads();
      if (u >= 2 * U) break;
      const int sweep = u / U, r = u % U, lvl = r / nblk, b = r % nblk;
      const int q = item_slot(blkmap, b);
      if (item_gated(blkmap, q)) continue;
      const InstDesc &d = Dd[blkmap.ids[q]];
      const int P = sweep == 0 ? lvl : npan_u - 1 - lvl;
      const bool need_fwd = sweep == 1 && first_sweep == 0;
      if (!trsv_panel<T>(d, b - blkmap.pre[q], P, sweep, need_fwd, epoch, err, ready_slot, calls,
                         tmp))
        return;
    }
    return;
  }
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int q = item_slot(map, item);
    if (item_gated(map, q)) continue;
    const InstDesc &d = Dd[map.ids[q]];
    const int local = item - map.pre[q];
    const int npan = d.npan, W = d.W;
    const int k = local / W, w = local % W;
    for (int sweep = first_sweep; sweep < 2; ++sweep) {
      const int Pfirst = sweep == 0 ? w : w + ((npan - 1 - w) / W) * W;
      for (int P = Pfirst; P >= 0 && P < npan; P += sweep == 0 ? W : -W)
        if (!trsv_panel<T>(d, k, P, sweep, false, epoch, err, ready_slot, calls, tmp)) return;
    }
  }
}

// ------------------------------------------------------------------------------------
// The band route (k_band.hip reduces J to H of lower bandwidth 64, J = Q H Q^T): LU with
// partial pivoting of C_k = lambda_k I - tau mu_k H, one 64-column panel per step.  At step j
// only block rows j and j + 1 hold entries in block column j (block row j carries the updates
// of step j - 1; block row j + 1 is still C_k's own and is formed from H when first read), so
// the pivots are chosen among those 128 rows and the step changes only those two block rows:
//   k_band_lu_panel  P_j [C_j; C_{j+1}][:, block j] = [L11; L21] U11 in LDS; L11 \ U11 into K
//                    block (j, j), M21 = L21 L11^{-1} into K block (j + 1, j), the row order
//                    after the exchanges into the permutation array (row i of the window came
//                    from row perm[i]), the inverses of L11 and U11 into dinv[..][0] and [1];
//   k_band_lu_rows   per 64-column tile of the trailing width, from the window's reordered top
//                    rows W: block row j + 1 <- bottom - M21 W, then block row j <- L11^{-1} W
//                    (= U12); bottom - L21 U12 = bottom - M21 W, so neither waits for the other;
//   k_band_lsolve    per step, from the reordered window y: y_top <- L11^{-1} y_top (final) and
//                    y_bottom <- y_bottom - M21 y_top (U^{-1} is the backward sweep of
//                    k_trsv_coop).
// Pivot: the largest |re| + |im| of the column (the lowest row on ties).
template <typename T>
__device__ __forceinline__ c_t<T> band_entry(const double *__restrict__ H, int mp, int m, double2 lam,
                                             double2 mu, double tau, int r, int c) {
  if (r >= m || c >= m) return mk<T>((T)(r == c ? 1.0 : 0.0), (T)0);
  const double h = H[(size_t)r * mp + c];
  double re = -tau * mu.x * h, im = -tau * mu.y * h;
  if (r == c) {
    re += lam.x;
    im += lam.y;
  }
  return mk<T>((T)re, (T)im);
}

template <typename T>
struct PanelLds {
  c_t<T> a[2 * PB][PB + 1];
  int perm[2 * PB];
  T wmax[2];
  int widx[2];
  int spiv;
  c_t<T> srec;
};

template <typename T, int NT>
__device__ __forceinline__ void band_lu_panel_body(const InstDesc *__restrict__ Dd, const ItemMap &map, int item,
                                                   int j, int *__restrict__ flag, PanelLds<T> &sp) {
  typedef c_t<T> C;
  C(*a)[PB + 1] = sp.a;
  int *perm = sp.perm;
  T *wmax = sp.wmax;
  int *widx = sp.widx;
  int &spiv = sp.spiv;
  C &srec = sp.srec;
  const int q = item_slot(map, item);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int blk = item - map.pre[q], tid = threadIdx.x;
  const int mp = d.mp, npan = d.npan, m = d.m, r0 = j * PB;
  const int nr = j + 1 < npan ? 2 * PB : PB;
  C *K = (C *)d.K + (size_t)blk * mp * mp;
  const double2 lam = d.lam[blk], mu = d.mu[blk];
  for (int e = tid; e < nr * PB; e += NT) {
    const int r = e / PB, c = e % PB;
    a[r][c] = (r < PB && j > 0) ? K[(size_t)(r0 + r) * mp + r0 + c]
                                : band_entry<T>(d.hH, mp, m, lam, mu, d.tau, r0 + r, r0 + c);
  }
  if (tid < 2 * PB) perm[tid] = tid;
  __syncthreads();
  int bad = 0;
  for (int k = 0; k < PB; ++k) {
    if (tid < 2 * PB) {  // waves 0 and 1: the candidates' magnitudes, arg-max per wave
      T v = (T)-1;
      if (tid >= k && tid < nr) v = fabs(a[tid][k].x) + fabs(a[tid][k].y);
      int ix = tid;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const T ov = __shfl_xor(v, o, 64);
        const int oi = __shfl_xor(ix, o, 64);
        if (ov > v || (ov == v && oi < ix)) {
          v = ov;
          ix = oi;
        }
      }
      if ((tid & 63) == 0) {
        wmax[tid >> 6] = v;
        widx[tid >> 6] = ix;
      }
    }
    __syncthreads();
    if (tid == 0) {
      const int p = wmax[1] > wmax[0] ? widx[1] : widx[0];
      spiv = p;
      const int t0 = perm[k];
      perm[k] = perm[p];
      perm[p] = t0;
    }
    __syncthreads();
    const int p = spiv;
    if (p != k && tid < PB) {
      const C t0 = a[k][tid];
      a[k][tid] = a[p][tid];
      a[p][tid] = t0;
    }
    __syncthreads();
    if (tid == 0) {
      bool ok;
      srec = recip_checked<T>(a[k][k], ok);
      bad |= ok ? 0 : 1;
    }
    __syncthreads();
    const C rp = srec;
    if (tid > k && tid < nr) a[tid][k] = tmul<T>(a[tid][k], rp);
    __syncthreads();
    const int rows = nr - k - 1, cols = PB - k - 1;
    for (int e = tid; e < rows * cols; e += NT) {
      const int r = k + 1 + e / cols, c = k + 1 + e % cols;
      a[r][c] = tsub<T>(a[r][c], tmul<T>(a[r][k], a[k][c]));
    }
    __syncthreads();
  }
  for (int e = tid; e < PB * PB; e += NT) {
    const int r = e / PB, c = e % PB;
    K[(size_t)(r0 + r) * mp + r0 + c] = a[r][c];
  }
  if (tid < nr) d.hpiv[((size_t)blk * npan + j) * 2 * PB + tid] = perm[tid];
  if (bad) atomicOr(flag, 1);
  __syncthreads();
  if (tid < PB) {
    bool ok;
    a[tid][tid] = recip_checked<T>(a[tid][tid], ok);
  }
  __syncthreads();
  tri_inv_doubling<T, NT, true>(a);
  C *Dl = (C *)d.dinv + ((size_t)(blk * npan + j) * 2 + 0) * PB * PB;
  C *Du = Dl + PB * PB;
  const C zero = mk<T>((T)0, (T)0), one = mk<T>((T)1, (T)0);
  for (int e = tid; e < PB * PB; e += NT) {
    const int r = e / PB, c = e % PB;
    const C v = a[r][c];
    Dl[e] = csel<T>(r > c, v, csel<T>(r == c, one, zero));
    Du[e] = csel<T>(r <= c, v, zero);
  }
  // M21 = L21 L11^{-1} into K block (j + 1, j): the bottom rows then need only the window's
  // top rows before their update (bottom - L21 U12 = bottom - M21 top), so the two block rows
  // of a step are computed independently
  if (nr == 2 * PB) {
    for (int e = tid; e < PB * PB; e += NT) {
      const int r = e / PB, c = e % PB;
      C acc = a[PB + r][c];  // L11^{-1}[c][c] = 1
      for (int k = c + 1; k < PB; ++k) acc = tfma<T>(a[PB + r][k], a[k][c], acc);
      K[(size_t)(r0 + PB + r) * mp + r0 + c] = acc;
    }
  }
}

// Rows of the step-j window [C_j; C_{j+1}] (block rows j and j + 1, 128 rows) after the row
// exchanges: row i is row perm[i] of the window, whose top half is K's block row j (j > 0; the
// entries of step j - 1's update) and whose bottom half is still C_k's own, formed from H.
template <typename T>
struct BandWin {
  const c_t<T> *Ktop;  // K block row j (row stride mp)
  const double *H;
  const int *perm;  // the window's row order, staged in LDS
  double2 lam, mu;
  double tau;
  int mp, m, r0;
  bool top_from_K;
  __device__ __forceinline__ c_t<T> get(int i, int c) const {
    const int sr = perm[i];
    return (sr < PB && top_from_K) ? Ktop[(size_t)sr * mp + c]
                                   : band_entry<T>(H, mp, m, lam, mu, tau, r0 + sr, c);
  }
};

// Item = (instance, block, tile t0 <= t < min(t1, npan - j - 1)): columns c0 = 64 (j + 1 + t) ..
// of the window.  Both products of the step share the window's reordered top rows W, gathered
// once into LDS slices: wavefronts 0-7 form block row j + 1 <- bottom - M21 W, wavefronts 8-15
// block row j <- L11^{-1} W = U12 (each a 32 x 16 part of its 64 x 64 tile, 3M complex MFMA
// products over 8-deep K slices, double-buffered in LDS, their loads issued two slices ahead).  The window's bottom rows are gathered into LDS with the first slices, so their
// latency overlaps the products; the new block row j + 1 is stored before a barrier after which
// block row j is overwritten, so every read of the window precedes the stores that replace it.
static constexpr int BR_NT = 1024;
template <typename T>
struct RowsLds {
  c_t<T> As[2][2][PB][US + 1];  // [product][buffer]: M21 (0), L11^{-1} (1) slices, 64 rows x US
  c_t<T> Bs[2][US][PB + 1];     // W slices: US x 64 columns
  c_t<T> Wb[PB][PB + 1];        // the window's reordered bottom rows, columns c0 .. c0 + 63
  int perm[2 * PB];             // the window's row order (row i came from row perm[i])
};

template <typename T>
__device__ __forceinline__ void band_lu_rows_body(const InstDesc *__restrict__ Dd, const ItemMap &map, int bid,
                                                  int nbid, int j, int t0, int t1, RowsLds<T> &sm) {
  typedef c_t<T> C;
  const int item = xcd_item(bid, nbid);  // the tiles of a block share an L2
  const int q = item_slot(map, item);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int mp = d.mp, npan = d.npan, nrem = npan - j - 1;
  const int ntile = (t1 < nrem ? t1 : nrem) - t0;
  const int local = item - map.pre[q];
  const int blk = local / ntile, tt = t0 + local % ntile;
  const int r0 = j * PB, c0 = (j + 1 + tt) * PB, tid = threadIdx.x;
  C *K = (C *)d.K + (size_t)blk * mp * mp;
  BandWin<T> win;
  win.Ktop = K + (size_t)r0 * mp;
  win.H = d.hH;
  win.perm = sm.perm;
  win.lam = d.lam[blk];
  win.mu = d.mu[blk];
  win.tau = d.tau;
  win.mp = mp;
  win.m = d.m;
  win.r0 = r0;
  win.top_from_K = j > 0;
  const int lane = tid & 63, li = lane & 15, lk = lane >> 4, wave = tid >> 6;
  const int prod = wave >> 3;  // 0: bottom (M21), 1: top (L11^{-1})
  const int pw = wave & 7, wr = (pw >> 2) * 32, wc = (pw & 3) * 16;
  // loaders: A slices, thread t: product t / 512, row (t % 512) / 8, column t % 8; W slice
  // (t < 512), row t / 64, column t % 64
  const int ap = tid >> 9, ar = (tid & 511) >> 3, ac = tid & 7, br = (tid & 511) >> 6, bc = tid & 63;
  const bool bl = tid < 512;
  const C *Ap = ap == 0 ? K + (size_t)(r0 + PB + ar) * mp + r0 + ac
                        : (const C *)d.dinv + ((size_t)(blk * npan + j) * 2 + 0) * PB * PB + (size_t)ar * PB + ac;
  // Slices in flight D ahead: the loads of slice sl + D are issued before slice sl is multiplied
  // and stored to LDS after it, so each has D slices' products to arrive; register slot s % (D + 1)
  // holds slice s.  FP64: D = 2.  FP32: D = 1, which keeps the kernel at 64 VGPRs with fewer
  // spills (two workgroups per CU).
  constexpr int nsl = PB / US, D = sizeof(T) == 8 ? 2 : 1, R = D + 1;
  static_assert(nsl >= D, "D slices are loaded before the loop");
  C qa[R], qb[R];
#pragma unroll
  for (int d = 0; d < D; ++d) qa[d] = ld_global<T>(Ap + d * US);
  // the window's row order into LDS first: every gather below then takes one global round trip
  if (tid < 2 * PB) sm.perm[tid] = d.hpiv[((size_t)blk * npan + j) * 2 * PB + tid];
  __syncthreads();
#pragma unroll
  for (int d = 0; d < D; ++d) qb[d] = bl ? win.get(d * US + br, c0 + bc) : mk<T>((T)0, (T)0);
  C wb[PB * PB / BR_NT];  // bottom rows: thread t takes rows t / 64 + 16 i, column t % 64
#pragma unroll
  for (int i = 0; i < PB * PB / BR_NT; ++i) wb[i] = win.get(PB + (tid >> 6) + 16 * i, c0 + (tid & 63));
  sm.As[ap][0][ar][ac] = qa[0];
  if (bl) sm.Bs[0][br][bc] = qb[0];
#pragma unroll
  for (int i = 0; i < PB * PB / BR_NT; ++i) sm.Wb[(tid >> 6) + 16 * i][tid & 63] = wb[i];
  __syncthreads();
  acc_t<T> p1[2], p2[2], p3[2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) p1[r][v] = p2[r][v] = p3[r][v] = (T)0;
#pragma unroll
  for (int sl = 0; sl < nsl; ++sl) {
    const int buf = sl & 1;
    if (sl + D < nsl) {
      const int k2 = (sl + D) * US;
      qa[(sl + D) % R] = ld_global<T>(Ap + k2);
      if (bl) qb[(sl + D) % R] = win.get(k2 + br, c0 + bc);
    }
#pragma unroll
    for (int kk = 0; kk < US; kk += 4) {
      const C b = sm.Bs[buf][kk + lk][wc + li];
      const T bs = b.x + b.y;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const C a = sm.As[prod][buf][wr + r * 16 + li][kk + lk];
        p1[r] = mfma16(a.x, b.x, p1[r]);
        p2[r] = mfma16(a.y, b.y, p2[r]);
        p3[r] = mfma16(a.x + a.y, bs, p3[r]);
      }
    }
    if (sl + 1 < nsl) {
      sm.As[ap][buf ^ 1][ar][ac] = qa[(sl + 1) % R];
      if (bl) sm.Bs[buf ^ 1][br][bc] = qb[(sl + 1) % R];
    }
    __syncthreads();
  }
  T cre[2][4], cim[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      cre[r][v] = p1[r][v] - p2[r][v];
      cim[r][v] = p3[r][v] - p1[r][v] - p2[r][v];
    }
  if (prod == 0) {  // block row j + 1 <- bottom - M21 W
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + r * 16 + mfma_row<T>(lk, v);
        const C z = sm.Wb[row][wc + li];
        K[(size_t)(r0 + PB + row) * mp + c0 + wc + li] = mk<T>(z.x - cre[r][v], z.y - cim[r][v]);
      }
  }
  __syncthreads();  // every read of the window (block row j included) is complete
  if (prod == 1) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + r * 16 + mfma_row<T>(lk, v);
        K[(size_t)(r0 + row) * mp + c0 + wc + li] = mk<T>(cre[r][v], cim[r][v]);
      }
  }
}

template <typename T>
__global__ __launch_bounds__(512) void k_band_lu_panel(const InstDesc *__restrict__ Dd, ItemMap map, int j,
                                                       int *__restrict__ flag) {
  __shared__ PanelLds<T> sp;
  band_lu_panel_body<T, 512>(Dd, map, blockIdx.x, j, flag, sp);
}

template <typename T>
__global__ __launch_bounds__(BR_NT) void k_band_lu_rows(const InstDesc *__restrict__ Dd, ItemMap map, int j, int t0,
                                                        int t1) {
  __shared__ RowsLds<T> sm;
  band_lu_rows_body<T>(Dd, map, blockIdx.x, gridDim.x, j, t0, t1, sm);
}

// Panel j + 1 and the row tiles t >= 1 of step j in one launch: the first npi workgroups take the
// panel (dispatched first, so it never waits for CUs behind the row tiles), the others the
// tiles.  The two touch disjoint parts of the factors (block column j + 1 against block columns
// >= j + 2), and the panel reads only what the first row tile of step j wrote before.
// FP32: 64 VGPRs (a few address spills) so that two 1024-thread workgroups share a CU (67 KB of
// LDS each), one's loads and stores overlapping the other's products: 288 to 271 us per step at
// 4095 x 256.  FP64 needs 122 VGPRs and 134 KB of LDS, one workgroup per CU either way.
template <typename T>
__global__ __launch_bounds__(BR_NT, sizeof(T) == 4 ? 8 : 1) void k_band_lu_step(const InstDesc *__restrict__ Dd, ItemMap pmap, int npi,
                                                        ItemMap rmap, int j, int *__restrict__ flag) {
  __shared__ union {
    PanelLds<T> p;
    RowsLds<T> r;
  } lds;
  if ((int)blockIdx.x < npi)
    band_lu_panel_body<T, BR_NT>(Dd, pmap, blockIdx.x, j + 1, flag, lds.p);
  else
    band_lu_rows_body<T>(Dd, rmap, blockIdx.x - npi, gridDim.x - npi, j, 1, 1 << 30, lds.r);
}

// One workgroup per block: the window [top; bottom] of step j (the top carried from step j-1,
// the bottom read from the vector), reordered; then top <- L11^{-1} top (final) and bottom <-
// bottom - M21 top (the next step's top), both from the reordered top.  Thread t: row t / 8,
// columns t % 8 + 8 c (c = 0 .. 7: each load instruction of a wavefront reads eight whole
// 128-byte lines, one per row, not 64 lines 16 bytes at a time).  What a step reads from memory does not depend on the solve (its
// entries of L11^{-1} and M21, its row order, the window's bottom rows of the vector, which only
// step j + 1 overwrites), so step j + 1's loads are issued before step j runs, into the other of
// two register sets: the steps then wait on barriers only, not on memory latency.
template <typename T>
struct LsolveRegs {
  c_t<T> li[8], mm[8];
  double2 vb;
  int pr;
};

template <typename T>
__global__ __launch_bounds__(512) void k_band_lsolve(const InstDesc *__restrict__ Dd, ItemMap map) {
  typedef c_t<T> C;
  __shared__ double2 ys[2 * PB];  // the window before the exchanges
  __shared__ double2 y[2 * PB];   // after them
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = Dd[map.ids[q]];
  const int blk = blockIdx.x - map.pre[q], tid = threadIdx.x;
  const int mp = d.mp, npan = d.npan;
  double2 *v = d.Vts + (size_t)blk * mp;
  const C *K = (const C *)d.K + (size_t)blk * mp * mp;
  const C *dinv = (const C *)d.dinv;
  const int *perm = d.hpiv + (size_t)blk * npan * 2 * PB;
  const int i = tid >> 3, qq = tid & 7;  // row i, columns qq + 8 c
  auto load = [&](int j, LsolveRegs<T> &R) {
    const int r0 = j * PB, nr = j + 1 < npan ? 2 * PB : PB;
    const C *Li = dinv + ((size_t)(blk * npan + j) * 2 + 0) * PB * PB + (size_t)i * PB + qq;
#pragma unroll
    for (int c = 0; c < 8; ++c) R.li[c] = gld(Li + 8 * c);
    if (nr == 2 * PB) {
      const C *M21 = K + (size_t)(r0 + PB + i) * mp + r0 + qq;
#pragma unroll
      for (int c = 0; c < 8; ++c) R.mm[c] = gld(M21 + 8 * c);
    } else {
#pragma unroll
      for (int c = 0; c < 8; ++c) R.mm[c] = mk<T>((T)0, (T)0);
    }
    if (tid < nr) R.pr = gld(perm + (size_t)j * 2 * PB + tid);
    if (tid >= PB && tid < nr) R.vb = gld(v + r0 + tid);
  };
  auto step = [&](int j, const LsolveRegs<T> &R) {
    const int r0 = j * PB, nr = j + 1 < npan ? 2 * PB : PB;
    if (tid >= PB && tid < nr) ys[tid] = R.vb;
    __syncthreads();
    if (tid < nr) y[tid] = ys[R.pr];
    __syncthreads();
    double2 s = make_double2(0.0, 0.0), t = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double2 yc = y[qq + 8 * c];
      s = cfma(widen(R.li[c]), yc, s);
      t = cfma(widen(R.mm[c]), yc, t);
    }
#pragma unroll
    for (int o = 1; o <= 4; o <<= 1) {
      s.x += __shfl_xor(s.x, o, 64);
      s.y += __shfl_xor(s.y, o, 64);
      t.x += __shfl_xor(t.x, o, 64);
      t.y += __shfl_xor(t.y, o, 64);
    }
    if (qq == 0) {
      gst(v + r0 + i, s);
      if (nr == 2 * PB) ys[i] = csub(y[PB + i], t);
    }
    __syncthreads();
  };
  LsolveRegs<T> ra, rb;
  if (tid < PB) ys[tid] = v[tid];
  load(0, ra);
  for (int j = 0; j < npan; j += 2) {
    if (j + 1 < npan) load(j + 1, rb);
    step(j, ra);
    if (j + 1 == npan) break;
    if (j + 2 < npan) load(j + 2, ra);
    step(j + 1, rb);
  }
}

// ------------------------------------------------------------------------------------
static constexpr int ASM_KCHUNK = 8;
int assemble_items(int mp, int nb) { return mp * ((nb + ASM_KCHUNK - 1) / ASM_KCHUNK); }
int assemble_lead() { return ASM_LEAD; }

template <typename T>
hipError_t launch_assemble(const InstDesc *D, const ItemMap &map, int items, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_assemble<T>, dim3(items), dim3(256), 0, st, D, map, ASM_KCHUNK);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lu_diag(const InstDesc *D, const ItemMap &map, int items, int p, int *flag,
                          hipStream_t st) {
  if (items <= 0) return hipSuccess;
  constexpr int NT = DiagThreads<T>::value;
  hipLaunchKernelGGL((k_lu_diag<T, NT>), dim3(items), dim3(NT), 0, st, D, map, p, flag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lu_panel(const InstDesc *D, const ItemMap &map, int items, int p,
                           hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lu_panel<T>, dim3(items), dim3(256), 0, st, D, map, p);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lu_update(const InstDesc *D, const ItemMap &map, int items, int p, int mode,
                            hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lu_update<T>, dim3(items), dim3(256), 0, st, D, map, p, mode);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_trsv(const InstDesc *D, const ItemMap &map, int items, int first_sweep,
                       hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsv<T>, dim3(items), dim3(256), 0, st, D, map, first_sweep);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_band_lu_panel(const InstDesc *D, const ItemMap &map, int items, int j, int *flag,
                                hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_band_lu_panel<T>, dim3(items), dim3(512), 0, st, D, map, j, flag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_band_lu_rows(const InstDesc *D, const ItemMap &map, int items, int j, int t0, int t1,
                               hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_band_lu_rows<T>, dim3(items), dim3(BR_NT), 0, st, D, map, j, t0, t1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_band_lu_step(const InstDesc *D, const ItemMap &pmap, int pitems, const ItemMap &rmap, int ritems,
                               int j, int *flag, hipStream_t st) {
  if (pitems + ritems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_band_lu_step<T>, dim3(pitems + ritems), dim3(BR_NT), 0, st, D, pmap, pitems, rmap, j, flag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_band_lsolve(const InstDesc *D, const ItemMap &map, int items, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_band_lsolve<T>, dim3(items), dim3(512), 0, st, D, map);
  return hipGetLastError();
}

static int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 0;
  }
  return cus;
}

template <typename T>
int trsv_coop_capacity() {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_trsv_coop<T>, 256, 0) != hipSuccess)
    return 0;
  return per * device_cus();
}

template <typename T>
hipError_t launch_trsv_coop(const InstDesc *D, const ItemMap &map, int items,
                            const unsigned long long *epoch, int *err, hipStream_t st,
                            int first_sweep, const ItemMap *blkmap, int nblk, int npan_u) {
  if (items <= 0) return hipSuccess;
  const int cap = trsv_coop_capacity<T>();
  if (cap <= 0) return hipErrorNotSupported;
  int grid = items < cap ? items : cap;
  ItemMap bm = map;
  if (blkmap && npan_u > 0 && nblk > 0) {
    // claimed units: any grid size works, so use whole multiples of the CU count (no CU gets
    // one workgroup more than the others)
    const int cus = device_cus();
    if (grid > cus) grid -= grid % cus;
    bm = *blkmap;
  } else {
    npan_u = 0;
    nblk = 0;
  }
  void *args[] = {(void *)&D,           (void *)&map,  (void *)&items, (void *)&epoch,
                  (void *)&err,         (void *)&first_sweep, (void *)&bm, (void *)&nblk,
                  (void *)&npan_u};
  return hipLaunchCooperativeKernel((const void *)k_trsv_coop<T>, dim3(grid), dim3(256), args, 0, st);
}

#define FDE_INST(T)                                                                              \
  template hipError_t launch_assemble<T>(const InstDesc *, const ItemMap &, int, hipStream_t);    \
  template hipError_t launch_lu_diag<T>(const InstDesc *, const ItemMap &, int, int, int *,        \
                                        hipStream_t);                                           \
  template hipError_t launch_lu_panel<T>(const InstDesc *, const ItemMap &, int, int, hipStream_t); \
  template hipError_t launch_lu_update<T>(const InstDesc *, const ItemMap &, int, int, int,        \
                                          hipStream_t);                                         \
  template hipError_t launch_trsv<T>(const InstDesc *, const ItemMap &, int, int, hipStream_t);    \
  template hipError_t launch_trsv_coop<T>(const InstDesc *, const ItemMap &, int,                 \
                                          const unsigned long long *, int *, hipStream_t, int,   \
                                          const ItemMap *, int, int);                             \
  template hipError_t launch_hess_uinv<T>(const InstDesc *, const ItemMap &, int, int *,          \
                                          hipStream_t);                                         \
  template hipError_t launch_band_lu_panel<T>(const InstDesc *, const ItemMap &, int, int, int *,  \
                                              hipStream_t);                                     \
  template hipError_t launch_band_lu_rows<T>(const InstDesc *, const ItemMap &, int, int, int, int, \
                                             hipStream_t);                                      \
  template hipError_t launch_band_lu_step<T>(const InstDesc *, const ItemMap &, int, const ItemMap &, int, \
                                             int, int *, hipStream_t);                          \
  template hipError_t launch_band_lsolve<T>(const InstDesc *, const ItemMap &, int, hipStream_t);   \
  template int trsv_coop_capacity<T>();
FDE_INST(double)
FDE_INST(float)
#undef FDE_INST

}  // namespace fde
