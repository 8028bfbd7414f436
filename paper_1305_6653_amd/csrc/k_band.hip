// The blocks of the Strang preconditioner through one band form of J (not in the paper).
//
// Every block K_k = lambda_k I - tau mu_k J (Section 3.2) is a shift of the same real matrix J.
// An orthogonal similarity J = Q H Q^T with H of lower bandwidth 64 (H[i][j] = 0 for
// i > j + 64: a block upper Hessenberg matrix with 64 x 64 blocks whose subdiagonal blocks are
// upper triangular) turns every block into C_k = lambda_k I - tau mu_k H = Q^T K_k Q.  Gaussian
// elimination with partial pivoting confined to the 128 rows of each 64-column panel factors
// C_k in O(64 m^2) operations instead of the O(m^3) of a dense LU (k_factor.hip), and the
// solves read L only inside the band.
//
// The reduction here is blocked so that its O(m^3) work runs as matrix products on the matrix
// cores.  For panel p (columns 64p .. 64p+63, c = 64(p+1), w = mp - c):
//   k_band_panel   the w x 64 block A[c:, 64p:c] is reduced to upper triangular form by 64
//                  Householder reflections H_j = I - beta_j v_j v_j^T (the sign choice of the
//                  textbook reflector, alpha = -sign(x_0) |x|), accumulated in compact WY form
//                  H_0 ... H_63 = I - V T V^T (T upper triangular, from V^T V by recursive
//                  doubling: T = [T1 -T1 V1^T V2 T2; 0 T2]).  Cooperative: workgroup g
//                  holds 128 rows of the block in LDS; per reflection one exchange of the
//                  column dot products x^T a between the workgroups (all of them at once, before
//                  the reflector is known: v^T a = x^T a - alpha a_0 and v^T v = 2 (x^T x -
//                  alpha x_0)).
//   right update   [A; Q][:, c:] -= ([A; Q][:, c:] V) T V^T   (A and Q stacked: one product)
//   left update    A[c:, c:] -= V T^T (V^T A[c:, c:])
// with FP64 MFMA products (k_dgemm; the long inner products are split over the K dimension
// into partial outputs that k_band_w2 / k_band_y2 sum in a fixed order together with the
// multiplication by T).  Q starts as I, so at the end Q H Q^T = J with H = A.
#include <algorithm>

#include "batch.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace fde {

static constexpr int BW = 64;           // bandwidth = panel width
static constexpr int BP_ROWS = 128;     // rows of the panel per workgroup
static constexpr int BP_MAXG = 32;      // workgroups of a panel reduction (mp <= 4096)
static constexpr int BP_SPIN_MAX = 1 << 21;

__device__ __forceinline__ void bst(double *p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double bld(const double *p) {
  return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Exchange slots.  Every value a workgroup publishes goes to a slot of its own (per reflection
// step, workgroup and column), written once per panel with a 64-bit atomic store; a slot holds
// the sentinel until then, so a reader waits on the value itself (no separate barrier): one
// round trip once the writer has stored.  Two slot sets alternate between consecutive panels;
// each panel refills the other set with the sentinel for the next one.  Waits are bounded:
// after BP_SPIN_MAX polls, or once any workgroup has raised *err, the reader gives up.
static constexpr unsigned long long BP_SENTINEL = 0x7ff4deadbeefcafeull;  // a NaN no sum produces

__device__ __forceinline__ bool bwait(const double *p, double *out, const int *err) {
  for (int it = 0;; ++it) {
    const unsigned long long u = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (u != BP_SENTINEL) {
      *out = __longlong_as_double((long long)u);
      return true;
    }
    if (it > BP_SPIN_MAX || ((it & 63) == 63 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)))
      return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

__global__ void k_band_fill(unsigned long long *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = BP_SENTINEL;
}

// ---- [A; Q] = [J padded with I; I] -------------------------------------------------------
// J[i][j] = dx^{-a} (d+_i g_{i-j+1} + d-_i g_{j-i+1}) (eq. (1.4)-(1.5)); the pad rows and
// columns (i or j >= m) carry the unit diagonal, which the reduction leaves untouched.
__global__ __launch_bounds__(256) void k_band_init(const InstDesc *__restrict__ Dd, int inst,
                                                   double *__restrict__ AQ) {
  const InstDesc &d = Dd[inst];
  const int mp = d.mp, m = d.m;
  const int i = blockIdx.y;  // row of [A; Q]
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= mp) return;
  double v;
  if (i < mp) {
    if (i < m && j < m) {
      const int dd = i - j;
      const double gp = (dd >= -1 && dd + 1 <= m) ? d.g[dd + 1] : 0.0;
      const double gm = (dd <= 1 && 1 - dd <= m) ? d.g[1 - dd] : 0.0;
      v = d.scale * fma(d.dp[i], gp, d.dm[i] * gm);
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
  } else {
    v = (i - mp == j) ? 1.0 : 0.0;
  }
  AQ[(size_t)i * mp + j] = v;
}

__global__ void k_band_zero_u32(unsigned *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---- panel reduction (workgroups cooperating through exchange slots) --------------------------
// Workgroup g holds panel rows [128 g, 128 g + 128) (local to the panel: row r is row c + r of
// A) in LDS; thread t works on column t % 64 and rows t / 64 + 16 i.  Per reflection step j each
// workgroup publishes its column dot products (and workgroup 0 the panel's row j) into the
// step's slots, then waits for all of them; wavefront 0 sums the published values in workgroup
// order, so all workgroups derive bitwise-equal reflectors.  Four barriers per step: after the
// local dot products, after the exchange, after the sums, after the update.
static constexpr int BP_NT = 1024, BP_RG = BP_NT / BW;  // threads, row groups
static constexpr int BP_RPT = BP_ROWS / BP_RG;          // rows per thread
// slot set layout (doubles): xpart [64 steps][BP_MAXG][64], xtop [64 steps][64], gpart
// [BP_MAXG][64][64], gflag [BP_MAXG] (raised once a workgroup's gpart is stored)
static constexpr size_t BP_XPART = (size_t)BW * BP_MAXG * BW, BP_XTOP = (size_t)BW * BW,
                        BP_GPART = (size_t)BP_MAXG * BW * BW,
                        BP_SET = BP_XPART + BP_XTOP + BP_GPART + BP_MAXG;
struct BandPanelArgs {
  double *AQ;           // [2 mp][mp]
  double *V;            // [w][64]: the Householder vectors (zero above the diagonal)
  double *T;            // [64][64]: the compact-WY factor (zero below the diagonal)
  double *slots;        // this panel's slot set (BP_SET doubles)
  double *next;         // the other set, refilled with the sentinel for the next panel
  int *err;
  int mp, p;
};

__global__ __launch_bounds__(BP_NT) void k_band_panel(BandPanelArgs a) {
  __shared__ double S[BP_ROWS][BW + 1];
  __shared__ double red[BP_RG][BW];
  __shared__ double xch[BP_MAXG][BW];
  __shared__ double sx[BW], tp[BW], rd[BW], bt[BW];
  __shared__ double tw[BW][BW + 1];  // W of the T recursion
  __shared__ int bad;
  const int G = gridDim.x, g = blockIdx.x, t = threadIdx.x, col = t & 63, rg = t >> 6;
  const int mp = a.mp, c = (a.p + 1) * BW, w = mp - c, pc = a.p * BW + col;
  const int rbase = g * BP_ROWS;  // first panel row of this workgroup
  double *xpart = a.slots, *xtop = a.slots + BP_XPART, *gpart = xtop + BP_XTOP, *gflag = gpart + BP_GPART;
  {  // this workgroup's share of the next panel's slots
    unsigned long long *nx = reinterpret_cast<unsigned long long *>(a.next);
    const size_t per = (BP_SET + G - 1) / G, lo = per * g, hi = lo + per < BP_SET ? lo + per : BP_SET;
    for (size_t i = lo + t; i < hi; i += BP_NT) nx[i] = BP_SENTINEL;
  }
  if (t == 0) bad = 0;
#pragma unroll
  for (int i = 0; i < BP_RPT; ++i) {
    const int sr = rg + BP_RG * i, r = rbase + sr;
    S[sr][col] = r < w ? a.AQ[(size_t)(c + r) * mp + pc] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < BW; ++j) {
    // column dot products of step j over this workgroup's rows r >= j: x^T a for every column
    // (four interleaved partial sums, combined in a fixed order)
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < BP_RPT; ++i) {
      const int sr = rg + BP_RG * i;
      const double x = rbase + sr >= j ? S[sr][j] : 0.0;
      s4[i & 3] = fma(x, S[sr][col], s4[i & 3]);
    }
    red[rg][col] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    __syncthreads();
    if (t < BW) {
      double q = 0.0;
#pragma unroll
      for (int h = 0; h < BP_RG; ++h) q += red[h][t];
      bst(&xpart[((size_t)j * BP_MAXG + g) * BW + t], q);
      if (g == 0) bst(&xtop[(size_t)j * BW + t], S[j][t]);  // panel row j lies in slab 0 (j < 128)
    }
    bool ok = true;
    for (int h = rg; h < G; h += BP_RG)
      ok = ok && bwait(&xpart[((size_t)j * BP_MAXG + h) * BW + col], &xch[h][col], a.err);
    if (t < BW) ok = ok && bwait(&xtop[(size_t)j * BW + t], &tp[t], a.err);
    if (!ok) {
      bad = 1;
      atomicOr(a.err, 1);
    }
    __syncthreads();
    if (bad) return;
    if (t < BW) {
      double q = 0.0;
      for (int h = 0; h < G; ++h) q += xch[h][t];
      sx[t] = q;
    }
    __syncthreads();
    const double sxx = sx[j], sxc = sx[col], x0 = tp[j];
    const double nrm = sqrt(sxx);
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    const double vtv = 2.0 * (sxx - alpha * x0);  // (x0 - alpha)^2 + sum_{r > j} x_r^2
    const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
    const double v0 = x0 - alpha;
    if (col > j) {
      const double f = beta * (sxc - alpha * tp[col]);  // beta v^T a
#pragma unroll
      for (int i = 0; i < BP_RPT; ++i) {
        const int sr = rg + BP_RG * i, r = rbase + sr;
        if (r >= j) {
          const double v = r == j ? v0 : S[sr][j];
          S[sr][col] = fma(-f, v, S[sr][col]);
        }
      }
    } else if (col == j && g == 0 && rg == j % BP_RG) {
      // v_j's first entry (no thread reads S[j][j] during this step: the update uses v0)
      S[j][j] = beta > 0.0 ? v0 : 0.0;
    }
    if (t == 0) {
      rd[j] = beta > 0.0 ? alpha : x0;  // R[j][j] (a zero column below j keeps x0)
      bt[j] = beta;
    }
    __syncthreads();
  }
  // V (zero above the diagonal, and the whole column when beta_j = 0) and the reduced panel:
  // R on and above the diagonal, zeros below.  Slab rows past the panel stay zero.
#pragma unroll
  for (int i = 0; i < BP_RPT; ++i) {
    const int sr = rg + BP_RG * i, r = rbase + sr;
    if (r >= w) continue;
    const double x = S[sr][col];
    const double vv = (r >= col && bt[col] > 0.0) ? x : 0.0;
    a.V[(size_t)r * BW + col] = vv;
    a.AQ[(size_t)(c + r) * mp + pc] = r < col ? x : (r == col ? rd[col] : 0.0);
    S[sr][col] = vv;
  }
  __syncthreads();
  {  // this workgroup's part of V^T V on the matrix cores: wavefront q computes the 16 x 16 tile
     // (q / 4, q % 4) over the 128 slab rows
    const int q = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
    const int u0 = (q >> 2) * 16, w0 = (q & 3) * 16;
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < BP_ROWS; k0 += 4) acc = mfma16(S[k0 + lk][u0 + li], S[k0 + lk][w0 + li], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      bst(&gpart[(size_t)g * BW * BW + (size_t)(u0 + mfma_row<double>(lk, v)) * BW + w0 + li], acc[v]);
  }
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have completed
  __syncthreads();
  if (t == 0) bst(&gflag[g], 1.0);
  if (g != 0) return;
  // T in workgroup 0 from Gm = V^T V (the workgroups' parts summed in order) by recursive
  // doubling: for V = [V1 V2], T = [T1 T12; 0 T2] with T12 = -T1 (V1^T V2) T2, over blocks of
  // 1, 2, ..., 32 columns (the product of the reflectors is I - V T V^T)
  if (t < G) {
    double y;
    if (!bwait(&gflag[t], &y, a.err)) {
      bad = 1;
      atomicOr(a.err, 1);
    }
  }
  __syncthreads();
  if (bad) return;
  double(*Gm)[BW + 1] = S;       // rows 0..63 of the slab buffer
  double(*Tm)[BW + 1] = S + BW;  // rows 64..127
  double(*Wm)[BW + 1] = tw;
  for (int e = t; e < BW * BW; e += BP_NT) {
    double v[BP_MAXG];
#pragma unroll
    for (int h = 0; h < BP_MAXG; ++h) v[h] = h < G ? bld(&gpart[(size_t)h * BW * BW + e]) : 0.0;
    double q = 0.0;
#pragma unroll
    for (int h = 0; h < BP_MAXG; ++h)
      if (h < G) q += v[h];
    Gm[e >> 6][e & 63] = q;
    Tm[e >> 6][e & 63] = (e >> 6) == (e & 63) ? bt[e & 63] : 0.0;
  }
  __syncthreads();
  for (int b = 1; b < BW; b *= 2) {
    const int nout = (BW / (2 * b)) * b * b;
    for (int e = t; e < nout; e += BP_NT) {  // W = (V1^T V2) T2 (T2 upper triangular)
      const int o = 2 * b * (e / (b * b)), i = (e % (b * b)) / b, jj = e % b;
      double q = 0.0;
      for (int l = 0; l <= jj; ++l) q = fma(Gm[o + i][o + b + l], Tm[o + b + l][o + b + jj], q);
      Wm[o + i][jj] = q;
    }
    __syncthreads();
    for (int e = t; e < nout; e += BP_NT) {  // T12 = -T1 W (T1 upper triangular)
      const int o = 2 * b * (e / (b * b)), i = (e % (b * b)) / b, jj = e % b;
      double q = 0.0;
      for (int l = i; l < b; ++l) q = fma(Tm[o + i][o + l], Wm[o + l][jj], q);
      Tm[o + i][o + b + jj] = -q;
    }
    __syncthreads();
  }
  for (int e = t; e < BW * BW; e += BP_NT) a.T[e] = Tm[e >> 6][e & 63];
}

// ---- FP64 matrix products on MFMA -----------------------------------------------------------
// C (M x N) = alpha op(A) op(B) over the K range of split z = blockIdx.z (kc per split):
//   MODE 0: store the partial product at C + z M N (row-major, leading dimension N);
//   MODE 1: C[i][j] += alpha * product (one split).
// op(A)(i, k) = TA ? A[k lda + i] : A[i lda + k];  op(B)(k, j) = TB ? B[j ldb + k] : B[k ldb + j].
// M, N multiples of 64 and kc of 16.  64 x 64 tile per workgroup; wavefront w computes the 32 x 32
// quarter (w / 2, w % 2) as 2 x 2 products of v_mfma_f64_16x16x4f64 from 16-deep K slices
// staged in LDS, the next slice loaded into registers while the current one is multiplied;
// in MODE 1 the tile of C is read before the K loop.  Fixed summation order (deterministic).
static constexpr int DG_KS = 16;

template <bool TA, bool TB, int MODE>
__global__ __launch_bounds__(256) void k_dgemm(int M, int N, int kc, int K, const double *__restrict__ A,
                                               int lda, const double *__restrict__ B, int ldb,
                                               double *__restrict__ C, int ldc, double alpha) {
  __shared__ double As[2][DG_KS][64 + 1];  // As[buf][k][i]
  __shared__ double Bs[2][DG_KS][64 + 1];  // Bs[buf][k][j]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
  const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  double cv[2][2][4];
  if (MODE == 1) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          cv[r][c][v] = C[(size_t)(row0 + wr + 16 * r + mfma_row<double>(lk, v)) * ldc + col0 + wc + 16 * c + li];
  }
  v4d acc[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[r][c] = v4d{0.0, 0.0, 0.0, 0.0};
  // loader roles: op(A)[row0 .. +64][k0 .. +16] and op(B)[k0 .. +16][col0 .. +64], 4 doubles each
  const int a_i = TA ? (tid & 15) * 4 : tid >> 2, a_k = TA ? tid >> 4 : (tid & 3) * 4;
  const int b_k = TB ? (tid & 3) * 4 : tid >> 4, b_j = TB ? tid >> 2 : (tid & 15) * 4;
  const double *Ap = TA ? A + (size_t)a_k * lda + row0 + a_i : A + (size_t)(row0 + a_i) * lda + a_k;
  const double *Bp = TB ? B + (size_t)(col0 + b_j) * ldb + b_k : B + (size_t)b_k * ldb + col0 + b_j;
  const size_t a_step = TA ? (size_t)DG_KS * lda : DG_KS, b_step = TB ? DG_KS : (size_t)DG_KS * ldb;
  double ra[4], rb[4];
  auto load = [&](int k0) {
    const double *pa = Ap + (size_t)(k0 / DG_KS) * a_step, *pb = Bp + (size_t)(k0 / DG_KS) * b_step;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ra[u] = pa[u];
      rb[u] = pb[u];
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (TA) As[buf][a_k][a_i + u] = ra[u]; else As[buf][a_k + u][a_i] = ra[u];
      if (TB) Bs[buf][b_k + u][b_j] = rb[u]; else Bs[buf][b_k][b_j + u] = rb[u];
    }
  };
  if (kb < ke) {
    load(kb);
    stage(0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kb; k0 < ke; k0 += DG_KS) {
    const bool more = k0 + DG_KS < ke;
    if (more) load(k0 + DG_KS);
#pragma unroll
    for (int kk = 0; kk < DG_KS; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) av[r] = As[buf][kk + lk][wr + 16 * r + li];
#pragma unroll
      for (int c = 0; c < 2; ++c) bv[c] = Bs[buf][kk + lk][wc + 16 * c + li];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[r][c] = mfma16(av[r], bv[c], acc[r][c]);
    }
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0 + wr + 16 * r + mfma_row<double>(lk, v), j = col0 + wc + 16 * c + li;
        if (MODE == 0)
          C[(size_t)blockIdx.z * M * N + (size_t)i * N + j] = acc[r][c][v];
        else
          C[(size_t)i * ldc + j] = fma(alpha, acc[r][c][v], cv[r][c][v]);
      }
}

// W2[i][:] = (sum_z P[z][i][:]) T for rows i < M (P: [nsplit][M][64]; T upper triangular).
__global__ __launch_bounds__(256) void k_band_w2(const double *__restrict__ P, int nsplit, int M,
                                                 const double *__restrict__ T, double *__restrict__ W2) {
  __shared__ double Ts[BW][BW + 1];
  __shared__ double rs[4][BW];
  const int t = threadIdx.x, col = t & 63, rr = t >> 6, i = blockIdx.x * 4 + rr;
  for (int e = t; e < BW * BW; e += 256) Ts[e >> 6][e & 63] = T[e];
  double q = 0.0;
  for (int z = 0; z < nsplit; ++z) q += P[((size_t)z * M + i) * BW + col];
  rs[rr][col] = q;
  __syncthreads();
  double o = 0.0;
  for (int k = 0; k <= col; ++k) o = fma(rs[rr][k], Ts[k][col], o);
  W2[(size_t)i * BW + col] = o;
}

// Y2[:, j] = T^T (sum_z P[z][:, j]) for columns j < N (P: [nsplit][64][N]).
__global__ __launch_bounds__(256) void k_band_y2(const double *__restrict__ P, int nsplit, int N,
                                                 const double *__restrict__ T, double *__restrict__ Y2) {
  __shared__ double Ts[BW][BW + 1];
  __shared__ double ys[BW][4 + 1];
  const int t = threadIdx.x, a = t & 63, cc = t >> 6, j = blockIdx.x * 4 + cc;
  for (int e = t; e < BW * BW; e += 256) Ts[e >> 6][e & 63] = T[e];
  double q = 0.0;
  for (int z = 0; z < nsplit; ++z) q += P[((size_t)z * BW + a) * N + j];
  ys[a][cc] = q;
  __syncthreads();
  double o = 0.0;
  for (int k = 0; k <= a; ++k) o = fma(Ts[k][a], ys[k][cc], o);
  Y2[(size_t)a * N + j] = o;
}

// Qt = Q^T ([mp][mp], 64 x 64 tiles through LDS).
__global__ __launch_bounds__(256) void k_band_transpose(const double *__restrict__ Q, double *__restrict__ Qt,
                                                        int mp) {
  __shared__ double tl[64][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64, t = threadIdx.x;
  for (int e = t; e < 64 * 64; e += 256) tl[e >> 6][e & 63] = Q[(size_t)(r0 + (e >> 6)) * mp + c0 + (e & 63)];
  __syncthreads();
  for (int e = t; e < 64 * 64; e += 256) Qt[(size_t)(c0 + (e >> 6)) * mp + r0 + (e & 63)] = tl[e & 63][e >> 6];
}

// ---- host side -------------------------------------------------------------------------------
static int dg_splits(int tiles, int K) {
  // enough workgroups to fill the device four times over, each with at least 128 of the K range
  int z = 1;
  while (tiles * z < 1024 && K / (2 * z) >= 128 && z < 16) z *= 2;
  return z;
}

size_t band_work_doubles(int mp) {
  const size_t w2 = (size_t)2 * mp * BW * 16;  // W partials: up to 16 splits of [2 mp][64]
  const size_t y1 = (size_t)BW * mp * 16;      // Y partials
  return 2 * ((size_t)mp * BW + BW * BW)      // V and T, one pair per panel parity
         + 2 * BP_SET                          // two slot sets
         + std::max(w2, y1)                    // partial products
         + (size_t)2 * mp * BW                 // W2
         + (size_t)BW * mp                     // Y2
         + (size_t)16 * BW * BW + BW * BW;     // Y partials and Y2 of the next panel's columns
}

template <bool TA, bool TB, int MODE>
static hipError_t dgemm(int M, int N, int K, int splits, const double *A, int lda, const double *B, int ldb,
                        double *C, int ldc, double alpha, hipStream_t st) {
  const int kc = ((K / splits + DG_KS - 1) / DG_KS) * DG_KS;
  hipLaunchKernelGGL((k_dgemm<TA, TB, MODE>), dim3(M / 64, N / 64, splits), dim3(256), 0, st, M, N, kc, K, A,
                     lda, B, ldb, C, ldc, alpha);
  return hipGetLastError();
}

// The reduction in parts, so that a caller can time the panels and the updates apart and run
// the next panel beside the current update: init ([A; Q] from J, slot set 0 filled), then per
// panel p = 0 .. mp/64 - 2 the panel and its two-sided update, then Qt = Q^T.  Panel p writes
// V and T of parity p & 1, so panel p + 1 may run while the update of panel p still reads its own.
struct BandPtrs {
  double *V, *T, *slots, *part, *W2, *Y2, *partn, *Y2n;
};
static BandPtrs band_ptrs(int mp, double *work, int p) {
  BandPtrs b;
  const size_t vt = (size_t)mp * BW + BW * BW;
  b.V = work + (size_t)(p & 1) * vt;
  b.T = b.V + (size_t)mp * BW;
  b.slots = work + 2 * vt;
  b.part = b.slots + 2 * BP_SET;
  const size_t w2 = (size_t)2 * mp * BW * 16, y1 = (size_t)BW * mp * 16;
  b.W2 = b.part + std::max(w2, y1);
  b.Y2 = b.W2 + (size_t)2 * mp * BW;
  b.partn = b.Y2 + (size_t)BW * mp;
  b.Y2n = b.partn + (size_t)16 * BW * BW;
  return b;
}

hipError_t launch_band_init(const InstDesc *D, int inst, int mp, double *AQ, double *work, hipStream_t st) {
  const BandPtrs b = band_ptrs(mp, work, 0);
  hipLaunchKernelGGL(k_band_init, dim3((mp + 255) / 256, 2 * mp), dim3(256), 0, st, D, inst, AQ);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_band_fill, dim3(64), dim3(256), 0, st, reinterpret_cast<unsigned long long *>(b.slots), BP_SET);
  return hipGetLastError();
}

hipError_t launch_band_panel(int mp, int p, double *AQ, double *work, int *err, hipStream_t st) {
  const BandPtrs b = band_ptrs(mp, work, p);
  const int c = (p + 1) * BW, w = mp - c;
  const int g = (w + BP_ROWS - 1) / BP_ROWS;
  BandPanelArgs pa{AQ, b.V, b.T, b.slots + (size_t)(p & 1) * BP_SET, b.slots + (size_t)((p + 1) & 1) * BP_SET,
                   err, mp, p};
  // An ordinary launch, so that it may run beside the previous panel's far update on another
  // stream: its at most 32 workgroups become co-resident as that update's short workgroups
  // retire, and every wait between them is bounded (BP_SPIN_MAX).
  hipLaunchKernelGGL(k_band_panel, dim3(g), dim3(BP_NT), 0, st, pa);
  return hipGetLastError();
}

// The two-sided update of panel p in two parts.  near: W = [A; Q][:, c:] V and W2 = W T (all of
// the trailing width), then the next panel's 64 columns c .. c + 63 in full: [A; Q][:, c:c+64]
// -= W2 V[0:64]^T, Y = V^T A[c:, c:c+64], Y2 = T^T Y, A[c:, c:c+64] -= V Y2.  far: the same for
// the columns from c + 64 on (nothing when w = 64).  The far part touches none of the next panel's
// columns and reads only this panel's V, T and W2, so it may run beside panel p + 1.
hipError_t launch_band_update(int mp, int p, bool far, double *AQ, double *work, hipStream_t st) {
  const BandPtrs b = band_ptrs(mp, work, p);
  const int c = (p + 1) * BW, w = mp - c;
  double *Ac = AQ + (size_t)c * mp + c;
  hipError_t e;
  if (!far) {
    const int zr = dg_splits(2 * mp / 64, w);
    if ((e = dgemm<false, false, 0>(2 * mp, BW, w, zr, AQ + c, mp, b.V, BW, b.part, BW, 1.0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_band_w2, dim3(2 * mp / 4), dim3(256), 0, st, b.part, zr, 2 * mp, b.T, b.W2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = dgemm<false, true, 1>(2 * mp, BW, BW, 1, b.W2, BW, b.V, BW, AQ + c, mp, -1.0, st)) != hipSuccess) return e;
    const int zn = dg_splits(1, w);
    if ((e = dgemm<true, false, 0>(BW, BW, w, zn, b.V, BW, Ac, mp, b.partn, BW, 1.0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_band_y2, dim3(BW / 4), dim3(256), 0, st, b.partn, zn, BW, b.T, b.Y2n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return dgemm<false, false, 1>(w, BW, BW, 1, b.V, BW, b.Y2n, BW, Ac, mp, -1.0, st);
  }
  const int wf = w - BW;  // the columns from c + 64 on
  if (wf <= 0) return hipSuccess;
  if ((e = dgemm<false, true, 1>(2 * mp, wf, BW, 1, b.W2, BW, b.V + (size_t)BW * BW, BW, AQ + c + BW, mp, -1.0,
                                 st)) != hipSuccess)
    return e;
  const int zl = dg_splits(wf / 64, w);
  if ((e = dgemm<true, false, 0>(BW, wf, w, zl, b.V, BW, Ac + BW, mp, b.part, wf, 1.0, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_band_y2, dim3(wf / 4), dim3(256), 0, st, b.part, zl, wf, b.T, b.Y2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return dgemm<false, false, 1>(w, wf, BW, 1, b.V, BW, b.Y2, wf, Ac + BW, mp, -1.0, st);
}

hipError_t launch_band_finish(int mp, double *AQ, double *Qt, hipStream_t st) {
  hipLaunchKernelGGL(k_band_transpose, dim3(mp / 64, mp / 64), dim3(256), 0, st, AQ + (size_t)mp * mp, Qt, mp);
  return hipGetLastError();
}

}  // namespace fde
