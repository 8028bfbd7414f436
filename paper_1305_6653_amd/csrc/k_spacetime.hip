// Space-time kernels of the all-at-once operator (gfx950), batched over instances:
//  * Toeplitz symbol of G_a (eq. (1.5)) by an LDS FFT of its circulant embedding,
//  * the fused product M z = (A (x) I) z - tau (B (x) J) z of eq. (1.10): for every time
//    level the banded BVM rows are combined first, then J is applied once through the
//    FFT (J sum_q b_q z_q = sum_q b_q J z_q because J is time-independent),
//  * the right-hand side of the s-form system,
//  * the real DFT along time that diagonalises s(A), s(B) (Section 3.2), two spatial
//    columns packed per complex FFT.
#include "batch.hpp"
#include "common.hpp"
#include "fft_lds.hpp"
#include "kernels.hpp"

namespace fde {

static constexpr int ST_NT = 256;

// chat_br = FFT_L(c), c real [L]; result left in bit-reversed order.
__global__ __launch_bounds__(ST_NT) void k_symbol(const double *__restrict__ cG,
                                                  double2 *__restrict__ chat_br, int log2L,
                                                  const double2 *__restrict__ twL) {
  extern __shared__ double2 buf[];
  const int L = 1 << log2L;
  for (int i = threadIdx.x; i < L; i += ST_NT) buf[i] = make_double2(cG[i], 0.0);
  __syncthreads();
  fft_dif<ST_NT>(buf, log2L, 1, twL);
  for (int i = threadIdx.x; i < L; i += ST_NT) chat_br[i] = buf[i];
}

// Item = (instance, row n).
// mode 0 (M z):  v = sum_q b[n][q] Z[col_q], u = sum_q a[n][q] Z[col_q]  (col_q = c[n]+q-1 >= 0)
//                W[n] = u - tau J v
// mode 1 (J x):  W[n] = J Z[n]
// mode 2 (S z):  the Strang circulant rows: every row carries the main formula on the
//                wrapped columns (n - nu + q) mod s:  W[n] = u_S - tau J v_S
// mode 3 ((S - M) z): W[n] = (u_S - u) - tau J (v_S - v); nonzero only on the nu + (mu-nu)
//                boundary rows where the circulant and the BVM matrices differ.
// J v = scale/L * (d+ Re + d- Im) of IFFT(chat*V + i conj(chat)*V) = L (G v + i G^T v).
// The combinations u, v above for the KU elements i = tid + NT k (k < KU) of a thread: the
// loads of one coefficient step are issued together and u, v stay in registers (elements
// i >= m come out as zeros and are not used).
template <int KU, int NT>
__device__ __forceinline__ void band_combo_k(const InstDesc &d, const double *__restrict__ Z, int n, int mode,
                                             int tid, double (&u)[KU], double (&v)[KU]) {
  const int m = d.m, s = d.s, mu1 = d.mu1;
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    u[k] = 0.0;
    v[k] = 0.0;
  }
  if (mode == 1) {
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      const int i = tid + NT * k;
      v[k] = i < m ? Z[(size_t)n * m + i] : 0.0;
    }
    return;
  }
  auto step = [&](int col, double a, double b) {
    double z[KU];
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      const int i = tid + NT * k;
      z[k] = i < m ? Z[(size_t)col * m + i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      u[k] = fma(a, z[k], u[k]);
      v[k] = fma(b, z[k], v[k]);
    }
  };
  if (mode != 2) {  // BVM rows (subtracted in mode 3)
    const int c0 = d.band_c[n] - 1;
    const double *ra = d.band_a + (size_t)n * mu1;
    const double *rb = d.band_b + (size_t)n * mu1;
    for (int t = 0; t < mu1; ++t) {
      const int col = c0 + t;
      if (col >= 0 && col < s) step(col, ra[t], rb[t]);
    }
    if (mode == 3) {
#pragma unroll
      for (int k = 0; k < KU; ++k) {
        u[k] = -u[k];
        v[k] = -v[k];
      }
    }
  }
  if (mode >= 2) {  // circulant rows: main formula (stored in s-form row nu-1) wrapped mod s
    const double *ra = d.band_a + (size_t)(d.nu - 1) * mu1;
    const double *rb = d.band_b + (size_t)(d.nu - 1) * mu1;
    for (int t = 0; t < mu1; ++t) {
      int col = (n - d.nu + t) % s;
      if (col < 0) col += s;
      step(col, ra[t], rb[t]);
    }
  }
}

// NT threads (1024 for transforms of 4096 points and more, whose LDS allows one workgroup per
// CU: more wavefronts to hide the LDS passes; 256 below), KU = elements per thread
// (m <= NT KU).  Rows are numbered contiguously per XCD (xcd_item), so the neighbouring time
// rows that share band columns read them through one L2; the band combination is formed once
// (u stays in registers for the output) and d+, d- are loaded before the transforms.  Each
// element sees the same operations whatever NT, so the result does not depend on it.
template <int KU, int NT>
__global__ __launch_bounds__(NT) void k_bvm_matvec(const InstDesc *__restrict__ D, ItemMap map,
                                                      int src_sel, int src_j, int dst_sel,
                                                      int dst_j, int mode) {
  extern __shared__ double2 buf[];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int q = item_slot(map, item);
  if (item_gated(map, q)) return;
  const InstDesc &d = D[map.ids[q]];
  const int n = item - map.pre[q];
  const int m = d.m, L = 1 << d.log2L, tid = threadIdx.x;
  const double *Z = vsel(d, src_sel, src_j);
  double *W = vsel(d, dst_sel, dst_j);
  if (mode == 3 && n >= d.nu && n < d.s - (d.mu1 - 1 - d.nu)) {
    // interior row: S and M apply the same main formula without wrap-around, so the
    // difference is exactly zero (uniform per workgroup, before any barrier)
    for (int i = tid; i < m; i += NT) W[(size_t)n * m + i] = 0.0;
    return;
  }
  double u[KU], v[KU], dpv[KU], dmv[KU];
  band_combo_k<KU, NT>(d, Z, n, mode, tid, u, v);
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int i = tid + NT * k;
    dpv[k] = i < m ? d.dp[i] : 0.0;
    dmv[k] = i < m ? d.dm[i] : 0.0;
  }
  for (int i = tid; i < L; i += NT) buf[i] = make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < KU; ++k) {  // the same thread wrote the zero first
    const int i = tid + NT * k;
    if (i < m) buf[i] = make_double2(v[k], 0.0);
  }
  __syncthreads();
  fft_dif<NT>(buf, d.log2L, 1, d.twL);
  for (int k = tid; k < L; k += NT) {
    const double2 x = buf[k], c = d.chat[k];
    const double2 P = cmul(c, x);
    const double2 Qv = cmulc(x, c);
    buf[k] = make_double2(P.x - Qv.y, P.y + Qv.x);
  }
  __syncthreads();
  fft_dit_inv<NT>(buf, d.log2L, 1, d.twL);
  const double coef = (mode == 1 ? 1.0 : -d.tau) * d.scale / (double)L;
#pragma unroll
  for (int k = 0; k < KU; ++k) {
    const int i = tid + NT * k;
    if (i < m) {
      const double2 y = buf[i];
      W[(size_t)n * m + i] = fma(coef, fma(dpv[k], y.x, dmv[k] * y.y), u[k]);
    }
  }
}

// Item = (instance, row n):  b[n] = tau sum_q bhat[n][q] f[c+q] - a0[n] u0 + tau b0[n] Ju0,
// where a0[n], b0[n] are the coefficients on u_0 (nonzero only when the band starts at u_0).
__global__ __launch_bounds__(ST_NT) void k_rhs(const InstDesc *__restrict__ D, ItemMap map,
                                               int use_ju0) {
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = D[map.ids[q]];
  const int n = blockIdx.x - map.pre[q];
  const int m = d.m, c = d.band_c[n];
  const double *ra = d.band_a + (size_t)n * d.mu1;
  const double *rb = d.band_b + (size_t)n * d.mu1;
  for (int i = threadIdx.x; i < m; i += ST_NT) {
    double acc = 0.0;
    for (int t = 0; t < d.mu1; ++t) acc = fma(rb[t], d.f[(size_t)(c + t) * m + i], acc);
    acc *= d.tau;
    if (c == 0) {
      acc = fma(-ra[0], d.u0[i], acc);
      if (use_ju0 && d.need_ju0) acc = fma(d.tau * rb[0], d.Ju0[i], acc);
    }
    d.b[(size_t)n * m + i] = acc;
  }
}

// Time-axis real DFT.  Item = (instance, group of 2*TP spatial columns); TP complex FFTs of
// length s per workgroup (TP = 2, 4 or 8, chosen per plan so that the launch has enough
// workgroups).  Items in XCD-contiguous order (xcd_item), so the column groups that share a
// cache line of a row are read through the same L2.  The twiddle table (s/2 entries) is copied
// into LDS behind the data.

// If epoch_ctr is set, the first workgroup also draws the next block-solve epoch from the
// device-wide counter into epoch_slot[0] (read by the block solve that follows on the stream),
// so a recorded launch sequence gets a fresh epoch on every replay, and clears the block
// solve's unit counter epoch_slot[1].
template <int TP>
__global__ __launch_bounds__(ST_NT) void k_time_rfft(const InstDesc *__restrict__ D, ItemMap map,
                                                     int src_sel, int src_j, int max_log2s,
                                                     unsigned long long *epoch_ctr,
                                                     unsigned long long *epoch_slot) {
  extern __shared__ double2 buf[];
  if (epoch_ctr && blockIdx.x == 0 && threadIdx.x == 0) {
    *epoch_slot = atomicAdd(epoch_ctr, 1ull) + 1ull;
    epoch_slot[1] = 0ull;  // the block solve's unit counter
  }
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int q = item_slot(map, item);
  if (item_gated(map, q)) return;
  const InstDesc &d = D[map.ids[q]];
  const int m = d.m, mp = d.mp, log2s = d.log2s, s = 1 << log2s;
  const double *V = vsel(d, src_sel, src_j);
  const int col0 = (item - map.pre[q]) * 2 * TP;
  double2 *twl = buf + ((size_t)TP << max_log2s);
  for (int i = threadIdx.x; i < s / 2; i += ST_NT) twl[i] = d.tws[i];
  for (int e = threadIdx.x; e < s * 2 * TP; e += ST_NT) {
    const int n = e / (2 * TP), c = e % (2 * TP);
    const int col = col0 + c;
    const double v = (col < m) ? V[(size_t)n * m + col] : 0.0;
    reinterpret_cast<double *>(&buf[(c >> 1) * s + n])[c & 1] = v;
  }
  __syncthreads();
  fft_dif<ST_NT>(buf, log2s, TP, twl);
  const int nbk = s / 2 + 1;
  for (int e = threadIdx.x; e < nbk * 2 * TP; e += ST_NT) {
    const int k = e / (2 * TP), c = e % (2 * TP), f = c >> 1;
    const int col = col0 + c;
    if (col >= mp) continue;
    const int kk = (s - k) & (s - 1);
    const double2 Zk = buf[f * s + bitrev(k, log2s)];
    const double2 Zn = cconj(buf[f * s + bitrev(kk, log2s)]);
    double2 o;
    if ((c & 1) == 0) {
      o = make_double2(0.5 * (Zk.x + Zn.x), 0.5 * (Zk.y + Zn.y));
    } else {  // (Zk - Zn) * (-i/2)
      o = make_double2(0.5 * (Zk.y - Zn.y), -0.5 * (Zk.x - Zn.x));
    }
    if (col >= m) o = make_double2(0.0, 0.0);
    d.Vh[(size_t)k * mp + col] = o;
  }
}

template <int TP>
__global__ __launch_bounds__(ST_NT) void k_time_irfft(const InstDesc *__restrict__ D, ItemMap map,
                                                      int dst_sel, int dst_j, int max_log2s) {
  extern __shared__ double2 buf[];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int q = item_slot(map, item);
  if (item_gated(map, q)) return;
  const InstDesc &d = D[map.ids[q]];
  const int m = d.m, mp = d.mp, log2s = d.log2s, s = 1 << log2s;
  double *W = vsel(d, dst_sel, dst_j);
  const double2 *Wh = d.Vh;
  const int col0 = (item - map.pre[q]) * 2 * TP;
  double2 *twl = buf + ((size_t)TP << max_log2s);
  for (int i = threadIdx.x; i < s / 2; i += ST_NT) twl[i] = d.tws[i];
  // position p of the bit-reversed input holds Z[k], k = bitrev(p); Z = What_a + i What_b
  for (int e = threadIdx.x; e < s * TP; e += ST_NT) {
    const int p = e / TP, f = e % TP;
    const int k = bitrev(p, log2s);
    const int ca = col0 + 2 * f;
    double2 a, b;
    if (k <= s / 2) {
      a = Wh[(size_t)k * mp + ca];
      b = Wh[(size_t)k * mp + ca + 1];
      if (k == 0 || k == s / 2) {
        a.y = 0.0;
        b.y = 0.0;
      }
    } else {
      a = cconj(Wh[(size_t)(s - k) * mp + ca]);
      b = cconj(Wh[(size_t)(s - k) * mp + ca + 1]);
    }
    buf[f * s + p] = make_double2(a.x - b.y, a.y + b.x);
  }
  __syncthreads();
  fft_dit_inv<ST_NT>(buf, log2s, TP, twl);
  const double inv_s = 1.0 / (double)s;
  for (int e = threadIdx.x; e < s * 2 * TP; e += ST_NT) {
    const int n = e / (2 * TP), c = e % (2 * TP);
    const int col = col0 + c;
    if (col >= m) continue;
    const double2 z = buf[(c >> 1) * s + n];
    W[(size_t)n * m + col] = ((c & 1) ? z.y : z.x) * inv_s;
  }
}

// BCCB preconditioners (the 2-D diagonalisation of Section 3.2): after the time DFT, each time
// frequency k needs Y = F_m^{-1} diag(1/(lam_k - tau mu_k lamx_j)) F_m X over the space index.
// DFT of order m (any m) by Bluestein's method: with w_n = e^{-i pi n^2/m} (nj = (n^2 + j^2 -
// (j-n)^2)/2),  X_j = w_j sum_n (x_n w_n) conj(w_{j-n}),  a linear convolution done through the
// power-of-two FFT of length L >= 2m - 1 with the stored spectrum of conj(w) (bit-reversed).
// The inverse uses F^{-1} y = conj(F conj(y)) / m.  Item = (instance, k); one LDS buffer.
__device__ __forceinline__ void chirp_filter(double2 *buf, const InstDesc &d) {
  fft_dif<ST_NT>(buf, d.log2L, 1, d.twL);
  const int L = 1 << d.log2L;
  for (int i = threadIdx.x; i < L; i += ST_NT) buf[i] = cmul(buf[i], d.bh[i]);
  __syncthreads();
  fft_dit_inv<ST_NT>(buf, d.log2L, 1, d.twL);
}

__global__ __launch_bounds__(ST_NT) void k_bccb_solve(const InstDesc *__restrict__ D, ItemMap map) {
  extern __shared__ double2 buf[];
  const int q = item_slot(map, blockIdx.x);
  if (item_gated(map, q)) return;
  const InstDesc &d = D[map.ids[q]];
  const int k = blockIdx.x - map.pre[q];
  const int m = d.m, L = 1 << d.log2L;
  double2 *v = d.Vh + (size_t)k * d.mp;
  const double invL = 1.0 / (double)L;
  double2 lk = d.lam[k];
  if (k == 0 && d.pc == 2) lk = make_double2(d.lam0s, 0.0);
  const double2 tmk = cscale(d.mu[k], -d.tau);
  for (int i = threadIdx.x; i < L; i += ST_NT) buf[i] = i < m ? cmul(v[i], d.chirp[i]) : make_double2(0.0, 0.0);
  __syncthreads();
  chirp_filter(buf, d);
  // X_j = w_j conv_j / L; Y_j = X_j / (lam_k - tau mu_k lamx_j); next input conj(Y_j) w_j
  for (int j = threadIdx.x; j < L; j += ST_NT) {
    double2 t = make_double2(0.0, 0.0);
    if (j < m) {
      const double2 X = cscale(cmul(d.chirp[j], buf[j]), invL);
      const double2 e = cadd(lk, cmul(tmk, d.lamx[j]));
      const double ee = e.x * e.x + e.y * e.y;
      const double2 Y = cscale(cmulc(X, e), 1.0 / ee);
      t = cmul(cconj(Y), d.chirp[j]);
    }
    buf[j] = t;
  }
  __syncthreads();
  chirp_filter(buf, d);
  const double sc = invL / (double)m;
  for (int n = threadIdx.x; n < m; n += ST_NT) v[n] = cscale(cconj(cmul(d.chirp[n], buf[n])), sc);
}

// ------------------------------------------------------------------------------------
static hipError_t set_lds(const void *fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_symbol(const double *cG, double2 *chat_br, int log2L, const double2 *twL,
                         hipStream_t st) {
  const size_t lds = sizeof(double2) << log2L;
  hipError_t e = set_lds((const void *)k_symbol, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_symbol, dim3(1), dim3(ST_NT), lds, st, cG, chat_br, log2L, twL);
  return hipGetLastError();
}

template <int KU, int NT>
static hipError_t bvm_matvec_ku(const InstDesc *D, const ItemMap &map, int items, size_t lds, int src_sel,
                                int src_j, int dst_sel, int dst_j, int mode, hipStream_t st) {
  hipError_t e = set_lds((const void *)k_bvm_matvec<KU, NT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_bvm_matvec<KU, NT>), dim3(items), dim3(NT), lds, st, D, map, src_sel, src_j, dst_sel,
                     dst_j, mode);
  return hipGetLastError();
}

hipError_t launch_bvm_matvec(const InstDesc *D, const ItemMap &map, int items, int max_log2L,
                             int src_sel, int src_j, int dst_sel, int dst_j, int mode,
                             hipStream_t st) {
  if (items <= 0) return hipSuccess;
  const size_t lds = sizeof(double2) << max_log2L;
  // every instance has m <= L / 2 <= NT KU
  switch (max_log2L) {
    case 13: return bvm_matvec_ku<4, 1024>(D, map, items, lds, src_sel, src_j, dst_sel, dst_j, mode, st);
    case 12: return bvm_matvec_ku<2, 1024>(D, map, items, lds, src_sel, src_j, dst_sel, dst_j, mode, st);
    case 11: return bvm_matvec_ku<4, ST_NT>(D, map, items, lds, src_sel, src_j, dst_sel, dst_j, mode, st);
    case 10: return bvm_matvec_ku<2, ST_NT>(D, map, items, lds, src_sel, src_j, dst_sel, dst_j, mode, st);
    default:
      if (max_log2L < 10) return bvm_matvec_ku<1, ST_NT>(D, map, items, lds, src_sel, src_j, dst_sel, dst_j, mode, st);
      return hipErrorInvalidValue;
  }
}

hipError_t launch_rhs(const InstDesc *D, const ItemMap &map, int items, int use_ju0,
                      hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rhs, dim3(items), dim3(ST_NT), 0, st, D, map, use_ju0);
  return hipGetLastError();
}

template <int TP>
static hipError_t rfft_tp(const InstDesc *D, const ItemMap &map, int items, int max_log2s,
                          int src_sel, int src_j, hipStream_t st, unsigned long long *epoch_ctr,
                          unsigned long long *epoch_slot) {
  const size_t lds = ((sizeof(double2) * (2 * TP + 1)) << max_log2s) / 2;
  hipError_t e = set_lds((const void *)k_time_rfft<TP>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_time_rfft<TP>, dim3(items), dim3(ST_NT), lds, st, D, map, src_sel, src_j,
                     max_log2s, epoch_ctr, epoch_slot);
  return hipGetLastError();
}

template <int TP>
static hipError_t irfft_tp(const InstDesc *D, const ItemMap &map, int items, int max_log2s,
                           int dst_sel, int dst_j, hipStream_t st) {
  const size_t lds = ((sizeof(double2) * (2 * TP + 1)) << max_log2s) / 2;
  hipError_t e = set_lds((const void *)k_time_irfft<TP>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_time_irfft<TP>, dim3(items), dim3(ST_NT), lds, st, D, map, dst_sel, dst_j,
                     max_log2s);
  return hipGetLastError();
}

hipError_t launch_time_rfft(const InstDesc *D, const ItemMap &map, int items, int max_log2s,
                            int cols, int src_sel, int src_j, hipStream_t st,
                            unsigned long long *epoch_ctr, unsigned long long *epoch_slot) {
  if (items <= 0) return hipSuccess;
  switch (cols) {
    case 4: return rfft_tp<2>(D, map, items, max_log2s, src_sel, src_j, st, epoch_ctr, epoch_slot);
    case 8: return rfft_tp<4>(D, map, items, max_log2s, src_sel, src_j, st, epoch_ctr, epoch_slot);
    case 16: return rfft_tp<8>(D, map, items, max_log2s, src_sel, src_j, st, epoch_ctr, epoch_slot);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_time_irfft(const InstDesc *D, const ItemMap &map, int items, int max_log2s,
                             int cols, int dst_sel, int dst_j, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  switch (cols) {
    case 4: return irfft_tp<2>(D, map, items, max_log2s, dst_sel, dst_j, st);
    case 8: return irfft_tp<4>(D, map, items, max_log2s, dst_sel, dst_j, st);
    case 16: return irfft_tp<8>(D, map, items, max_log2s, dst_sel, dst_j, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bccb_solve(const InstDesc *D, const ItemMap &map, int items, int max_log2L,
                             hipStream_t st) {
  if (items <= 0) return hipSuccess;
  const size_t lds = sizeof(double2) << max_log2L;
  hipError_t e = set_lds((const void *)k_bccb_solve, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bccb_solve, dim3(items), dim3(ST_NT), lds, st, D, map);
  return hipGetLastError();
}

// Spatial columns per time-FFT workgroup: 16 (128-byte row segments) while that still gives
// the launch at least two workgroups per CU, else 8, else 4.
int time_fft_cols_per_item(long long total_mp, int cus) {
  for (int cols = 16; cols > 4; cols >>= 1)
    if (total_mp / cols >= 2LL * cus) return cols;
  return 4;
}

}  // namespace fde
