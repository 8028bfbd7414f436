// Space-time kernels of the all-at-once operator (gfx950):
//  * Toeplitz symbol of G_a (eq. (1.5)) by an LDS FFT of its circulant embedding,
//  * the fused product M z = (A (x) I) z - tau (B (x) J) z of eq. (1.10): for every time
//    level the banded BVM rows are combined first, then J is applied once through the
//    FFT (J sum_q b_q z_q = sum_q b_q J z_q because J is time-independent),
//  * the right-hand side of the s-form system,
//  * the real DFT along time that diagonalises s(A), s(B) (Section 3.2), two spatial
//    columns packed per complex FFT.
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

// One workgroup per time level n.
//   v = sum_q b[n][q] Z[col_q],  u = sum_q a[n][q] Z[col_q]   (col_q = c[n]+q-1, skip < 0)
//   FFT(v);  X = chat*V + i conj(chat)*V;  IFFT(X) = L (G v + i G^T v)
//   W[n][i] = u_i + coefJ * scale/L * (d+_i Re + d-_i Im)
__global__ __launch_bounds__(ST_NT) void k_bvm_matvec(const double *__restrict__ Z,
                                                      double *__restrict__ W, DevSpace sp,
                                                      DevBand bd, double coef) {
  extern __shared__ double2 buf[];
  const int n = blockIdx.x;
  const int m = sp.m, L = 1 << sp.log2L;
  const int c0 = bd.c[n] - 1;
  const double *ra = bd.a + (size_t)n * bd.mu1;
  const double *rb = bd.b + (size_t)n * bd.mu1;
  for (int i = threadIdx.x; i < L; i += ST_NT) {
    double v = 0.0;
    if (i < m) {
      for (int q = 0; q < bd.mu1; ++q) {
        const int col = c0 + q;
        if (col >= 0 && col < bd.s) v = fma(rb[q], Z[(size_t)col * m + i], v);
      }
    }
    buf[i] = make_double2(v, 0.0);
  }
  __syncthreads();
  fft_dif<ST_NT>(buf, sp.log2L, 1, sp.twL);
  for (int k = threadIdx.x; k < L; k += ST_NT) {
    const double2 x = buf[k], c = sp.chat_br[k];
    const double2 P = cmul(c, x);
    const double2 Q = cmulc(x, c);
    buf[k] = make_double2(P.x - Q.y, P.y + Q.x);
  }
  __syncthreads();
  fft_dit_inv<ST_NT>(buf, sp.log2L, 1, sp.twL);
  for (int i = threadIdx.x; i < m; i += ST_NT) {
    double u = 0.0;
    for (int q = 0; q < bd.mu1; ++q) {
      const int col = c0 + q;
      if (col >= 0 && col < bd.s) u = fma(ra[q], Z[(size_t)col * m + i], u);
    }
    const double2 y = buf[i];
    W[(size_t)n * m + i] = fma(coef, fma(sp.dplus[i], y.x, sp.dminus[i] * y.y), u);
  }
}

__global__ __launch_bounds__(ST_NT) void k_rhs(const double *__restrict__ f,
                                               const double *__restrict__ u0,
                                               const double *__restrict__ Ju0,
                                               double *__restrict__ b, int m, DevBand bd,
                                               double tau) {
  const int n = blockIdx.y;
  const int i = blockIdx.x * ST_NT + threadIdx.x;
  if (i >= m) return;
  const int c = bd.c[n];
  const double *ra = bd.a + (size_t)n * bd.mu1;
  const double *rb = bd.b + (size_t)n * bd.mu1;
  double acc = 0.0;
  for (int q = 0; q < bd.mu1; ++q) acc = fma(rb[q], f[(size_t)(c + q) * m + i], acc);
  acc *= tau;
  if (c == 0) {
    acc = fma(-ra[0], u0[i], acc);
    if (Ju0 != nullptr) acc = fma(tau * rb[0], Ju0[i], acc);
  }
  b[(size_t)n * m + i] = acc;
}

// Time-axis real DFT.  Workgroup = 2*TP spatial columns, TP complex FFTs of length s.
static constexpr int TP = 8;

__global__ __launch_bounds__(ST_NT) void k_time_rfft(const double *__restrict__ V,
                                                     double2 *__restrict__ Vh, int m, int mp,
                                                     int log2s, const double2 *__restrict__ tw) {
  extern __shared__ double2 buf[];
  const int s = 1 << log2s;
  const int col0 = blockIdx.x * 2 * TP;
  for (int e = threadIdx.x; e < s * 2 * TP; e += ST_NT) {
    const int n = e / (2 * TP), c = e % (2 * TP);
    const int col = col0 + c;
    const double v = (col < m) ? V[(size_t)n * m + col] : 0.0;
    reinterpret_cast<double *>(&buf[(c >> 1) * s + n])[c & 1] = v;
  }
  __syncthreads();
  fft_dif<ST_NT>(buf, log2s, TP, tw);
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
    Vh[(size_t)k * mp + col] = o;
  }
}

__global__ __launch_bounds__(ST_NT) void k_time_irfft(const double2 *__restrict__ Wh,
                                                      double *__restrict__ W, int m, int mp,
                                                      int log2s, const double2 *__restrict__ tw) {
  extern __shared__ double2 buf[];
  const int s = 1 << log2s;
  const int col0 = blockIdx.x * 2 * TP;
  // position p of the bit-reversed input holds Z[k], k = bitrev(p); Z = What_a + i What_b
  for (int e = threadIdx.x; e < s * TP; e += ST_NT) {
    const int p = e / TP, f = e % TP;
    const int k = bitrev(p, log2s);
    const int ca = col0 + 2 * f;
    double2 a, b;
    if (k <= s / 2) {
      a = Wh[(size_t)k * mp + ca];
      b = Wh[(size_t)k * mp + ca + 1];
      if (k == 0 || k == s / 2) { a.y = 0.0; b.y = 0.0; }
    } else {
      a = cconj(Wh[(size_t)(s - k) * mp + ca]);
      b = cconj(Wh[(size_t)(s - k) * mp + ca + 1]);
    }
    buf[f * s + p] = make_double2(a.x - b.y, a.y + b.x);
  }
  __syncthreads();
  fft_dit_inv<ST_NT>(buf, log2s, TP, tw);
  const double inv_s = 1.0 / (double)s;
  for (int e = threadIdx.x; e < s * 2 * TP; e += ST_NT) {
    const int n = e / (2 * TP), c = e % (2 * TP);
    const int col = col0 + c;
    if (col >= m) continue;
    const double2 z = buf[(c >> 1) * s + n];
    W[(size_t)n * m + col] = ((c & 1) ? z.y : z.x) * inv_s;
  }
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

hipError_t launch_bvm_matvec(const double *Z, double *W, const DevSpace &sp, const DevBand &bd,
                             double coefJ, hipStream_t st) {
  const size_t lds = sizeof(double2) << sp.log2L;
  hipError_t e = set_lds((const void *)k_bvm_matvec, lds);
  if (e != hipSuccess) return e;
  const double coef = coefJ * sp.scale / (double)(1 << sp.log2L);
  hipLaunchKernelGGL(k_bvm_matvec, dim3(bd.s), dim3(ST_NT), lds, st, Z, W, sp, bd, coef);
  return hipGetLastError();
}

hipError_t launch_rhs(const double *f, const double *u0, const double *Ju0, double *b, int m,
                      const DevBand &bd, double tau, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs, dim3((m + ST_NT - 1) / ST_NT, bd.s), dim3(ST_NT), 0, st, f, u0, Ju0,
                     b, m, bd, tau);
  return hipGetLastError();
}

hipError_t launch_time_rfft(const double *V, double2 *Vh, int m, int mp, int log2s,
                            const double2 *tws, hipStream_t st) {
  const size_t lds = (sizeof(double2) * TP) << log2s;
  hipError_t e = set_lds((const void *)k_time_rfft, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_time_rfft, dim3(mp / (2 * TP)), dim3(ST_NT), lds, st, V, Vh, m, mp, log2s,
                     tws);
  return hipGetLastError();
}

hipError_t launch_time_irfft(const double2 *Wh, double *W, int m, int mp, int log2s,
                             const double2 *tws, hipStream_t st) {
  const size_t lds = (sizeof(double2) * TP) << log2s;
  hipError_t e = set_lds((const void *)k_time_irfft, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_time_irfft, dim3(mp / (2 * TP)), dim3(ST_NT), lds, st, Wh, W, m, mp,
                     log2s, tws);
  return hipGetLastError();
}

}  // namespace fde
