// LDS-resident radix-2 complex FFTs (FP64) for power-of-two lengths, batched over
// `nbatch` contiguous sequences buf[f*N + t].
//
// fft_dif: natural order in, bit-reversed order out, kernel e^{-2 pi i jk/N}
//          (Gentleman-Sande decimation in frequency).
// fft_dit_inv: bit-reversed order in, natural order out, kernel e^{+2 pi i jk/N},
//          unnormalised (Cooley-Tukey decimation in time).
// Pairing the two needs no permutation at all: a spectrum is multiplied pointwise in
// bit-reversed order (the multiplier is stored bit-reversed), which is how the
// Toeplitz products through a circulant embedding use them.
//
// tw[t] = e^{-2 pi i t/N}, t < N/2, precomputed in FP64 on the host.
// Every thread of the block must call these (they contain __syncthreads()).
#pragma once
#include "common.hpp"

namespace fde {

// Two consecutive radix-2 stages are done together in registers (a radix-4 pass: a thread
// loads the four elements i, i+h, i+2h, i+3h of a group of 4h, applies both stages and stores
// them back), so a length-N transform takes ceil(log2 N / 2) barriers instead of log2 N.  Each
// element sees exactly the operations of the radix-2 stages, in the same order.

template <int NT>
__device__ __forceinline__ void fft_dif(double2 *buf, int log2N, int nbatch,
                                        const double2 *__restrict__ tw) {
  const int N = 1 << log2N;
  int lh = log2N - 1;  // half-span of the next radix-2 stage is 2^lh
  for (; lh >= 1; lh -= 2) {
    // stages with half-spans 2h (= 2^lh) and h: groups of 4h
    const int h = 1 << (lh - 1);
    const int q4 = N >> 2, tsh1 = log2N - 1 - lh, tsh2 = tsh1 + 1;
    const int total = nbatch * q4;
    for (int b = threadIdx.x; b < total; b += NT) {
      const int f = b >> (log2N - 2), bb = b & (q4 - 1);
      const int j = bb & (h - 1), grp = bb >> (lh - 1);
      const int i0 = (f << log2N) + (grp << (lh + 1)) + j;
      const double2 x0 = buf[i0], x1 = buf[i0 + h], x2 = buf[i0 + 2 * h], x3 = buf[i0 + 3 * h];
      const double2 w1 = tw[j << tsh1], w1b = tw[(j + h) << tsh1], w2 = tw[j << tsh2];
      const double2 a0 = cadd(x0, x2), a2 = cmul(csub(x0, x2), w1);
      const double2 a1 = cadd(x1, x3), a3 = cmul(csub(x1, x3), w1b);
      buf[i0] = cadd(a0, a1);
      buf[i0 + h] = cmul(csub(a0, a1), w2);
      buf[i0 + 2 * h] = cadd(a2, a3);
      buf[i0 + 3 * h] = cmul(csub(a2, a3), w2);
    }
    __syncthreads();
  }
  if (lh == 0) {  // odd log2N: the last radix-2 stage (half-span 1, twiddle 1)
    const int half = N >> 1, total = nbatch * half;
    for (int b = threadIdx.x; b < total; b += NT) {
      const int i0 = b << 1;
      const double2 a = buf[i0], c = buf[i0 + 1];
      buf[i0] = cadd(a, c);
      buf[i0 + 1] = csub(a, c);
    }
    __syncthreads();
  }
}

template <int NT>
__device__ __forceinline__ void fft_dit_inv(double2 *buf, int log2N, int nbatch,
                                            const double2 *__restrict__ tw) {
  const int N = 1 << log2N;
  int lh = 0;  // half-span of the next radix-2 stage is 2^lh
  if (log2N & 1) {  // odd log2N: the first radix-2 stage (half-span 1, twiddle 1)
    const int half = N >> 1, total = nbatch * half;
    for (int b = threadIdx.x; b < total; b += NT) {
      const int i0 = b << 1;
      const double2 a = buf[i0], c = buf[i0 + 1];
      buf[i0] = cadd(a, c);
      buf[i0 + 1] = csub(a, c);
    }
    __syncthreads();
    lh = 1;
  }
  for (; lh + 1 < log2N + 1 && lh < log2N; lh += 2) {
    // stages with half-spans h (= 2^lh) and 2h: groups of 4h
    const int h = 1 << lh;
    const int q4 = N >> 2, tsh1 = log2N - 1 - lh, tsh2 = tsh1 - 1;
    const int total = nbatch * q4;
    for (int b = threadIdx.x; b < total; b += NT) {
      const int f = b >> (log2N - 2), bb = b & (q4 - 1);
      const int j = bb & (h - 1), grp = bb >> lh;
      const int i0 = (f << log2N) + (grp << (lh + 2)) + j;
      const double2 x0 = buf[i0], x1 = buf[i0 + h], x2 = buf[i0 + 2 * h], x3 = buf[i0 + 3 * h];
      const double2 w1 = tw[j << tsh1], w2 = tw[j << tsh2], w2b = tw[(j + h) << tsh2];
      const double2 c1 = cmulc(x1, w1), c3 = cmulc(x3, w1);  // times e^{+2 pi i ...}
      const double2 a0 = cadd(x0, c1), a1 = csub(x0, c1), a2 = cadd(x2, c3), a3 = csub(x2, c3);
      const double2 c2 = cmulc(a2, w2), c4 = cmulc(a3, w2b);
      buf[i0] = cadd(a0, c2);
      buf[i0 + 2 * h] = csub(a0, c2);
      buf[i0 + h] = cadd(a1, c4);
      buf[i0 + 3 * h] = csub(a1, c4);
    }
    __syncthreads();
  }
}

}  // namespace fde
