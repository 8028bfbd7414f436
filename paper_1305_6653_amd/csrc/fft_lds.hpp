// LDS-resident complex FFTs (FP64) for power-of-two lengths, made of radix-2 stages (applied
// three at a time), batched over `nbatch` contiguous sequences buf[f*N + t].
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

// Consecutive radix-2 stages are done together in registers: three per pass (a radix-8 pass:
// a thread loads the eight elements i + r h, r < 8, of a group of 8h, applies the three stages
// and stores them back), the one or two left over in a radix-2 or radix-4 pass, so a length-N
// transform takes about log2(N) / 3 barriers instead of log2 N.  Each element sees exactly the
// operations of the radix-2 stages, in the same order.

// DIF stage with half-span H on a pair at offset o of its group: (a, c) -> (a + c, (a - c) w),
// w = tw[o << (log2 N - 1 - log2 H)].
template <int NT>
__device__ __forceinline__ void fft_dif(double2 *buf, int log2N, int nbatch,
                                        const double2 *__restrict__ tw) {
  const int N = 1 << log2N;
  int lh = log2N - 1;  // half-span of the next radix-2 stage is 2^lh
  for (; lh >= 2; lh -= 3) {
    // stages with half-spans 4h (= 2^lh), 2h and h: groups of 8h
    const int h = 1 << (lh - 2);
    const int q8 = N >> 3, tsh = log2N - 1 - lh;
    const int total = nbatch * q8;
    for (int b = threadIdx.x; b < total; b += NT) {
      const int f = b >> (log2N - 3), bb = b & (q8 - 1);
      const int j = bb & (h - 1), grp = bb >> (lh - 2);
      const int i0 = (f << log2N) + (grp << (lh + 1)) + j;
      double2 x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) x[r] = buf[i0 + r * h];
#pragma unroll
      for (int r = 0; r < 4; ++r) {  // half-span 4h, offset j + r h
        const double2 a = x[r], c = x[r + 4];
        x[r] = cadd(a, c);
        x[r + 4] = cmul(csub(a, c), tw[(j + r * h) << tsh]);
      }
#pragma unroll
      for (int r = 0; r < 8; r += (r & 1) ? 3 : 1) {  // r = 0, 1, 4, 5: half-span 2h, offset j + (r & 1) h
        const double2 a = x[r], c = x[r + 2];
        x[r] = cadd(a, c);
        x[r + 2] = cmul(csub(a, c), tw[(j + (r & 1) * h) << (tsh + 1)]);
      }
#pragma unroll
      for (int r = 0; r < 8; r += 2) {  // half-span h, offset j
        const double2 a = x[r], c = x[r + 1];
        x[r] = cadd(a, c);
        x[r + 1] = cmul(csub(a, c), tw[j << (tsh + 2)]);
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) buf[i0 + r * h] = x[r];
    }
    __syncthreads();
  }
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

// DIT stage with half-span H on a pair at offset o of its group: (a, c) -> (a + c w*, a - c w*),
// w = tw[o << (log2 N - 1 - log2 H)], w* its conjugate.  The one or two stages that log2 N
// leaves over when divided by three come first (radix-2 / radix-4), then radix-8 passes.
template <int NT>
__device__ __forceinline__ void fft_dit_inv(double2 *buf, int log2N, int nbatch,
                                            const double2 *__restrict__ tw) {
  const int N = 1 << log2N;
  int lh = 0;  // half-span of the next radix-2 stage is 2^lh
  if (log2N % 3 == 1) {  // the first radix-2 stage (half-span 1, twiddle 1)
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
  for (; log2N % 3 == 2 && lh == 0; lh += 2) {
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
  for (; lh < log2N; lh += 3) {
    // stages with half-spans h (= 2^lh), 2h and 4h: groups of 8h
    const int h = 1 << lh;
    const int q8 = N >> 3, tsh = log2N - 1 - lh;
    const int total = nbatch * q8;
    for (int b = threadIdx.x; b < total; b += NT) {
      const int f = b >> (log2N - 3), bb = b & (q8 - 1);
      const int j = bb & (h - 1), grp = bb >> lh;
      const int i0 = (f << log2N) + (grp << (lh + 3)) + j;
      double2 x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) x[r] = buf[i0 + r * h];
#pragma unroll
      for (int r = 0; r < 8; r += 2) {  // half-span h, offset j
        const double2 a = x[r], c = cmulc(x[r + 1], tw[j << tsh]);
        x[r] = cadd(a, c);
        x[r + 1] = csub(a, c);
      }
#pragma unroll
      for (int r = 0; r < 8; r += (r & 1) ? 3 : 1) {  // r = 0, 1, 4, 5: half-span 2h, offset j + (r & 1) h
        const double2 a = x[r], c = cmulc(x[r + 2], tw[(j + (r & 1) * h) << (tsh - 1)]);
        x[r] = cadd(a, c);
        x[r + 2] = csub(a, c);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {  // half-span 4h, offset j + r h
        const double2 a = x[r], c = cmulc(x[r + 4], tw[(j + r * h) << (tsh - 2)]);
        x[r] = cadd(a, c);
        x[r + 4] = csub(a, c);
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) buf[i0 + r * h] = x[r];
    }
    __syncthreads();
  }
}

}  // namespace fde
