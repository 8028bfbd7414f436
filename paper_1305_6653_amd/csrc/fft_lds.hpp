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

template <int NT>
__device__ __forceinline__ void fft_dif(double2 *buf, int log2N, int nbatch,
                                        const double2 *__restrict__ tw) {
  const int half = 1 << (log2N - 1);
  const int total = nbatch * half;
  for (int lh = log2N - 1; lh >= 0; --lh) {
    const int h = 1 << lh;
    const int tsh = log2N - 1 - lh;  // twiddle stride N/(2h)
    for (int b = threadIdx.x; b < total; b += NT) {
      const int f = b >> (log2N - 1), bb = b & (half - 1);
      const int j = bb & (h - 1), grp = bb >> lh;
      const int i0 = (f << log2N) + (grp << (lh + 1)) + j, i1 = i0 + h;
      const double2 a = buf[i0], c = buf[i1];
      const double2 w = tw[j << tsh];
      buf[i0] = cadd(a, c);
      buf[i1] = cmul(csub(a, c), w);
    }
    __syncthreads();
  }
}

template <int NT>
__device__ __forceinline__ void fft_dit_inv(double2 *buf, int log2N, int nbatch,
                                            const double2 *__restrict__ tw) {
  const int half = 1 << (log2N - 1);
  const int total = nbatch * half;
  for (int lh = 0; lh < log2N; ++lh) {
    const int h = 1 << lh;
    const int tsh = log2N - 1 - lh;
    for (int b = threadIdx.x; b < total; b += NT) {
      const int f = b >> (log2N - 1), bb = b & (half - 1);
      const int j = bb & (h - 1), grp = bb >> lh;
      const int i0 = (f << log2N) + (grp << (lh + 1)) + j, i1 = i0 + h;
      const double2 a = buf[i0];
      const double2 c = cmulc(buf[i1], tw[j << tsh]);  // times e^{+2 pi i ...}
      buf[i0] = cadd(a, c);
      buf[i1] = csub(a, c);
    }
    __syncthreads();
  }
}

}  // namespace fde
