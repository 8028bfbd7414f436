// Device helpers shared by the gfx950 kernels: complex arithmetic on interleaved
// (re, im) pairs, MFMA wrappers, wavefront (64-lane) reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fde {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct ctype;
template <> struct ctype<double> { typedef double2 type; typedef v4d acc; };
template <> struct ctype<float> { typedef float2 type; typedef v4f acc; };

template <typename T> using c_t = typename ctype<T>::type;
template <typename T> using acc_t = typename ctype<T>::acc;

template <typename T> __device__ __forceinline__ c_t<T> mk(T re, T im) { c_t<T> r; r.x = re; r.y = im; return r; }

// Loads through a global-address-space pointer.  A pointer read from memory (a descriptor's
// arrays) is generic, and a load through it is a flat load, which counts in lgkmcnt as well as
// vmcnt: the next wait for an LDS access would wait for it too, so a load issued ahead of LDS work
// would not stay in flight.  These are global loads (and stores), counted in vmcnt only.
template <typename V> __device__ __forceinline__ V gld(const V *p) {
  typedef __attribute__((address_space(1))) const V gV;
  return *(gV *)p;
}
template <typename V> __device__ __forceinline__ void gst(V *p, V v) {
  typedef __attribute__((address_space(1))) V gV;
  *(gV *)p = v;
}
// the HIP vector types copy through a generic this pointer: load and store them as native vectors
#define FDE_GLD_VEC(V, E)                                                   \
  template <> __device__ __forceinline__ V gld<V>(const V *p) {            \
    typedef E nv __attribute__((ext_vector_type(2)));                      \
    typedef __attribute__((address_space(1))) const nv gnv;                \
    const nv v = *(gnv *)p;                                                \
    V r;                                                                   \
    r.x = v.x;                                                             \
    r.y = v.y;                                                             \
    return r;                                                              \
  }                                                                        \
  template <> __device__ __forceinline__ void gst<V>(V * p, V v) {         \
    typedef E nv __attribute__((ext_vector_type(2)));                      \
    typedef __attribute__((address_space(1))) nv gnv;                      \
    nv w;                                                                  \
    w.x = v.x;                                                             \
    w.y = v.y;                                                             \
    *(gnv *)p = w;                                                         \
  }
FDE_GLD_VEC(double2, double)
FDE_GLD_VEC(float2, float)
#undef FDE_GLD_VEC

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// acc += a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ double2 widen(double2 a) { return a; }
__device__ __forceinline__ double2 widen(float2 a) { return make_double2((double)a.x, (double)a.y); }

// Generic complex ops for the factor type T (float or double), computed in T.
template <typename T> __device__ __forceinline__ c_t<T> tmul(c_t<T> a, c_t<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ c_t<T> tsub(c_t<T> a, c_t<T> b) {
  return mk<T>(a.x - b.x, a.y - b.y);
}
// 1 / a (scaled to avoid overflow; pivots here are far from the extremes)
template <typename T> __device__ __forceinline__ c_t<T> trecip(c_t<T> a) {
  T d = a.x * a.x + a.y * a.y;
  return mk<T>(a.x / d, -a.y / d);
}

// MFMA 16x16x4: D = A(16x4) * B(4x16) + C.  Operand lane layout on gfx950 (measured):
//   A[i][k] in lane i + 16k, B[k][j] in lane j + 16k for both types;
//   D element v of lane l is D[mfma_row<T>(l/16, v)][l%16] with
//   f32: row 4*(l/16) + v,   f64: row (l/16) + 4v.
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ constexpr int mfma_row(int lk, int v);
template <> __device__ __forceinline__ constexpr int mfma_row<float>(int lk, int v) { return 4 * lk + v; }
template <> __device__ __forceinline__ constexpr int mfma_row<double>(int lk, int v) { return lk + 4 * v; }

// 64-lane sum reductions (result valid in every lane).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double2 wave_sum(double2 v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

// 64-lane sum with DPP lane permutes instead of LDS shuffles: butterflies inside each 16-lane
// row (quad_perm [1,0,3,2], quad_perm [2,3,0,1], half-row mirror, row mirror leave the row sum
// in every lane of the row), then the four row sums in row order (fixed order; result valid
// in every lane).  Needs all 64 lanes active.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  const long long b = __double_as_longlong(v);
  const int lo = (int)(b & 0xffffffff), hi = (int)(b >> 32);
  double r = 0.0;
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    const long long x = ((long long)__builtin_amdgcn_readlane(hi, 16 * row) << 32) |
                        (unsigned)__builtin_amdgcn_readlane(lo, 16 * row);
    r += __longlong_as_double(x);
  }
  return r;
}

// Block sum in a fixed order (deterministic): wave tree, then waves in index order.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red /* >= NT/64 */) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += red[i];
  __syncthreads();
  return t;
}

__device__ __forceinline__ int bitrev(int k, int log2n) {
  return (int)(__brev((unsigned)k) >> (32 - log2n));
}

}  // namespace fde
