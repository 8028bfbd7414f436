// Learned warm start: a small network that maps one problem instance (alpha, d+(x), d-(x),
// f(x,t) on the grid) to an initial guess of the all-at-once solution.  Everything runs
// here on gfx950: feature packing, bf16 MFMA GEMMs with FP32 accumulation (convolutions
// as im2col + GEMM), ReLU, the fixed synthesis basis, relative-MSE loss, backward pass and
// Adam.  Weights are kept as FP32 masters plus bf16 copies used by the GEMMs.
//
// Network (activations position-major, channels last):
//   X [B][256][Cin]                     Cin = (s+1) f-levels + d+ + d- + alpha
//   conv 5/2 -> relu -> [B][128][C1]    conv 5/2 -> relu -> [B][64][C2]
//   conv 5/2 -> relu -> [B][32][C3]     fc -> relu -> [B][F1]   fc -> relu -> [B][F2]
//   fc -> [B][NC] coefficients          synthesis U = c Bsyn, Bsyn [NC][s*m] fixed
// f is normalised by its RMS (the solution is linear in f when u0 = 0), and the target
// solution is divided by the same RMS.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fdebvm.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x) {
  // round to nearest even
  unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

// ---------------------------------------------------------------------------------------
// GEMM  C[M][N] (+)= op(A)[M][K] op(B)[K][N]; element (i,k) of op(A) is A[i*sa0 + k*sa1],
// element (k,j) of op(B) is B[k*sb0 + j*sb1].  A, B are FP32 or bf16 (TA/TB), converted to
// bf16 in LDS; v_mfma_f32_16x16x16_bf16 with FP32 accumulation.  64x64 tile per workgroup,
// 4 waves of 32x32.  Epilogue: + bias[j] (optional), ReLU (optional), accumulate into C
// (beta = 1) or overwrite.  Lane layout (measured): A[i][k] in lane i + 16*(k/4), element
// k%4; B[k][j] in lane j + 16*(k/4), element k%4; D[4*(lane/16) + v][lane%16].
template <typename T> __device__ __forceinline__ float ldf(const T *p, size_t i);
template <> __device__ __forceinline__ float ldf<float>(const float *p, size_t i) { return p[i]; }
template <> __device__ __forceinline__ float ldf<unsigned short>(const unsigned short *p, size_t i) {
  return bf2f(p[i]);
}

// Split-K: blockIdx.z handles k in [z*kc, (z+1)*kc); with gridDim.z > 1 the raw products go
// to ws[z][M][N] and k_splitk_reduce applies the epilogue after summing z in order.
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_gemm(const TA *__restrict__ A, long sa0, long sa1,
                                              const TB *__restrict__ B, long sb0, long sb1,
                                              float *__restrict__ Cm, int M, int N, int K,
                                              const float *__restrict__ bias, int relu, int beta,
                                              int kc, float *__restrict__ ws) {
  __shared__ unsigned short As[64][17];
  __shared__ unsigned short Bs[16][65];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int kbeg = blockIdx.z * kc, kend = min(K, kbeg + kc);
  v4f acc[2][2];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c)
      for (int v = 0; v < 4; ++v) acc[r][c][v] = 0.0f;
  for (int k0 = kbeg; k0 < kend; k0 += 16) {
    for (int e = tid; e < 64 * 16; e += 256) {
      const int ii = e >> 4, kk = e & 15;
      const int gi = i0 + ii, gk = k0 + kk;
      float a = 0.0f;
      if (gi < M && gk < kend) a = ldf<TA>(A, (size_t)gi * sa0 + (size_t)gk * sa1);
      As[ii][kk] = f2bf(a);
      const int jj = e & 63, kb = e >> 6;
      const int gj = j0 + jj, gkb = k0 + kb;
      float b = 0.0f;
      if (gj < N && gkb < kend) b = ldf<TB>(B, (size_t)gkb * sb0 + (size_t)gj * sb1);
      Bs[kb][jj] = f2bf(b);
    }
    __syncthreads();
    const int li = lane & 15, lk = (lane >> 4) * 4;
    v4s a[2], b[2];
    for (int r = 0; r < 2; ++r)
      for (int e = 0; e < 4; ++e) a[r][e] = (short)As[wr + r * 16 + li][lk + e];
    for (int c = 0; c < 2; ++c)
      for (int e = 0; e < 4; ++e) b[c][e] = (short)Bs[lk + e][wc + c * 16 + li];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c)
        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[r], b[c], acc[r][c], 0, 0, 0);
    __syncthreads();
  }
  const int li = lane & 15, lg = lane >> 4;
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c)
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wr + r * 16 + 4 * lg + v, gj = j0 + wc + c * 16 + li;
        if (gi >= M || gj >= N) continue;
        float x = acc[r][c][v];
        if (gridDim.z > 1) {
          ws[((size_t)blockIdx.z * M + gi) * N + gj] = x;
          continue;
        }
        if (bias) x += bias[gj];
        if (relu) x = x > 0.0f ? x : 0.0f;
        float *dst = Cm + (size_t)gi * N + gj;
        *dst = beta ? *dst + x : x;
      }
}

__global__ void k_splitk_reduce(const float *__restrict__ ws, int splits, int M, int N,
                                float *__restrict__ Cm, const float *__restrict__ bias, int relu,
                                int beta) {
  const size_t total = (size_t)M * N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    float x = 0.0f;
    for (int z = 0; z < splits; ++z) x += ws[(size_t)z * total + e];
    if (bias) x += bias[e % N];
    if (relu) x = x > 0.0f ? x : 0.0f;
    Cm[e] = beta ? Cm[e] + x : x;
  }
}

// im2col for a stride-2, width-5, pad-2 convolution over positions:
// cols[b*Lo + o][t*C + c] = X[b][2o + t - 2][c] (0 outside), X given as [B][L][C] with an
// optional row index map (rows of X taken from idx[b]).
__global__ void k_im2col(const float *__restrict__ X, const int *__restrict__ idx, int B, int L,
                         int C, int Lo, float *__restrict__ cols) {
  const size_t total = (size_t)B * Lo * 5 * C;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const size_t r = e / C;
    const int t = (int)(r % 5);
    const size_t ro = r / 5;
    const int o = (int)(ro % Lo), b = (int)(ro / Lo);
    const int src = 2 * o + t - 2;
    const int bb = idx ? idx[b] : b;
    cols[e] = (src >= 0 && src < L) ? X[((size_t)bb * L + src) * C + c] : 0.0f;
  }
}

// col2im (gather form): dX[b][i][c] = sum over taps t with (i + 2 - t) = 2o, 0 <= o < Lo, of
// dcols[b*Lo + o][t*C + c].
__global__ void k_col2im(const float *__restrict__ dcols, int B, int L, int C, int Lo,
                         float *__restrict__ dX) {
  const size_t total = (size_t)B * L * C;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const size_t r = e / C;
    const int i = (int)(r % L), b = (int)(r / L);
    float acc = 0.0f;
    for (int t = 0; t < 5; ++t) {
      const int num = i + 2 - t;
      if (num < 0 || (num & 1)) continue;
      const int o = num >> 1;
      if (o >= Lo) continue;
      acc += dcols[((size_t)b * Lo + o) * 5 * C + (size_t)t * C + c];
    }
    dX[e] = acc;
  }
}

// dpre = dY * (Y > 0)
__global__ void k_relu_bwd(const float *__restrict__ Y, float *__restrict__ dY, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    if (!(Y[e] > 0.0f)) dY[e] = 0.0f;
}

// db[j] = sum_i dY[i][j]  (fixed order)
__global__ void k_colsum(const float *__restrict__ dY, int rows, int cols, float *__restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float acc = 0.0f;
  for (int i = 0; i < rows; ++i) acc += dY[(size_t)i * cols + j];
  db[j] = acc;
}

// Relative MSE: loss_b = ||U_b - T_b/r_b||^2 / ||T_b/r_b||^2; dU = 2 (U - T/r) / (||T/r||^2 B).
// One workgroup per instance (rows of T taken through idx).  part[b] = loss_b.
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ U, const double *__restrict__ T,
                                              const float *__restrict__ rms, const int *__restrict__ idx,
                                              int n, int B, float *__restrict__ dU,
                                              float *__restrict__ part) {
  __shared__ float red[2][4];
  const int b = blockIdx.x;
  const int bb = idx ? idx[b] : b;
  const float inv = 1.0f / rms[bb];
  const float *u = U + (size_t)b * n;
  const double *t = T + (size_t)bb * n;
  float se = 0.0f, st = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float tv = (float)t[i] * inv, d = u[i] - tv;
    se += d * d;
    st += tv * tv;
  }
  for (int o = 32; o > 0; o >>= 1) {
    se += __shfl_xor(se, o, 64);
    st += __shfl_xor(st, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = se;
    red[1][threadIdx.x >> 6] = st;
  }
  __syncthreads();
  se = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  st = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  const float sc = 2.0f / (fmaxf(st, 1e-30f) * (float)B);
  if (dU)
    for (int i = threadIdx.x; i < n; i += 256) dU[(size_t)b * n + i] = sc * (u[i] - (float)t[i] * inv);
  if (threadIdx.x == 0) part[b] = se / fmaxf(st, 1e-30f);
}

// Adam on FP32 masters; refreshes the bf16 copies of the weights.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, unsigned short *__restrict__ pb, size_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const float gv = g[e];
    const float a = b1 * m1[e] + (1.0f - b1) * gv;
    const float v = b2 * m2[e] + (1.0f - b2) * gv * gv;
    m1[e] = a;
    m2[e] = v;
    const float x = p[e] - lr * (a / c1) / (sqrtf(v / c2) + eps);
    p[e] = x;
    pb[e] = f2bf(x);
  }
}

__global__ void k_to_bf16(const float *__restrict__ p, unsigned short *__restrict__ pb, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    pb[e] = f2bf(p[e]);
}

// Features of instance b: X[b][i][c] for i < 256 (i >= m is zero padding):
//   c <= s: f[c][i] / r, r = RMS of f over the (s+1) x m grid;  c = s+1: d+[i];  c = s+2: d-[i];
//   c = s+3: alpha - 1.5.   r is stored in rms[b].  f, dp, dm are FP64 [B] arrays of pointers.
__global__ __launch_bounds__(256) void k_features(const double *const *__restrict__ f,
                                                  const double *const *__restrict__ dp,
                                                  const double *const *__restrict__ dm,
                                                  const double *__restrict__ alpha, int m, int s,
                                                  float *__restrict__ X, float *__restrict__ rms) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  const int C = s + 4;
  const double *fb = f[b];
  const size_t nf = (size_t)(s + 1) * m;
  double acc = 0.0;
  for (size_t e = threadIdx.x; e < nf; e += 256) acc += fb[e] * fb[e];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  double r = sqrt((red[0] + red[1] + red[2] + red[3]) / (double)nf);
  if (!(r > 0.0)) r = 1.0;
  if (threadIdx.x == 0) rms[b] = (float)r;
  const double inv = 1.0 / r;
  float *xb = X + (size_t)b * 256 * C;
  for (int e = threadIdx.x; e < 256 * C; e += 256) {
    const int i = e / C, c = e % C;
    float v = 0.0f;
    if (i < m) {
      if (c <= s) v = (float)(fb[(size_t)c * m + i] * inv);
      else if (c == s + 1) v = (float)dp[b][i];
      else if (c == s + 2) v = (float)dm[b][i];
      else v = (float)(alpha[b] - 1.5);
    }
    xb[e] = v;
  }
}

// x0[b] = U[b] * rms[row b] (FP64 out, [s][m]); row b of the dataset is idx[b] (or b)
__global__ void k_scale_out(const float *__restrict__ U, const float *__restrict__ rms,
                            const int *__restrict__ idx, int n, double *const *__restrict__ out) {
  const int b = blockIdx.y;
  const float r = rms[idx ? idx[b] : b];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x)
    out[b][e] = (double)U[(size_t)b * n + e] * (double)r;
}

int grid1(size_t n) {
  size_t g = (n + 255) / 256;
  return (int)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

}  // namespace

// =========================================================================================
// host side
// =========================================================================================
static thread_local std::string g_nn_err;
static fde_status nn_fail(fde_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_nn_err = buf;
  return st;
}
#define NNCHK(...)                                                                                    \
  do {                                                                                                \
    hipError_t e_ = (__VA_ARGS__);                                                                    \
    if (e_ != hipSuccess) return nn_fail(FDE_EDEVICE, "%s: %s", #__VA_ARGS__, hipGetErrorString(e_)); \
  } while (0)

struct Layer {
  int kin, kout;     // GEMM K and N (conv: kin = 5 * Cin)
  int lin, lout;     // positions (conv) or 1 (fc)
  int cin;           // conv input channels
  bool conv, relu;
  size_t w_off, b_off;  // into the parameter vector (W [kin][kout] row-major, b [kout])
};

struct fde_nn {
  fde_nn_config cfg;
  int cin = 0, nc = 0, nout = 0;
  std::vector<Layer> layers;
  size_t nparam = 0;
  float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr, *bsyn = nullptr;
  unsigned short *pb = nullptr, *bsyn_b = nullptr;
  int maxB = 0;
  std::vector<float *> act;   // act[0] = X rows [B][256][Cin]; act[l+1] = layer l output
  std::vector<float *> cols;  // im2col buffers of conv layers
  float *coef = nullptr, *U = nullptr, *dU = nullptr, *dcoef = nullptr, *dA = nullptr,
        *dB = nullptr, *dcols = nullptr, *part = nullptr, *rms = nullptr;
  float *X = nullptr;  // features of the last fde_nn_features call
  float *ws = nullptr; // split-K partial products
  int *idx = nullptr;
  int step = 0;
  hipStream_t stream = nullptr;
  std::vector<void *> allocs;
};

static fde_status nn_alloc(fde_nn *n, void **p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return nn_fail(FDE_ENOMEM, "hipMalloc(%zu) failed", bytes);
  }
  n->allocs.push_back(*p);
  return FDE_OK;
}
template <typename P>
static fde_status nn_alloc_t(fde_nn *n, P **p, size_t count) {
  void *q = nullptr;
  fde_status st = nn_alloc(n, &q, count * sizeof(P));
  *p = (P *)q;
  return st;
}

static void nn_free(fde_nn *n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  for (void *p : n->allocs) (void)hipFree(p);
  delete n;
}

// Split-K workspace shared by all GEMMs of one network (stream-ordered use).
static constexpr size_t NN_WS_FLOATS = (size_t)16 << 20;

template <typename TA, typename TB>
static hipError_t gemm(hipStream_t st, float *ws, const TA *A, long sa0, long sa1, const TB *B,
                       long sb0, long sb1, float *Cm, int M, int N, int K, const float *bias,
                       int relu, int beta) {
  const int tiles = ((N + 63) / 64) * ((M + 63) / 64);
  int splits = 1;
  // fill the chip when the output has few tiles and K is long (>= 512 per split)
  while (splits < 64 && tiles * splits < 512 && K / (splits * 2) >= 512 &&
         (size_t)splits * 2 * M * N <= NN_WS_FLOATS)
    splits *= 2;
  const int kc = ((K + splits - 1) / splits + 15) / 16 * 16;
  splits = (K + kc - 1) / kc;
  dim3 grid((N + 63) / 64, (M + 63) / 64, splits);
  hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(256), 0, st, A, sa0, sa1, B, sb0, sb1, Cm, M, N, K,
                     bias, relu, beta, kc, ws);
  if (splits > 1) {
    hipLaunchKernelGGL(k_splitk_reduce, dim3(grid1((size_t)M * N)), dim3(256), 0, st, ws, splits, M,
                       N, Cm, bias, relu, beta);
  }
  return hipGetLastError();
}

extern "C" fde_status fde_nn_create(const fde_nn_config *c, fde_nn **out) {
  if (!c || !out) return nn_fail(FDE_EINVAL, "NULL argument");
  *out = nullptr;
  if (c->m < 1 || c->m > 256 || c->s < 2 || c->s > 512 || c->max_batch < 1 || c->conv_ch[0] < 1 ||
      c->conv_ch[1] < 1 || c->conv_ch[2] < 1 || c->fc[0] < 1 || c->fc[1] < 1 || c->nx < 1 || c->nt < 1)
    return nn_fail(FDE_EINVAL, "invalid network configuration");
  fde_nn *n = new fde_nn();
  n->cfg = *c;
  n->cin = c->s + 4;
  n->nc = c->nx * c->nt;
  n->nout = c->s * c->m;
  n->maxB = c->max_batch;
  const int ch[4] = {n->cin, c->conv_ch[0], c->conv_ch[1], c->conv_ch[2]};
  const int pos[4] = {256, 128, 64, 32};
  size_t off = 0;
  for (int l = 0; l < 3; ++l) {
    Layer L{5 * ch[l], ch[l + 1], pos[l], pos[l + 1], ch[l], true, true, 0, 0};
    L.w_off = off;
    off += (size_t)L.kin * L.kout;
    L.b_off = off;
    off += L.kout;
    n->layers.push_back(L);
  }
  const int fin[3] = {32 * ch[3], c->fc[0], c->fc[1]};
  const int fout[3] = {c->fc[0], c->fc[1], n->nc};
  for (int l = 0; l < 3; ++l) {
    Layer L{fin[l], fout[l], 1, 1, 0, false, l < 2, 0, 0};
    L.w_off = off;
    off += (size_t)L.kin * L.kout;
    L.b_off = off;
    off += L.kout;
    n->layers.push_back(L);
  }
  n->nparam = off;
  fde_status st = FDE_OK;
  auto bail = [&](fde_status s_) {
    nn_free(n);
    return s_;
  };
  if (hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking) != hipSuccess)
    return bail(nn_fail(FDE_EDEVICE, "stream creation failed"));
  const int B = n->maxB;
#define NA(ptr, cnt) \
  if ((st = nn_alloc_t(n, &(ptr), (cnt))) != FDE_OK) return bail(st)
  NA(n->p, off);
  NA(n->g, off);
  NA(n->m1, off);
  NA(n->m2, off);
  NA(n->pb, off);
  NA(n->bsyn, (size_t)n->nc * n->nout);
  NA(n->bsyn_b, (size_t)n->nc * n->nout);
  n->act.assign(7, nullptr);
  n->cols.assign(3, nullptr);
  NA(n->act[0], (size_t)B * 256 * n->cin);
  NA(n->X, (size_t)B * 256 * n->cin);
  size_t maxcols = 0;
  for (int l = 0; l < 6; ++l) {
    const Layer &L = n->layers[l];
    NA(n->act[l + 1], (size_t)B * L.lout * L.kout);
    if (L.conv) {
      NA(n->cols[l], (size_t)B * L.lout * L.kin);
      maxcols = std::max(maxcols, (size_t)B * L.lout * L.kin);
    }
  }
  size_t maxact = (size_t)B * 256 * n->cin;
  for (int l = 0; l < 6; ++l) maxact = std::max(maxact, (size_t)B * n->layers[l].lout * n->layers[l].kout);
  NA(n->U, (size_t)B * n->nout);
  NA(n->dU, (size_t)B * n->nout);
  NA(n->dA, maxact);
  NA(n->dB, maxact);
  NA(n->dcols, maxcols);
  NA(n->part, B);
  NA(n->rms, B);
  NA(n->idx, B);
  NA(n->ws, NN_WS_FLOATS);
#undef NA
  n->coef = n->act[6];
  // fixed synthesis basis Bsyn[q*nx + p][t*m + i] = cos(q pi t_{t+1}) sin((p+1) pi x_i / 2) / norm
  std::vector<float> bs((size_t)n->nc * n->nout);
  for (int q = 0; q < c->nt; ++q)
    for (int pp = 0; pp < c->nx; ++pp)
      for (int t = 0; t < c->s; ++t)
        for (int i = 0; i < c->m; ++i) {
          const double tt = (double)(t + 1) / c->s, xx = 2.0 * (i + 1) / (c->m + 1);
          bs[((size_t)(q * c->nx + pp)) * n->nout + (size_t)t * c->m + i] =
              (float)(std::cos(q * M_PI * tt) * std::sin((pp + 1) * M_PI * xx / 2.0) *
                      std::sqrt(2.0 / (c->s * c->m)));
        }
  if (hipMemcpy(n->bsyn, bs.data(), bs.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
    return bail(nn_fail(FDE_EDEVICE, "upload failed"));
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(bs.size())), dim3(256), 0, n->stream, n->bsyn, n->bsyn_b, bs.size());
  // He-style initialisation from a fixed-seed LCG (biases zero)
  std::vector<float> w(off, 0.0f);
  unsigned long long st64 = 0x9E3779B97F4A7C15ull ^ (unsigned long long)c->seed;
  auto urand = [&]() {
    st64 = st64 * 6364136223846793005ull + 1442695040888963407ull;
    return ((st64 >> 11) & ((1ull << 53) - 1)) * (1.0 / 9007199254740992.0);
  };
  for (const Layer &L : n->layers) {
    const double a = std::sqrt(6.0 / L.kin) * (L.relu ? 1.0 : 0.5);
    for (size_t e = 0; e < (size_t)L.kin * L.kout; ++e) w[L.w_off + e] = (float)((2.0 * urand() - 1.0) * a);
  }
  if (hipMemcpy(n->p, w.data(), off * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(n->m1, 0, off * sizeof(float)) != hipSuccess ||
      hipMemset(n->m2, 0, off * sizeof(float)) != hipSuccess ||
      hipMemset(n->g, 0, off * sizeof(float)) != hipSuccess)
    return bail(nn_fail(FDE_EDEVICE, "initialisation failed"));
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(off)), dim3(256), 0, n->stream, n->p, n->pb, off);
  if (hipStreamSynchronize(n->stream) != hipSuccess) return bail(nn_fail(FDE_EDEVICE, "sync failed"));
  *out = n;
  return FDE_OK;
}

extern "C" void fde_nn_destroy(fde_nn *n) { nn_free(n); }
extern "C" const char *fde_nn_last_error(void) { return g_nn_err.c_str(); }

extern "C" fde_status fde_nn_num_params(const fde_nn *n, long long *count) {
  if (!n || !count) return nn_fail(FDE_EINVAL, "NULL argument");
  *count = (long long)n->nparam;
  return FDE_OK;
}

extern "C" fde_status fde_nn_set_params(fde_nn *n, const float *host) {
  if (!n || !host) return nn_fail(FDE_EINVAL, "NULL argument");
  NNCHK(hipMemcpy(n->p, host, n->nparam * sizeof(float), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(n->nparam)), dim3(256), 0, n->stream, n->p, n->pb, n->nparam);
  NNCHK(hipStreamSynchronize(n->stream));
  return FDE_OK;
}

extern "C" fde_status fde_nn_set_basis(fde_nn *n, const float *host) {
  if (!n || !host) return nn_fail(FDE_EINVAL, "NULL argument");
  const size_t cnt = (size_t)n->nc * n->nout;
  NNCHK(hipMemcpy(n->bsyn, host, cnt * sizeof(float), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(cnt)), dim3(256), 0, n->stream, n->bsyn, n->bsyn_b, cnt);
  NNCHK(hipStreamSynchronize(n->stream));
  return FDE_OK;
}

extern "C" fde_status fde_nn_get_params(const fde_nn *n, float *host, int which) {
  if (!n || !host) return nn_fail(FDE_EINVAL, "NULL argument");
  const float *src = which == 0 ? n->p : which == 1 ? n->g : which == 2 ? n->m1 : which == 3 ? n->m2 : nullptr;
  if (!src) return nn_fail(FDE_EINVAL, "which must be 0 (params), 1 (grads), 2, 3 (Adam moments)");
  NNCHK(hipStreamSynchronize(n->stream));
  NNCHK(hipMemcpy(host, src, n->nparam * sizeof(float), hipMemcpyDeviceToHost));
  return FDE_OK;
}

extern "C" fde_status fde_nn_set_state(fde_nn *n, const float *m1, const float *m2, int step) {
  if (!n || !m1 || !m2 || step < 0) return nn_fail(FDE_EINVAL, "invalid argument");
  NNCHK(hipMemcpy(n->m1, m1, n->nparam * sizeof(float), hipMemcpyHostToDevice));
  NNCHK(hipMemcpy(n->m2, m2, n->nparam * sizeof(float), hipMemcpyHostToDevice));
  n->step = step;
  return FDE_OK;
}

extern "C" fde_status fde_nn_get_step(const fde_nn *n, int *step) {
  if (!n || !step) return nn_fail(FDE_EINVAL, "NULL argument");
  *step = n->step;
  return FDE_OK;
}

extern "C" fde_status fde_nn_features(fde_nn *n, int B, const double *const *f, const double *const *dp,
                                      const double *const *dm, const double *alpha, float *X,
                                      float *rms) {
  if (!n || !f || !dp || !dm || !alpha || !X || !rms || B < 1)
    return nn_fail(FDE_EINVAL, "invalid argument");
  // pointer arrays and alpha are host arrays; f, dp, dm point to device FP64 data
  std::vector<const double *> pf(f, f + B), pp(dp, dp + B), pm(dm, dm + B);
  const double **d_ptr = nullptr;
  double *d_alpha = nullptr;
  NNCHK(hipMalloc((void **)&d_ptr, 3 * B * sizeof(void *)));
  NNCHK(hipMalloc((void **)&d_alpha, B * sizeof(double)));
  std::vector<const double *> all;
  all.insert(all.end(), pf.begin(), pf.end());
  all.insert(all.end(), pp.begin(), pp.end());
  all.insert(all.end(), pm.begin(), pm.end());
  hipError_t e = hipMemcpy(d_ptr, all.data(), all.size() * sizeof(void *), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_alpha, alpha, B * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_features, dim3(B), dim3(256), 0, n->stream, d_ptr, d_ptr + B, d_ptr + 2 * B,
                       d_alpha, n->cfg.m, n->cfg.s, X, rms);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  (void)hipFree(d_ptr);
  (void)hipFree(d_alpha);
  if (e != hipSuccess) return nn_fail(FDE_EDEVICE, "features: %s", hipGetErrorString(e));
  return FDE_OK;
}

// forward over rows idx[0..B) of X (device features [*][256][Cin]); result in n->U, n->coef
static fde_status nn_forward(fde_nn *n, const float *X, const int *idx, int B) {
  hipStream_t st = n->stream;
  const float *in = X;
  const int *rows = idx;
  for (int l = 0; l < 6; ++l) {
    const Layer &L = n->layers[l];
    float *outp = n->act[l + 1];
    const float *bias = n->p + L.b_off;
    const unsigned short *W = n->pb + L.w_off;
    if (L.conv) {
      const size_t tot = (size_t)B * L.lout * L.kin;
      hipLaunchKernelGGL(k_im2col, dim3(grid1(tot)), dim3(256), 0, st, in, rows, B, L.lin, L.cin,
                         L.lout, n->cols[l]);
      NNCHK(hipGetLastError());
      NNCHK(gemm<float, unsigned short>(st, n->ws, n->cols[l], L.kin, 1, W, L.kout, 1, outp, B * L.lout,
                                        L.kout, L.kin, bias, L.relu ? 1 : 0, 0));
    } else {
      NNCHK(gemm<float, unsigned short>(st, n->ws, in, L.kin, 1, W, L.kout, 1, outp, B, L.kout, L.kin, bias,
                                        L.relu ? 1 : 0, 0));
    }
    in = outp;
    rows = nullptr;
  }
  // synthesis U = coef Bsyn
  NNCHK(gemm<float, unsigned short>(st, n->ws, n->coef, n->nc, 1, n->bsyn_b, n->nout, 1, n->U, B, n->nout,
                                    n->nc, nullptr, 0, 0));
  return FDE_OK;
}

static fde_status nn_backward(fde_nn *n, const float *X, const int *idx, int B) {
  hipStream_t st = n->stream;
  NNCHK(hipMemsetAsync(n->g, 0, n->nparam * sizeof(float), st));
  // dcoef = dU Bsyn^T
  float *dY = n->dA, *dX = n->dB;
  NNCHK(gemm<float, unsigned short>(st, n->ws, n->dU, n->nout, 1, n->bsyn_b, 1, n->nout, dY, B, n->nc,
                                    n->nout, nullptr, 0, 0));
  for (int l = 5; l >= 0; --l) {
    const Layer &L = n->layers[l];
    const float *Y = n->act[l + 1];
    const int rowsN = L.conv ? B * L.lout : B;
    if (L.relu) {
      hipLaunchKernelGGL(k_relu_bwd, dim3(grid1((size_t)rowsN * L.kout)), dim3(256), 0, st, Y, dY,
                         (size_t)rowsN * L.kout);
      NNCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_colsum, dim3((L.kout + 255) / 256), dim3(256), 0, st, dY, rowsN, L.kout,
                       n->g + L.b_off);
    NNCHK(hipGetLastError());
    // dW = in^T dY   (in = cols for conv, previous activation for fc)
    const float *in = L.conv ? n->cols[l] : n->act[l];
    NNCHK(gemm<float, float>(st, n->ws, in, 1, L.kin, dY, L.kout, 1, n->g + L.w_off, L.kin, L.kout, rowsN,
                             nullptr, 0, 0));
    if (l == 0) break;
    // d(in) = dY W^T
    const unsigned short *W = n->pb + L.w_off;
    if (L.conv) {
      NNCHK(gemm<float, unsigned short>(st, n->ws, dY, L.kout, 1, W, 1, L.kout, n->dcols, rowsN, L.kin,
                                        L.kout, nullptr, 0, 0));
      const size_t tot = (size_t)B * L.lin * L.cin;
      hipLaunchKernelGGL(k_col2im, dim3(grid1(tot)), dim3(256), 0, st, n->dcols, B, L.lin, L.cin,
                         L.lout, dX);
      NNCHK(hipGetLastError());
    } else {
      NNCHK(gemm<float, unsigned short>(st, n->ws, dY, L.kout, 1, W, 1, L.kout, dX, rowsN, L.kin, L.kout,
                                        nullptr, 0, 0));
    }
    std::swap(dY, dX);
  }
  (void)X;
  (void)idx;
  return FDE_OK;
}

static fde_status upload_idx(fde_nn *n, const int *idx, int B, const int **didx) {
  if (!idx) {
    *didx = nullptr;
    return FDE_OK;
  }
  NNCHK(hipMemcpyAsync(n->idx, idx, B * sizeof(int), hipMemcpyHostToDevice, n->stream));
  NNCHK(hipStreamSynchronize(n->stream));
  *didx = n->idx;
  return FDE_OK;
}

extern "C" fde_status fde_nn_loss_grad(fde_nn *n, const float *X, const double *T, const float *rms,
                                       const int *idx, int B, float *loss) {
  if (!n || !X || !T || !rms || B < 1 || B > n->maxB) return nn_fail(FDE_EINVAL, "invalid argument");
  const int *didx = nullptr;
  fde_status s0 = upload_idx(n, idx, B, &didx);
  if (s0 != FDE_OK) return s0;
  s0 = nn_forward(n, X, didx, B);
  if (s0 != FDE_OK) return s0;
  hipLaunchKernelGGL(k_loss, dim3(B), dim3(256), 0, n->stream, n->U, T, rms, didx, n->nout, B, n->dU, n->part);
  NNCHK(hipGetLastError());
  s0 = nn_backward(n, X, didx, B);
  if (s0 != FDE_OK) return s0;
  if (loss) {
    std::vector<float> part(B);
    NNCHK(hipMemcpyAsync(part.data(), n->part, B * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    NNCHK(hipStreamSynchronize(n->stream));
    double t = 0;
    for (float v : part) t += v;
    *loss = (float)(t / B);
  }
  return FDE_OK;
}

extern "C" fde_status fde_nn_adam(fde_nn *n, float lr, float beta1, float beta2, float eps) {
  if (!n || !(lr > 0)) return nn_fail(FDE_EINVAL, "invalid argument");
  n->step += 1;
  const float c1 = 1.0f - std::pow(beta1, (float)n->step), c2 = 1.0f - std::pow(beta2, (float)n->step);
  hipLaunchKernelGGL(k_adam, dim3(grid1(n->nparam)), dim3(256), 0, n->stream, n->p, n->g, n->m1, n->m2,
                     n->pb, n->nparam, lr, beta1, beta2, eps, c1, c2);
  NNCHK(hipGetLastError());
  return FDE_OK;
}

extern "C" fde_status fde_nn_predict(fde_nn *n, const float *X, const float *rms, const int *idx, int B,
                                     double *const *x0) {
  if (!n || !X || !rms || !x0 || B < 1 || B > n->maxB) return nn_fail(FDE_EINVAL, "invalid argument");
  const int *didx = nullptr;
  fde_status s0 = upload_idx(n, idx, B, &didx);
  if (s0 != FDE_OK) return s0;
  s0 = nn_forward(n, X, didx, B);
  if (s0 != FDE_OK) return s0;
  double **d_out = nullptr;
  NNCHK(hipMalloc((void **)&d_out, B * sizeof(double *)));
  hipError_t e = hipMemcpy(d_out, x0, B * sizeof(double *), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_scale_out, dim3((n->nout + 255) / 256, B), dim3(256), 0, n->stream, n->U, rms,
                       didx, n->nout, d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  (void)hipFree(d_out);
  if (e != hipSuccess) return nn_fail(FDE_EDEVICE, "predict: %s", hipGetErrorString(e));
  return FDE_OK;
}

extern "C" fde_status fde_nn_output(const fde_nn *n, float *host, int B) {
  if (!n || !host || B < 1 || B > n->maxB) return nn_fail(FDE_EINVAL, "invalid argument");
  NNCHK(hipStreamSynchronize(n->stream));
  NNCHK(hipMemcpy(host, n->U, (size_t)B * n->nout * sizeof(float), hipMemcpyDeviceToHost));
  return FDE_OK;
}

extern "C" fde_status fde_nn_sync(fde_nn *n) {
  if (!n) return nn_fail(FDE_EINVAL, "NULL argument");
  NNCHK(hipStreamSynchronize(n->stream));
  return FDE_OK;
}
