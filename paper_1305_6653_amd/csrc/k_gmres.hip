// Restarted GMRES control on the device: the small per-instance updates between the
// Arnoldi launches (Givens rotations of the new Hessenberg column, the residual estimate,
// the least-squares back substitution, restart decisions).  Keeping them on the device
// lets a whole restart cycle run as a fixed launch sequence with no host round trip; the
// gate arrays written here switch off the items of instances that have finished, so
// batched instances that converge at different iterations share the sequence.
//
// The arithmetic is the textbook one of Saad's GMRES (right preconditioning, flexible
// form): rotation r of column j acts on rows (r, r+1); the new rotation zeroes H[j+1][j];
// |g[j+1]| is the residual norm of the current iterate; y solves the k x k upper
// triangular system H y = g.
#include "batch.hpp"
#include "kernels.hpp"

namespace fde {

static constexpr int GM_NT = 64;

__global__ __launch_bounds__(GM_NT) void k_gm_restart(const InstDesc *__restrict__ D,
                                                      GmresCtl *__restrict__ ctl,
                                                      GmresWork *__restrict__ work,
                                                      int *__restrict__ gates, int count) {
  const int i = blockIdx.x * GM_NT + threadIdx.x;
  if (i >= count) return;
  GmresCtl &c = ctl[i];
  int *live = gates + GATE_LIVE * count, *act = gates + GATE_ACTIVE * count;
  act[i] = 0;
  c.active = 0;
  c.k = 0;
  if (c.done) {
    live[i] = 0;
    return;
  }
  const double beta = D[i].nrm[0];
  c.truer = beta / c.bnorm;
  bool stop = false;
  if (!isfinite(beta)) {
    c.fail = 1;
    stop = true;
  } else if (beta <= c.tol * c.bnorm) {
    c.conv = 1;
    stop = true;
  } else if (c.its >= c.maxit) {
    stop = true;
  }
  if (stop) {
    c.done = 1;
    live[i] = 0;
    return;
  }
  GmresWork &w = work[i];
  w.g[0] = beta;
  for (int r = 1; r <= GM_RMAX; ++r) w.g[r] = 0.0;
  live[i] = 1;
  act[i] = 1;
  c.active = 1;
}

__global__ __launch_bounds__(GM_NT) void k_gm_givens(const InstDesc *__restrict__ D,
                                                     GmresCtl *__restrict__ ctl,
                                                     GmresWork *__restrict__ work,
                                                     int *__restrict__ gates, int count, int j,
                                                     int R) {
  const int i = blockIdx.x * GM_NT + threadIdx.x;
  if (i >= count) return;
  int *live = gates + GATE_LIVE * count, *act = gates + GATE_ACTIVE * count;
  if (!act[i]) return;
  GmresCtl &c = ctl[i];
  GmresWork &w = work[i];
  const double *hc = D[i].H;  // h_{0..j+1, j} from the Arnoldi launches
  c.its += 1;
  // the column and the previous rotations are loaded together into registers (unrolled with
  // constant indices), then rotated through a carried value: no memory round trip per rotation
  double h[GM_RMAX + 1], cs[GM_RMAX], sn[GM_RMAX];
#pragma unroll
  for (int r = 0; r <= GM_RMAX; ++r) h[r] = r <= j + 1 ? hc[r] : 0.0;
#pragma unroll
  for (int r = 0; r < GM_RMAX; ++r) {
    cs[r] = r < j ? w.cs[r] : 0.0;
    sn[r] = r < j ? w.sn[r] : 0.0;
  }
  double a = h[0], b = h[1];  // rows j and j+1 of the column once rotation j-1 is applied
#pragma unroll
  for (int r = 0; r < GM_RMAX; ++r) {
    if (r < j) {
      const double hb = h[r + 1];
      w.H[r][j] = cs[r] * a + sn[r] * hb;
      a = -sn[r] * a + cs[r] * hb;
    }
    if (r == j) b = h[r + 1];
  }
  const double dd = hypot(a, b);
  w.cs[j] = dd > 0.0 ? a / dd : 1.0;
  w.sn[j] = dd > 0.0 ? b / dd : 0.0;
  w.H[j][j] = dd;
  w.H[j + 1][j] = 0.0;
  w.g[j + 1] = -w.sn[j] * w.g[j];
  w.g[j] = w.cs[j] * w.g[j];
  c.k = j + 1;
  c.est = fabs(w.g[j + 1]) / c.bnorm;
  if (!isfinite(c.est)) {  // the cycle is discarded; the solve reports the failure
    c.fail = 1;
    c.done = 1;
    c.k = 0;
    c.active = 0;
    act[i] = 0;
    live[i] = 0;
    return;
  }
  if (fabs(w.g[j + 1]) <= c.tol * c.bnorm || c.its >= c.maxit || j + 1 >= R) {
    act[i] = 0;
    c.active = 0;
  }
}

__global__ __launch_bounds__(GM_NT) void k_gm_backsolve(const InstDesc *__restrict__ D,
                                                        GmresCtl *__restrict__ ctl,
                                                        GmresWork *__restrict__ work, int count) {
  const int i = blockIdx.x * GM_NT + threadIdx.x;
  if (i >= count) return;
  GmresCtl &c = ctl[i];
  const GmresWork &w = work[i];
  double *y = D[i].y;
  const int k = c.k;
  y[0] = (double)k;
  for (int r = k - 1; r >= 0; --r) {
    double t = w.g[r];
    for (int q = r + 1; q < k; ++q) t -= w.H[r][q] * y[1 + q];
    y[1 + r] = t / w.H[r][r];
  }
  if (k > 0) c.restarts += 1;
  c.k = 0;
}

static inline dim3 gm_grid(int count) { return dim3((count + GM_NT - 1) / GM_NT); }

hipError_t launch_gm_restart(const InstDesc *D, GmresCtl *ctl, GmresWork *work, int *gates,
                             int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gm_restart, gm_grid(count), dim3(GM_NT), 0, st, D, ctl, work, gates, count);
  return hipGetLastError();
}

hipError_t launch_gm_givens(const InstDesc *D, GmresCtl *ctl, GmresWork *work, int *gates,
                            int count, int j, int R, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gm_givens, gm_grid(count), dim3(GM_NT), 0, st, D, ctl, work, gates, count,
                     j, R);
  return hipGetLastError();
}

hipError_t launch_gm_backsolve(const InstDesc *D, GmresCtl *ctl, GmresWork *work, int count,
                               hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gm_backsolve, gm_grid(count), dim3(GM_NT), 0, st, D, ctl, work, count);
  return hipGetLastError();
}

}  // namespace fde
