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
#include "gmres_step.hpp"
#include "kernels.hpp"

namespace fde {

static constexpr int GM_NT = 64;

__global__ __launch_bounds__(GM_NT) void k_gm_restart(const InstDesc *__restrict__ D,
                                                      GmresCtl *__restrict__ ctl,
                                                      GmresWork *__restrict__ work,
                                                      int *__restrict__ gates, int count) {
  const int i = blockIdx.x * GM_NT + threadIdx.x;
  if (i >= count) return;
  gm_restart_one(D[i], ctl[i], work[i], gates, count, i);
}

__global__ __launch_bounds__(GM_NT) void k_gm_givens(const InstDesc *__restrict__ D,
                                                     GmresCtl *__restrict__ ctl,
                                                     GmresWork *__restrict__ work,
                                                     int *__restrict__ gates, int count, int j,
                                                     int R) {
  const int i = blockIdx.x * GM_NT + threadIdx.x;
  if (i >= count) return;
  if (!gates[GATE_ACTIVE * count + i]) return;
  gm_givens_one(D[i], ctl[i], work[i], gates, count, i, j, R);
}

__global__ __launch_bounds__(GM_NT) void k_gm_backsolve(const InstDesc *__restrict__ D,
                                                        GmresCtl *__restrict__ ctl,
                                                        GmresWork *__restrict__ work, int count) {
  const int i = blockIdx.x * GM_NT + threadIdx.x;
  if (i >= count) return;
  gm_backsolve_one(D[i], ctl[i], work[i]);
}

// Control records and gates of a zero-start solve, on the device: ||b|| from the partials of
// the preceding dot launch (summed in index order, as the host does), tolerance and iteration
// limit; b = 0 ends the instance at once (x is already zero); a non-finite ||b|| ends it with
// badrhs set, for the host to report.
__global__ __launch_bounds__(GM_NT) void k_gm_init(const InstDesc *__restrict__ D,
                                                   GmresCtl *__restrict__ ctl,
                                                   int *__restrict__ gates, int count, double tol,
                                                   int maxit) {
  const int i = blockIdx.x * GM_NT + threadIdx.x;
  if (i >= count) return;
  const InstDesc &d = D[i];
  double t = 0.0;
  for (int q = 0; q < d.nblk; ++q) t += d.part0[q];
  GmresCtl c{};
  c.bnorm = sqrt(t);
  c.tol = tol;
  c.maxit = maxit;
  if (!isfinite(c.bnorm)) {
    c.badrhs = 1;
    c.done = 1;
  } else if (c.bnorm == 0.0) {
    c.done = c.conv = 1;
  }
  ctl[i] = c;
  gates[GATE_LIVE * count + i] = c.done ? 0 : 1;
  gates[GATE_ACTIVE * count + i] = 0;
  gates[GATE_X0 * count + i] = 0;
}

hipError_t launch_gm_init(const InstDesc *D, GmresCtl *ctl, int *gates, int count, double tol,
                          int maxit, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gm_init, dim3((count + GM_NT - 1) / GM_NT), dim3(GM_NT), 0, st, D, ctl, gates,
                     count, tol, maxit);
  return hipGetLastError();
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
