// The per-instance control steps of restarted GMRES (Saad's GMRES, right preconditioning,
// flexible form), each run by one thread per instance: from the small launches of k_gmres.hip
// and from the fused one-chunk kernels of k_krylov.hip, so both give the same bits.  Every
// multiply-add is an explicit fma (or an explicitly rounded product), so that the compiler
// has no contraction to choose differently in the kernels these are inlined into.
#pragma once
#include "batch.hpp"

namespace fde {

// Restart decision from beta = ||r|| (nrm[0]): converged, failed, out of iterations, or a new
// cycle with g = beta e_1.
__device__ __forceinline__ void gm_restart_one(const InstDesc &d, GmresCtl &c, GmresWork &w,
                                               int *__restrict__ gates, int count, int i) {
  int *live = gates + GATE_LIVE * count, *act = gates + GATE_ACTIVE * count;
  act[i] = 0;
  c.active = 0;
  c.k = 0;
  if (c.done) {
    live[i] = 0;
    return;
  }
  const double beta = d.nrm[0];
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
  w.g[0] = beta;
  for (int r = 1; r <= GM_RMAX; ++r) w.g[r] = 0.0;
  live[i] = 1;
  act[i] = 1;
  c.active = 1;
}

// y = H^{-1} g for the k columns of the cycle (upper triangular back substitution), y[0] = k.
__device__ __forceinline__ void gm_backsolve_one(const InstDesc &d, GmresCtl &c, const GmresWork &w) {
  double *y = d.y;
  const int k = c.k;
  y[0] = (double)k;
  for (int r = k - 1; r >= 0; --r) {
    double t = w.g[r];
    for (int q = r + 1; q < k; ++q) t = fma(-w.H[r][q], y[1 + q], t);
    y[1 + r] = t / w.H[r][r];
  }
  if (k > 0) c.restarts += 1;
  c.k = 0;
}

// The same back substitution on a copy of H's k x k triangle and of g in LDS (Hs[r][q],
// gs[r]); y (y[0] = k, then the k coefficients) into ys.  The arithmetic of gm_backsolve_one.
__device__ __forceinline__ void gm_backsolve_lds(GmresCtl &c, const double (*Hs)[GM_RMAX + 1],
                                                 const double *gs, double *ys) {
  const int k = c.k;
  ys[0] = (double)k;
  for (int r = k - 1; r >= 0; --r) {
    double t = gs[r];
    for (int q = r + 1; q < k; ++q) t = fma(-Hs[r][q], ys[1 + q], t);
    ys[1 + r] = t / Hs[r][r];
  }
  if (k > 0) c.restarts += 1;
  c.k = 0;
}

// Givens update after Arnoldi step j: the previous rotations applied to the new Hessenberg
// column h_{0..j+1, j} (written by the orthogonalisation), the rotation that zeroes
// H[j+1][j], the residual estimate |g[j+1]| / ||b|| and the end-of-cycle decision.  The column
// hc, the previous rotations csp/snp and g[j] come in as arguments (global memory, or copies
// in LDS), the results go to w.
__device__ __forceinline__ void gm_givens_core(const double *hc, const double *csp, const double *snp,
                                               double gj, GmresCtl &c, GmresWork &w,
                                               int *__restrict__ gates, int count, int i, int j,
                                               int R) {
  int *live = gates + GATE_LIVE * count, *act = gates + GATE_ACTIVE * count;
  c.its += 1;
  // the column and the previous rotations are loaded together into registers (unrolled with
  // constant indices), then rotated through a carried value: no memory round trip per rotation
  double h[GM_RMAX + 1], cs[GM_RMAX], sn[GM_RMAX];
#pragma unroll
  for (int r = 0; r <= GM_RMAX; ++r) h[r] = r <= j + 1 ? hc[r] : 0.0;
#pragma unroll
  for (int r = 0; r < GM_RMAX; ++r) {
    cs[r] = r < j ? csp[r] : 0.0;
    sn[r] = r < j ? snp[r] : 0.0;
  }
  double a = h[0], b = h[1];  // rows j and j+1 of the column once rotation j-1 is applied
#pragma unroll
  for (int r = 0; r < GM_RMAX; ++r) {
    if (r < j) {
      const double hb = h[r + 1];
      w.H[r][j] = fma(cs[r], a, sn[r] * hb);
      a = fma(-sn[r], a, cs[r] * hb);
    }
    if (r == j) b = h[r + 1];
  }
  const double dd = hypot(a, b);
  const double cj = dd > 0.0 ? a / dd : 1.0, sj = dd > 0.0 ? b / dd : 0.0;
  w.cs[j] = cj;
  w.sn[j] = sj;
  w.H[j][j] = dd;
  w.H[j + 1][j] = 0.0;
  const double g1 = -sj * gj;
  w.g[j + 1] = g1;
  w.g[j] = cj * gj;
  c.k = j + 1;
  c.est = fabs(g1) / c.bnorm;
  if (!isfinite(c.est)) {  // the cycle is discarded; the solve reports the failure
    c.fail = 1;
    c.done = 1;
    c.k = 0;
    c.active = 0;
    act[i] = 0;
    live[i] = 0;
    return;
  }
  if (fabs(g1) <= c.tol * c.bnorm || c.its >= c.maxit || j + 1 >= R) {
    act[i] = 0;
    c.active = 0;
  }
}

// The same with every input read from global memory (the Givens launch).
__device__ __forceinline__ void gm_givens_one(const InstDesc &d, GmresCtl &c, GmresWork &w,
                                              int *__restrict__ gates, int count, int i, int j,
                                              int R) {
  gm_givens_core(d.H, w.cs, w.sn, w.g[j], c, w, gates, count, i, j, R);
}

}  // namespace fde
