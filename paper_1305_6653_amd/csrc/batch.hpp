// Per-instance descriptors shared by every kernel.  A launch covers a set of instances: the
// host passes, per launch, the prefix sums of the number of work items each instance
// contributes (`pre[0] = 0, pre[i+1] = pre[i] + items_i`) and the instance ids; a workgroup
// finds its instance by binary search and decodes its local item from that instance's sizes.
// A single solve is a batch of one.
#pragma once
#include <hip/hip_runtime.h>

namespace fde {

struct InstDesc {
  // sizes
  int m, s, mp, nb, npan, log2L, log2s, mu1, nu;
  int W;     // workgroups per block in the cooperative block solve
  int nblk;  // Krylov reduction blocks
  int need_ju0;  // the right-hand side uses J u_0 (a u_0 coefficient in B)
  double tau, scale;
  // operator tables
  const double *dp, *dm, *g;
  const double2 *chat, *twL, *tws, *lam, *mu;
  const int *band_c;
  const double *band_a, *band_b;
  // factors (complex FP64 or FP32 per the plan), block-solve flags (epoch of the last
  // published panel, [nb][npan][2])
  void *K, *dinv;
  unsigned long long *tsflags;
  // BCCB preconditioners (pc = 1: S2, 2: S2~ with the zero time frequency moved to lam0s):
  // chirp w_n = e^{-i pi n^2/m} [m], FFT_L of the chirp filter in bit-reversed order [L], and
  // the eigenvalues of s(J) [m]
  int pc;
  double lam0s;
  const double2 *chirp, *bh, *lamx;
  // Hessenberg route to the blocks (blk = 1): H, Q and Q^T of J = Q H Q^T (real, [m][mp]);
  // per block the multipliers and row exchanges of the shifted Hessenberg LU ([nb][mp]).
  // Vts is the frequency-domain vector the block solve works on: Vh for the LU route, a
  // second [nb][mp] buffer for the Hessenberg route (Q^T is applied out of place).
  int blk;
  const double *hH, *hQ, *hQt;
  double2 *hl;
  int *hpiv;
  double2 *Vts;
  // vectors (FP64, [s][m] unless noted)
  double *V, *Z;              // (R+1) and R vectors
  double *w, *x, *b, *tmp, *sio;
  double *u0, *f, *Ju0;       // [m], [s+1][m], [m]
  double2 *Vh;                // [nb][mp]
  double *part0, *part1;      // [nblk] reduction partials
  double *partm;              // [R+1][nblk] partials of the Gram-Schmidt projections
  double *H, *y, *nrm;        // Hessenberg column [R+2], LSQ solution [R], norms [2]
  double *h2;                 // [R+2] second Gram-Schmidt pass of the current column
  unsigned *gctr;             // [1] chunks done in the current Gram-Schmidt launch (0 between)
};

// vector selectors resolved on the device
enum VSel : int { VS_V = 0, VS_Z, VS_W, VS_X, VS_B, VS_TMP, VS_SIO, VS_U0, VS_JU0 };

__device__ __forceinline__ double *vsel(const InstDesc &d, int sel, int j) {
  const size_t n = (size_t)d.s * d.m;
  switch (sel) {
    case VS_V: return d.V + (size_t)j * n;
    case VS_Z: return d.Z + (size_t)j * n;
    case VS_W: return d.w;
    case VS_X: return d.x;
    case VS_B: return d.b;
    case VS_TMP: return d.tmp;
    case VS_SIO: return d.sio;
    case VS_U0: return d.u0;
    default: return d.Ju0;
  }
}

// Launch-wide item map: instance ids[count], prefix pre[count+1].  If gate is set, the
// items of instance i are skipped unless gate[i] != 0 (a device array written by earlier
// launches, so a fixed launch sequence can follow the instances' progress).
struct ItemMap {
  const int *ids;
  const int *pre;
  int count;
  const int *gate;
};

__device__ __forceinline__ bool item_gated(const ItemMap &mp, int q) {
  return mp.gate != nullptr && mp.gate[mp.ids[q]] == 0;
}

// Restarted GMRES control, one record per instance of a plan, advanced on the device between
// launches.  Restart lengths up to GM_RMAX.
static constexpr int GM_RMAX = 64;

struct GmresCtl {
  double bnorm;     // ||b||
  double tol;       // relative tolerance on ||b - M x|| / ||b||
  double truer;     // last true relative residual
  double est;       // Givens estimate of the relative residual
  int maxit, its, k, restarts;
  int conv, done, fail, active;  // active: taking part in the current cycle (mirrors the gate)
  int badrhs, pad;               // badrhs: ||b|| is not finite (set by k_gm_init)
};

struct GmresWork {
  double H[GM_RMAX + 1][GM_RMAX];  // rotated Hessenberg matrix of the current cycle
  double cs[GM_RMAX], sn[GM_RMAX], g[GM_RMAX + 1];
};

// gate arrays of a plan, [GATE_COUNT][count]
enum GateSel : int { GATE_LIVE = 0, GATE_ACTIVE, GATE_X0, GATE_COUNT };

// Returns the position q in the map with pre[q] <= item < pre[q+1].
// Workgroups are dispatched to the eight XCDs in turn (workgroup b to XCD b mod 8).  This
// bijection of [0, n) gives XCD x a contiguous range of item indices, so items that share data
// (neighbouring columns, the tiles of one block) are served by the same L2.
__device__ __forceinline__ int xcd_item(int bid, int n) {
  const int per = n >> 3, rem = n & 7, x = bid & 7;
  return x * per + (x < rem ? x : rem) + (bid >> 3);
}

__device__ __forceinline__ int item_slot(const ItemMap &mp, int item) {
  int lo = 0, hi = mp.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (mp.pre[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace fde
