// Host-callable launchers of the gfx950 kernels.  All pointers are device pointers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace fde {

// Spatial operator J = dx^{-a} (D+ G + D- G^T) in Toeplitz-symbol form.
struct DevSpace {
  int m;
  int log2L;                // circulant embedding length L = 2^log2L >= 2m-1
  const double *dplus;      // [m]
  const double *dminus;     // [m]
  const double2 *chat_br;   // [L]  FFT_L of the first column of the embedding, bit-reversed order
  const double2 *twL;       // [L/2] e^{-2 pi i t/L}
  double scale;             // dx^{-alpha}
};

// BVM band tables of the s-form system: s-form row n is (s+1)-form row n+1, whose
// coefficients sit on (s+1)-form columns c[n] .. c[n]+mu.
struct DevBand {
  int s;
  int mu1;                  // mu + 1
  const int *c;             // [s]
  const double *a;          // [s][mu1]  Ahat coefficients
  const double *b;          // [s][mu1]  Bhat coefficients
};

hipError_t launch_symbol(const double *cG, double2 *chat_br, int log2L, const double2 *twL,
                         hipStream_t st);
// W[n] = sum_q a[n][q] Z[c+q-1] + coefJ * J (sum_q b[n][q] Z[c+q-1]),  columns < 0 skipped.
hipError_t launch_bvm_matvec(const double *Z, double *W, const DevSpace &sp, const DevBand &bd,
                             double coefJ, hipStream_t st);
// b[n] = tau sum_q b[n][q] f[c+q] - a0[n] u0 + tau b0[n] Ju0   (a0, b0: coefficient on u_0)
hipError_t launch_rhs(const double *f, const double *u0, const double *Ju0, double *b, int m,
                      const DevBand &bd, double tau, hipStream_t st);
hipError_t launch_time_rfft(const double *V, double2 *Vh, int m, int mp, int log2s,
                            const double2 *tws, hipStream_t st);
hipError_t launch_time_irfft(const double2 *Wh, double *W, int m, int mp, int log2s,
                             const double2 *tws, hipStream_t st);

// ---- preconditioner blocks (T = double or float factor storage) ----
template <typename T>
hipError_t launch_assemble(void *K, int m, int mp, int nb, const double2 *lam, const double2 *mu,
                           double tau, double scale, const double *g, const double *dp,
                           const double *dm, hipStream_t st);
template <typename T>
hipError_t launch_lu_diag(void *K, int mp, int nb, int p, void *dinv, int *flag, hipStream_t st);
template <typename T>
hipError_t launch_lu_panel(void *K, int mp, int nb, int p, const void *dinv, hipStream_t st);
template <typename T>
hipError_t launch_lu_update(void *K, int mp, int nb, int p, hipStream_t st);
template <typename T>
hipError_t launch_trsv(const void *K, const void *dinv, double2 *Vh, int mp, int nb, hipStream_t st);
// Several workgroups per block, cooperative launch; flags [nb][mp/64][2] hold the epoch of
// the last published panel; *err is raised if a dependency wait had to be abandoned.
template <typename T>
hipError_t launch_trsv_coop(const void *K, const void *dinv, double2 *Vh, int *flags, int mp,
                            int nb, int epoch, int *err, hipStream_t st);

// ---- Krylov BLAS-1 (FP64, deterministic reductions) ----
int krylov_blocks(size_t n);
hipError_t launch_mgs_step(int i, int j, double *V, double *w, size_t n, const double *part_in,
                           double *part_out, int nblk, double *Hcol, hipStream_t st);
hipError_t launch_normalize(const double *src, double *dst, size_t n, const double *part, int nblk,
                            double *out_norm, hipStream_t st);
hipError_t launch_residual(const double *b, const double *Mx, double *r, size_t n, double *part,
                           int nblk, hipStream_t st);
hipError_t launch_dot_partial(const double *x, const double *y, size_t n, double *part, int nblk,
                              hipStream_t st);
hipError_t launch_update_x(double *x, const double *Z, const double *y, int k, size_t n,
                           hipStream_t st);

}  // namespace fde
