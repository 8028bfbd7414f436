// Host-callable launchers of the gfx950 kernels.  Every launcher takes the device array of
// instance descriptors, the launch's item map (device pointers) and the total item count;
// all other pointers are device pointers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "batch.hpp"

namespace fde {

hipError_t launch_symbol(const double *cG, double2 *chat_br, int log2L, const double2 *twL,
                         hipStream_t st);

// mode 0: W[n] = sum_q a[n][q] Z[c+q-1] - tau J (sum_q b[n][q] Z[c+q-1]),  items = s per instance
// mode 1: W[n] = J Z[n],                                                  items = rows per instance
hipError_t launch_bvm_matvec(const InstDesc *D, const ItemMap &map, int items, int max_log2L,
                             int src_sel, int src_j, int dst_sel, int dst_j, int mode,
                             hipStream_t st);
// b = tau Bhat f - a0 u0 (+ tau b0 J u0), items = s per instance
hipError_t launch_rhs(const InstDesc *D, const ItemMap &map, int items, int use_ju0, hipStream_t st);
// items = mp / cols per instance, cols = time_fft_cols_per_item(sum of mp, CUs) (4, 8 or 16).
// With epoch_ctr set, the launch also draws the next block-solve epoch into *epoch_slot (see
// launch_trsv_coop).
hipError_t launch_time_rfft(const InstDesc *D, const ItemMap &map, int items, int max_log2s,
                            int cols, int src_sel, int src_j, hipStream_t st,
                            unsigned long long *epoch_ctr = nullptr,
                            unsigned long long *epoch_slot = nullptr);
hipError_t launch_time_irfft(const InstDesc *D, const ItemMap &map, int items, int max_log2s,
                             int cols, int dst_sel, int dst_j, hipStream_t st);
int time_fft_cols_per_item(long long total_mp, int cus);
// BCCB preconditioner solve in the time-frequency domain: for every time frequency k < nb,
// Vh[k] <- F_m^{-1} diag(1 / (lam_k - tau mu_k lamx)) F_m Vh[k] (space DFTs of order m by
// Bluestein's chirp method on the power-of-two FFT of length L).  items = nb per instance.
hipError_t launch_bccb_solve(const InstDesc *D, const ItemMap &map, int items, int max_log2L,
                             hipStream_t st);

// ---- preconditioner blocks (T = double or float factor storage) ----
int assemble_items(int mp, int nb);
// rows and columns of every block written by the assembly (the first trailing update forms
// the rest)
int assemble_lead();
template <typename T>
hipError_t launch_assemble(const InstDesc *D, const ItemMap &map, int items, hipStream_t st);
// items: nb (diag), 2 nrem nb (panel), nrem^2 nb (update) per instance, nrem = mp/64 - p - 1
template <typename T>
hipError_t launch_lu_diag(const InstDesc *D, const ItemMap &map, int items, int p, int *flag,
                          hipStream_t st);
template <typename T>
hipError_t launch_lu_panel(const InstDesc *D, const ItemMap &map, int items, int p, hipStream_t st);
// trailing update of panel step p, mode 0: every tile (nrem^2 items per block, K = 64);
// 1: the first tile row and column (2 nrem - 1); 2: the other tiles with the updates of steps
// p and p + 1 together ((nrem - 1)^2, K = 128)
template <typename T>
hipError_t launch_lu_update(const InstDesc *D, const ItemMap &map, int items, int p, int mode,
                            hipStream_t st);
// one workgroup per block, an ordinary launch with no flags: items = nb W per instance (the
// item k W solves block k); the same panel arithmetic as launch_trsv_coop, so the same bits.
// first_sweep = 1 runs the U sweep only.
template <typename T>
hipError_t launch_trsv(const InstDesc *D, const ItemMap &map, int items, int first_sweep,
                       hipStream_t st);
// several workgroups per block (descriptor field W), cooperative launch: items = nb W per
// instance; flags in the descriptors hold the epoch of the last published panel; the epoch of
// this launch is read from *epoch (device memory, written by the preceding time FFT); *err is
// raised if a dependency wait had to be abandoned.  first_sweep = 1 runs the U sweep only (the
// Hessenberg route, whose lower factor is applied by launch_hess_lsolve).  With blkmap (items =
// nb per instance, nblk in all) and npan_u > 0 (every instance has npan_u panels) the panels
// are claimed from the counter epoch[1] instead, which the preceding time FFT resets.
template <typename T>
hipError_t launch_trsv_coop(const InstDesc *D, const ItemMap &map, int items,
                            const unsigned long long *epoch, int *err, hipStream_t st,
                            int first_sweep = 0, const ItemMap *blkmap = nullptr, int nblk = 0,
                            int npan_u = 0);
// co-resident workgroups of the cooperative block solve on this device (0 if unknown)
template <typename T>
int trsv_coop_capacity();

// ---- Krylov BLAS-1 (FP64, deterministic reductions), items = nblk per instance ----
int krylov_blocks(size_t n);
// largest vector length that krylov_blocks makes one chunk
size_t krylov_one_max();
// Arnoldi step j in one launch when every instance's vectors are one chunk (n <= max_n <=
// krylov_one_max()): the MGS projections, the norm, v_{j+1} and the Givens update of the
// control record (the work of launch_mgs_step i = 0..j+1, launch_normalize and
// launch_gm_givens), with the same bits.  items = 1 per instance (the Krylov map).
hipError_t launch_arnoldi1(const InstDesc *D, const ItemMap &map, int items, size_t max_n, int j,
                           GmresCtl *ctl, GmresWork *work, int *gates, int count, int R,
                           hipStream_t st);
// The same for the restart step's tail (residual, its norm, v_0, the restart decision) and
// for the end of a cycle (back substitution, x += Q y), one-chunk instances only; items = 1
// per instance (the Krylov map; its gate is ignored: the kernels read the live gate).
hipError_t launch_restart1(const InstDesc *D, const ItemMap &map, int items, size_t max_n,
                           GmresCtl *ctl, GmresWork *work, int *gates, int count, hipStream_t st);
hipError_t launch_finish1(const InstDesc *D, const ItemMap &map, int items, size_t max_n,
                          GmresCtl *ctl, const GmresWork *work, const int *gates, int count,
                          int basis_sel, hipStream_t st);
// Modified Gram-Schmidt step i of Arnoldi column j (i = 0..j+1, one launch each): h_{i-1} from
// the partials of launch i-1, w -= h_{i-1} v_{i-1}, partial <v_i, w> (<w, w> for i = j+1).
hipError_t launch_mgs_step(const InstDesc *D, const ItemMap &map, int items, int i, int j,
                           hipStream_t st);
// Arnoldi orthogonalisation by classical Gram-Schmidt twice (k_krylov.hip), items = chunks:
// V^T w (the last chunk writes H[0..j]); w -= V H then pass 0: V^T w again (the last chunk
// writes h2 and adds it to H), pass 1: w -= V h2 and the norm partial.
hipError_t launch_cgs_dot(const InstDesc *D, const ItemMap &map, int items, int j, hipStream_t st);
hipError_t launch_cgs_update(const InstDesc *D, const ItemMap &map, int items, int j, int pass,
                             hipStream_t st);
hipError_t launch_normalize(const InstDesc *D, const ItemMap &map, int items, int src_sel,
                            int src_j, int dst_sel, int dst_j, int psel, int hidx, hipStream_t st);
hipError_t launch_residual(const InstDesc *D, const ItemMap &map, int items, hipStream_t st);
hipError_t launch_dot_partial(const InstDesc *D, const ItemMap &map, int items, int xsel, int ysel,
                              int psel, hipStream_t st);
// dst += a src (vector selectors)
hipError_t launch_axpy(const InstDesc *D, const ItemMap &map, int items, int dst_sel, int src_sel,
                       double a, hipStream_t st);
// x *= y[0] per instance
hipError_t launch_scale_x(const InstDesc *D, const ItemMap &map, int items, hipStream_t st);
hipError_t launch_update_x(const InstDesc *D, const ItemMap &map, int items, int basis_sel,
                           hipStream_t st);
hipError_t launch_copy(const InstDesc *D, const ItemMap &map, int items, int src_sel, int src_j,
                       int dst_sel, int dst_j, hipStream_t st);

// ---- restarted GMRES control on the device (one thread per instance of the plan) ----
// restart: beta = nrm[0] of every live instance -> converged / out of iterations / new cycle;
// sets gate[GATE_LIVE] and gate[GATE_ACTIVE].
// control records and gates of a zero-start solve from the partials of <b, b> in part0
hipError_t launch_gm_init(const InstDesc *D, GmresCtl *ctl, int *gates, int count, double tol,
                          int maxit, hipStream_t st);
hipError_t launch_gm_restart(const InstDesc *D, GmresCtl *ctl, GmresWork *work, int *gates,
                             int count, hipStream_t st);
// Arnoldi step j done: rotate the new Hessenberg column, update the residual estimate and
// retire instances that converged, ran out of iterations or reached the end of the cycle.
hipError_t launch_gm_givens(const InstDesc *D, GmresCtl *ctl, GmresWork *work, int *gates,
                            int count, int j, int R, hipStream_t st);
// end of cycle: y = H^{-1} g into the descriptors' y (y[0] = k, 0 if the instance did not run)
hipError_t launch_gm_backsolve(const InstDesc *D, GmresCtl *ctl, GmresWork *work, int count,
                               hipStream_t st);

// ---- Hessenberg route to the blocks (k_hessenberg.hip) ----
// Workspace of one reduction of an instance of order m (mp padded, G workgroups):
// sync [G] (arrival flags), err [1], vbuf [mp] (column snapshot), part [G][2][mp],
// ybuf [2][mp]; outputs H, Q, Q^T [m][mp] row-major.
struct HessWork {
  unsigned *sync;
  int *err;
  double *vbuf, *part, *ybuf;
  double *H, *Q, *Qt;
};
int hess_reduce_groups(int m);   // G
int hess_reduce_max_m();         // largest order the register-resident reduction takes
// J = Q H Q^T of instance `inst` of D (cooperative launch; err set if it could not finish)
hipError_t launch_hess_reduce(const InstDesc *D, int inst, int m, const HessWork &wk, hipStream_t st);
// item = (instance, block): pivoted LU of lambda_k I - tau mu_k H into K (upper part), hl, hpiv
template <typename T>
hipError_t launch_hess_lu(const InstDesc *D, const ItemMap &map, int items, int max_mp, int *flag,
                          hipStream_t st);
// item = (instance, block, panel): inverse of U's diagonal 64x64 tile into dinv[..][1]
template <typename T>
hipError_t launch_hess_uinv(const InstDesc *D, const ItemMap &map, int items, int *flag,
                            hipStream_t st);
// ---- the band route: J = Q H Q^T with H of lower bandwidth 64 (k_band.hip) ----
size_t band_work_doubles(int mp);  // workspace of the reduction
// J = Q H Q^T of instance `inst` in [A; Q] ([2 mp][mp]): init ([J; I]), then for p = 0 .. mp/64-2
// the panel (cooperative; *err set if a wait between its workgroups had to be abandoned) and its
// two-sided update, then Qt = Q^T
hipError_t launch_band_init(const InstDesc *D, int inst, int mp, double *AQ, double *work, hipStream_t st);
hipError_t launch_band_panel(int mp, int p, double *AQ, double *work, int *err, hipStream_t st);
// far = false: the update's products over the whole trailing width and the next panel's columns;
// far = true: the rest of the columns (may run beside launch_band_panel(p + 1))
hipError_t launch_band_update(int mp, int p, bool far, double *AQ, double *work, hipStream_t st);
hipError_t launch_band_finish(int mp, double *AQ, double *Qt, hipStream_t st);
// step j of the pivoted band LU: item = (instance, block) for the panel, (instance, block, tile)
// for the rows, tiles t0 <= t < min(t1, npan - j - 1) of each block; permutations in hpiv
// [nb][npan][128]
template <typename T>
hipError_t launch_band_lu_panel(const InstDesc *D, const ItemMap &map, int items, int j, int *flag,
                                hipStream_t st);
template <typename T>
hipError_t launch_band_lu_rows(const InstDesc *D, const ItemMap &map, int items, int j, int t0, int t1,
                               hipStream_t st);
// panel j + 1 (pitems workgroups first) and the row tiles t >= 1 of step j in one launch
template <typename T>
hipError_t launch_band_lu_step(const InstDesc *D, const ItemMap &pmap, int pitems, const ItemMap &rmap, int ritems,
                               int j, int *flag, hipStream_t st);
// item = (instance, block): y <- L^{-1} P y on Vts in place
template <typename T>
hipError_t launch_band_lsolve(const InstDesc *D, const ItemMap &map, int items, hipStream_t st);
// item = (instance, block): the exchanges and eliminations applied to Vts in place
hipError_t launch_hess_lsolve(const InstDesc *D, const ItemMap &map, int items, int max_mp,
                              hipStream_t st);
// Vts = Vh Q (trans 0, src2 0) or Vh = Vts Q^T (trans 1, src2 1)
int qgemm_items(int nb, int mp);
hipError_t launch_qgemm(const InstDesc *D, const ItemMap &map, int items, int trans, int src2,
                        hipStream_t st);

// ---- streaming-read probe: out has `blocks` floats; reads bytes (a multiple of 16) of x ----
hipError_t launch_read_probe(const void *x, size_t bytes, float *out, int blocks, hipStream_t st);
// back-to-back 16x16x4 MFMAs (FP64 if fp64, else FP32) in `blocks` workgroups of 256 threads;
// mfma_probe_flops gives the real flops of one launch
hipError_t launch_mfma_probe(int fp64, int iters, float *out, int blocks, hipStream_t st);
double mfma_probe_flops(int iters, int blocks);

}  // namespace fde
