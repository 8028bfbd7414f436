/*
 * fdebvm — Strang block-circulant preconditioned GMRES for the all-at-once
 * boundary-value-method (BVM) discretisation of the 1-D two-sided space-fractional
 * diffusion equation, on AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 2, eq. (1.1)):
 *   u_t = d+(x) D+^a u + d-(x) D-^a u + f(x,t),  x in (xL,xR), t in (t0,T],
 *   u(xL,t) = u(xR,t) = 0,  u(x,t0) = u0(x),  1 < a < 2,  d+- >= 0, d+ + d- > 0.
 * Space: shifted Grunwald formula on x_i = xL + i dx, dx = (xR-xL)/(m+1), i = 1..m,
 *   J = dx^{-a} (D+ G_a + D- G_a^T)  (eq. (1.2)-(1.5)).
 * Time: a mu-step BVM with (nu1, nu2) = (nu, mu-nu) on t_n = t0 + n tau, tau = (T-t0)/s
 *   (eq. (1.7)-(1.9)).  u_0 is moved to the right-hand side, so the unknowns are
 *   u_1..u_s and the all-at-once system (eq. (1.10)) is
 *     M u = (A (x) I_m - tau B (x) J) u = b,
 *     b   = tau (Bhat[1:,:] (x) I) f - a0 (x) u0 + tau b0 (x) (J u0),
 *   with Ahat, Bhat the (s+1)x(s+1) BVM matrices, A = Ahat[1:,1:], a0 = Ahat[1:,0], etc.
 * Preconditioner (Section 3.1, eq. (1.11)):  S = s(A) (x) I - tau s(B) (x) J, applied
 *   through the time-axis DFT as s independent blocks K_k = lambda_k I - tau mu_k J
 *   (Section 3.2), K_{s-k} = conj(K_k).
 *
 * Layouts.  All space-time vectors are FP64, time-major: element (n, i) at n*m + i.
 *   f is [s+1][m] (f_0..f_s); u and b are [s][m] (rows 1..s); u0 is [m].
 * Memory spaces.  Calls that take a `mem_space` argument accept host pointers
 *   (FDE_MEM_HOST; copied through the handle's staging buffers) or device pointers
 *   (FDE_MEM_DEVICE; used in place, must stay valid until the call returns).
 * Ownership.  Every input array is copied or consumed during the call; the caller may
 *   free it on return.  The handle owns all device memory until fde_bvm_destroy().
 * Errors.  Status codes only (no exceptions, no abort across the ABI); the message of
 *   the last failure on the calling thread is returned by fde_last_error().
 * Streams.  Work is enqueued on the handle's stream (fde_set_stream, default: a stream
 *   the library creates, which does not synchronise with the null stream) and every call
 *   returns after that stream is synchronised.  FDE_MEM_DEVICE inputs are read on the
 *   handle's stream: work that produces them on another stream must be complete, or
 *   ordered before the call by passing the producer's stream to fde_set_stream.
 *   A handle is not thread-safe; distinct handles may be used from distinct threads.
 */
#ifndef FDEBVM_H
#define FDEBVM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fde_bvm fde_bvm; /* opaque handle */

typedef enum {
  FDE_OK = 0,
  FDE_EINVAL = -1,       /* invalid argument or call order                          */
  FDE_ENOMEM = -2,       /* device allocation failed                                 */
  FDE_ESINGULAR = -3,    /* zero/non-finite pivot in a preconditioner block          */
  FDE_ENOCONV = -4,      /* maxit reached; u holds the last iterate, info is filled  */
  FDE_EDEVICE = -5,      /* HIP runtime error                                        */
  FDE_EUNSUPPORTED = -6  /* valid input the library does not handle (e.g. s not 2^k)*/
} fde_status;

/* Built-in BVMs (Section 2.2; the paper prints no coefficients, so each is stated here):
 *   FDE_BVM_TRAPEZOIDAL  (nu1, nu2) = (1, 0): u_n - u_{n-1} = tau/2 (g_{n-1} + g_n), order 2.
 *   FDE_BVM_GBDF3        (2, 1): third-order generalized BDF; main formula on u_{n-2..n+1}
 *                        with beta at u_n, one initial and one final (BDF3) formula.
 *   FDE_BVM_GAM5         (2, 2): fifth-order generalized Adams method, the BVM of the
 *                        experiments of Section 4.  Every row is u_r - u_{r-1} = tau sum_i
 *                        beta_i g_{c+i}, beta integrating over [t_{r-1}, t_r] the quartic
 *                        through five consecutive nodes: centred on u_r for the main formula,
 *                        the first five nodes for row 1, the last five for rows s-1 and s.
 *   FDE_BVM_CUSTOM       the formula in fde_problem.custom. */
typedef enum {
  FDE_BVM_TRAPEZOIDAL = 0,
  FDE_BVM_GBDF3 = 1,
  FDE_BVM_CUSTOM = 2,
  FDE_BVM_GAM5 = 3
} fde_bvm_kind;

/* A mu-step BVM, mu = nu1 + nu2 (eq. (1.7)-(1.9)).  Coefficient i of the main formula
 * multiplies u_{n-nu1+i}; of initial formula j (1 <= j < nu1, row j-1 of the *_init
 * arrays) multiplies u_i; of final formula r (0 <= r < nu2) multiplies u_{s-mu+i}.
 * Arrays are row-major with mu+1 columns.  The main formula must be consistent:
 * rho(1) = 0 and rho'(1) = sigma(1) (Section 3.1). */
typedef struct {
  int nu1, nu2;
  const double *alpha, *beta;           /* [mu+1]          */
  const double *alpha_init, *beta_init; /* [nu1-1][mu+1]   */
  const double *alpha_fin, *beta_fin;   /* [nu2][mu+1]     */
} fde_bvm_formula;

/* The problem statement of eq. (1.1) on the grid of Section 2.1.  d_plus, d_minus are
 * sampled at the interior nodes x_1..x_m (time-independent).  `custom` is read only
 * when kind == FDE_BVM_CUSTOM. */
typedef struct {
  double alpha, xL, xR, t0, T;
  int m, s;
  const double *d_plus, *d_minus; /* host pointers, [m] */
  fde_bvm_kind kind;
  const fde_bvm_formula *custom;
} fde_problem;

typedef enum { FDE_FP64 = 0, FDE_MIXED_C32 = 1 } fde_precision;
typedef enum { FDE_MEM_HOST = 0, FDE_MEM_DEVICE = 1 } fde_mem_space;

/* rtol: stop when ||b - M u||_2 <= rtol ||b||_2 (true residual, recomputed in FP64).
 * restart: GMRES restart length (1..64).  maxit: total iteration cap.
 * x0: initial guess [s][m] in mem_space, or NULL for zero.  A guess is first scaled by the
 *     gamma that minimises ||b - gamma M x0|| (so ||r_0|| <= ||b||: a poor guess never
 *     starts worse than the zero start).
 * x0_kind: FDE_X0_SOLUTION (the guess approximates u) or FDE_X0_LOWRANK (the guess
 *     approximates c = (S - M) u, the part of S u that differs from b; the start is then
 *     S^{-1}(b + c), which equals u when c is exact).  By Theorem 3.3 S^{-1} M = I + L with
 *     L supported on the nu + (mu - nu) boundary block rows, so c has only those rows. */
typedef enum { FDE_X0_SOLUTION = 0, FDE_X0_LOWRANK = 1 } fde_x0_kind;
typedef struct {
  double rtol;
  int restart, maxit;
  const double *x0;
  int mem_space;
  int x0_kind;
} fde_solve_opts;

typedef struct {
  int iters, restarts, converged, precision;
  double true_relres; /* ||b - M u|| / ||b|| of the returned u, FP64 */
  double est_relres;  /* GMRES least-squares estimate at exit        */
  double t_factor_ms, t_solve_ms;
} fde_solve_info;

/* Validates the problem (1 < alpha < 2; d+- >= 0 and d+ + d- > 0 at every node; m >= 1;
 * s >= mu+1 and a power of two (else FDE_EUNSUPPORTED); xR > xL; T > t0; consistent
 * custom formula), builds the Grunwald weights (eq. (1.2)), the BVM tables and the Strang
 * eigenvalues (closed form after eq. (1.13)), allocates the device workspace and computes
 * the Toeplitz symbol FFT of G_a on the device.  On success *out owns a new handle. */
fde_status fde_bvm_setup(const fde_problem *p, fde_bvm **out);

/* Assembles the floor(s/2)+1 distinct blocks K_k = lambda_k I - tau mu_k J and factors them
 * by pivot-free blocked LU on the GPU (Section 3.2), in complex FP64 (FDE_FP64) or complex
 * FP32 (FDE_MIXED_C32).  Pivot-free elimination is safe because every K_k is strictly row
 * diagonally dominant for an A_{nu,mu-nu}-stable formula (Prop 2.2, Definition 3.1); a zero
 * or non-finite pivot returns FDE_ESINGULAR.  May be called again to switch precision. */
fde_status fde_precond_factor(fde_bvm *h, fde_precision prec);

/* Solves M u = b (b built on the GPU from u0 [m] and f [s+1][m]) by right-preconditioned
 * restarted GMRES (flexible form; FP64 Arnoldi with modified Gram-Schmidt, Givens rotations
 * and true residual).  u0, f, u are in o->mem_space.  Requires fde_precond_factor first. */
fde_status fde_bvm_solve(fde_bvm *h, const double *u0, const double *f, double *u,
                         const fde_solve_opts *o, fde_solve_info *info);

/* Factors the blocks of `count` handles together: every phase of the blocked LU is one
 * launch covering the blocks of all instances (uneven m and s allowed).  Same numerics
 * and errors as fde_precond_factor; the handles must be distinct. */
fde_status fde_precond_factor_batch(fde_bvm *const *h, int count, fde_precision prec);

/* Solves `count` independent handles factored with the same precision.  Every phase is
 * one launch over all instances that take part in it (a device table of per-instance
 * descriptors drives the kernels); restart cycles run in lockstep and each instance stops
 * on its own true residual.  Arrays of pointers are host arrays; the pointed-to data is in
 * o->mem_space; o->x0 must be NULL (use fde_bvm_solve_batch_x0).  info is [count].
 * Returns FDE_ENOCONV if any instance hit maxit (its info says which). */
fde_status fde_bvm_solve_batch(fde_bvm *const *h, int count, const double *const *u0,
                               const double *const *f, double *const *u,
                               const fde_solve_opts *o, fde_solve_info *info);
/* As fde_bvm_solve_batch with per-instance initial guesses x0[i] (NULL entries: zero). */
fde_status fde_bvm_solve_batch_x0(fde_bvm *const *h, int count, const double *const *u0,
                                  const double *const *f, const double *const *x0,
                                  double *const *u, const fde_solve_opts *o, fde_solve_info *info);

void fde_bvm_destroy(fde_bvm *h);
const char *fde_last_error(void);

/* ---- stream and sizes ------------------------------------------------------------ */
/* Use `stream` (a hipStream_t, or NULL for the library's own stream) for all later work. */
fde_status fde_set_stream(fde_bvm *h, void *stream);
/* dims[0..5] = m, s, mu, nu1, nb = s/2+1, padded block order mp. */
fde_status fde_get_dims(const fde_bvm *h, int *dims);

/* ---- execution options -------------------------------------------------------------
 * A solve runs its restart steps and restart cycles as fixed launch sequences driven by
 * per-instance control records on the device (Givens rotations, convergence tests and the
 * least-squares update happen there; finished instances are gated off), so the host reads
 * the state once per cycle.  The sequences are recorded once per plan as hipGraphs and
 * replayed; if recording fails they are launched directly, with identical results.
 *   FDE_OPT_GRAPHS        1 (default): replay recorded sequences; 0: launch directly.
 *   FDE_OPT_AUTOTUNE      1 (default): on the first solve of a shape (the sizes of all
 *                         instances of the call and the precision), time the block solve in
 *                         its ordinary one-workgroup-per-block launch and in the cooperative
 *                         launch for every candidate number of workgroups per block, and the
 *                         time FFTs for 4, 8 and 16 spatial columns per workgroup, and keep the
 *                         fastest for the life of the process.  Every launch form gives the
 *                         same bits.
 *   FDE_OPT_TRSV_W        0 (default): autotuned or the largest co-resident value;
 *                         k > 0: cooperative, at most k workgroups per block (clamped to what
 *                         fits); -1: the ordinary launch, one workgroup per block, no flags.
 *   FDE_OPT_TRSV_W_IN_USE read-only: workgroups per block of the handle's last plan's
 *                         cooperative block solve, 0 for the ordinary launch.
 *   FDE_OPT_GRAPHS_IN_USE read-only: 1 if the handle's solves replay recorded sequences.
 * Options of the first handle of a batch call apply to the call.  Setting an option
 * synchronises the handle's stream.  Unknown options return FDE_EINVAL. */
typedef enum {
  FDE_OPT_GRAPHS = 0,
  FDE_OPT_AUTOTUNE = 1,
  FDE_OPT_TRSV_W = 2,
  FDE_OPT_TRSV_W_IN_USE = 3,
  FDE_OPT_GRAPHS_IN_USE = 4,
  FDE_OPT_PRECOND = 5,
  FDE_OPT_SIDE = 6,
  FDE_OPT_BLOCKS = 7,
  FDE_OPT_ORTHO = 8,
  FDE_OPT_BLOCKS_IN_USE = 9,
  FDE_OPT_X0_GATE = 10,
  FDE_OPT_X0_KEPT = 11
} fde_option;
/* FDE_OPT_X0_GATE decides whether an initial guess is used, in millionths: after the scaling by
 * gamma (see fde_solve_opts), a guess with ||b - gamma M x0|| > gate 1e-6 ||b|| is dropped and
 * the instance starts from zero.  Default 10000 (1e-2): with the Strang preconditioner the
 * iteration count is set by the few outlying eigenvalues of S^{-1} M (the rank of S^{-1} M - I
 * is at most 2 m mu, Section 3.3), not by the starting residual, and guesses that reduce the
 * residual less than about a hundredfold do not save iterations (they can cost one or two).
 * 0 keeps every guess.  FDE_OPT_X0_KEPT (read-only): 1 if the handle's last solve used its
 * guess, else 0. */
/* FDE_OPT_PRECOND selects the preconditioner built by the next fde_precond_factor (changing it
 * discards the current factorization):
 *   FDE_PC_STRANG        S = s(A) (x) I - tau s(B) (x) J, eq. (1.11) (default): s/2+1 block LUs.
 *   FDE_PC_BCCB          S2 = s(A) (x) I - tau s(B) (x) s(J), eq. (x1), with s(J) the Strang
 *                        circulant of J built on the mean coefficients dbar+- (Section 3.1);
 *                        diagonalised by the 2-D DFT (Section 3.2): no block factors, an apply
 *                        costs O(s m log m).  Always FP64; the precision argument is recorded.
 *   FDE_PC_BCCB_SHIFTED  S2~ of eq. (xc): as S2 with the zero eigenvalue of s(A) moved to
 *                        Re of its last eigenvalue, invertible even if s(J) is singular.
 *   FDE_PC_NONE          no preconditioner (column I of the tables of Section 4).
 * All instances of a batch call must use the same kind. */
typedef enum {
  FDE_PC_STRANG = 0,
  FDE_PC_BCCB = 1,
  FDE_PC_BCCB_SHIFTED = 2,
  FDE_PC_NONE = 3
} fde_precond_kind;
/* FDE_OPT_SIDE selects how GMRES uses the preconditioner P:
 *   FDE_SIDE_RIGHT (default)  flexible right preconditioning, M P^{-1} y = b, x = P^{-1} y; the
 *                             stopping test is on the true residual ||b - M x|| <= rtol ||b||.
 *   FDE_SIDE_LEFT             GMRES on P^{-1} M x = P^{-1} b (the form of the convergence
 *                             theorem of Section 3.3 and of the iteration counts of Section 4):
 *                             the Krylov basis updates x directly and the stopping test is on
 *                             the preconditioned residual, ||P^{-1}(b - M x)|| <= rtol
 *                             ||P^{-1} b||.  fde_solve_info.true_relres is still ||b - M x|| /
 *                             ||b||, computed once after the last cycle. */
typedef enum { FDE_SIDE_RIGHT = 0, FDE_SIDE_LEFT = 1 } fde_precond_side;
/* FDE_OPT_BLOCKS selects how the blocks K_k = lambda_k I - tau mu_k J of S are factored and
 * solved (the operator S^{-1} is the same up to rounding; changing it discards the current
 * factorization):
 *   FDE_BLOCKS_LU          a pivot-free LU of every block (s/2+1 dense LUs on MFMA);
 *                          the solves read the full L and U factors.
 *   FDE_BLOCKS_HESSENBERG  every block is a shift of J: one Householder reduction J = Q H Q^T
 *                          (H upper Hessenberg, Q orthogonal; FP64) and, per block, Gaussian
 *                          elimination with partial pivoting of lambda_k I - tau mu_k H (rows i
 *                          and i+1 compete in step i).  An apply is Q^T v_k, the exchanges and
 *                          eliminations, U^{-1}, Q: the solves read only the U factors (half the
 *                          bytes).  Not in the paper.  m <= 1024 (FDE_EUNSUPPORTED beyond);
 *                          needs cooperative launches.
 *   FDE_BLOCKS_BAND        as FDE_BLOCKS_HESSENBERG with H of lower bandwidth 64 instead of 1:
 *                          a blocked Householder reduction J = Q H Q^T whose O(m^3) work runs
 *                          as matrix products (FP64), then per block an LU of lambda_k I -
 *                          tau mu_k H with partial pivoting among the 128 rows of each 64-column
 *                          panel (O(64 m^2)); the solves read U and the band of L.  Any m the
 *                          library takes; needs cooperative launches.  Not in the paper. */
/*   FDE_BLOCKS_AUTO        (default) FDE_BLOCKS_BAND when m >= FDE_BAND_MIN_M_FP64 (FP64 blocks;
 *                          FDE_BAND_MIN_M_FP64_LONG when s / 2 + 1 >= FDE_BAND_LONG_NB) or
 *                          m >= FDE_BAND_MIN_M_MIXED (FP32 blocks), else FDE_BLOCKS_LU (for a
 *                          batch: the band route only if every instance qualifies).  Measured on
 *                          MI355X at s = 256 (factor + solve): in FP64 block LU is 7% faster at
 *                          m = 1023 and the band route 12% faster at m = 1279, 1.7x at m = 2047
 *                          and 2.5x at m = 3071; with FP32 blocks block LU is 4% faster at
 *                          m = 1535 and the band route 1.2x faster at m = 2047.  Block LU's
 *                          factorization grows with s and the band reduction does not: for
 *                          s = 512 the band route is 10% faster at m = 1023 in FP64.
 * FDE_OPT_BLOCKS_IN_USE (read-only) is the route of the current factorization. */
typedef enum { FDE_BLOCKS_LU = 0, FDE_BLOCKS_HESSENBERG = 1, FDE_BLOCKS_BAND = 2, FDE_BLOCKS_AUTO = 3 } fde_block_solver;
#define FDE_BAND_MIN_M_FP64 1152
#define FDE_BAND_MIN_M_FP64_LONG 960
#define FDE_BAND_LONG_NB 257
#define FDE_BAND_MIN_M_MIXED 1792
/* FDE_OPT_ORTHO selects the Arnoldi orthogonalisation (FP64 either way):
 *   FDE_ORTHO_MGS   (default) modified Gram-Schmidt, j + 2 dependent launches at step j.
 *   FDE_ORTHO_CGS2  classical Gram-Schmidt applied twice: three launches per step whatever j;
 *                   the same basis in exact arithmetic, orthogonal to working precision. */
typedef enum { FDE_ORTHO_MGS = 0, FDE_ORTHO_CGS2 = 1 } fde_ortho;
fde_status fde_bvm_set_option(fde_bvm *h, int option, int value);
fde_status fde_bvm_get_option(fde_bvm *h, int option, int *value);
/* Autotuned choices of this process into buf (NUL-terminated), ';'-separated: "shape=W" for
 * the block solve (W = -1: the ordinary one-workgroup-per-block launch) and "shape/tfft=c" for
 * the time FFTs' spatial columns per workgroup (4, 8 or 16); FDE_EINVAL if len is too small. */
fde_status fde_autotune_report(char *buf, int len);
/* Measurement aid: the best of `reps` timed passes of a plain streaming-read kernel over a
 * `bytes`-byte device buffer (allocated and freed by the call), in GB/s: the read bandwidth
 * that bandwidth-bound kernels can practically reach on the current device.  FDE_EINVAL for
 * bytes < 1 MiB or reps < 1; FDE_ENOMEM if the buffer cannot be allocated. */
fde_status fde_read_bandwidth_probe(size_t bytes, int reps, double *gbs);
/* Measurement aid: the best of `reps` timed launches of a kernel that issues back-to-back
 * 16x16x4 MFMA products on register operands (FP64 if fp64 != 0, else FP32 — the instructions
 * of the blocked LU) on every SIMD, in TFLOP/s: the matrix-core rate MFMA-bound kernels can
 * practically reach on the current device.  FDE_EINVAL for reps < 1 or a null tflops. */
fde_status fde_mfma_peak_probe(int fp64, int reps, double *tflops);

/* ---- device buffers ------------------------------------------------------------------
 * For callers that hold no device allocator of their own (a C program, or a Python process
 * that must not load a second HIP runtime, e.g. under a profiler that preloads the system
 * one): plain device memory on the current device, usable wherever FDE_MEM_DEVICE pointers
 * are accepted.  fde_device_alloc returns FDE_EINVAL for bytes == 0 and FDE_ENOMEM when the
 * allocation fails (*ptr is then NULL); fde_device_free(NULL) is a no-op.  fde_memcpy is
 * synchronous (it returns after the copy has completed on the device); kind is one of
 * FDE_COPY_H2D, FDE_COPY_D2H, FDE_COPY_D2D.  fde_device_synchronize waits for all work on
 * the current device, every stream included. */
typedef enum { FDE_COPY_H2D = 0, FDE_COPY_D2H = 1, FDE_COPY_D2D = 2 } fde_copy_kind;
fde_status fde_device_alloc(size_t bytes, void **ptr);
fde_status fde_device_free(void *ptr);
fde_status fde_memcpy(void *dst, const void *src, size_t bytes, int kind);
fde_status fde_device_synchronize(void);

/* ---- the individual steps of the path, for per-kernel checks ----------------------- */
/* b = right-hand side of eq. (1.10) in s-form, [s][m]. */
fde_status fde_build_rhs(fde_bvm *h, const double *u0, const double *f, double *b, int mem_space);
/* w = M z (Toeplitz FFT product with J at every time level, then the banded A, B
 * coupling), z and w [s][m]. */
fde_status fde_apply_matvec(fde_bvm *h, const double *z, double *w, int mem_space);
/* y = J x for `count` vectors, x and y [count][m] (LDS radix-2 FFT, circulant embedding). */
fde_status fde_toeplitz_apply(fde_bvm *h, const double *x, double *y, int count, int mem_space);
/* vhat[k][i] = sum_n v[n][i] e^{-2 pi i nk/s}, k = 0..s/2; v [s][m] real, vhat
 * [s/2+1][m] complex interleaved (re, im). */
fde_status fde_time_rfft(fde_bvm *h, const double *v, double *vhat, int mem_space);
/* z = S^{-1} v (time DFT, block solves with the stored factors, inverse DFT), [s][m]. */
fde_status fde_apply_precond(fde_bvm *h, const double *v, double *z, int mem_space);
/* z = S^{-1} v like fde_apply_precond, allocating nothing: for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  v and z are DEVICE pointers ([s][m]); the handle must have been factored with
 * the Strang preconditioner and block LU factors (the default).  The working memory of the
 * call (the frequency-domain vector, the block-solve flags and counters, the launch
 * descriptor) is one fixed static device array of FDE_NOALLOC_SCRATCH_BYTES per GPU, held
 * until the process ends; its address is looked up once per device at fde_bvm_setup.  Every
 * call on a GPU shares that array: calls that overlap on one GPU (from other threads or on
 * other streams) race, so a caller serialises them.  The result equals fde_apply_precond's
 * bit for bit (same kernels, same launch shapes).  Errors: FDE_EINVAL for NULL arguments or an
 * unfactored handle; FDE_EUNSUPPORTED when (s/2+1) * mp * 16 bytes of frequency vector (mp =
 * m rounded up to 64) plus its flags exceed the array (m = 4095 fits up to s = 256, m = 1023
 * up to s = 1024), or for another preconditioner or block solver; FDE_EDEVICE if the block
 * solve had to abandon a dependency wait. */
#define FDE_NOALLOC_SCRATCH_BYTES (16u << 20)
fde_status fde_apply_precond_noalloc(fde_bvm *h, const double *v, double *z);
/* Copies the stored LU factors of block k (unit-lower L below the diagonal, U on and above
 * it, complex interleaved, [m][m] row-major, widened to FP64) to the host array out. */
fde_status fde_get_factor_block(fde_bvm *h, int k, double *out);
/* With FDE_BLOCKS_HESSENBERG factors stored: copies H and Q of J = Q H Q^T ([m][m] row-major,
 * host arrays) to the caller; the factor block of fde_get_factor_block then holds U on and
 * above the diagonal (below it: unspecified).  FDE_EINVAL without such a factorization. */
fde_status fde_get_hessenberg(fde_bvm *h, double *H, double *Q);

/* ---- per-kernel timing ------------------------------------------------------------- */
/* When enabled, every kernel launch is bracketed by HIP events on the handle's stream and
 * its duration is added to a per-kernel-name total.  Enabling clears the totals. */
fde_status fde_profile_enable(fde_bvm *h, int enable);
/* Total milliseconds, launch count and algorithmic work (flops or bytes, per the kernel:
 * FLOP for the LU kernels, bytes for the others) recorded for the kernel named `name`. */
fde_status fde_profile_query(const fde_bvm *h, const char *name, double *total_ms, int *count,
                             double *work);

/* ---- learned warm start ------------------------------------------------------------
 * A small network predicts an initial guess x0 of the all-at-once solution from one
 * instance's data (alpha, d+, d-, f on the grid, u0 = 0); GMRES started from it converges
 * to the same solution (the true FP64 residual decides), so a poor guess costs iterations,
 * never accuracy.  Network: three stride-2 width-5 convolutions over the 256 padded
 * spatial positions (channels = the s+1 time levels of f normalised by its RMS, d+, d-,
 * alpha-1.5), three fully connected layers, and a fixed synthesis basis
 * cos(q pi t) sin(p pi x/2) (q < nt, p < nx) that maps the nx*nt coefficients to [s][m].
 * Convolutions are im2col + GEMM; every GEMM runs on bf16 MFMA with FP32 accumulation;
 * weights are FP32 masters with bf16 copies; Adam updates the masters.
 * Parameter layout (FP32 vector): per layer l = conv1..3, fc1..3, W_l [kin][kout] row-major
 * then b_l [kout]; conv kin = 5*Cin with element (t, c) at t*Cin + c (tap t reads position
 * 2o + t - 2).  Device arrays: X [N][256][s+4] features, rms [N], T [N][s*m] FP64 targets. */
typedef struct fde_nn fde_nn;
typedef struct {
  int m, s;          /* grid of the instances the network serves (m <= 256)        */
  int max_batch;     /* largest batch passed to the calls below                     */
  int conv_ch[3];    /* output channels of the three convolutions                   */
  int fc[2];         /* widths of the two hidden fully connected layers            */
  int nx, nt;        /* synthesis basis: nx sine modes in x, nt cosine modes in t  */
  int seed;          /* initialisation seed                                         */
} fde_nn_config;

fde_status fde_nn_create(const fde_nn_config *c, fde_nn **out);
void fde_nn_destroy(fde_nn *n);
const char *fde_nn_last_error(void);
fde_status fde_nn_num_params(const fde_nn *n, long long *count);
/* host FP32 parameter vector in, refreshes the bf16 copies */
fde_status fde_nn_set_params(fde_nn *n, const float *host);
/* Replaces the fixed synthesis matrix: host FP32 [nx*nt][s*m] (output = coefficients x basis). */
fde_status fde_nn_set_basis(fde_nn *n, const float *host);
/* which = 0 parameters, 1 gradients of the last fde_nn_loss_grad, 2/3 Adam moments */
fde_status fde_nn_get_params(const fde_nn *n, float *host, int which);
/* restores Adam moments and step count (checkpoint resume) */
fde_status fde_nn_set_state(fde_nn *n, const float *m1, const float *m2, int step);
fde_status fde_nn_get_step(const fde_nn *n, int *step);
/* Features of B instances: f[b], dp[b], dm[b] are device FP64 arrays ([s+1][m], [m], [m]),
 * the pointer arrays and alpha[B] are host arrays; X [B][256][s+4] and rms [B] are device. */
fde_status fde_nn_features(fde_nn *n, int B, const double *const *f, const double *const *dp,
                           const double *const *dm, const double *alpha, float *X, float *rms);
/* Forward, relative-MSE loss against T/rms and backward for the rows idx[0..B) (host array,
 * NULL = rows 0..B-1); gradients are averaged over the batch; *loss (nullable) is the mean. */
fde_status fde_nn_loss_grad(fde_nn *n, const float *X, const double *T, const float *rms,
                            const int *idx, int B, float *loss);
/* One Adam step with the gradients of the last fde_nn_loss_grad. */
fde_status fde_nn_adam(fde_nn *n, float lr, float beta1, float beta2, float eps);
/* x0[b] (device FP64 [s][m], host array of pointers) = prediction for row idx[b] times rms. */
fde_status fde_nn_predict(fde_nn *n, const float *X, const float *rms, const int *idx, int B,
                          double *const *x0);
/* host copy of the last forward output (normalised), [B][s*m] FP32 */
fde_status fde_nn_output(const fde_nn *n, float *host, int B);
fde_status fde_nn_sync(fde_nn *n);

/* w = S z (the Strang block-circulant of eq. (1.11) applied forward), z and w [s][m]. */
fde_status fde_bvm_strang_apply(fde_bvm *h, const double *z, double *w, int mem_space);
/* c = (S - M) z, nonzero only on the nu + (mu - nu) boundary time rows (Theorem 3.3). */
fde_status fde_bvm_lowrank_correction(fde_bvm *h, const double *z, double *c, int mem_space);

/* Replaces alpha and d+- of a set-up handle (same m, s, grid and formula), recomputing the
 * weights, the symbol and the eigen-free tables; the stored factorization is discarded. */
fde_status fde_bvm_set_coefficients(fde_bvm *h, double alpha, const double *d_plus,
                                    const double *d_minus);

#ifdef __cplusplus
}
#endif
#endif /* FDEBVM_H */
