// Host runtime behind the C ABI of include/fdebvm.h: input validation, the BVM tables
// (eq. (1.7)-(1.10)), the Strang eigenvalues (closed form after eq. (1.13)), device
// workspace, the restarted GMRES driver and per-kernel timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "fdebvm.h"
#include "kernels.hpp"

using namespace fde;
typedef std::complex<double> cd;

static thread_local std::string g_err;

static fde_status fail(fde_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(FDE_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                 \
  } while (0)

#define STCHK(expr)                 \
  do {                              \
    fde_status s_ = (expr);         \
    if (s_ != FDE_OK) return s_;    \
  } while (0)

namespace {

struct HostFormula {
  int nu = 0, mu = 0;
  std::vector<double> a, b;    // main [mu+1]
  std::vector<double> ai, bi;  // [nu-1][mu+1]
  std::vector<double> af, bf;  // [mu-nu][mu+1]
};

// Trapezoidal rule as a BVM with (nu, mu-nu) = (1, 0).
HostFormula formula_trapezoidal() {
  HostFormula F;
  F.nu = 1;
  F.mu = 1;
  F.a = {-1.0, 1.0};
  F.b = {0.5, 0.5};
  return F;
}

// Third-order generalized BDF, (nu, mu-nu) = (2, 1): main formula on u_{n-2..n+1} with beta
// on u_n, one initial formula on u_0..u_3 (beta on u_1), one final formula = BDF3 on
// u_{s-3..s}.  Each is the four-point formula of order 3 with beta only at the derivative node.
HostFormula formula_gbdf3() {
  HostFormula F;
  F.nu = 2;
  F.mu = 3;
  F.a = {1.0 / 6.0, -1.0, 0.5, 1.0 / 3.0};
  F.b = {0.0, 0.0, 1.0, 0.0};
  F.ai = {-1.0 / 3.0, -0.5, 1.0, -1.0 / 6.0};
  F.bi = {0.0, 1.0, 0.0, 0.0};
  F.af = {-1.0 / 3.0, 1.5, -3.0, 11.0 / 6.0};
  F.bf = {0.0, 0.0, 0.0, 1.0};
  return F;
}

struct ProfEntry {
  double ms = 0.0;
  int count = 0;
  double work = 0.0;
};
struct Pending {
  std::string name;
  double work;
  hipEvent_t a, b;
};

}  // namespace

struct fde_bvm {
  // ---- problem
  int m = 0, s = 0, mu = 0, nu = 0, nb = 0, mp = 0, npan = 0, log2L = 0, log2s = 0, L = 0;
  double alpha = 0, dx = 0, tau = 0, scale = 0;
  HostFormula F;
  std::vector<double> g, dp, dm;
  std::vector<int> band_c;
  std::vector<double> band_a, band_b;
  std::vector<cd> lam, muk;
  bool need_Ju0 = false;
  // ---- device
  hipStream_t stream = nullptr, own_stream = nullptr;
  std::vector<void *> allocs;
  double *d_g = nullptr, *d_dp = nullptr, *d_dm = nullptr, *d_cG = nullptr;
  double2 *d_chat = nullptr, *d_twL = nullptr, *d_tws = nullptr, *d_lam = nullptr, *d_mu = nullptr;
  int *d_band_c = nullptr, *d_bandJ_c = nullptr, *d_flag = nullptr;
  double *d_band_a = nullptr, *d_band_b = nullptr, *d_bandJ_a = nullptr, *d_bandJ_b = nullptr;
  DevSpace sp{};
  DevBand bd{}, bdJ{};
  // ---- factors
  void *d_K = nullptr, *d_dinv = nullptr;
  size_t K_bytes = 0, dinv_bytes = 0;
  int *d_tsflags = nullptr, *d_tserr = nullptr;  // block-solve dependency flags, error flag
  int ts_epoch = 0;
  bool ts_coop = true;
  int prec = -1;
  double t_factor_ms = 0.0;
  // ---- Krylov workspace
  int R = 0, nblk = 1;
  double *d_V = nullptr, *d_Z = nullptr;
  double *d_w = nullptr, *d_x = nullptr, *d_b = nullptr, *d_tmp = nullptr, *d_Ju0 = nullptr;
  double *d_part[2] = {nullptr, nullptr}, *d_H = nullptr, *d_y = nullptr, *d_nrm = nullptr;
  double2 *d_Vh = nullptr;
  double *d_su0 = nullptr, *d_sf = nullptr, *d_sio = nullptr;
  // ---- profiling
  bool prof = false;
  std::map<std::string, ProfEntry> prof_tab;
  std::vector<Pending> pend;
  std::vector<hipEvent_t> evpool;

  size_t n() const { return (size_t)s * m; }
};

// ====================================================================================
// helpers
// ====================================================================================
static fde_status dalloc(fde_bvm *h, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(FDE_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
  }
  h->allocs.push_back(*p);
  return FDE_OK;
}

template <typename P>
static fde_status dalloc_t(fde_bvm *h, P **p, size_t count) {
  void *q = nullptr;
  fde_status st = dalloc(h, &q, count * sizeof(P));
  *p = (P *)q;
  return st;
}

static void dfree(fde_bvm *h, void *p) {
  if (!p) return;
  for (size_t i = 0; i < h->allocs.size(); ++i)
    if (h->allocs[i] == p) {
      h->allocs.erase(h->allocs.begin() + i);
      break;
    }
  (void)hipFree(p);
}

static hipEvent_t get_event(fde_bvm *h) {
  if (!h->evpool.empty()) {
    hipEvent_t e = h->evpool.back();
    h->evpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

template <typename Fn>
static hipError_t run(fde_bvm *h, const char *name, double work, Fn &&launch) {
  if (!h->prof) return launch();
  hipEvent_t a = get_event(h), b = get_event(h);
  (void)hipEventRecord(a, h->stream);
  hipError_t e = launch();
  (void)hipEventRecord(b, h->stream);
  h->pend.push_back({name, work, a, b});
  return e;
}

static fde_status sync_and_flush(fde_bvm *h) {
  HIPCHK(hipStreamSynchronize(h->stream));
  for (auto &p : h->pend) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ProfEntry &e = h->prof_tab[p.name];
      e.ms += ms;
      e.count += 1;
      e.work += p.work;
    }
    h->evpool.push_back(p.a);
    h->evpool.push_back(p.b);
  }
  h->pend.clear();
  return FDE_OK;
}

static int ilog2_exact(long v) {
  if (v <= 0 || (v & (v - 1))) return -1;
  int l = 0;
  while ((1L << l) < v) ++l;
  return l;
}

static bool finite_all(const double *x, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

static fde_status validate_formula(const HostFormula &F) {
  const int mu1 = F.mu + 1;
  double rho1 = 0, drho1 = 0, sig1 = 0, scale = 0;
  for (int i = 0; i < mu1; ++i) {
    rho1 += F.a[i];
    drho1 += i * F.a[i];
    sig1 += F.b[i];
    scale += std::fabs(F.a[i]) + std::fabs(F.b[i]);
  }
  const double tol = 1e-12 * (scale > 1 ? scale : 1);
  if (std::fabs(rho1) > tol || std::fabs(drho1 - sig1) > tol)
    return fail(FDE_EINVAL, "BVM formula is not consistent: rho(1)=%g, rho'(1)-sigma(1)=%g", rho1,
                drho1 - sig1);
  return FDE_OK;
}

// ====================================================================================
// setup
// ====================================================================================
static fde_status build_tables(fde_bvm *h) {
  const int m = h->m, s = h->s, mu = h->mu, nu = h->nu, mu1 = mu + 1;
  const HostFormula &F = h->F;
  // Grunwald weights, eq. (1.2): g_0 = 1, g_{k+1} = (1 - (alpha+1)/(k+1)) g_k.
  h->g.assign(m + 1, 0.0);
  h->g[0] = 1.0;
  for (int k = 0; k < m; ++k) h->g[k + 1] = (1.0 - (h->alpha + 1.0) / (k + 1.0)) * h->g[k];
  // BVM rows of the s-form system (s-form row n = (s+1)-form row r = n+1).
  h->band_c.assign(s, 0);
  h->band_a.assign((size_t)s * mu1, 0.0);
  h->band_b.assign((size_t)s * mu1, 0.0);
  h->need_Ju0 = false;
  for (int n = 0; n < s; ++n) {
    const int r = n + 1;
    const double *ra, *rb;
    int c;
    if (r < nu) {
      c = 0;
      ra = &F.ai[(size_t)(r - 1) * mu1];
      rb = &F.bi[(size_t)(r - 1) * mu1];
    } else if (r <= s - mu + nu) {
      c = r - nu;
      ra = F.a.data();
      rb = F.b.data();
    } else {
      const int fr = r - (s - mu + nu + 1);
      c = s - mu;
      ra = &F.af[(size_t)fr * mu1];
      rb = &F.bf[(size_t)fr * mu1];
    }
    h->band_c[n] = c;
    for (int q = 0; q < mu1; ++q) {
      h->band_a[(size_t)n * mu1 + q] = ra[q];
      h->band_b[(size_t)n * mu1 + q] = rb[q];
    }
    if (c == 0 && rb[0] != 0.0) h->need_Ju0 = true;
  }
  // Strang eigenvalues: lambda_k = sum_i alpha_i w^{(i-nu)k}, w = e^{2 pi i/s}; same for mu_k.
  h->lam.assign(h->nb, cd(0, 0));
  h->muk.assign(h->nb, cd(0, 0));
  for (int k = 0; k < h->nb; ++k) {
    for (int i = 0; i < mu1; ++i) {
      long t = ((long)(i - nu) * k) % s;
      if (t < 0) t += s;
      const double th = 2.0 * M_PI * (double)t / (double)s;
      const cd w(std::cos(th), std::sin(th));
      h->lam[k] += F.a[i] * w;
      h->muk[k] += F.b[i] * w;
    }
  }
  return FDE_OK;
}

static std::vector<double2> twiddles(int N) {
  std::vector<double2> t(N / 2 > 0 ? N / 2 : 1);
  for (int j = 0; j < N / 2; ++j) {
    const double th = -2.0 * M_PI * (double)j / (double)N;
    t[j] = make_double2(std::cos(th), std::sin(th));
  }
  return t;
}

static void destroy_handle(fde_bvm *h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (void *p : h->allocs) (void)hipFree(p);
  for (auto &p : h->pend) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : h->evpool) (void)hipEventDestroy(e);
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  delete h;
}

extern "C" fde_status fde_bvm_setup(const fde_problem *p, fde_bvm **out) {
  if (!out) return fail(FDE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return fail(FDE_EINVAL, "problem is NULL");
  if (!(p->alpha > 1.0 && p->alpha < 2.0)) return fail(FDE_EINVAL, "alpha must lie in (1,2), got %g", p->alpha);
  if (!(p->xR > p->xL) || !std::isfinite(p->xR - p->xL)) return fail(FDE_EINVAL, "need xR > xL");
  if (!(p->T > p->t0) || !std::isfinite(p->T - p->t0)) return fail(FDE_EINVAL, "need T > t0");
  if (p->m < 1) return fail(FDE_EINVAL, "m must be >= 1, got %d", p->m);
  if (!p->d_plus || !p->d_minus) return fail(FDE_EINVAL, "d_plus and d_minus are required");
  if (!finite_all(p->d_plus, p->m) || !finite_all(p->d_minus, p->m))
    return fail(FDE_EINVAL, "non-finite diffusion coefficient");
  for (int i = 0; i < p->m; ++i) {
    if (p->d_plus[i] < 0.0 || p->d_minus[i] < 0.0)
      return fail(FDE_EINVAL, "d+- must be nonnegative (node %d)", i + 1);
    if (!(p->d_plus[i] + p->d_minus[i] > 0.0))
      return fail(FDE_EINVAL, "d+ + d- must be positive (node %d)", i + 1);
  }
  HostFormula F;
  if (p->kind == FDE_BVM_TRAPEZOIDAL) {
    F = formula_trapezoidal();
  } else if (p->kind == FDE_BVM_GBDF3) {
    F = formula_gbdf3();
  } else if (p->kind == FDE_BVM_CUSTOM) {
    const fde_bvm_formula *c = p->custom;
    if (!c) return fail(FDE_EINVAL, "custom formula is NULL");
    if (c->nu1 < 1 || c->nu2 < 0 || c->nu1 + c->nu2 > 16)
      return fail(FDE_EINVAL, "need nu1 >= 1, nu2 >= 0, nu1 + nu2 <= 16");
    F.nu = c->nu1;
    F.mu = c->nu1 + c->nu2;
    const int mu1 = F.mu + 1;
    if (!c->alpha || !c->beta) return fail(FDE_EINVAL, "custom formula: alpha/beta are required");
    if (F.nu > 1 && (!c->alpha_init || !c->beta_init))
      return fail(FDE_EINVAL, "custom formula: %d initial formulas required", F.nu - 1);
    if (c->nu2 > 0 && (!c->alpha_fin || !c->beta_fin))
      return fail(FDE_EINVAL, "custom formula: %d final formulas required", c->nu2);
    F.a.assign(c->alpha, c->alpha + mu1);
    F.b.assign(c->beta, c->beta + mu1);
    if (F.nu > 1) {
      F.ai.assign(c->alpha_init, c->alpha_init + (size_t)(F.nu - 1) * mu1);
      F.bi.assign(c->beta_init, c->beta_init + (size_t)(F.nu - 1) * mu1);
    }
    if (c->nu2 > 0) {
      F.af.assign(c->alpha_fin, c->alpha_fin + (size_t)c->nu2 * mu1);
      F.bf.assign(c->beta_fin, c->beta_fin + (size_t)c->nu2 * mu1);
    }
  } else {
    return fail(FDE_EINVAL, "unknown BVM kind %d", (int)p->kind);
  }
  STCHK(validate_formula(F));
  if (p->s < F.mu + 1) return fail(FDE_EINVAL, "s = %d must be at least mu+1 = %d", p->s, F.mu + 1);
  const int log2s = ilog2_exact(p->s);
  if (log2s < 0) return fail(FDE_EUNSUPPORTED, "s = %d is not a power of two", p->s);
  if (p->s > 1024) return fail(FDE_EUNSUPPORTED, "s = %d exceeds 1024", p->s);
  if (p->m > 4096) return fail(FDE_EUNSUPPORTED, "m = %d exceeds 4096", p->m);

  fde_bvm *h = new fde_bvm();
  h->m = p->m;
  h->s = p->s;
  h->F = F;
  h->mu = F.mu;
  h->nu = F.nu;
  h->nb = p->s / 2 + 1;
  h->mp = ((p->m + 63) / 64) * 64;
  h->npan = h->mp / 64;
  h->log2s = log2s;
  h->L = 2;
  h->log2L = 1;
  while (h->L < 2 * p->m) {
    h->L <<= 1;
    h->log2L++;
  }
  h->alpha = p->alpha;
  h->dx = (p->xR - p->xL) / (p->m + 1);
  h->tau = (p->T - p->t0) / p->s;
  h->scale = std::pow(h->dx, -p->alpha);
  h->dp.assign(p->d_plus, p->d_plus + p->m);
  h->dm.assign(p->d_minus, p->d_minus + p->m);
  build_tables(h);

  auto bail = [&](fde_status st) {
    destroy_handle(h);
    return st;
  };
  if (hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess) {
    h->own_stream = nullptr;
    return bail(fail(FDE_EDEVICE, "hipStreamCreate failed"));
  }
  h->stream = h->own_stream;
  const int m = h->m, s = h->s, mu1 = h->mu + 1, nb = h->nb, L = h->L;
  const size_t n = h->n();
  fde_status st = FDE_OK;
#define ALLOC(ptr, cnt) \
  if ((st = dalloc_t(h, &(ptr), (cnt))) != FDE_OK) return bail(st)
  ALLOC(h->d_g, m + 1);
  ALLOC(h->d_dp, m);
  ALLOC(h->d_dm, m);
  ALLOC(h->d_cG, L);
  ALLOC(h->d_chat, L);
  ALLOC(h->d_twL, L / 2);
  ALLOC(h->d_tws, s / 2);
  ALLOC(h->d_band_c, s);
  ALLOC(h->d_band_a, (size_t)s * mu1);
  ALLOC(h->d_band_b, (size_t)s * mu1);
  ALLOC(h->d_bandJ_c, 1);
  ALLOC(h->d_bandJ_a, 1);
  ALLOC(h->d_bandJ_b, 1);
  ALLOC(h->d_lam, nb);
  ALLOC(h->d_mu, nb);
  ALLOC(h->d_flag, 1);
  ALLOC(h->d_tserr, 1);
  ALLOC(h->d_tsflags, (size_t)h->nb * h->npan * 2);
  ALLOC(h->d_w, n);
  ALLOC(h->d_x, n);
  ALLOC(h->d_b, n);
  ALLOC(h->d_tmp, n);
  ALLOC(h->d_Ju0, m);
  ALLOC(h->d_part[0], 1024);
  ALLOC(h->d_part[1], 1024);
  ALLOC(h->d_H, 72);
  ALLOC(h->d_y, 72);
  ALLOC(h->d_nrm, 8);
  ALLOC(h->d_Vh, (size_t)nb * h->mp);
  ALLOC(h->d_su0, m);
  ALLOC(h->d_sf, (size_t)(s + 1) * m);
  ALLOC(h->d_sio, n);
#undef ALLOC
  h->nblk = krylov_blocks(n);

  std::vector<double> cG(L, 0.0);
  for (int i = 0; i < m; ++i) cG[i] = h->g[i + 1];
  cG[L - 1] = h->g[0];
  std::vector<double2> lam(nb), muk(nb);
  for (int k = 0; k < nb; ++k) {
    lam[k] = make_double2(h->lam[k].real(), h->lam[k].imag());
    muk[k] = make_double2(h->muk[k].real(), h->muk[k].imag());
  }
  const std::vector<double2> twL = twiddles(L), tws = twiddles(s);
  const int cJ = 1;
  const double aJ = 0.0, bJ = 1.0;
  hipStream_t q = h->stream;
#define H2D(dst, src, bytes)                                                      \
  if (hipMemcpyAsync((dst), (src), (bytes), hipMemcpyHostToDevice, q) != hipSuccess) \
  return bail(fail(FDE_EDEVICE, "upload failed"))
  H2D(h->d_g, h->g.data(), sizeof(double) * (m + 1));
  H2D(h->d_dp, h->dp.data(), sizeof(double) * m);
  H2D(h->d_dm, h->dm.data(), sizeof(double) * m);
  H2D(h->d_cG, cG.data(), sizeof(double) * L);
  H2D(h->d_twL, twL.data(), sizeof(double2) * (L / 2));
  H2D(h->d_tws, tws.data(), sizeof(double2) * (s / 2));
  H2D(h->d_band_c, h->band_c.data(), sizeof(int) * s);
  H2D(h->d_band_a, h->band_a.data(), sizeof(double) * s * mu1);
  H2D(h->d_band_b, h->band_b.data(), sizeof(double) * s * mu1);
  H2D(h->d_bandJ_c, &cJ, sizeof(int));
  H2D(h->d_bandJ_a, &aJ, sizeof(double));
  H2D(h->d_bandJ_b, &bJ, sizeof(double));
  H2D(h->d_lam, lam.data(), sizeof(double2) * nb);
  H2D(h->d_mu, muk.data(), sizeof(double2) * nb);
#undef H2D
  h->sp = DevSpace{m, h->log2L, h->d_dp, h->d_dm, h->d_chat, h->d_twL, h->scale};
  h->bd = DevBand{s, mu1, h->d_band_c, h->d_band_a, h->d_band_b};
  h->bdJ = DevBand{1, 1, h->d_bandJ_c, h->d_bandJ_a, h->d_bandJ_b};
  if (hipMemsetAsync(h->d_tsflags, 0, sizeof(int) * h->nb * h->npan * 2, q) != hipSuccess ||
      hipMemsetAsync(h->d_tserr, 0, sizeof(int), q) != hipSuccess)
    return bail(fail(FDE_EDEVICE, "flag initialisation failed"));
  if (launch_symbol(h->d_cG, h->d_chat, h->log2L, h->d_twL, q) != hipSuccess)
    return bail(fail(FDE_EDEVICE, "symbol FFT launch failed: %s", hipGetErrorString(hipGetLastError())));
  if (hipStreamSynchronize(q) != hipSuccess) return bail(fail(FDE_EDEVICE, "setup synchronisation failed"));
  *out = h;
  return FDE_OK;
}

extern "C" void fde_bvm_destroy(fde_bvm *h) { destroy_handle(h); }
extern "C" const char *fde_last_error(void) { return g_err.c_str(); }

extern "C" fde_status fde_set_stream(fde_bvm *h, void *stream) {
  if (!h) return fail(FDE_EINVAL, "handle is NULL");
  HIPCHK(hipStreamSynchronize(h->stream));
  h->stream = stream ? (hipStream_t)stream : h->own_stream;
  return FDE_OK;
}

extern "C" fde_status fde_get_dims(const fde_bvm *h, int *dims) {
  if (!h || !dims) return fail(FDE_EINVAL, "NULL argument");
  dims[0] = h->m;
  dims[1] = h->s;
  dims[2] = h->mu;
  dims[3] = h->nu;
  dims[4] = h->nb;
  dims[5] = h->mp;
  return FDE_OK;
}

// ====================================================================================
// factorization
// ====================================================================================
template <typename T>
static fde_status factor_impl(fde_bvm *h) {
  const int m = h->m, mp = h->mp, nb = h->nb;
  const double esz = (double)sizeof(T) * 2.0;
  HIPCHK(run(h, "assemble", (double)nb * m * m * esz, [&] {
    return launch_assemble<T>(h->d_K, m, mp, nb, h->d_lam, h->d_mu, h->tau, h->scale, h->d_g,
                              h->d_dp, h->d_dm, h->stream);
  }));
  for (int p = 0; p < h->npan; ++p) {
    // algorithmic flops (complex = 8 real flops per multiply-add) on the unpadded order m
    const double rem = std::max(0, m - (p + 1) * 64);
    const double w = std::min(64, m - p * 64);
    HIPCHK(run(h, "lu_diag", nb * 8.0 * w * w * w / 3.0, [&] {
      return launch_lu_diag<T>(h->d_K, mp, nb, p, h->d_dinv, h->d_flag, h->stream);
    }));
    if (p + 1 < h->npan) {
      HIPCHK(run(h, "lu_panel", nb * 8.0 * 64.0 * 64.0 * rem, [&] {
        return launch_lu_panel<T>(h->d_K, mp, nb, p, h->d_dinv, h->stream);
      }));
      HIPCHK(run(h, "lu_update", nb * 8.0 * 64.0 * rem * rem, [&] {
        return launch_lu_update<T>(h->d_K, mp, nb, p, h->stream);
      }));
    }
  }
  return FDE_OK;
}

extern "C" fde_status fde_precond_factor(fde_bvm *h, fde_precision prec) {
  if (!h) return fail(FDE_EINVAL, "handle is NULL");
  if (prec != FDE_FP64 && prec != FDE_MIXED_C32) return fail(FDE_EINVAL, "unknown precision %d", (int)prec);
  const size_t esz = prec == FDE_FP64 ? sizeof(double2) : sizeof(float2);
  const size_t Kb = (size_t)h->nb * h->mp * h->mp * esz;
  const size_t Db = (size_t)h->nb * h->npan * 2 * 64 * 64 * esz;
  if (h->K_bytes != Kb) {
    HIPCHK(hipStreamSynchronize(h->stream));
    dfree(h, h->d_K);
    dfree(h, h->d_dinv);
    h->d_K = h->d_dinv = nullptr;
    h->K_bytes = h->dinv_bytes = 0;
    h->prec = -1;
    STCHK(dalloc(h, &h->d_K, Kb));
    STCHK(dalloc(h, &h->d_dinv, Db));
    h->K_bytes = Kb;
    h->dinv_bytes = Db;
  }
  h->prec = -1;
  hipEvent_t e0 = get_event(h), e1 = get_event(h);
  HIPCHK(hipMemsetAsync(h->d_flag, 0, sizeof(int), h->stream));
  HIPCHK(hipEventRecord(e0, h->stream));
  fde_status st = prec == FDE_FP64 ? factor_impl<double>(h) : factor_impl<float>(h);
  if (st != FDE_OK) return st;
  HIPCHK(hipEventRecord(e1, h->stream));
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  STCHK(sync_and_flush(h));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  h->evpool.push_back(e0);
  h->evpool.push_back(e1);
  h->t_factor_ms = ms;
  if (flag) return fail(FDE_ESINGULAR, "zero or non-finite pivot in a preconditioner block");
  h->prec = prec;
  return FDE_OK;
}

// ====================================================================================
// operators
// ====================================================================================
static fde_status op_matvec(fde_bvm *h, const double *z, double *w) {
  const double bytes = 16.0 * (double)h->n();
  HIPCHK(run(h, "bvm_matvec", bytes,
             [&] { return launch_bvm_matvec(z, w, h->sp, h->bd, -h->tau, h->stream); }));
  return FDE_OK;
}

static fde_status op_precond(fde_bvm *h, const double *v, double *z) {
  const int m = h->m, nb = h->nb;
  const double vbytes = 8.0 * h->n() + 16.0 * nb * m;
  HIPCHK(run(h, "time_rfft", vbytes, [&] {
    return launch_time_rfft(v, h->d_Vh, m, h->mp, h->log2s, h->d_tws, h->stream);
  }));
  const double esz = h->prec == FDE_FP64 ? 16.0 : 8.0;
  if (h->ts_epoch >= 0x7ffffff0) {  // epochs are compared for equality; restart the count
    HIPCHK(hipMemsetAsync(h->d_tsflags, 0, sizeof(int) * h->nb * h->npan * 2, h->stream));
    h->ts_epoch = 0;
  }
  const int epoch = ++h->ts_epoch;
  HIPCHK(run(h, "trsv", (double)nb * m * m * esz + 32.0 * nb * m, [&] {
    hipError_t e = hipErrorNotSupported;
    if (h->ts_coop) {
      e = h->prec == FDE_FP64 ? launch_trsv_coop<double>(h->d_K, h->d_dinv, h->d_Vh, h->d_tsflags,
                                                         h->mp, nb, epoch, h->d_tserr, h->stream)
                              : launch_trsv_coop<float>(h->d_K, h->d_dinv, h->d_Vh, h->d_tsflags,
                                                        h->mp, nb, epoch, h->d_tserr, h->stream);
      if (e != hipSuccess) {  // cooperative launch refused: one workgroup per block instead
        (void)hipGetLastError();
        h->ts_coop = false;
      }
    }
    if (!h->ts_coop)
      e = h->prec == FDE_FP64 ? launch_trsv<double>(h->d_K, h->d_dinv, h->d_Vh, h->mp, nb, h->stream)
                              : launch_trsv<float>(h->d_K, h->d_dinv, h->d_Vh, h->mp, nb, h->stream);
    return e;
  }));
  HIPCHK(run(h, "time_irfft", vbytes, [&] {
    return launch_time_irfft(h->d_Vh, z, m, h->mp, h->log2s, h->d_tws, h->stream);
  }));
  return FDE_OK;
}

static fde_status op_rhs(fde_bvm *h, const double *u0, const double *f, double *b) {
  const double *Ju0 = nullptr;
  if (h->need_Ju0) {
    HIPCHK(run(h, "toeplitz", 16.0 * h->m, [&] {
      return launch_bvm_matvec(u0, h->d_Ju0, h->sp, h->bdJ, 1.0, h->stream);
    }));
    Ju0 = h->d_Ju0;
  }
  HIPCHK(run(h, "rhs", 8.0 * (2.0 * h->s + 1.0) * h->m, [&] {
    return launch_rhs(f, u0, Ju0, b, h->m, h->bd, h->tau, h->stream);
  }));
  return FDE_OK;
}

// The block solve raises d_tserr if it had to abandon a dependency wait (never expected).
static fde_status check_trsv_err(fde_bvm *h) {
  int err = 0;
  HIPCHK(hipMemcpyAsync(&err, h->d_tserr, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (err) {
    (void)hipMemsetAsync(h->d_tserr, 0, sizeof(int), h->stream);
    return fail(FDE_EDEVICE, "block solve abandoned a dependency wait");
  }
  return FDE_OK;
}

static fde_status stage_in(fde_bvm *h, const double *src, size_t count, int mem, double *staging,
                           const double **dev) {
  if (mem == FDE_MEM_DEVICE) {
    *dev = src;
    return FDE_OK;
  }
  if (mem != FDE_MEM_HOST) return fail(FDE_EINVAL, "unknown mem_space %d", mem);
  HIPCHK(hipMemcpyAsync(staging, src, count * sizeof(double), hipMemcpyHostToDevice, h->stream));
  *dev = staging;
  return FDE_OK;
}

static fde_status copy_out(fde_bvm *h, double *dst, const double *dev, size_t count, int mem) {
  HIPCHK(hipMemcpyAsync(dst, dev, count * sizeof(double),
                        mem == FDE_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        h->stream));
  return FDE_OK;
}

static fde_status host_norm(fde_bvm *h, const double *x, double *out) {
  const size_t n = h->n();
  HIPCHK(run(h, "dot", 8.0 * n, [&] { return launch_dot_partial(x, x, n, h->d_part[0], h->nblk, h->stream); }));
  std::vector<double> part(h->nblk);
  HIPCHK(hipMemcpyAsync(part.data(), h->d_part[0], sizeof(double) * h->nblk, hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  double t = 0.0;
  for (double v : part) t += v;
  *out = std::sqrt(t);
  return FDE_OK;
}

static fde_status ensure_krylov(fde_bvm *h, int R) {
  if (h->R >= R && h->d_V) return FDE_OK;
  HIPCHK(hipStreamSynchronize(h->stream));
  dfree(h, h->d_V);
  dfree(h, h->d_Z);
  h->d_V = h->d_Z = nullptr;
  h->R = 0;
  const size_t n = h->n();
  STCHK(dalloc_t(h, &h->d_V, (size_t)(R + 1) * n));
  STCHK(dalloc_t(h, &h->d_Z, (size_t)R * n));
  h->R = R;
  return FDE_OK;
}

// ====================================================================================
// GMRES (right preconditioning, flexible form, MGS Arnoldi, Givens least squares)
// ====================================================================================
static fde_status gmres(fde_bvm *h, const fde_solve_opts &o, fde_solve_info *info) {
  const size_t n = h->n();
  const int R = o.restart;
  const double tol = o.rtol;
  STCHK(ensure_krylov(h, R));
  double bnorm = 0.0;
  STCHK(host_norm(h, h->d_b, &bnorm));
  if (!std::isfinite(bnorm)) return fail(FDE_EINVAL, "right-hand side is not finite");
  int its = 0, restarts = 0;
  bool conv = false;
  double truer = 0.0, est = 0.0;
  if (bnorm == 0.0) {
    HIPCHK(hipMemsetAsync(h->d_x, 0, n * sizeof(double), h->stream));
    conv = true;
  }
  std::vector<double> H((size_t)(R + 1) * R), cs(R), sn(R), gv(R + 1), hcol(R + 2), y(R);
  const double vb = 8.0 * n;
  while (!conv) {
    STCHK(op_matvec(h, h->d_x, h->d_tmp));
    HIPCHK(run(h, "residual", 3 * vb, [&] {
      return launch_residual(h->d_b, h->d_tmp, h->d_V, n, h->d_part[0], h->nblk, h->stream);
    }));
    HIPCHK(run(h, "normalize", 2 * vb, [&] {
      return launch_normalize(h->d_V, h->d_V, n, h->d_part[0], h->nblk, h->d_nrm, h->stream);
    }));
    double beta = 0.0;
    HIPCHK(hipMemcpyAsync(&beta, h->d_nrm, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    STCHK(sync_and_flush(h));
    truer = beta / bnorm;
    if (!std::isfinite(beta)) {
      if (info) info->true_relres = truer;
      return fail(FDE_ENOCONV, "residual is not finite");
    }
    if (beta <= tol * bnorm) {
      conv = true;
      break;
    }
    if (its >= o.maxit) break;
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int k = 0;
    for (int j = 0; j < R; ++j) {
      double *vj = h->d_V + (size_t)j * n, *zj = h->d_Z + (size_t)j * n;
      STCHK(op_precond(h, vj, zj));
      STCHK(op_matvec(h, zj, h->d_w));
      for (int i = 0; i <= j + 1; ++i) {
        HIPCHK(run(h, "mgs", (i == 0 ? 2 : 4) * vb, [&] {
          return launch_mgs_step(i, j, h->d_V, h->d_w, n, h->d_part[(i + 1) & 1], h->d_part[i & 1],
                                 h->nblk, h->d_H, h->stream);
        }));
      }
      HIPCHK(run(h, "normalize", 2 * vb, [&] {
        return launch_normalize(h->d_w, h->d_V + (size_t)(j + 1) * n, n, h->d_part[(j + 1) & 1],
                                h->nblk, h->d_H + j + 1, h->stream);
      }));
      HIPCHK(hipMemcpyAsync(hcol.data(), h->d_H, sizeof(double) * (j + 2), hipMemcpyDeviceToHost,
                            h->stream));
      STCHK(sync_and_flush(h));
      ++its;
      for (int i = 0; i <= j + 1; ++i) H[(size_t)i * R + j] = hcol[i];
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * R + j], b = H[(size_t)(i + 1) * R + j];
        H[(size_t)i * R + j] = cs[i] * a + sn[i] * b;
        H[(size_t)(i + 1) * R + j] = -sn[i] * a + cs[i] * b;
      }
      const double a = H[(size_t)j * R + j], b = H[(size_t)(j + 1) * R + j];
      const double d = std::hypot(a, b);
      cs[j] = d > 0 ? a / d : 1.0;
      sn[j] = d > 0 ? b / d : 0.0;
      H[(size_t)j * R + j] = d;
      H[(size_t)(j + 1) * R + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      k = j + 1;
      est = std::fabs(gv[j + 1]) / bnorm;
      if (!std::isfinite(est)) return fail(FDE_ENOCONV, "Arnoldi produced a non-finite value");
      if (std::fabs(gv[j + 1]) <= tol * bnorm || its >= o.maxit) break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double t = gv[i];
      for (int c = i + 1; c < k; ++c) t -= H[(size_t)i * R + c] * y[c];
      y[i] = t / H[(size_t)i * R + i];
    }
    HIPCHK(hipMemcpyAsync(h->d_y, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, h->stream));
    HIPCHK(run(h, "update_x", (2.0 + k) * vb,
               [&] { return launch_update_x(h->d_x, h->d_Z, h->d_y, k, n, h->stream); }));
    ++restarts;
  }
  STCHK(check_trsv_err(h));
  if (info) {
    info->iters = its;
    info->restarts = restarts;
    info->converged = conv ? 1 : 0;
    info->true_relres = truer;
    info->est_relres = est;
  }
  if (!conv) return fail(FDE_ENOCONV, "GMRES reached maxit=%d with relative residual %.3e", o.maxit, truer);
  return FDE_OK;
}

static fde_status check_opts(const fde_bvm *h, const fde_solve_opts *o, fde_solve_opts *out) {
  fde_solve_opts d{1e-10, 20, 1000, nullptr, FDE_MEM_HOST};
  if (o) d = *o;
  if (!(d.rtol > 0.0) || !std::isfinite(d.rtol)) return fail(FDE_EINVAL, "rtol must be positive");
  if (d.restart < 1 || d.restart > 64) return fail(FDE_EINVAL, "restart must be in 1..64");
  if (d.maxit < 0) return fail(FDE_EINVAL, "maxit must be >= 0");
  if (d.mem_space != FDE_MEM_HOST && d.mem_space != FDE_MEM_DEVICE)
    return fail(FDE_EINVAL, "unknown mem_space %d", d.mem_space);
  (void)h;
  *out = d;
  return FDE_OK;
}

static fde_status solve_one(fde_bvm *h, const double *u0, const double *f, double *u,
                            const fde_solve_opts &o, fde_solve_info *info) {
  if (h->prec < 0) return fail(FDE_EINVAL, "fde_precond_factor must succeed before fde_bvm_solve");
  if (!u0 || !f || !u) return fail(FDE_EINVAL, "u0, f and u are required");
  const size_t n = h->n();
  if (info) {
    std::memset(info, 0, sizeof *info);
    info->precision = h->prec;
    info->t_factor_ms = h->t_factor_ms;
  }
  hipEvent_t e0 = get_event(h), e1 = get_event(h);
  HIPCHK(hipEventRecord(e0, h->stream));
  const double *du0, *df;
  STCHK(stage_in(h, u0, h->m, o.mem_space, h->d_su0, &du0));
  STCHK(stage_in(h, f, (size_t)(h->s + 1) * h->m, o.mem_space, h->d_sf, &df));
  STCHK(op_rhs(h, du0, df, h->d_b));
  if (o.x0) {
    HIPCHK(hipMemcpyAsync(h->d_x, o.x0, n * sizeof(double),
                          o.mem_space == FDE_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          h->stream));
  } else {
    HIPCHK(hipMemsetAsync(h->d_x, 0, n * sizeof(double), h->stream));
  }
  fde_status st = gmres(h, o, info);
  if (st != FDE_OK && st != FDE_ENOCONV) return st;
  const std::string msg = g_err;
  STCHK(copy_out(h, u, h->d_x, n, o.mem_space));
  HIPCHK(hipEventRecord(e1, h->stream));
  STCHK(sync_and_flush(h));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  h->evpool.push_back(e0);
  h->evpool.push_back(e1);
  if (info) info->t_solve_ms = ms;
  if (st != FDE_OK) g_err = msg;
  return st;
}

extern "C" fde_status fde_bvm_solve(fde_bvm *h, const double *u0, const double *f, double *u,
                                    const fde_solve_opts *o, fde_solve_info *info) {
  if (!h) return fail(FDE_EINVAL, "handle is NULL");
  fde_solve_opts oo;
  STCHK(check_opts(h, o, &oo));
  return solve_one(h, u0, f, u, oo, info);
}

extern "C" fde_status fde_bvm_solve_batch(fde_bvm *const *hs, int count, const double *const *u0,
                                          const double *const *f, double *const *u,
                                          const fde_solve_opts *o, fde_solve_info *info) {
  if (count < 0 || (count > 0 && (!hs || !u0 || !f || !u)))
    return fail(FDE_EINVAL, "invalid batch arguments");
  fde_status worst = FDE_OK;
  std::string msg;
  for (int i = 0; i < count; ++i) {
    if (!hs[i]) return fail(FDE_EINVAL, "handle %d is NULL", i);
    fde_solve_opts oo;
    STCHK(check_opts(hs[i], o, &oo));
    fde_status st = solve_one(hs[i], u0[i], f[i], u[i], oo, info ? &info[i] : nullptr);
    if (st != FDE_OK && st != FDE_ENOCONV) return st;
    if (st != FDE_OK && worst == FDE_OK) {
      worst = st;
      msg = g_err;
    }
  }
  if (worst != FDE_OK) g_err = msg;
  return worst;
}

// ====================================================================================
// single steps (per-kernel checks)
// ====================================================================================
extern "C" fde_status fde_build_rhs(fde_bvm *h, const double *u0, const double *f, double *b,
                                    int mem_space) {
  if (!h || !u0 || !f || !b) return fail(FDE_EINVAL, "NULL argument");
  const double *du0, *df;
  STCHK(stage_in(h, u0, h->m, mem_space, h->d_su0, &du0));
  STCHK(stage_in(h, f, (size_t)(h->s + 1) * h->m, mem_space, h->d_sf, &df));
  STCHK(op_rhs(h, du0, df, h->d_tmp));
  STCHK(copy_out(h, b, h->d_tmp, h->n(), mem_space));
  return sync_and_flush(h);
}

extern "C" fde_status fde_apply_matvec(fde_bvm *h, const double *z, double *w, int mem_space) {
  if (!h || !z || !w) return fail(FDE_EINVAL, "NULL argument");
  const double *dz;
  STCHK(stage_in(h, z, h->n(), mem_space, h->d_sio, &dz));
  STCHK(op_matvec(h, dz, h->d_tmp));
  STCHK(copy_out(h, w, h->d_tmp, h->n(), mem_space));
  return sync_and_flush(h);
}

extern "C" fde_status fde_apply_precond(fde_bvm *h, const double *v, double *z, int mem_space) {
  if (!h || !v || !z) return fail(FDE_EINVAL, "NULL argument");
  if (h->prec < 0) return fail(FDE_EINVAL, "fde_precond_factor must succeed first");
  const double *dv;
  STCHK(stage_in(h, v, h->n(), mem_space, h->d_sio, &dv));
  STCHK(op_precond(h, dv, h->d_tmp));
  STCHK(copy_out(h, z, h->d_tmp, h->n(), mem_space));
  STCHK(sync_and_flush(h));
  return check_trsv_err(h);
}

extern "C" fde_status fde_time_rfft(fde_bvm *h, const double *v, double *vhat, int mem_space) {
  if (!h || !v || !vhat) return fail(FDE_EINVAL, "NULL argument");
  const double *dv;
  STCHK(stage_in(h, v, h->n(), mem_space, h->d_sio, &dv));
  HIPCHK(launch_time_rfft(dv, h->d_Vh, h->m, h->mp, h->log2s, h->d_tws, h->stream));
  HIPCHK(hipMemcpy2DAsync(vhat, sizeof(double2) * h->m, h->d_Vh, sizeof(double2) * h->mp,
                          sizeof(double2) * h->m, h->nb,
                          mem_space == FDE_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          h->stream));
  return sync_and_flush(h);
}

extern "C" fde_status fde_toeplitz_apply(fde_bvm *h, const double *x, double *y, int count,
                                         int mem_space) {
  if (!h || !x || !y || count < 1) return fail(FDE_EINVAL, "invalid argument");
  const size_t cnt = (size_t)count * h->m;
  std::vector<int> c(count);
  std::vector<double> a(count, 0.0), b(count, 1.0);
  for (int i = 0; i < count; ++i) c[i] = i + 1;
  int *dc = nullptr;
  double *da = nullptr, *db = nullptr, *dx = nullptr, *dy = nullptr;
  fde_status st = FDE_OK;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(h->stream);
    dfree(h, dc);
    dfree(h, da);
    dfree(h, db);
    dfree(h, dx);
    dfree(h, dy);
  };
  if ((st = dalloc_t(h, &dc, count)) || (st = dalloc_t(h, &da, count)) || (st = dalloc_t(h, &db, count)) ||
      (st = dalloc_t(h, &dx, cnt)) || (st = dalloc_t(h, &dy, cnt))) {
    cleanup();
    return st;
  }
  const hipMemcpyKind in = mem_space == FDE_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const hipMemcpyKind outk = mem_space == FDE_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  hipError_t e = hipMemcpyAsync(dc, c.data(), sizeof(int) * count, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(da, a.data(), sizeof(double) * count, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(db, b.data(), sizeof(double) * count, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dx, x, sizeof(double) * cnt, in, h->stream);
  DevBand bd{count, 1, dc, da, db};
  if (e == hipSuccess)
    e = run(h, "toeplitz", 16.0 * cnt, [&] { return launch_bvm_matvec(dx, dy, h->sp, bd, 1.0, h->stream); });
  if (e == hipSuccess) e = hipMemcpyAsync(y, dy, sizeof(double) * cnt, outk, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  cleanup();
  if (e != hipSuccess) return fail(FDE_EDEVICE, "toeplitz apply failed: %s", hipGetErrorString(e));
  return sync_and_flush(h);
}

extern "C" fde_status fde_get_factor_block(fde_bvm *h, int k, double *out) {
  if (!h || !out) return fail(FDE_EINVAL, "NULL argument");
  if (h->prec < 0) return fail(FDE_EINVAL, "no factorization stored");
  if (k < 0 || k >= h->nb) return fail(FDE_EINVAL, "block %d out of range 0..%d", k, h->nb - 1);
  const int m = h->m, mp = h->mp;
  const size_t esz = h->prec == FDE_FP64 ? sizeof(double2) : sizeof(float2);
  std::vector<char> raw((size_t)mp * mp * esz);
  HIPCHK(hipMemcpyAsync(raw.data(), (char *)h->d_K + (size_t)k * mp * mp * esz, raw.size(),
                        hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const size_t src = (size_t)i * mp + j, dst = ((size_t)i * m + j) * 2;
      if (h->prec == FDE_FP64) {
        const double *p = (const double *)raw.data() + 2 * src;
        out[dst] = p[0];
        out[dst + 1] = p[1];
      } else {
        const float *p = (const float *)raw.data() + 2 * src;
        out[dst] = p[0];
        out[dst + 1] = p[1];
      }
    }
  return FDE_OK;
}

// ====================================================================================
// profiling
// ====================================================================================
extern "C" fde_status fde_profile_enable(fde_bvm *h, int enable) {
  if (!h) return fail(FDE_EINVAL, "handle is NULL");
  STCHK(sync_and_flush(h));
  h->prof = enable != 0;
  if (h->prof) h->prof_tab.clear();
  return FDE_OK;
}

extern "C" fde_status fde_profile_query(const fde_bvm *h, const char *name, double *total_ms,
                                        int *count, double *work) {
  if (!h || !name) return fail(FDE_EINVAL, "NULL argument");
  auto it = h->prof_tab.find(name);
  const ProfEntry e = it == h->prof_tab.end() ? ProfEntry() : it->second;
  if (total_ms) *total_ms = e.ms;
  if (count) *count = e.count;
  if (work) *work = e.work;
  return FDE_OK;
}
