// Host runtime behind the C ABI of include/fdebvm.h: input validation, the BVM tables
// (eq. (1.7)-(1.10)), the Strang eigenvalues (closed form after eq. (1.13)), device
// workspace, launch plans over one or many instances, the restarted GMRES driver and
// per-kernel timing.
//
// A plan is a set of set-up handles solved together: a device table of per-instance
// descriptors and, per launch kind, an item map (instance ids + prefix sums of item
// counts).  Every kernel launch covers all instances of the plan that take part in that
// phase, so a batch of uneven instances costs one launch per phase; a single solve is a
// plan of one.
#include <hip/hip_runtime.h>

#include <algorithm>
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

#define STCHK(expr)              \
  do {                           \
    fde_status s_ = (expr);      \
    if (s_ != FDE_OK) return s_; \
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

// Process-wide epoch of the cooperative block solve.  Flags hold the epoch of the last
// published panel; every launch uses a new value.  On wrap-around the generation changes
// and every handle clears its flags before its next solve.
int g_epoch = 0;
int g_epoch_gen = 0;

}  // namespace

struct Plan;

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
  int *d_band_c = nullptr;
  double *d_band_a = nullptr, *d_band_b = nullptr;
  // ---- factors
  void *d_K = nullptr, *d_dinv = nullptr;
  size_t K_bytes = 0;
  int *d_tsflags = nullptr;
  int flag_gen = -1;
  int prec = -1;
  double t_factor_ms = 0.0;
  // ---- vectors
  int R = 0, nblk = 1;
  double *d_V = nullptr, *d_Z = nullptr;
  double *d_w = nullptr, *d_x = nullptr, *d_b = nullptr, *d_tmp = nullptr, *d_sio = nullptr;
  double *d_u0 = nullptr, *d_f = nullptr, *d_Ju0 = nullptr;
  double2 *d_Vh = nullptr;
  // ---- the plan of this handle alone
  Plan *self = nullptr;
  // ---- profiling
  bool prof = false;
  std::map<std::string, ProfEntry> prof_tab;
  std::vector<Pending> pend;
  std::vector<hipEvent_t> evpool;

  size_t n() const { return (size_t)s * m; }
};

// ====================================================================================
// device memory helpers
// ====================================================================================
static fde_status dalloc_raw(void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(FDE_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
  }
  return FDE_OK;
}

static fde_status dalloc(fde_bvm *h, void **p, size_t bytes) {
  STCHK(dalloc_raw(p, bytes));
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

// ====================================================================================
// plans: descriptor table + item maps
// ====================================================================================
struct HostMap {
  std::vector<int> ids, pre;
  int items = 0;
};

struct Plan {
  std::vector<fde_bvm *> hs;
  fde_bvm *lead = nullptr;  // stream and profiling owner
  int R = 0;
  InstDesc *d_desc = nullptr;
  double *d_part = nullptr, *d_H = nullptr, *d_y = nullptr, *d_nrm = nullptr;
  int *d_err = nullptr, *d_flag = nullptr;
  int *d_arena = nullptr;
  size_t arena_ints = 0;
  std::vector<InstDesc> desc;
  std::vector<int> arena_host;  // kept alive until the next rebuild (async upload source)
  std::vector<size_t> part_off;
  std::vector<void *> allocs;
  bool desc_dirty = true;
};

static void plan_free(Plan *P) {
  if (!P) return;
  for (void *p : P->allocs) (void)hipFree(p);
  delete P;
}

static fde_status plan_alloc(Plan *P, void **p, size_t bytes) {
  STCHK(dalloc_raw(p, bytes));
  P->allocs.push_back(*p);
  return FDE_OK;
}

static HostMap make_map(const std::vector<int> &slots, const std::vector<int> &items_per_slot) {
  HostMap m;
  m.pre.push_back(0);
  for (size_t q = 0; q < slots.size(); ++q) {
    if (items_per_slot[q] <= 0) continue;
    m.ids.push_back(slots[q]);
    m.pre.push_back(m.pre.back() + items_per_slot[q]);
  }
  m.items = m.pre.back();
  if (m.ids.empty()) m.ids.push_back(0);
  return m;
}

// Upload several maps into the plan's arena; returns device ItemMaps.
static fde_status upload_maps(Plan *P, const std::vector<HostMap> &maps, std::vector<ItemMap> &out) {
  size_t need = 0;
  for (const HostMap &m : maps) need += m.ids.size() + m.pre.size();
  HIPCHK(hipStreamSynchronize(P->lead->stream));  // previous users of the arena are done
  if (need > P->arena_ints) {
    if (P->d_arena) {
      auto it = std::find(P->allocs.begin(), P->allocs.end(), (void *)P->d_arena);
      if (it != P->allocs.end()) P->allocs.erase(it);
      (void)hipFree(P->d_arena);
      P->d_arena = nullptr;
    }
    size_t cap = std::max<size_t>(need, 1024);
    void *p = nullptr;
    STCHK(plan_alloc(P, &p, cap * sizeof(int)));
    P->d_arena = (int *)p;
    P->arena_ints = cap;
  }
  P->arena_host.clear();
  out.clear();
  for (const HostMap &m : maps) {
    const size_t oi = P->arena_host.size();
    P->arena_host.insert(P->arena_host.end(), m.ids.begin(), m.ids.end());
    const size_t op = P->arena_host.size();
    P->arena_host.insert(P->arena_host.end(), m.pre.begin(), m.pre.end());
    out.push_back(ItemMap{P->d_arena + oi, P->d_arena + op, (int)m.ids.size()});
  }
  HIPCHK(hipMemcpy(P->d_arena, P->arena_host.data(), P->arena_host.size() * sizeof(int),
                   hipMemcpyHostToDevice));
  return FDE_OK;
}

static InstDesc make_desc(fde_bvm *h) {
  InstDesc d;
  std::memset(&d, 0, sizeof d);
  d.m = h->m;
  d.s = h->s;
  d.mp = h->mp;
  d.nb = h->nb;
  d.npan = h->npan;
  d.log2L = h->log2L;
  d.log2s = h->log2s;
  d.mu1 = h->mu + 1;
  d.nu = h->nu;
  d.W = 1;
  d.nblk = h->nblk;
  d.need_ju0 = h->need_Ju0 ? 1 : 0;
  d.tau = h->tau;
  d.scale = h->scale;
  d.dp = h->d_dp;
  d.dm = h->d_dm;
  d.g = h->d_g;
  d.chat = h->d_chat;
  d.twL = h->d_twL;
  d.tws = h->d_tws;
  d.lam = h->d_lam;
  d.mu = h->d_mu;
  d.band_c = h->d_band_c;
  d.band_a = h->d_band_a;
  d.band_b = h->d_band_b;
  d.K = h->d_K;
  d.dinv = h->d_dinv;
  d.tsflags = h->d_tsflags;
  d.V = h->d_V;
  d.Z = h->d_Z;
  d.w = h->d_w;
  d.x = h->d_x;
  d.b = h->d_b;
  d.tmp = h->d_tmp;
  d.sio = h->d_sio;
  d.u0 = h->d_u0;
  d.f = h->d_f;
  d.Ju0 = h->d_Ju0;
  d.Vh = h->d_Vh;
  return d;
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
  if (h->self) h->self->desc_dirty = true;
  return FDE_OK;
}

// (Re)builds descriptors and plan-level buffers for restart length R; uploads descriptors.
static fde_status plan_prepare(Plan *P, int R, int trsv_cap) {
  const int count = (int)P->hs.size();
  for (fde_bvm *h : P->hs) STCHK(ensure_krylov(h, R));
  if (P->R < R || !P->d_H) {
    for (void *p : {(void *)P->d_part, (void *)P->d_H, (void *)P->d_y, (void *)P->d_nrm}) {
      if (!p) continue;
      auto it = std::find(P->allocs.begin(), P->allocs.end(), p);
      if (it != P->allocs.end()) P->allocs.erase(it);
      (void)hipFree(p);
    }
    size_t parts = 0;
    P->part_off.assign(count, 0);
    for (int i = 0; i < count; ++i) {
      P->part_off[i] = parts;
      parts += 2 * (size_t)P->hs[i]->nblk;
    }
    void *p = nullptr;
    STCHK(plan_alloc(P, &p, parts * sizeof(double)));
    P->d_part = (double *)p;
    STCHK(plan_alloc(P, &p, (size_t)count * (R + 2) * sizeof(double)));
    P->d_H = (double *)p;
    STCHK(plan_alloc(P, &p, (size_t)count * (R + 1) * sizeof(double)));
    P->d_y = (double *)p;
    STCHK(plan_alloc(P, &p, (size_t)count * 2 * sizeof(double)));
    P->d_nrm = (double *)p;
    P->R = R;
    P->desc_dirty = true;
  }
  // workgroups per block of the cooperative solve: all items co-resident when they fit
  long total_nb = 0;
  for (fde_bvm *h : P->hs) total_nb += h->nb;
  const int Wu = (trsv_cap > 0 && total_nb <= trsv_cap) ? (int)(trsv_cap / total_nb) : 1;
  P->desc.resize(count);
  for (int i = 0; i < count; ++i) {
    fde_bvm *h = P->hs[i];
    InstDesc d = make_desc(h);
    d.W = std::max(1, std::min(h->npan, Wu));
    d.part0 = P->d_part + P->part_off[i];
    d.part1 = d.part0 + h->nblk;
    d.H = P->d_H + (size_t)i * (R + 2);
    d.y = P->d_y + (size_t)i * (R + 1);
    d.nrm = P->d_nrm + (size_t)i * 2;
    if (std::memcmp(&d, &P->desc[i], sizeof d) != 0) P->desc_dirty = true;
    P->desc[i] = d;
  }
  if (P->desc_dirty) {
    HIPCHK(hipStreamSynchronize(P->lead->stream));
    HIPCHK(hipMemcpy(P->d_desc, P->desc.data(), sizeof(InstDesc) * count, hipMemcpyHostToDevice));
    P->desc_dirty = false;
  }
  return FDE_OK;
}

static fde_status plan_create(const std::vector<fde_bvm *> &hs, Plan **out) {
  Plan *P = new Plan();
  P->hs = hs;
  P->lead = hs[0];
  void *p = nullptr;
  fde_status st;
  if ((st = plan_alloc(P, &p, sizeof(InstDesc) * hs.size())) != FDE_OK) {
    plan_free(P);
    return st;
  }
  P->d_desc = (InstDesc *)p;
  if ((st = plan_alloc(P, &p, 2 * sizeof(int))) != FDE_OK) {
    plan_free(P);
    return st;
  }
  P->d_err = (int *)p;
  P->d_flag = P->d_err + 1;
  if (hipMemset(P->d_err, 0, 2 * sizeof(int)) != hipSuccess) {
    plan_free(P);
    return fail(FDE_EDEVICE, "plan flag initialisation failed");
  }
  P->desc.resize(hs.size());
  std::memset(P->desc.data(), 0, sizeof(InstDesc) * hs.size());
  *out = P;
  return FDE_OK;
}

// ====================================================================================
// validation and tables
// ====================================================================================
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

static void build_tables(fde_bvm *h) {
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
  plan_free(h->self);
  h->self = nullptr;
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
  ALLOC(h->d_lam, nb);
  ALLOC(h->d_mu, nb);
  ALLOC(h->d_tsflags, (size_t)nb * h->npan * 2);
  ALLOC(h->d_w, n);
  ALLOC(h->d_x, n);
  ALLOC(h->d_b, n);
  ALLOC(h->d_tmp, n);
  ALLOC(h->d_sio, n);
  ALLOC(h->d_u0, m);
  ALLOC(h->d_f, (size_t)(s + 1) * m);
  ALLOC(h->d_Ju0, m);
  ALLOC(h->d_Vh, (size_t)nb * h->mp);
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
  hipStream_t q = h->stream;
#define H2D(dst, src, bytes)                                                                  \
  if (hipMemcpy((dst), (src), (bytes), hipMemcpyHostToDevice) != hipSuccess)                   \
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
  H2D(h->d_lam, lam.data(), sizeof(double2) * nb);
  H2D(h->d_mu, muk.data(), sizeof(double2) * nb);
#undef H2D
  if (hipMemsetAsync(h->d_tsflags, 0, sizeof(int) * nb * h->npan * 2, q) != hipSuccess ||
      hipMemsetAsync(h->d_Ju0, 0, sizeof(double) * m, q) != hipSuccess)
    return bail(fail(FDE_EDEVICE, "initialisation failed"));
  h->flag_gen = g_epoch_gen;
  if (launch_symbol(h->d_cG, h->d_chat, h->log2L, h->d_twL, q) != hipSuccess)
    return bail(fail(FDE_EDEVICE, "symbol FFT launch failed: %s", hipGetErrorString(hipGetLastError())));
  if (hipStreamSynchronize(q) != hipSuccess) return bail(fail(FDE_EDEVICE, "setup synchronisation failed"));
  if ((st = plan_create({h}, &h->self)) != FDE_OK) return bail(st);
  *out = h;
  return FDE_OK;
}

extern "C" fde_status fde_bvm_set_coefficients(fde_bvm *h, double alpha, const double *d_plus,
                                               const double *d_minus) {
  if (!h || !d_plus || !d_minus) return fail(FDE_EINVAL, "NULL argument");
  if (!(alpha > 1.0 && alpha < 2.0)) return fail(FDE_EINVAL, "alpha must lie in (1,2), got %g", alpha);
  if (!finite_all(d_plus, h->m) || !finite_all(d_minus, h->m))
    return fail(FDE_EINVAL, "non-finite diffusion coefficient");
  for (int i = 0; i < h->m; ++i)
    if (d_plus[i] < 0.0 || d_minus[i] < 0.0 || !(d_plus[i] + d_minus[i] > 0.0))
      return fail(FDE_EINVAL, "d+- must be nonnegative with a positive sum (node %d)", i + 1);
  HIPCHK(hipStreamSynchronize(h->stream));
  h->alpha = alpha;
  h->scale = std::pow(h->dx, -alpha);
  h->dp.assign(d_plus, d_plus + h->m);
  h->dm.assign(d_minus, d_minus + h->m);
  h->g.assign(h->m + 1, 0.0);
  h->g[0] = 1.0;
  for (int k = 0; k < h->m; ++k) h->g[k + 1] = (1.0 - (alpha + 1.0) / (k + 1.0)) * h->g[k];
  std::vector<double> cG(h->L, 0.0);
  for (int i = 0; i < h->m; ++i) cG[i] = h->g[i + 1];
  cG[h->L - 1] = h->g[0];
  HIPCHK(hipMemcpy(h->d_g, h->g.data(), sizeof(double) * (h->m + 1), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->d_dp, h->dp.data(), sizeof(double) * h->m, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->d_dm, h->dm.data(), sizeof(double) * h->m, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->d_cG, cG.data(), sizeof(double) * h->L, hipMemcpyHostToDevice));
  HIPCHK(launch_symbol(h->d_cG, h->d_chat, h->log2L, h->d_twL, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->prec = -1;
  h->self->desc_dirty = true;
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
static fde_status factor_plan_impl(Plan *P) {
  fde_bvm *L = P->lead;
  const int count = (int)P->hs.size();
  std::vector<int> slots(count);
  int maxpan = 0;
  double asm_bytes = 0.0;
  std::vector<int> it(count);
  for (int i = 0; i < count; ++i) {
    slots[i] = i;
    maxpan = std::max(maxpan, P->hs[i]->npan);
    asm_bytes += (double)P->hs[i]->nb * P->hs[i]->m * P->hs[i]->m * sizeof(T) * 2.0;
  }
  // maps: assemble, then (diag, panel, update) for every panel step
  std::vector<HostMap> hm;
  for (int i = 0; i < count; ++i) it[i] = assemble_items(P->hs[i]->mp, P->hs[i]->nb);
  hm.push_back(make_map(slots, it));
  for (int p = 0; p < maxpan; ++p) {
    for (int i = 0; i < count; ++i) it[i] = p < P->hs[i]->npan ? P->hs[i]->nb : 0;
    hm.push_back(make_map(slots, it));
    for (int i = 0; i < count; ++i) {
      const int nrem = P->hs[i]->npan - p - 1;
      it[i] = nrem > 0 ? 2 * nrem * P->hs[i]->nb : 0;
    }
    hm.push_back(make_map(slots, it));
    for (int i = 0; i < count; ++i) {
      const int nrem = P->hs[i]->npan - p - 1;
      it[i] = nrem > 0 ? nrem * nrem * P->hs[i]->nb : 0;
    }
    hm.push_back(make_map(slots, it));
  }
  std::vector<ItemMap> dm;
  STCHK(upload_maps(P, hm, dm));
  hipStream_t st = L->stream;
  HIPCHK(run(L, "assemble", asm_bytes, [&] { return launch_assemble<T>(P->d_desc, dm[0], hm[0].items, st); }));
  for (int p = 0; p < maxpan; ++p) {
    // algorithmic flops (complex multiply-add = 8 real flops) on the unpadded orders m
    double wd = 0, wp = 0, wu = 0;
    for (fde_bvm *h : P->hs) {
      if (p >= h->npan) continue;
      const double rem = std::max(0, h->m - (p + 1) * 64);
      const double w = std::min(64, h->m - p * 64);
      wd += h->nb * 8.0 * w * w * w / 3.0;
      wp += h->nb * 8.0 * 64.0 * 64.0 * rem;
      wu += h->nb * 8.0 * 64.0 * rem * rem;
    }
    const HostMap &hd = hm[1 + 3 * p], &hp = hm[2 + 3 * p], &hu = hm[3 + 3 * p];
    HIPCHK(run(L, "lu_diag", wd, [&] { return launch_lu_diag<T>(P->d_desc, dm[1 + 3 * p], hd.items, p, P->d_flag, st); }));
    if (hp.items > 0) {
      HIPCHK(run(L, "lu_panel", wp, [&] { return launch_lu_panel<T>(P->d_desc, dm[2 + 3 * p], hp.items, p, st); }));
      HIPCHK(run(L, "lu_update", wu, [&] { return launch_lu_update<T>(P->d_desc, dm[3 + 3 * p], hu.items, p, st); }));
    }
  }
  return FDE_OK;
}

static fde_status factor_plan(Plan *P, fde_precision prec) {
  if (prec != FDE_FP64 && prec != FDE_MIXED_C32) return fail(FDE_EINVAL, "unknown precision %d", (int)prec);
  fde_bvm *L = P->lead;
  const size_t esz = prec == FDE_FP64 ? sizeof(double2) : sizeof(float2);
  for (fde_bvm *h : P->hs) {
    const size_t Kb = (size_t)h->nb * h->mp * h->mp * esz;
    const size_t Db = (size_t)h->nb * h->npan * 2 * 64 * 64 * esz;
    h->prec = -1;
    if (h->K_bytes != Kb) {
      HIPCHK(hipStreamSynchronize(h->stream));
      dfree(h, h->d_K);
      dfree(h, h->d_dinv);
      h->d_K = h->d_dinv = nullptr;
      h->K_bytes = 0;
      STCHK(dalloc(h, &h->d_K, Kb));
      STCHK(dalloc(h, &h->d_dinv, Db));
      h->K_bytes = Kb;
      if (h->self) h->self->desc_dirty = true;
    }
  }
  P->desc_dirty = true;
  STCHK(plan_prepare(P, std::max(P->R, 1), 0));
  hipEvent_t e0 = get_event(L), e1 = get_event(L);
  HIPCHK(hipMemsetAsync(P->d_flag, 0, sizeof(int), L->stream));
  HIPCHK(hipEventRecord(e0, L->stream));
  STCHK(prec == FDE_FP64 ? factor_plan_impl<double>(P) : factor_plan_impl<float>(P));
  HIPCHK(hipEventRecord(e1, L->stream));
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, P->d_flag, sizeof(int), hipMemcpyDeviceToHost, L->stream));
  STCHK(sync_and_flush(L));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  L->evpool.push_back(e0);
  L->evpool.push_back(e1);
  if (flag) return fail(FDE_ESINGULAR, "zero or non-finite pivot in a preconditioner block");
  for (fde_bvm *h : P->hs) {
    h->prec = prec;
    h->t_factor_ms = ms;
  }
  return FDE_OK;
}

extern "C" fde_status fde_precond_factor(fde_bvm *h, fde_precision prec) {
  if (!h) return fail(FDE_EINVAL, "handle is NULL");
  return factor_plan(h->self, prec);
}

// ====================================================================================
// solve-phase maps and operators over a plan
// ====================================================================================
struct SolveMaps {
  ItemMap mv, tfft, trsv, kry, rhs, ju0;
  int n_mv = 0, n_tfft = 0, n_trsv = 0, n_kry = 0, n_rhs = 0, n_ju0 = 0;
  int max_log2L = 1, max_log2s = 1, max_mp = 64;
  int prec = -1;
  double trsv_bytes = 0, vec_bytes = 0, tfft_bytes = 0;
};

static fde_status build_solve_maps(Plan *P, const std::vector<int> &active, SolveMaps &S) {
  const int count = (int)active.size();
  std::vector<int> a(count), b(count), c(count), d(count), e(count), f(count);
  S.max_log2L = S.max_log2s = 1;
  S.max_mp = 64;
  S.trsv_bytes = S.vec_bytes = S.tfft_bytes = 0;
  for (int q = 0; q < count; ++q) {
    fde_bvm *h = P->hs[active[q]];
    const InstDesc &ds = P->desc[active[q]];
    a[q] = h->s;
    b[q] = h->mp / time_fft_cols_per_item();
    c[q] = h->nb * ds.W;
    d[q] = h->nblk;
    e[q] = h->s;
    f[q] = h->need_Ju0 ? 1 : 0;
    S.max_log2L = std::max(S.max_log2L, h->log2L);
    S.max_log2s = std::max(S.max_log2s, h->log2s);
    S.max_mp = std::max(S.max_mp, h->mp);
    const double esz = h->prec == FDE_FP64 ? 16.0 : 8.0;
    S.trsv_bytes += (double)h->nb * h->m * h->m * esz + 32.0 * h->nb * h->m;
    S.vec_bytes += 8.0 * h->n();
    S.tfft_bytes += 8.0 * h->n() + 16.0 * h->nb * h->m;
  }
  std::vector<HostMap> hm = {make_map(active, a), make_map(active, b), make_map(active, c),
                             make_map(active, d), make_map(active, e), make_map(active, f)};
  std::vector<ItemMap> dm;
  STCHK(upload_maps(P, hm, dm));
  S.mv = dm[0];
  S.tfft = dm[1];
  S.trsv = dm[2];
  S.kry = dm[3];
  S.rhs = dm[4];
  S.ju0 = dm[5];
  S.n_mv = hm[0].items;
  S.n_tfft = hm[1].items;
  S.n_trsv = hm[2].items;
  S.n_kry = hm[3].items;
  S.n_rhs = hm[4].items;
  S.n_ju0 = hm[5].items;
  S.prec = P->hs[active[0]]->prec;
  return FDE_OK;
}

static fde_status op_matvec(Plan *P, const SolveMaps &S, int src, int sj, int dst, int dj) {
  fde_bvm *L = P->lead;
  HIPCHK(run(L, "bvm_matvec", 2.0 * S.vec_bytes, [&] {
    return launch_bvm_matvec(P->d_desc, S.mv, S.n_mv, S.max_log2L, src, sj, dst, dj, 0, L->stream);
  }));
  return FDE_OK;
}

static fde_status op_precond(Plan *P, const SolveMaps &S, int src, int sj, int dst, int dj) {
  fde_bvm *L = P->lead;
  hipStream_t st = L->stream;
  HIPCHK(run(L, "time_rfft", S.tfft_bytes, [&] {
    return launch_time_rfft(P->d_desc, S.tfft, S.n_tfft, S.max_log2s, src, sj, st);
  }));
  for (fde_bvm *h : P->hs)
    if (h->flag_gen != g_epoch_gen) {
      HIPCHK(hipMemsetAsync(h->d_tsflags, 0, sizeof(int) * h->nb * h->npan * 2, st));
      h->flag_gen = g_epoch_gen;
    }
  if (g_epoch >= 0x7ffffff0) {
    g_epoch = 0;
    ++g_epoch_gen;
    for (fde_bvm *h : P->hs) {
      HIPCHK(hipMemsetAsync(h->d_tsflags, 0, sizeof(int) * h->nb * h->npan * 2, st));
      h->flag_gen = g_epoch_gen;
    }
  }
  const int epoch = ++g_epoch;
  static bool coop_ok = true;
  HIPCHK(run(L, "trsv", S.trsv_bytes, [&] {
    hipError_t e = hipErrorNotSupported;
    if (coop_ok) {
      e = S.prec == FDE_FP64
              ? launch_trsv_coop<double>(P->d_desc, S.trsv, S.n_trsv, epoch, P->d_err, st)
              : launch_trsv_coop<float>(P->d_desc, S.trsv, S.n_trsv, epoch, P->d_err, st);
      if (e != hipSuccess) {  // cooperative launch refused: one workgroup per block instead
        (void)hipGetLastError();
        coop_ok = false;
      }
    }
    if (!coop_ok) {
      // one workgroup per block: W = 1 items; the trsv map counts nb W, so rebuild counts
      e = S.prec == FDE_FP64 ? launch_trsv<double>(P->d_desc, S.trsv, S.n_trsv, S.max_mp, st)
                             : launch_trsv<float>(P->d_desc, S.trsv, S.n_trsv, S.max_mp, st);
    }
    return e;
  }));
  HIPCHK(run(L, "time_irfft", S.tfft_bytes, [&] {
    return launch_time_irfft(P->d_desc, S.tfft, S.n_tfft, S.max_log2s, dst, dj, st);
  }));
  return FDE_OK;
}

static fde_status op_rhs(Plan *P, const SolveMaps &S) {
  fde_bvm *L = P->lead;
  if (S.n_ju0 > 0) {
    HIPCHK(run(L, "toeplitz", 16.0 * S.n_ju0, [&] {
      return launch_bvm_matvec(P->d_desc, S.ju0, S.n_ju0, S.max_log2L, VS_U0, 0, VS_JU0, 0, 1,
                               L->stream);
    }));
  }
  HIPCHK(run(L, "rhs", 2.0 * S.vec_bytes, [&] {
    return launch_rhs(P->d_desc, S.rhs, S.n_rhs, S.n_ju0 > 0 ? 1 : 0, L->stream);
  }));
  return FDE_OK;
}

// The block solve raises the plan's error flag if it had to abandon a dependency wait.
static fde_status check_trsv_err(Plan *P) {
  int err = 0;
  HIPCHK(hipMemcpy(&err, P->d_err, sizeof(int), hipMemcpyDeviceToHost));
  if (err) {
    (void)hipMemset(P->d_err, 0, sizeof(int));
    return fail(FDE_EDEVICE, "block solve abandoned a dependency wait");
  }
  return FDE_OK;
}

// ====================================================================================
// GMRES over a plan: lockstep restart cycles (right preconditioning, flexible form, MGS
// Arnoldi, Givens rotations; convergence only on the recomputed true residual)
// ====================================================================================
struct InstState {
  double bnorm = 0, truer = 0, est = 0;
  int its = 0, restarts = 0, k = 0;
  bool done = false, conv = false, in_cycle = false;
  std::vector<double> H, cs, sn, g, y;
};

// Sum of an instance's chunk partials (part0 or part1) in index order.
static double part_sum(const Plan *P, const std::vector<double> &parts, int i, int psel) {
  double t = 0.0;
  const size_t base = P->part_off[i] + (psel ? P->hs[i]->nblk : 0);
  for (int q = 0; q < P->hs[i]->nblk; ++q) t += parts[base + q];
  return t;
}

static fde_status gmres_plan(Plan *P, const fde_solve_opts &o, const std::vector<char> &has_x0,
                             std::vector<InstState> &st) {
  fde_bvm *L = P->lead;
  const int count = (int)P->hs.size();
  const int R = o.restart;
  const double tol = o.rtol;
  hipStream_t stream = L->stream;
  std::vector<int> all(count);
  for (int i = 0; i < count; ++i) all[i] = i;
  SolveMaps S;
  STCHK(build_solve_maps(P, all, S));
  // right-hand sides and their norms
  STCHK(op_rhs(P, S));
  HIPCHK(run(L, "dot", S.vec_bytes, [&] { return launch_dot_partial(P->d_desc, S.kry, S.n_kry, VS_B, VS_B, 0, stream); }));
  size_t nparts = 0;
  for (fde_bvm *h : P->hs) nparts += 2 * (size_t)h->nblk;
  std::vector<double> parts(nparts), hbuf((size_t)count * (R + 2)), nrm((size_t)count * 2);
  HIPCHK(hipMemcpyAsync(parts.data(), P->d_part, nparts * sizeof(double), hipMemcpyDeviceToHost, stream));
  STCHK(sync_and_flush(L));
  std::vector<double> bsq(count);
  for (int i = 0; i < count; ++i) bsq[i] = part_sum(P, parts, i, 0);
  // An initial guess is first scaled by the gamma minimising ||b - gamma M x0|| (one step of
  // minimal residual along x0), so that ||r_0|| <= ||b||: a poor guess never starts worse
  // than the zero start.
  std::vector<int> with_x0;
  for (int i = 0; i < count; ++i)
    if (has_x0[i]) with_x0.push_back(i);
  if (!with_x0.empty()) {
    STCHK(build_solve_maps(P, with_x0, S));
    if (o.x0_kind == FDE_X0_LOWRANK) {  // x holds c: start from S^{-1}(b + c)
      HIPCHK(run(L, "axpy", 3.0 * S.vec_bytes, [&] { return launch_axpy(P->d_desc, S.kry, S.n_kry, VS_X, VS_B, 1.0, stream); }));
      STCHK(op_precond(P, S, VS_X, 0, VS_X, 0));
    }
    STCHK(op_matvec(P, S, VS_X, 0, VS_TMP, 0));
    HIPCHK(run(L, "dot", S.vec_bytes, [&] { return launch_dot_partial(P->d_desc, S.kry, S.n_kry, VS_B, VS_TMP, 0, stream); }));
    HIPCHK(run(L, "dot", S.vec_bytes, [&] { return launch_dot_partial(P->d_desc, S.kry, S.n_kry, VS_TMP, VS_TMP, 1, stream); }));
    HIPCHK(hipMemcpyAsync(parts.data(), P->d_part, nparts * sizeof(double), hipMemcpyDeviceToHost, stream));
    STCHK(sync_and_flush(L));
    std::vector<double> ybuf((size_t)count * (R + 1), 0.0);
    for (int i : with_x0) {
      const double bm = part_sum(P, parts, i, 0), mm = part_sum(P, parts, i, 1);
      ybuf[(size_t)i * (R + 1)] = (mm > 0.0 && std::isfinite(bm / mm)) ? bm / mm : 0.0;
    }
    HIPCHK(hipMemcpy(P->d_y, ybuf.data(), ybuf.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(run(L, "scale_x", 2.0 * S.vec_bytes, [&] { return launch_scale_x(P->d_desc, S.kry, S.n_kry, stream); }));
    STCHK(build_solve_maps(P, all, S));
  }
  for (int i = 0; i < count; ++i) {
    st[i].bnorm = std::sqrt(bsq[i]);
    st[i].H.assign((size_t)(R + 1) * R, 0.0);
    st[i].cs.assign(R, 0.0);
    st[i].sn.assign(R, 0.0);
    st[i].g.assign(R + 1, 0.0);
    st[i].y.assign(R + 1, 0.0);
    if (!std::isfinite(st[i].bnorm)) return fail(FDE_EINVAL, "right-hand side %d is not finite", i);
    if (st[i].bnorm == 0.0) {
      HIPCHK(hipMemsetAsync(P->hs[i]->d_x, 0, P->hs[i]->n() * sizeof(double), stream));
      st[i].done = st[i].conv = true;
    }
  }
  std::vector<int> active;
  for (int i = 0; i < count; ++i)
    if (!st[i].done) active.push_back(i);
  std::vector<int> built = all;
  for (;;) {
    if (active.empty()) break;
    if (active != built) {
      STCHK(build_solve_maps(P, active, S));
      built = active;
    }
    // true residual of every active instance: V_0 = b - M x, beta = ||V_0||
    STCHK(op_matvec(P, S, VS_X, 0, VS_TMP, 0));
    HIPCHK(run(L, "residual", 3.0 * S.vec_bytes, [&] { return launch_residual(P->d_desc, S.kry, S.n_kry, stream); }));
    HIPCHK(run(L, "normalize", 2.0 * S.vec_bytes, [&] {
      return launch_normalize(P->d_desc, S.kry, S.n_kry, VS_V, 0, VS_V, 0, 0, -1, stream);
    }));
    HIPCHK(hipMemcpyAsync(nrm.data(), P->d_nrm, nrm.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    STCHK(sync_and_flush(L));
    std::vector<int> cyc;
    for (int i : active) {
      InstState &s = st[i];
      const double beta = nrm[(size_t)i * 2];
      s.truer = beta / s.bnorm;
      if (!std::isfinite(beta)) return fail(FDE_ENOCONV, "residual of instance %d is not finite", i);
      if (beta <= tol * s.bnorm) {
        s.done = s.conv = true;
        continue;
      }
      if (s.its >= o.maxit) {
        s.done = true;
        continue;
      }
      std::fill(s.g.begin(), s.g.end(), 0.0);
      s.g[0] = beta;
      s.k = 0;
      s.in_cycle = true;
      cyc.push_back(i);
    }
    if (cyc.empty()) break;
    if (cyc != built) {
      STCHK(build_solve_maps(P, cyc, S));
      built = cyc;
    }
    for (int j = 0; j < R && !cyc.empty(); ++j) {
      STCHK(op_precond(P, S, VS_V, j, VS_Z, j));
      STCHK(op_matvec(P, S, VS_Z, j, VS_W, 0));
      for (int i = 0; i <= j + 1; ++i) {
        HIPCHK(run(L, "mgs", (i == 0 ? 2.0 : 4.0) * S.vec_bytes,
                   [&] { return launch_mgs_step(P->d_desc, S.kry, S.n_kry, i, j, stream); }));
      }
      HIPCHK(run(L, "normalize", 2.0 * S.vec_bytes, [&] {
        return launch_normalize(P->d_desc, S.kry, S.n_kry, VS_W, 0, VS_V, j + 1, (j + 1) & 1, j + 1, stream);
      }));
      HIPCHK(hipMemcpyAsync(hbuf.data(), P->d_H, hbuf.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
      STCHK(sync_and_flush(L));
      std::vector<int> next;
      for (int i : cyc) {
        InstState &s = st[i];
        const double *hc = &hbuf[(size_t)i * (R + 2)];
        ++s.its;
        for (int r = 0; r <= j + 1; ++r) s.H[(size_t)r * R + j] = hc[r];
        for (int r = 0; r < j; ++r) {
          const double a = s.H[(size_t)r * R + j], b = s.H[(size_t)(r + 1) * R + j];
          s.H[(size_t)r * R + j] = s.cs[r] * a + s.sn[r] * b;
          s.H[(size_t)(r + 1) * R + j] = -s.sn[r] * a + s.cs[r] * b;
        }
        const double a = s.H[(size_t)j * R + j], b = s.H[(size_t)(j + 1) * R + j];
        const double dd = std::hypot(a, b);
        s.cs[j] = dd > 0 ? a / dd : 1.0;
        s.sn[j] = dd > 0 ? b / dd : 0.0;
        s.H[(size_t)j * R + j] = dd;
        s.H[(size_t)(j + 1) * R + j] = 0.0;
        s.g[j + 1] = -s.sn[j] * s.g[j];
        s.g[j] = s.cs[j] * s.g[j];
        s.k = j + 1;
        s.est = std::fabs(s.g[j + 1]) / s.bnorm;
        if (!std::isfinite(s.est)) return fail(FDE_ENOCONV, "Arnoldi of instance %d produced a non-finite value", i);
        if (std::fabs(s.g[j + 1]) <= tol * s.bnorm || s.its >= o.maxit) continue;
        next.push_back(i);
      }
      if (next != cyc) {
        cyc = next;
        if (!cyc.empty()) {
          STCHK(build_solve_maps(P, cyc, S));
          built = cyc;
        }
      }
    }
    // x += Z y for every instance of the cycle (y[0] carries k)
    std::vector<double> ybuf((size_t)count * (R + 1), 0.0);
    for (int i : active) {
      InstState &s = st[i];
      if (!s.in_cycle) continue;
      double *y = &ybuf[(size_t)i * (R + 1)];
      y[0] = s.k;
      for (int r = s.k - 1; r >= 0; --r) {
        double t = s.g[r];
        for (int c = r + 1; c < s.k; ++c) t -= s.H[(size_t)r * R + c] * y[1 + c];
        y[1 + r] = t / s.H[(size_t)r * R + r];
      }
      s.in_cycle = false;
      ++s.restarts;
    }
    HIPCHK(hipMemcpy(P->d_y, ybuf.data(), ybuf.size() * sizeof(double), hipMemcpyHostToDevice));
    if (active != built) {
      STCHK(build_solve_maps(P, active, S));
      built = active;
    }
    HIPCHK(run(L, "update_x", 3.0 * S.vec_bytes, [&] { return launch_update_x(P->d_desc, S.kry, S.n_kry, stream); }));
    std::vector<int> still;
    for (int i : active)
      if (!st[i].done) still.push_back(i);
    active = still;
  }
  STCHK(sync_and_flush(L));
  return check_trsv_err(P);
}

static fde_status check_opts(const fde_solve_opts *o, fde_solve_opts *out) {
  fde_solve_opts d{1e-10, 20, 1000, nullptr, FDE_MEM_HOST, FDE_X0_SOLUTION};
  if (o) d = *o;
  if (d.x0_kind != FDE_X0_SOLUTION && d.x0_kind != FDE_X0_LOWRANK)
    return fail(FDE_EINVAL, "unknown x0_kind %d", d.x0_kind);
  if (!(d.rtol > 0.0) || !std::isfinite(d.rtol)) return fail(FDE_EINVAL, "rtol must be positive");
  if (d.restart < 1 || d.restart > 64) return fail(FDE_EINVAL, "restart must be in 1..64");
  if (d.maxit < 0) return fail(FDE_EINVAL, "maxit must be >= 0");
  if (d.mem_space != FDE_MEM_HOST && d.mem_space != FDE_MEM_DEVICE)
    return fail(FDE_EINVAL, "unknown mem_space %d", d.mem_space);
  *out = d;
  return FDE_OK;
}

static fde_status copy_in(fde_bvm *h, double *dst, const double *src, size_t count, int mem) {
  HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(double),
                        mem == FDE_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        h->stream));
  return FDE_OK;
}

static fde_status copy_out(fde_bvm *h, double *dst, const double *src, size_t count, int mem) {
  HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(double),
                        mem == FDE_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        h->stream));
  return FDE_OK;
}

static fde_status solve_plan(Plan *P, const double *const *u0, const double *const *f,
                             double *const *u, const double *const *x0, const fde_solve_opts &o,
                             fde_solve_info *info) {
  fde_bvm *L = P->lead;
  const int count = (int)P->hs.size();
  const int prec = P->hs[0]->prec;
  for (int i = 0; i < count; ++i) {
    fde_bvm *h = P->hs[i];
    if (h->prec < 0) return fail(FDE_EINVAL, "fde_precond_factor must succeed before solving (instance %d)", i);
    if (h->prec != prec) return fail(FDE_EINVAL, "all instances of a batch need the same precision");
    if (!u0[i] || !f[i] || !u[i]) return fail(FDE_EINVAL, "u0, f and u are required (instance %d)", i);
    if (h->stream != L->stream) HIPCHK(hipStreamSynchronize(h->stream));
  }
  const int cap = prec == FDE_FP64 ? trsv_coop_capacity<double>() : trsv_coop_capacity<float>();
  STCHK(plan_prepare(P, o.restart, cap));
  hipEvent_t e0 = get_event(L), e1 = get_event(L);
  HIPCHK(hipEventRecord(e0, L->stream));
  for (int i = 0; i < count; ++i) {
    fde_bvm *h = P->hs[i];
    STCHK(copy_in(L, h->d_u0, u0[i], h->m, o.mem_space));
    STCHK(copy_in(L, h->d_f, f[i], (size_t)(h->s + 1) * h->m, o.mem_space));
    if (x0 && x0[i]) STCHK(copy_in(L, h->d_x, x0[i], h->n(), o.mem_space));
    else HIPCHK(hipMemsetAsync(h->d_x, 0, h->n() * sizeof(double), L->stream));
  }
  std::vector<InstState> st(count);
  std::vector<char> has_x0(count, 0);
  for (int i = 0; i < count; ++i) has_x0[i] = (x0 && x0[i]) ? 1 : 0;
  fde_status gs = gmres_plan(P, o, has_x0, st);
  if (gs != FDE_OK && gs != FDE_ENOCONV) return gs;
  const std::string msg = g_err;
  for (int i = 0; i < count; ++i) STCHK(copy_out(L, u[i], P->hs[i]->d_x, P->hs[i]->n(), o.mem_space));
  HIPCHK(hipEventRecord(e1, L->stream));
  STCHK(sync_and_flush(L));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  L->evpool.push_back(e0);
  L->evpool.push_back(e1);
  bool all_conv = true;
  for (int i = 0; i < count; ++i) {
    if (!st[i].conv) all_conv = false;
    if (!info) continue;
    fde_solve_info &f_ = info[i];
    std::memset(&f_, 0, sizeof f_);
    f_.iters = st[i].its;
    f_.restarts = st[i].restarts;
    f_.converged = st[i].conv ? 1 : 0;
    f_.precision = prec;
    f_.true_relres = st[i].truer;
    f_.est_relres = st[i].est;
    f_.t_factor_ms = P->hs[i]->t_factor_ms;
    f_.t_solve_ms = ms;
  }
  if (gs != FDE_OK) {
    g_err = msg;
    return gs;
  }
  if (!all_conv) return fail(FDE_ENOCONV, "GMRES reached maxit=%d before rtol=%.1e", o.maxit, o.rtol);
  return FDE_OK;
}

extern "C" fde_status fde_bvm_solve(fde_bvm *h, const double *u0, const double *f, double *u,
                                    const fde_solve_opts *o, fde_solve_info *info) {
  if (!h) return fail(FDE_EINVAL, "handle is NULL");
  fde_solve_opts oo;
  STCHK(check_opts(o, &oo));
  const double *x0 = oo.x0;
  return solve_plan(h->self, &u0, &f, &u, &x0, oo, info);
}

static fde_status batch_plan(fde_bvm *const *hs, int count, Plan **P) {
  std::vector<fde_bvm *> v(hs, hs + count);
  for (int i = 0; i < count; ++i) {
    if (!hs[i]) return fail(FDE_EINVAL, "handle %d is NULL", i);
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(FDE_EINVAL, "handle %d appears twice in the batch", i);
  }
  return plan_create(v, P);
}

extern "C" fde_status fde_precond_factor_batch(fde_bvm *const *hs, int count, fde_precision prec) {
  if (count < 0 || (count > 0 && !hs)) return fail(FDE_EINVAL, "invalid batch arguments");
  if (count == 0) return FDE_OK;
  Plan *P = nullptr;
  STCHK(batch_plan(hs, count, &P));
  fde_status st = factor_plan(P, prec);
  plan_free(P);
  return st;
}

extern "C" fde_status fde_bvm_solve_batch(fde_bvm *const *hs, int count, const double *const *u0,
                                          const double *const *f, double *const *u,
                                          const fde_solve_opts *o, fde_solve_info *info) {
  if (count < 0 || (count > 0 && (!hs || !u0 || !f || !u)))
    return fail(FDE_EINVAL, "invalid batch arguments");
  if (count == 0) return FDE_OK;
  fde_solve_opts oo;
  STCHK(check_opts(o, &oo));
  if (oo.x0) return fail(FDE_EINVAL, "batch solves take no x0 in opts; use fde_bvm_solve_batch_x0");
  Plan *P = nullptr;
  STCHK(batch_plan(hs, count, &P));
  std::vector<const double *> x0(count, nullptr);
  fde_status st = solve_plan(P, u0, f, u, x0.data(), oo, info);
  plan_free(P);
  return st;
}

extern "C" fde_status fde_bvm_solve_batch_x0(fde_bvm *const *hs, int count, const double *const *u0,
                                             const double *const *f, const double *const *x0,
                                             double *const *u, const fde_solve_opts *o,
                                             fde_solve_info *info) {
  if (count < 0 || (count > 0 && (!hs || !u0 || !f || !u || !x0)))
    return fail(FDE_EINVAL, "invalid batch arguments");
  if (count == 0) return FDE_OK;
  fde_solve_opts oo;
  STCHK(check_opts(o, &oo));
  Plan *P = nullptr;
  STCHK(batch_plan(hs, count, &P));
  fde_status st = solve_plan(P, u0, f, u, x0, oo, info);
  plan_free(P);
  return st;
}

// ====================================================================================
// single steps (per-kernel checks), all through the handle's own plan
// ====================================================================================
static fde_status self_maps(fde_bvm *h, SolveMaps &S) {
  const int cap = h->prec == FDE_MIXED_C32 ? trsv_coop_capacity<float>() : trsv_coop_capacity<double>();
  STCHK(plan_prepare(h->self, std::max(h->self->R, 1), cap));
  return build_solve_maps(h->self, {0}, S);
}

extern "C" fde_status fde_build_rhs(fde_bvm *h, const double *u0, const double *f, double *b,
                                    int mem_space) {
  if (!h || !u0 || !f || !b) return fail(FDE_EINVAL, "NULL argument");
  if (mem_space != FDE_MEM_HOST && mem_space != FDE_MEM_DEVICE) return fail(FDE_EINVAL, "bad mem_space");
  SolveMaps S;
  STCHK(self_maps(h, S));
  STCHK(copy_in(h, h->d_u0, u0, h->m, mem_space));
  STCHK(copy_in(h, h->d_f, f, (size_t)(h->s + 1) * h->m, mem_space));
  STCHK(op_rhs(h->self, S));
  STCHK(copy_out(h, b, h->d_b, h->n(), mem_space));
  return sync_and_flush(h);
}

extern "C" fde_status fde_apply_matvec(fde_bvm *h, const double *z, double *w, int mem_space) {
  if (!h || !z || !w) return fail(FDE_EINVAL, "NULL argument");
  if (mem_space != FDE_MEM_HOST && mem_space != FDE_MEM_DEVICE) return fail(FDE_EINVAL, "bad mem_space");
  SolveMaps S;
  STCHK(self_maps(h, S));
  STCHK(copy_in(h, h->d_sio, z, h->n(), mem_space));
  STCHK(op_matvec(h->self, S, VS_SIO, 0, VS_TMP, 0));
  STCHK(copy_out(h, w, h->d_tmp, h->n(), mem_space));
  return sync_and_flush(h);
}

static fde_status self_band_op(fde_bvm *h, const double *z, double *w, int mem_space, int mode,
                               const char *name) {
  if (!h || !z || !w) return fail(FDE_EINVAL, "NULL argument");
  if (mem_space != FDE_MEM_HOST && mem_space != FDE_MEM_DEVICE) return fail(FDE_EINVAL, "bad mem_space");
  SolveMaps S;
  STCHK(self_maps(h, S));
  STCHK(copy_in(h, h->d_sio, z, h->n(), mem_space));
  HIPCHK(run(h, name, 16.0 * h->n(), [&] {
    return launch_bvm_matvec(h->self->d_desc, S.mv, S.n_mv, S.max_log2L, VS_SIO, 0, VS_TMP, 0, mode,
                             h->stream);
  }));
  STCHK(copy_out(h, w, h->d_tmp, h->n(), mem_space));
  return sync_and_flush(h);
}

extern "C" fde_status fde_bvm_strang_apply(fde_bvm *h, const double *z, double *w, int mem_space) {
  return self_band_op(h, z, w, mem_space, 2, "strang_apply");
}

extern "C" fde_status fde_bvm_lowrank_correction(fde_bvm *h, const double *z, double *c, int mem_space) {
  return self_band_op(h, z, c, mem_space, 3, "lowrank_correction");
}

extern "C" fde_status fde_apply_precond(fde_bvm *h, const double *v, double *z, int mem_space) {
  if (!h || !v || !z) return fail(FDE_EINVAL, "NULL argument");
  if (mem_space != FDE_MEM_HOST && mem_space != FDE_MEM_DEVICE) return fail(FDE_EINVAL, "bad mem_space");
  if (h->prec < 0) return fail(FDE_EINVAL, "fde_precond_factor must succeed first");
  SolveMaps S;
  STCHK(self_maps(h, S));
  STCHK(copy_in(h, h->d_sio, v, h->n(), mem_space));
  STCHK(op_precond(h->self, S, VS_SIO, 0, VS_TMP, 0));
  STCHK(copy_out(h, z, h->d_tmp, h->n(), mem_space));
  STCHK(sync_and_flush(h));
  return check_trsv_err(h->self);
}

extern "C" fde_status fde_time_rfft(fde_bvm *h, const double *v, double *vhat, int mem_space) {
  if (!h || !v || !vhat) return fail(FDE_EINVAL, "NULL argument");
  if (mem_space != FDE_MEM_HOST && mem_space != FDE_MEM_DEVICE) return fail(FDE_EINVAL, "bad mem_space");
  SolveMaps S;
  STCHK(self_maps(h, S));
  STCHK(copy_in(h, h->d_sio, v, h->n(), mem_space));
  HIPCHK(launch_time_rfft(h->self->d_desc, S.tfft, S.n_tfft, S.max_log2s, VS_SIO, 0, h->stream));
  HIPCHK(hipMemcpy2DAsync(vhat, sizeof(double2) * h->m, h->d_Vh, sizeof(double2) * h->mp,
                          sizeof(double2) * h->m, h->nb,
                          mem_space == FDE_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          h->stream));
  return sync_and_flush(h);
}

extern "C" fde_status fde_toeplitz_apply(fde_bvm *h, const double *x, double *y, int count,
                                         int mem_space) {
  if (!h || !x || !y || count < 1) return fail(FDE_EINVAL, "invalid argument");
  if (count > h->s) return fail(FDE_EINVAL, "count must be <= s (%d)", h->s);
  if (mem_space != FDE_MEM_HOST && mem_space != FDE_MEM_DEVICE) return fail(FDE_EINVAL, "bad mem_space");
  SolveMaps S;
  STCHK(self_maps(h, S));
  const size_t cnt = (size_t)count * h->m;
  std::vector<HostMap> hm = {make_map({0}, {count})};
  std::vector<ItemMap> dm;
  STCHK(upload_maps(h->self, hm, dm));
  STCHK(copy_in(h, h->d_sio, x, cnt, mem_space));
  HIPCHK(run(h, "toeplitz", 16.0 * cnt, [&] {
    return launch_bvm_matvec(h->self->d_desc, dm[0], count, h->log2L, VS_SIO, 0, VS_TMP, 0, 1, h->stream);
  }));
  STCHK(copy_out(h, y, h->d_tmp, cnt, mem_space));
  return sync_and_flush(h);
}

extern "C" fde_status fde_get_factor_block(fde_bvm *h, int k, double *out) {
  if (!h || !out) return fail(FDE_EINVAL, "NULL argument");
  if (h->prec < 0) return fail(FDE_EINVAL, "no factorization stored");
  if (k < 0 || k >= h->nb) return fail(FDE_EINVAL, "block %d out of range 0..%d", k, h->nb - 1);
  const int m = h->m, mp = h->mp;
  const size_t esz = h->prec == FDE_FP64 ? sizeof(double2) : sizeof(float2);
  std::vector<char> raw((size_t)mp * mp * esz);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipMemcpy(raw.data(), (char *)h->d_K + (size_t)k * mp * mp * esz, raw.size(), hipMemcpyDeviceToHost));
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
