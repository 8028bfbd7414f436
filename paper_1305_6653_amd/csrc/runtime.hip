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
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "fdebvm.h"
#include "kernels.hpp"

// Named host-side ranges for timeline tools (roctx; rocprofv3 --marker-trace shows them).
// Without a tool attached the calls return at once.  The factor and solve entry points wait
// for their device work before returning, so their outer ranges span it; inner ranges mark
// where the host issues each phase.
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

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

// Fifth-order generalized Adams method, (nu, mu-nu) = (2, 2).  Each row r reads
// u_r - u_{r-1} = tau sum_i beta_i g_{c+i}, where beta_i is the integral over the step
// [r-1, r] of the Lagrange basis polynomial of node i of the five nodes c..c+4 (in units of
// tau).  Main formula: nodes centred on r (c = r-2); row 1: nodes 0..4; rows s-1, s: nodes
// s-4..s.  Weights in 720ths; e.g. the main formula's are those of the quartic integrated
// over its second panel, the mirror image of the third.
HostFormula formula_gam5() {
  HostFormula F;
  F.nu = 2;
  F.mu = 4;
  const double d = 720.0;
  F.a = {0.0, -1.0, 1.0, 0.0, 0.0};
  F.b = {-19.0 / d, 346.0 / d, 456.0 / d, -74.0 / d, 11.0 / d};
  F.ai = {-1.0, 1.0, 0.0, 0.0, 0.0};
  F.bi = {251.0 / d, 646.0 / d, -264.0 / d, 106.0 / d, -19.0 / d};
  F.af = {0.0, 0.0, -1.0, 1.0, 0.0,  // row s-1: step [2, 3] of the last five nodes
          0.0, 0.0, 0.0, -1.0, 1.0};  // row s:   step [3, 4]
  F.bf = {11.0 / d, -74.0 / d, 456.0 / d, 346.0 / d, -19.0 / d,
          -19.0 / d, 106.0 / d, -264.0 / d, 646.0 / d, 251.0 / d};
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
  bool owned;  // false: the events belong to a recorded graph and are reused by its replays
  int step;    // Arnoldi step of a restart cycle (-1 outside the cycle)
};

// A recorded launch sequence (hipGraph) and the timing events recorded inside it.
struct GraphSeg {
  hipGraphExec_t exec = nullptr;
  std::vector<Pending> prof;
};

// Set while a launch sequence is being recorded on this thread.
thread_local GraphSeg *g_capture = nullptr;
// Arnoldi step whose launches are being issued (-1 outside a restart cycle).
thread_local int g_step = -1;

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
  // band route: a second stream for the reduction's next panel, which runs beside the rest of
  // the current panel's update, and the two events that order it
  hipStream_t side_stream = nullptr;
  hipEvent_t side_ev[2] = {nullptr, nullptr};
  std::vector<void *> allocs;
  double *d_g = nullptr, *d_dp = nullptr, *d_dm = nullptr, *d_cG = nullptr;
  double2 *d_chat = nullptr, *d_twL = nullptr, *d_tws = nullptr, *d_lam = nullptr, *d_mu = nullptr;
  int *d_band_c = nullptr;
  double *d_band_a = nullptr, *d_band_b = nullptr;
  // ---- factors
  void *d_K = nullptr, *d_dinv = nullptr;
  size_t K_bytes = 0;
  unsigned long long *d_tsflags = nullptr;
  int prec = -1;
  double t_factor_ms = 0.0;
  // ---- vectors
  int R = 0, nblk = 1;
  double *d_V = nullptr, *d_Z = nullptr;
  double *d_w = nullptr, *d_x = nullptr, *d_b = nullptr, *d_tmp = nullptr, *d_sio = nullptr;
  double *d_u0 = nullptr, *d_f = nullptr, *d_Ju0 = nullptr;
  double2 *d_Vh = nullptr;
  // ---- Hessenberg route to the blocks (allocated when first factored that way): H, Q, Q^T
  // [m][mp], multipliers and exchanges [nb][mp], the block-solve vector [nb][mp], and the
  // reduction's workspace
  int blk_route = FDE_BLOCKS_LU;
  double *d_hH = nullptr, *d_hQ = nullptr, *d_hQt = nullptr;
  double2 *d_hl = nullptr, *d_Vh2 = nullptr;
  int *d_hpiv = nullptr;
  HessWork hwk{};
  // ---- band route to the blocks (allocated when first factored that way): [H; Q] [2 mp][mp]
  // of J = Q H Q^T (H of lower bandwidth 64), Q^T [mp][mp], the row orders of the pivoted band
  // LU [nb][npan][128], the reduction's workspace and error flag
  double *d_bAQ = nullptr, *d_bQt = nullptr, *d_bwork = nullptr;
  int *d_bpiv = nullptr, *d_berr = nullptr;
  // ---- BCCB preconditioner tables (allocated when a BCCB preconditioner is factored)
  double2 *d_chirp = nullptr, *d_bh = nullptr, *d_lamx = nullptr;
  double lam0s = 0.0;
  // ---- the plan of this handle alone
  Plan *self = nullptr;
  // ---- options (fde_bvm_set_option)
  int opt_graphs = 1, opt_autotune = 1, opt_trsv_w = 0;
  int opt_precond = FDE_PC_STRANG;  // chosen kind; pc = the kind of the current factorization
  int pc = FDE_PC_STRANG;
  int opt_side = FDE_SIDE_RIGHT;
  int opt_blocks = FDE_BLOCKS_AUTO;
  int opt_ortho = FDE_ORTHO_MGS;
  int opt_x0_gate = 10000;  // millionths of ||b||
  int x0_kept = 0;          // the last solve used its initial guess
  // ---- profiling
  bool prof = false;
  int prof_step_limit = 1 << 30;  // launches of cycle steps >= this were gated off: not counted
  std::map<std::string, ProfEntry> prof_tab;
  std::vector<Pending> pend;
  std::vector<hipEvent_t> evpool;

  size_t n() const { return (size_t)s * m; }
};

// ====================================================================================
// device memory helpers
// ====================================================================================
static fde_status noalloc_scratch(void **out);

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

// Launch with optional timing: HIP events around the launch on the handle's stream.  While a
// launch sequence is recorded, the events are recorded into the graph as event nodes and
// are read after every replay.
template <typename Fn>
static hipError_t run(fde_bvm *h, const char *name, double work, Fn &&launch,
                      hipStream_t on = nullptr) {
  if (!h->prof) return launch();
  const hipStream_t st = on ? on : h->stream;
  hipEvent_t a = get_event(h), b = get_event(h);
  if (g_capture) {
    hipError_t e = hipEventRecordWithFlags(a, st, hipEventRecordExternal);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecordWithFlags(b, st, hipEventRecordExternal);
    g_capture->prof.push_back({name, work, a, b, false, g_step});
    return e;
  }
  (void)hipEventRecord(a, st);
  hipError_t e = launch();
  (void)hipEventRecord(b, st);
  h->pend.push_back({name, work, a, b, true, g_step});
  return e;
}

static fde_status sync_and_flush(fde_bvm *h) {
  HIPCHK(hipStreamSynchronize(h->stream));
  for (auto &p : h->pend) {
    float ms = 0.0f;
    if (p.step < h->prof_step_limit && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ProfEntry &e = h->prof_tab[p.name];
      e.ms += ms;
      e.count += 1;
      e.work += p.work;
    }
    if (p.owned) {
      h->evpool.push_back(p.a);
      h->evpool.push_back(p.b);
    }
  }
  h->pend.clear();
  return FDE_OK;
}

// Device-wide counter of block-solve epochs, one per GPU (64-bit: never wraps in practice).
// Every preconditioner apply draws a new value on the device, so flags left by earlier
// applies (of any plan, eager or replayed) never match.
static std::mutex g_epoch_mu;
static unsigned long long *g_epoch_ctr[64] = {};

static fde_status epoch_counter(unsigned long long **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(FDE_EUNSUPPORTED, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_epoch_mu);
  if (!g_epoch_ctr[dev]) {
    void *p = nullptr;
    STCHK(dalloc_raw(&p, sizeof(unsigned long long)));
    if (hipMemset(p, 0, sizeof(unsigned long long)) != hipSuccess) {
      (void)hipFree(p);
      return fail(FDE_EDEVICE, "epoch counter initialisation failed");
    }
    g_epoch_ctr[dev] = (unsigned long long *)p;  // kept for the life of the process
  }
  *out = g_epoch_ctr[dev];
  return FDE_OK;
}

// ====================================================================================
// plans: descriptor table + item maps
// ====================================================================================
struct HostMap {
  std::vector<int> ids, pre;
  int items = 0;
};

// Item maps of the solve-phase launches over every instance of a plan.
struct SolveMaps {
  ItemMap mv, tfft, trsv, kry, rhs, ju0, blk, qg;
  int n_mv = 0, n_tfft = 0, n_trsv = 0, n_kry = 0, n_rhs = 0, n_ju0 = 0, n_blk = 0, n_qg = 0;
  int pc = 0, route = FDE_BLOCKS_LU;
  int max_log2L = 1, max_log2s = 1, max_mp = 64;
  int tfft_cols = 16;  // spatial columns per time-FFT workgroup
  int npan_u = 0;      // panels per block if every instance has the same count, else 0
  int prec = -1;
  int trsv_solo = 0;   // block solve by one workgroup per block, an ordinary launch (k_trsv)
  size_t kry_one_n = 0;  // largest vector if every instance's vectors are one chunk, else 0
  double trsv_bytes = 0, vec_bytes = 0, tfft_bytes = 0, bccb_bytes = 0, qg_flops = 0, band_l_bytes = 0;
};

// The same maps with their items skipped for instances whose gate entry is zero.
static SolveMaps gated(const SolveMaps &S, const int *gate) {
  SolveMaps G = S;
  for (ItemMap *m : {&G.mv, &G.tfft, &G.trsv, &G.kry, &G.rhs, &G.ju0, &G.blk, &G.qg}) m->gate = gate;
  return G;
}

struct Plan {
  std::vector<fde_bvm *> hs;
  fde_bvm *lead = nullptr;  // stream and profiling owner
  int R = 0;
  InstDesc *d_desc = nullptr;
  double *d_part = nullptr, *d_H = nullptr, *d_y = nullptr, *d_nrm = nullptr, *d_h2 = nullptr;
  unsigned *d_gctr = nullptr;
  int *d_err = nullptr, *d_flag = nullptr;
  int *d_arena = nullptr;
  size_t arena_ints = 0;
  std::vector<InstDesc> desc;
  std::vector<int> arena_host;  // kept alive until the next rebuild (async upload source)
  std::vector<size_t> part_off;
  std::vector<void *> allocs;
  bool desc_dirty = true;
  // device GMRES control
  GmresCtl *d_ctl = nullptr;
  GmresWork *d_work = nullptr;
  int *d_gates = nullptr;             // [GATE_COUNT][count]
  unsigned long long *d_epoch = nullptr;  // epoch of this plan's current block solve
  std::vector<GmresCtl> ctl_host;
  std::vector<int> gates_host;
  // pinned host staging: the control records and the block-solve error flag read back once
  // per cycle (the factorization's pivot flag in the int after that flag), the control
  // records and gates uploaded once per solve (pin_* byte offsets)
  void *pin = nullptr;
  size_t pin_err = 0, pin_ctl_up = 0, pin_gates_up = 0;
  double *pin_parts = nullptr;  // the reduction partials read back for the norms of b
  // solve maps over all instances, in their own allocation (recorded graphs refer to them)
  SolveMaps full;
  bool full_ok = false;
  bool trsv_solo = false;  // the block solve's launch form (see trsv_solo_choice)
  int *d_fullmaps = nullptr;
  size_t fullmaps_ints = 0;
  std::vector<int> fullmaps_host;
  // recorded launch sequences: the first restart step, Arnoldi steps [j0, j1) of a cycle,
  // and the end of a cycle (least-squares update) followed by the next restart step
  GraphSeg seg_restart, seg_finish;
  std::map<std::pair<int, int>, GraphSeg> seg_steps;
  int graph_R = -1, graph_prec = -1, graph_side = -1, graph_ortho = -1;
  bool graph_off = false;
  std::vector<int> pred_steps;  // Arnoldi steps of each cycle of the previous solve
};

static void graph_release(Plan *P, GraphSeg &g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g.exec = nullptr;
  for (Pending &p : g.prof) {
    P->lead->evpool.push_back(p.a);
    P->lead->evpool.push_back(p.b);
  }
  g.prof.clear();
}

static bool graphs_recorded(const Plan *P) {
  if (P->seg_restart.exec || P->seg_finish.exec) return true;
  for (auto &kv : P->seg_steps)
    if (kv.second.exec) return true;
  return false;
}

static void graphs_invalidate(Plan *P) {
  graph_release(P, P->seg_restart);
  graph_release(P, P->seg_finish);
  for (auto &kv : P->seg_steps) graph_release(P, kv.second);
  P->seg_steps.clear();
  P->graph_R = P->graph_prec = P->graph_side = P->graph_ortho = -1;
}

static void plan_free(Plan *P) {
  if (!P) return;
  if (graphs_recorded(P)) (void)hipStreamSynchronize(P->lead->stream);
  graphs_invalidate(P);
  for (void *p : P->allocs) (void)hipFree(p);
  if (P->pin) (void)hipHostFree(P->pin);
  if (P->pin_parts) (void)hipHostFree(P->pin_parts);
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
    out.push_back(ItemMap{P->d_arena + oi, P->d_arena + op, (int)m.ids.size(), nullptr});
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
  d.blk = h->blk_route;
  if (h->blk_route == FDE_BLOCKS_BAND) {
    d.hH = h->d_bAQ;
    d.hQ = h->d_bAQ ? h->d_bAQ + (size_t)h->mp * h->mp : nullptr;
    d.hQt = h->d_bQt;
    d.hpiv = h->d_bpiv;
  } else {
    d.hH = h->d_hH;
    d.hQ = h->d_hQ;
    d.hQt = h->d_hQt;
    d.hpiv = h->d_hpiv;
  }
  d.hl = h->d_hl;
  d.Vts = h->blk_route != FDE_BLOCKS_LU ? h->d_Vh2 : h->d_Vh;
  d.pc = h->pc;
  d.lam0s = h->lam0s;
  d.chirp = h->d_chirp;
  d.bh = h->d_bh;
  d.lamx = h->d_lamx;
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
// ---- workgroups per block of the cooperative block solve --------------------------------
// All items of a launch must be co-resident (W * sum(nb) <= capacity), so that a block's
// workgroups never wait on a workgroup that has not started.  Within that limit the value
// comes from, in order: the lead handle's option, the autotuner's table for the plan's shape
// (sizes of all instances and the precision), or the largest value that fits.
static std::mutex g_tune_mu;
static std::map<std::string, int> g_tuned_w;
static std::map<std::string, int> g_tuned_cols;  // time-FFT spatial columns per workgroup

static std::string plan_shape_key(const Plan *P, int prec) {
  std::string k = prec == FDE_FP64 ? "f64" : "c32";
  if (!P->hs.empty() && P->hs[0]->blk_route == FDE_BLOCKS_HESSENBERG) k += "h";
  if (!P->hs.empty() && P->hs[0]->blk_route == FDE_BLOCKS_BAND) k += "b";
  char buf[32];
  for (const fde_bvm *h : P->hs) {
    snprintf(buf, sizeof buf, ":%dx%d", h->m, h->s);
    k += buf;
  }
  return k;
}

// Autotuned choices so far, "shape=W" separated by ';' (for reports).
// The time-FFT column groups appear as "shape/tfft=cols".
static std::string tuned_summary() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  std::string out;
  for (auto &kv : g_tuned_w) {
    if (!out.empty()) out += ";";
    out += kv.first + "=" + std::to_string(kv.second);
  }
  for (auto &kv : g_tuned_cols) {
    if (!out.empty()) out += ";";
    out += kv.first + "/tfft=" + std::to_string(kv.second);
  }
  return out;
}

static int trsv_capacity(int prec) {
  return prec == FDE_MIXED_C32 ? trsv_coop_capacity<float>() : trsv_coop_capacity<double>();
}

static int trsv_wmax(const Plan *P, const fde_bvm *h, int prec) {
  long total_nb = 0;
  for (const fde_bvm *q : P->hs) total_nb += q->nb;
  const int cap = trsv_capacity(prec);
  const long w = (cap > 0 && total_nb <= cap) ? cap / total_nb : 1;
  return (int)std::max(1L, std::min<long>(h->npan, w));
}

// The value -1 (option or autotuner) selects the ordinary one-workgroup-per-block launch.
static int trsv_choice(const Plan *P, int prec, int wmax) {
  if (P->lead->opt_trsv_w != 0) return P->lead->opt_trsv_w;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tuned_w.find(plan_shape_key(P, prec));
  return it != g_tuned_w.end() ? it->second : wmax;
}

static int trsv_workgroups(const Plan *P, const fde_bvm *h, int prec) {
  const int wmax = trsv_wmax(P, h, prec);
  return std::max(1, std::min(wmax, trsv_choice(P, prec, wmax)));
}

static bool trsv_solo_choice(const Plan *P, int prec) { return trsv_choice(P, prec, 1) == -1; }

static fde_status plan_prepare(Plan *P, int R, int prec) {
  const int count = (int)P->hs.size();
  for (fde_bvm *h : P->hs) STCHK(ensure_krylov(h, R));
  if (P->R < R || !P->d_H) {
    for (void *p : {(void *)P->d_part, (void *)P->d_H, (void *)P->d_y, (void *)P->d_nrm, (void *)P->d_h2,
                    (void *)P->d_gctr}) {
      if (!p) continue;
      auto it = std::find(P->allocs.begin(), P->allocs.end(), p);
      if (it != P->allocs.end()) P->allocs.erase(it);
      (void)hipFree(p);
    }
    size_t parts = 0;
    P->part_off.assign(count, 0);
    for (int i = 0; i < count; ++i) {  // part0, part1, then the [R+1][nblk] projection partials
      P->part_off[i] = parts;
      parts += (size_t)(R + 3) * P->hs[i]->nblk;
    }
    void *p = nullptr;
    STCHK(plan_alloc(P, &p, parts * sizeof(double)));
    P->d_part = (double *)p;
    if (P->pin_parts) (void)hipHostFree(P->pin_parts);
    P->pin_parts = nullptr;
    HIPCHK(hipHostMalloc((void **)&P->pin_parts, parts * sizeof(double), hipHostMallocDefault));
    STCHK(plan_alloc(P, &p, (size_t)count * (R + 2) * sizeof(double)));
    P->d_H = (double *)p;
    STCHK(plan_alloc(P, &p, (size_t)count * (R + 1) * sizeof(double)));
    P->d_y = (double *)p;
    STCHK(plan_alloc(P, &p, (size_t)count * 2 * sizeof(double)));
    P->d_nrm = (double *)p;
    STCHK(plan_alloc(P, &p, (size_t)count * (R + 2) * sizeof(double)));
    P->d_h2 = (double *)p;
    STCHK(plan_alloc(P, &p, (size_t)count * sizeof(unsigned)));
    P->d_gctr = (unsigned *)p;
    HIPCHK(hipMemset(P->d_gctr, 0, (size_t)count * sizeof(unsigned)));
    P->R = R;
    P->desc_dirty = true;
  }
  P->desc.resize(count);
  const bool solo = trsv_solo_choice(P, prec);
  if (solo != P->trsv_solo) P->full_ok = false;  // the launch sequence changes: new graphs
  P->trsv_solo = solo;
  for (int i = 0; i < count; ++i) {
    fde_bvm *h = P->hs[i];
    InstDesc d = make_desc(h);
    d.W = trsv_workgroups(P, h, prec);
    if (d.W != P->desc[i].W) P->full_ok = false;  // item counts change: new maps, new graphs
    d.part0 = P->d_part + P->part_off[i];
    d.part1 = d.part0 + h->nblk;
    d.partm = d.part0 + 2 * (size_t)h->nblk;
    d.h2 = P->d_h2 + (size_t)i * (R + 2);
    d.gctr = P->d_gctr + i;
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
  const size_t count = hs.size();
  const size_t ctl_bytes = (sizeof(GmresCtl) * count + 255) / 256 * 256;
  const size_t gate_bytes = (sizeof(int) * GATE_COUNT * count + 255) / 256 * 256;
  if ((st = plan_alloc(P, &p, ctl_bytes + gate_bytes + 256 + sizeof(GmresWork) * count)) != FDE_OK) {
    plan_free(P);
    return st;
  }
  char *base = (char *)p;
  P->d_ctl = (GmresCtl *)base;
  P->d_gates = (int *)(base + ctl_bytes);
  P->d_epoch = (unsigned long long *)(base + ctl_bytes + gate_bytes);
  P->d_work = (GmresWork *)(base + ctl_bytes + gate_bytes + 256);
  if (hipMemset(base, 0, ctl_bytes + gate_bytes + 256) != hipSuccess) {
    plan_free(P);
    return fail(FDE_EDEVICE, "plan control initialisation failed");
  }
  P->ctl_host.assign(count, GmresCtl{});
  P->gates_host.assign(GATE_COUNT * count, 0);
  P->pin_err = ctl_bytes;
  P->pin_ctl_up = ctl_bytes + 256;
  P->pin_gates_up = 2 * ctl_bytes + 256;
  if (hipHostMalloc(&P->pin, 2 * ctl_bytes + 256 + gate_bytes, hipHostMallocDefault) != hipSuccess) {
    P->pin = nullptr;
    plan_free(P);
    return fail(FDE_EDEVICE, "pinned host buffer allocation failed");
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

// In-place radix-2 FFT (e^{-2 pi i jk/N}, N a power of two), natural order in and out.
static void host_fft(std::vector<cd> &a) {
  const size_t N = a.size();
  for (size_t i = 1, j = 0; i < N; ++i) {
    size_t bit = N >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= N; len <<= 1) {
    const double th = -2.0 * M_PI / (double)len;
    for (size_t i = 0; i < N; i += len)
      for (size_t k = 0; k < len / 2; ++k) {
        const cd w = std::polar(1.0, th * (double)k);
        const cd u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
}

// Tables of the BCCB preconditioners (Section 3.1, eq. (x1) and (xc)):
//  * s(J) = dx^{-alpha} (dbar+ s(G) + dbar- s(G)^T), dbar the means of d+-, s(G) the order-m
//    circulant with first column g_1..g_{floor((m+1)/2)}, 0.., g_0 (s(G^T) read as s(G)^T);
//    its eigenvalues lamx_j = DFT of the first column (by the same Bluestein route as on the
//    device, through the host FFT of length L);
//  * the chirp w_n = e^{-i pi n^2/m} (n^2 taken mod 2m, exact) and the FFT of the chirp filter
//    b_k = conj(w_k), b_{L-k} = conj(w_k), stored bit-reversed for the device's DIF/DIT pair;
//  * for S2~ the zero time frequency lam_0 = rho(1) = 0 becomes Re(lam_{s-1}).
static fde_status bccb_prepare(fde_bvm *h) {
  const int m = h->m, L = h->L;
  std::vector<cd> w(m);
  for (int n = 0; n < m; ++n) {
    const long long r = ((long long)n * n) % (2LL * m);
    w[n] = std::polar(1.0, -M_PI * (double)r / (double)m);
  }
  std::vector<cd> bf(L, cd(0.0, 0.0));
  for (int k = 0; k < m; ++k) {
    bf[k] = std::conj(w[k]);
    if (k > 0) bf[L - k] = std::conj(w[k]);
  }
  host_fft(bf);
  std::vector<double2> bh(L);
  for (int i = 0; i < L; ++i) {
    int r = 0;
    for (int b = 0; b < h->log2L; ++b) r |= ((i >> b) & 1) << (h->log2L - 1 - b);
    bh[i] = make_double2(bf[r].real(), bf[r].imag());  // position i holds frequency bitrev(i)
  }
  // first column of s(J)
  std::vector<double> cG(m, 0.0);
  const int hh = (m + 1) / 2;
  for (int i = 0; i < hh; ++i) cG[i] = h->g[i + 1];
  if (m - 1 >= hh) cG[m - 1] = h->g[0];
  double dbp = 0.0, dbm = 0.0;
  for (int i = 0; i < m; ++i) {
    dbp += h->dp[i];
    dbm += h->dm[i];
  }
  dbp /= m;
  dbm /= m;
  std::vector<cd> a(L, cd(0.0, 0.0));
  for (int n = 0; n < m; ++n) {
    const double cJ = h->scale * (dbp * cG[n] + dbm * cG[(m - n) % m]);
    a[n] = cJ * w[n];
  }
  host_fft(a);
  std::vector<cd> bnat(L, cd(0.0, 0.0));
  for (int k = 0; k < m; ++k) {
    bnat[k] = std::conj(w[k]);
    if (k > 0) bnat[L - k] = std::conj(w[k]);
  }
  host_fft(bnat);
  for (int i = 0; i < L; ++i) a[i] = std::conj(a[i] * bnat[i]);  // inverse FFT via conj(FFT(conj))
  host_fft(a);
  std::vector<double2> lamx(m);
  for (int j = 0; j < m; ++j) {
    const cd X = w[j] * std::conj(a[j]) / (double)L;
    lamx[j] = make_double2(X.real(), X.imag());
  }
  h->lam0s = h->lam[h->s - 1 < h->nb ? h->s - 1 : 1].real();  // Re(lam_{s-1}) = Re(lam_1)
  if (!h->d_chirp) {
    STCHK(dalloc_t(h, &h->d_chirp, (size_t)m));
    STCHK(dalloc_t(h, &h->d_bh, (size_t)L));
    STCHK(dalloc_t(h, &h->d_lamx, (size_t)m));
  }
  std::vector<double2> wd(m);
  for (int n = 0; n < m; ++n) wd[n] = make_double2(w[n].real(), w[n].imag());
  HIPCHK(hipMemcpy(h->d_chirp, wd.data(), sizeof(double2) * m, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->d_bh, bh.data(), sizeof(double2) * L, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->d_lamx, lamx.data(), sizeof(double2) * m, hipMemcpyHostToDevice));
  return FDE_OK;
}

static void destroy_handle(fde_bvm *h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  plan_free(h->self);
  h->self = nullptr;
  for (void *p : h->allocs) (void)hipFree(p);
  for (auto &p : h->pend)
    if (p.owned) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
  for (auto e : h->evpool) (void)hipEventDestroy(e);
  for (auto e : h->side_ev)
    if (e) (void)hipEventDestroy(e);
  if (h->side_stream) (void)hipStreamDestroy(h->side_stream);
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  delete h;
}

extern "C" fde_status fde_bvm_setup(const fde_problem *p, fde_bvm **out) {
  TraceRange tr_setup("fde_bvm_setup");
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
  // the kind as the int a C caller stored: a value outside the enumeration is rejected below,
  // and reading it through the enumeration type would already be undefined in C++
  static_assert(sizeof(fde_bvm_kind) == sizeof(int), "fde_bvm_kind is stored as an int");
  int kind = 0;
  std::memcpy(&kind, &p->kind, sizeof kind);
  HostFormula F;
  if (kind == FDE_BVM_TRAPEZOIDAL) {
    F = formula_trapezoidal();
  } else if (kind == FDE_BVM_GBDF3) {
    F = formula_gbdf3();
  } else if (kind == FDE_BVM_GAM5) {
    F = formula_gam5();
  } else if (kind == FDE_BVM_CUSTOM) {
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
    return fail(FDE_EINVAL, "unknown BVM kind %d", kind);
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
  {
    void *na = nullptr;  // the allocation-free apply's array: address looked up once per device
    fde_status sst = noalloc_scratch(&na);
    if (sst != FDE_OK) return bail(sst);
  }
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
  ALLOC(h->d_tsflags, (size_t)nb * h->npan * 2);  // 0: no epoch drawn yet (epochs start at 1)
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
  if (hipMemsetAsync(h->d_tsflags, 0, sizeof(unsigned long long) * nb * h->npan * 2, q) != hipSuccess ||
      hipMemsetAsync(h->d_Ju0, 0, sizeof(double) * m, q) != hipSuccess)
    return bail(fail(FDE_EDEVICE, "initialisation failed"));
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

extern "C" fde_status fde_bvm_set_option(fde_bvm *h, int option, int value) {
  if (!h) return fail(FDE_EINVAL, "handle is NULL");
  HIPCHK(hipStreamSynchronize(h->stream));
  switch (option) {
    case FDE_OPT_GRAPHS:
      h->opt_graphs = value ? 1 : 0;
      graphs_invalidate(h->self);
      h->self->graph_off = false;
      return FDE_OK;
    case FDE_OPT_AUTOTUNE:
      h->opt_autotune = value ? 1 : 0;
      return FDE_OK;
    case FDE_OPT_TRSV_W:
      if (value < -1 || value > 1024) return fail(FDE_EINVAL, "FDE_OPT_TRSV_W must be in -1..1024");
      h->opt_trsv_w = value;
      return FDE_OK;
    case FDE_OPT_PRECOND:
      if (value != FDE_PC_STRANG && value != FDE_PC_BCCB && value != FDE_PC_BCCB_SHIFTED &&
          value != FDE_PC_NONE)
        return fail(FDE_EINVAL, "unknown preconditioner %d", value);
      if (value != h->opt_precond) h->prec = -1;  // factor again before the next solve
      h->opt_precond = value;
      return FDE_OK;
    case FDE_OPT_SIDE:
      if (value != FDE_SIDE_RIGHT && value != FDE_SIDE_LEFT)
        return fail(FDE_EINVAL, "FDE_OPT_SIDE must be FDE_SIDE_RIGHT or FDE_SIDE_LEFT");
      h->opt_side = value;
      return FDE_OK;
    case FDE_OPT_ORTHO:
      if (value != FDE_ORTHO_MGS && value != FDE_ORTHO_CGS2)
        return fail(FDE_EINVAL, "FDE_OPT_ORTHO must be FDE_ORTHO_MGS or FDE_ORTHO_CGS2");
      h->opt_ortho = value;
      return FDE_OK;
    case FDE_OPT_X0_GATE:
      if (value < 0) return fail(FDE_EINVAL, "FDE_OPT_X0_GATE must be >= 0");
      h->opt_x0_gate = value;
      return FDE_OK;
    case FDE_OPT_BLOCKS:
      if (value != FDE_BLOCKS_LU && value != FDE_BLOCKS_HESSENBERG && value != FDE_BLOCKS_BAND &&
          value != FDE_BLOCKS_AUTO)
        return fail(FDE_EINVAL, "FDE_OPT_BLOCKS must be FDE_BLOCKS_LU, _HESSENBERG, _BAND or _AUTO");
      if (value != h->opt_blocks) h->prec = -1;  // factor again before the next solve
      h->opt_blocks = value;
      return FDE_OK;
    default:
      return fail(FDE_EINVAL, "unknown or read-only option %d", option);
  }
}

extern "C" fde_status fde_bvm_get_option(fde_bvm *h, int option, int *value) {
  if (!h || !value) return fail(FDE_EINVAL, "NULL argument");
  switch (option) {
    case FDE_OPT_GRAPHS: *value = h->opt_graphs; return FDE_OK;
    case FDE_OPT_AUTOTUNE: *value = h->opt_autotune; return FDE_OK;
    case FDE_OPT_TRSV_W: *value = h->opt_trsv_w; return FDE_OK;
    case FDE_OPT_TRSV_W_IN_USE:
      *value = h->self->desc.empty() || h->self->trsv_solo ? 0 : h->self->desc[0].W;
      return FDE_OK;
    case FDE_OPT_GRAPHS_IN_USE: *value = graphs_recorded(h->self) ? 1 : 0; return FDE_OK;
    case FDE_OPT_SIDE: *value = h->opt_side; return FDE_OK;
    case FDE_OPT_BLOCKS: *value = h->opt_blocks; return FDE_OK;
    case FDE_OPT_BLOCKS_IN_USE: *value = h->blk_route; return FDE_OK;
    case FDE_OPT_ORTHO: *value = h->opt_ortho; return FDE_OK;
    case FDE_OPT_PRECOND: *value = h->opt_precond; return FDE_OK;
    case FDE_OPT_X0_GATE: *value = h->opt_x0_gate; return FDE_OK;
    case FDE_OPT_X0_KEPT: *value = h->x0_kept; return FDE_OK;
    default: return fail(FDE_EINVAL, "unknown option %d", option);
  }
}

extern "C" fde_status fde_read_bandwidth_probe(size_t bytes, int reps, double *gbs) {
  if (!gbs || reps < 1 || bytes < (1u << 20)) return fail(FDE_EINVAL, "need bytes >= 1 MiB, reps >= 1, gbs");
  bytes &= ~(size_t)15;
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = 8 * std::max(cus, 1);
  void *x = nullptr, *out = nullptr;
  STCHK(dalloc_raw(&x, bytes));
  fde_status st = dalloc_raw(&out, sizeof(float) * blocks);
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float best = 1e30f;
  if (st == FDE_OK && (hipMemset(x, 0, bytes) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
                       hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    st = fail(FDE_EDEVICE, "probe set-up failed");
  for (int r = 0; st == FDE_OK && r <= reps; ++r) {  // the first run warms up
    float ms = 0.0f;
    if (hipEventRecord(e0, s) != hipSuccess || launch_read_probe(x, bytes, (float *)out, blocks, s) != hipSuccess ||
        hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      st = fail(FDE_EDEVICE, "probe launch failed");
    else if (r > 0)
      best = std::min(best, ms);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(out);
  (void)hipFree(x);
  if (st == FDE_OK) *gbs = (double)bytes / (best * 1e-3) / 1e9;
  return st;
}

extern "C" fde_status fde_mfma_peak_probe(int fp64, int reps, double *tflops) {
  if (!tflops || reps < 1) return fail(FDE_EINVAL, "need reps >= 1, tflops");
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = 4 * std::max(cus, 1), iters = 2048;  // four waves per SIMD
  void *out = nullptr;
  STCHK(dalloc_raw(&out, sizeof(float) * blocks));
  fde_status st = FDE_OK;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float best = 1e30f;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    st = fail(FDE_EDEVICE, "probe set-up failed");
  for (int r = 0; st == FDE_OK && r <= reps; ++r) {  // the first run warms up
    float ms = 0.0f;
    if (hipEventRecord(e0, s) != hipSuccess || launch_mfma_probe(fp64, iters, (float *)out, blocks, s) != hipSuccess ||
        hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      st = fail(FDE_EDEVICE, "probe launch failed");
    else if (r > 0)
      best = std::min(best, ms);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(out);
  if (st == FDE_OK) *tflops = mfma_probe_flops(iters, blocks) / (best * 1e-3) / 1e12;
  return st;
}

// ---- device buffers for callers without a device allocator of their own ------------------
extern "C" fde_status fde_device_alloc(size_t bytes, void **ptr) {
  if (!ptr) return fail(FDE_EINVAL, "ptr is NULL");
  *ptr = nullptr;
  if (bytes == 0) return fail(FDE_EINVAL, "bytes must be positive");
  return dalloc_raw(ptr, bytes);
}

extern "C" fde_status fde_device_free(void *ptr) {
  if (ptr) HIPCHK(hipFree(ptr));
  return FDE_OK;
}

extern "C" fde_status fde_memcpy(void *dst, const void *src, size_t bytes, int kind) {
  if (bytes == 0) return FDE_OK;
  if (!dst || !src) return fail(FDE_EINVAL, "NULL pointer");
  hipMemcpyKind k;
  switch (kind) {
    case FDE_COPY_H2D: k = hipMemcpyHostToDevice; break;
    case FDE_COPY_D2H: k = hipMemcpyDeviceToHost; break;
    case FDE_COPY_D2D: k = hipMemcpyDeviceToDevice; break;
    default: return fail(FDE_EINVAL, "unknown copy kind %d", kind);
  }
  HIPCHK(hipMemcpy(dst, src, bytes, k));
  return FDE_OK;
}

extern "C" fde_status fde_device_synchronize(void) {
  HIPCHK(hipDeviceSynchronize());
  return FDE_OK;
}

extern "C" fde_status fde_autotune_report(char *buf, int len) {
  if (!buf || len < 1) return fail(FDE_EINVAL, "invalid buffer");
  const std::string r = tuned_summary();
  std::snprintf(buf, (size_t)len, "%s", r.c_str());
  return (int)r.size() < len ? FDE_OK : fail(FDE_EINVAL, "buffer too small (%zu bytes needed)", r.size() + 1);
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
// Blocked right-looking LU of every block of every instance, two panel steps at a time (one
// launch per phase over all blocks of all instances):
//   diag(p), panel(p), band update of p (row and column p + 1), diag(p+1), panel(p+1),
//   then the rest of the trailing matrix with the updates of steps p and p + 1 together,
// so the trailing matrix is read and written once per pair of steps.
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
    // the assembly writes the first two block rows and columns (the rest is formed by the
    // first trailing update)
    const double mm = P->hs[i]->m, rest = std::max(0.0, mm - assemble_lead());
    asm_bytes += (double)P->hs[i]->nb * (mm * mm - rest * rest) * sizeof(T) * 2.0;
  }
  auto nrem_of = [&](int i, int p) { return P->hs[i]->npan - p - 1; };
  // maps: assemble, then per pair (diag p, panel p, band p, diag p+1, panel p+1, rest p)
  std::vector<HostMap> hm;
  for (int i = 0; i < count; ++i) it[i] = assemble_items(P->hs[i]->mp, P->hs[i]->nb);
  hm.push_back(make_map(slots, it));
  for (int p = 0; p < maxpan; p += 2) {
    for (int pp = p; pp <= p + 1; ++pp) {
      for (int i = 0; i < count; ++i) it[i] = nrem_of(i, pp) >= 0 ? P->hs[i]->nb : 0;
      hm.push_back(make_map(slots, it));  // diag pp
      for (int i = 0; i < count; ++i) it[i] = nrem_of(i, pp) > 0 ? 2 * nrem_of(i, pp) * P->hs[i]->nb : 0;
      hm.push_back(make_map(slots, it));  // panel pp
      if (pp == p) {
        for (int i = 0; i < count; ++i) it[i] = nrem_of(i, p) > 0 ? (2 * nrem_of(i, p) - 1) * P->hs[i]->nb : 0;
        hm.push_back(make_map(slots, it));  // band p
      }
    }
    for (int i = 0; i < count; ++i) {
      const int n1 = nrem_of(i, p) - 1;
      it[i] = n1 > 0 ? n1 * n1 * P->hs[i]->nb : 0;
    }
    hm.push_back(make_map(slots, it));  // rest p
  }
  std::vector<ItemMap> dm;
  STCHK(upload_maps(P, hm, dm));
  hipStream_t st = L->stream;
  HIPCHK(run(L, "assemble", asm_bytes, [&] { return launch_assemble<T>(P->d_desc, dm[0], hm[0].items, st); }));
  // algorithmic flops (complex multiply-add = 8 real flops) on the unpadded orders m
  auto wdiag = [&](int p) {
    double w = 0;
    for (fde_bvm *h : P->hs)
      if (p < h->npan) {
        const double c = std::min(64, h->m - p * 64);
        w += h->nb * 8.0 * c * c * c / 3.0;
      }
    return w;
  };
  auto wpanel = [&](int p) {
    double w = 0;
    for (fde_bvm *h : P->hs)
      if (p < h->npan) w += h->nb * 8.0 * 64.0 * 64.0 * std::max(0, h->m - (p + 1) * 64);
    return w;
  };
  size_t mi = 1;
  for (int p = 0; p < maxpan; p += 2) {
    double wband = 0, wrest = 0;
    for (fde_bvm *h : P->hs) {
      if (p >= h->npan) continue;
      const double rem = std::max(0, h->m - (p + 1) * 64), rem2 = std::max(0.0, rem - 64.0);
      wband += h->nb * 8.0 * 64.0 * (rem * rem - rem2 * rem2);
      wrest += h->nb * 8.0 * 128.0 * rem2 * rem2;
    }
    for (int pp = p; pp <= p + 1; ++pp) {
      const size_t id = mi++, ip = mi++;
      if (hm[id].items > 0)
        HIPCHK(run(L, "lu_diag", wdiag(pp), [&] { return launch_lu_diag<T>(P->d_desc, dm[id], hm[id].items, pp, P->d_flag, st); }));
      if (hm[ip].items > 0)
        HIPCHK(run(L, "lu_panel", wpanel(pp), [&] { return launch_lu_panel<T>(P->d_desc, dm[ip], hm[ip].items, pp, st); }));
      if (pp == p) {
        const size_t ib = mi++;
        if (hm[ib].items > 0)
          HIPCHK(run(L, "lu_update", wband, [&] { return launch_lu_update<T>(P->d_desc, dm[ib], hm[ib].items, p, 1, st); }));
      }
    }
    const size_t ir = mi++;
    if (hm[ir].items > 0)
      HIPCHK(run(L, "lu_update", wrest, [&] { return launch_lu_update<T>(P->d_desc, dm[ir], hm[ir].items, p, 2, st); }));
  }
  return FDE_OK;
}

// The Hessenberg route: J = Q H Q^T per instance (one cooperative launch each), then the
// shifted Hessenberg LUs of all blocks of all instances and the inverses of U's diagonal
// tiles (one launch each).
template <typename T>
static fde_status hess_factor(Plan *P) {
  fde_bvm *L = P->lead;
  const int count = (int)P->hs.size();
  hipStream_t st = L->stream;
  std::vector<int> slots(count), a(count), b(count);
  int max_mp = 64;
  double wlu = 0.0;
  for (int i = 0; i < count; ++i) {
    fde_bvm *h = P->hs[i];
    const double m = h->m;
    HIPCHK(run(L, "hess_reduce", 10.0 / 3.0 * m * m * m + 4.0 * m * m * m, [&] {
      return launch_hess_reduce(P->d_desc, i, h->m, h->hwk, st);
    }));
    slots[i] = i;
    a[i] = h->nb;
    b[i] = h->nb * h->npan;
    max_mp = std::max(max_mp, h->mp);
    wlu += h->nb * 8.0 * m * m / 2.0;
  }
  std::vector<HostMap> hm = {make_map(slots, a), make_map(slots, b)};
  std::vector<ItemMap> dm;
  STCHK(upload_maps(P, hm, dm));
  HIPCHK(run(L, "hess_lu", wlu, [&] { return launch_hess_lu<T>(P->d_desc, dm[0], hm[0].items, max_mp, P->d_flag, st); }));
  double winv = 0.0;
  for (fde_bvm *h : P->hs) winv += h->nb * h->npan * 8.0 * 64.0 * 64.0 * 64.0 / 6.0;
  HIPCHK(run(L, "hess_uinv", winv, [&] { return launch_hess_uinv<T>(P->d_desc, dm[1], hm[1].items, P->d_flag, st); }));
  return FDE_OK;
}

static fde_status hess_alloc(fde_bvm *h) {
  if (h->d_hH) return FDE_OK;
  const size_t mp = h->mp, nb = h->nb, G = hess_reduce_groups(h->m);
  STCHK(dalloc_t(h, &h->d_hH, mp * mp));
  STCHK(dalloc_t(h, &h->d_hQ, mp * mp));
  STCHK(dalloc_t(h, &h->d_hQt, mp * mp));
  STCHK(dalloc_t(h, &h->d_hl, nb * mp));
  STCHK(dalloc_t(h, &h->d_hpiv, nb * mp));
  STCHK(dalloc_t(h, &h->d_Vh2, nb * mp));
  HIPCHK(hipMemsetAsync(h->d_Vh2, 0, nb * mp * sizeof(double2), h->stream));
  HessWork &w = h->hwk;
  STCHK(dalloc_t(h, &w.sync, G + 4));
  w.err = (int *)(w.sync + G);
  STCHK(dalloc_t(h, &w.vbuf, mp));
  STCHK(dalloc_t(h, &w.part, G * 2 * mp));
  STCHK(dalloc_t(h, &w.ybuf, 2 * mp));
  w.H = h->d_hH;
  w.Q = h->d_hQ;
  w.Qt = h->d_hQt;
  return FDE_OK;
}

// The band route: J = Q H Q^T with H of lower bandwidth 64 per instance (blocked Householder
// reduction, k_band.hip), then the pivoted band LU of every block, one panel step at a time
// (a panel launch over the blocks of all instances, then a launch over their row tiles).
static fde_status band_alloc(fde_bvm *h) {
  if (h->d_bAQ) return FDE_OK;
  const size_t mp = h->mp, nb = h->nb;
  STCHK(dalloc_t(h, &h->d_bAQ, 2 * mp * mp));
  STCHK(dalloc_t(h, &h->d_bQt, mp * mp));
  STCHK(dalloc_t(h, &h->d_bpiv, nb * mp * 2));
  STCHK(dalloc_t(h, &h->d_bwork, band_work_doubles(h->mp)));
  STCHK(dalloc_t(h, &h->d_berr, 64));
  HIPCHK(hipMemsetAsync(h->d_berr, 0, 64 * sizeof(int), h->stream));
  if (!h->side_stream) {
    HIPCHK(hipStreamCreateWithFlags(&h->side_stream, hipStreamNonBlocking));
    for (auto &e : h->side_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  if (!h->d_Vh2) {
    STCHK(dalloc_t(h, &h->d_Vh2, nb * mp));
    HIPCHK(hipMemsetAsync(h->d_Vh2, 0, nb * mp * sizeof(double2), h->stream));
  }
  return FDE_OK;
}

template <typename T>
static fde_status band_factor(Plan *P) {
  fde_bvm *L = P->lead;
  const int count = (int)P->hs.size();
  hipStream_t st = L->stream;
  int maxpan = 0;
  for (int i = 0; i < count; ++i) {
    TraceRange tr("band reduction of J");
    fde_bvm *h = P->hs[i];
    maxpan = std::max(maxpan, h->npan);
    // algorithmic flops: the panel QR of a w x 64 block 2 * 64^2 (w - 64/3); the two-sided update
    // with its product into Q 4 (2 mp) w 64 + 4 w^2 64 (right update of [A; Q], left update)
    const int mp = h->mp;
    HIPCHK(run(L, "band_init", 16.0 * mp * mp, [&] { return launch_band_init(P->d_desc, i, mp, h->d_bAQ, h->d_bwork, st); }));
    // Panels 0 .. np - 1.  Look-ahead: the update of panel p first finishes the next panel's 64
    // columns (near), then panel p + 1 runs on the side stream while the rest of the update
    // (far, the columns after those) runs on the main one; the main stream waits for the panel
    // before the next update.
    const int np = h->npan - 1;
    hipStream_t side = L->side_stream;
    auto panel_work = [&](int p) { return 2.0 * 64.0 * 64.0 * (mp - 64.0 * (p + 1) - 64.0 / 3.0); };
    if (np > 0)
      HIPCHK(run(L, "band_panel", panel_work(0), [&] {
        return launch_band_panel(mp, 0, h->d_bAQ, h->d_bwork, h->d_berr, st);
      }));
    for (int p = 0; p < np; ++p) {
      const double w = mp - 64.0 * (p + 1);
      const double all = 4.0 * 2.0 * mp * w * 64.0 + 4.0 * w * w * 64.0;
      const double near = 2.0 * 2.0 * mp * w * 64.0 + 2.0 * 2.0 * mp * 64.0 * 64.0 + 4.0 * w * 64.0 * 64.0;
      HIPCHK(run(L, "band_update", near, [&] { return launch_band_update(mp, p, false, h->d_bAQ, h->d_bwork, st); }));
      const bool next = p + 1 < np;
      if (next) {
        HIPCHK(hipEventRecord(L->side_ev[0], st));
        HIPCHK(hipStreamWaitEvent(side, L->side_ev[0], 0));
        HIPCHK(run(L, "band_panel", panel_work(p + 1), [&] {
          return launch_band_panel(mp, p + 1, h->d_bAQ, h->d_bwork, h->d_berr, side);
        }, side));
        HIPCHK(hipEventRecord(L->side_ev[1], side));
      }
      if (w > 64.0)
        HIPCHK(run(L, "band_update", all - near, [&] { return launch_band_update(mp, p, true, h->d_bAQ, h->d_bwork, st); }));
      if (next) HIPCHK(hipStreamWaitEvent(st, L->side_ev[1], 0));
    }
    HIPCHK(run(L, "band_finish", 16.0 * mp * mp, [&] { return launch_band_finish(mp, h->d_bAQ, h->d_bQt, st); }));
  }
  // Step j of the LU: panel j, then the row tiles of step j.  Look-ahead: the first row tile
  // (block column j + 1, all that panel j + 1 reads) runs first; panel j + 1 then runs in the
  // same launch as the other row tiles of step j (which touch block rows j and j + 1 at block
  // columns >= j + 2 only), its workgroups first.
  std::vector<int> slots(count), it(count);
  for (int i = 0; i < count; ++i) slots[i] = i;
  std::vector<HostMap> hm;
  for (int j = 0; j < maxpan; ++j) {
    for (int i = 0; i < count; ++i) it[i] = j < P->hs[i]->npan ? P->hs[i]->nb : 0;
    hm.push_back(make_map(slots, it));  // panel j
    for (int i = 0; i < count; ++i) it[i] = P->hs[i]->npan - j - 1 >= 1 ? P->hs[i]->nb : 0;
    hm.push_back(make_map(slots, it));  // row tile 0 of step j
    for (int i = 0; i < count; ++i) it[i] = std::max(0, P->hs[i]->npan - j - 2) * P->hs[i]->nb;
    hm.push_back(make_map(slots, it));  // row tiles 1 .. of step j
  }
  std::vector<ItemMap> dm;
  STCHK(upload_maps(P, hm, dm));
  // algorithmic flops (complex multiply-add = 8 real flops): the 128 x 64 panel LU, and per
  // tile of the trailing width the two 64 x 64 x 64 products
  auto panel_work = [&](int j) {
    double w = 0.0;
    for (fde_bvm *h : P->hs) {
      if (j >= h->npan) continue;
      const double nr = j + 1 < h->npan ? 128.0 : 64.0;
      w += h->nb * 8.0 * 64.0 * 64.0 * (nr - 64.0 / 3.0) / 2.0;
    }
    return w;
  };
  auto rows_work = [&](size_t mi) { return hm[mi].items * 2.0 * 8.0 * 64.0 * 64.0 * 64.0; };
  TraceRange tr("band LU of the shifted blocks");
  if (hm[0].items > 0)
    HIPCHK(run(L, "band_lu_panel", panel_work(0), [&] { return launch_band_lu_panel<T>(P->d_desc, dm[0], hm[0].items, 0, P->d_flag, st); }));
  for (int j = 0; j < maxpan; ++j) {
    const size_t i0 = 3 * j + 1, i1 = 3 * j + 2, ip = 3 * (j + 1);
    if (hm[i0].items > 0)
      HIPCHK(run(L, "band_lu_rows", rows_work(i0), [&] { return launch_band_lu_rows<T>(P->d_desc, dm[i0], hm[i0].items, j, 0, 1, st); }));
    const int pitems = j + 1 < maxpan ? hm[ip].items : 0;
    if (pitems + hm[i1].items > 0)
      HIPCHK(run(L, "band_lu_step", (pitems ? panel_work(j + 1) : 0.0) + rows_work(i1), [&] {
        return launch_band_lu_step<T>(P->d_desc, dm[j + 1 < maxpan ? ip : i1], pitems, dm[i1], hm[i1].items, j, P->d_flag, st);
      }));
  }
  return FDE_OK;
}

static fde_status bccb_prepare(fde_bvm *h);

static fde_status factor_plan(Plan *P, fde_precision prec) {
  if (prec != FDE_FP64 && prec != FDE_MIXED_C32) return fail(FDE_EINVAL, "unknown precision %d", (int)prec);
  TraceRange tr_factor("fde_precond_factor");
  fde_bvm *L = P->lead;
  const int kind = P->hs[0]->opt_precond;
  for (fde_bvm *h : P->hs)
    if (h->opt_precond != kind) return fail(FDE_EINVAL, "all instances of a batch need the same preconditioner");
  if (kind != FDE_PC_STRANG) {
    // BCCB: no block factors; the "factorization" is the space symbol and the chirp tables.
    // No preconditioner: nothing to build.
    hipEvent_t e0 = get_event(L), e1 = get_event(L);
    HIPCHK(hipEventRecord(e0, L->stream));
    for (fde_bvm *h : P->hs) {
      h->prec = -1;
      h->pc = kind;
      if (kind != FDE_PC_NONE) STCHK(bccb_prepare(h));
      if (h->self) h->self->desc_dirty = true;
    }
    P->desc_dirty = true;
    STCHK(plan_prepare(P, std::max(P->R, 1), prec));
    HIPCHK(hipEventRecord(e1, L->stream));
    STCHK(sync_and_flush(L));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    L->evpool.push_back(e0);
    L->evpool.push_back(e1);
    for (fde_bvm *h : P->hs) {
      h->prec = prec;
      h->t_factor_ms = ms;
    }
    return FDE_OK;
  }
  int route = P->hs[0]->opt_blocks;
  for (fde_bvm *h : P->hs)
    if (h->opt_blocks != route) return fail(FDE_EINVAL, "all instances of a batch need the same block solver");
  if (route == FDE_BLOCKS_AUTO) {  // the band route once every instance is large enough
    bool band = true;
    for (fde_bvm *h : P->hs) {
      const int mmin = prec != FDE_FP64              ? FDE_BAND_MIN_M_MIXED
                       : h->nb >= FDE_BAND_LONG_NB ? FDE_BAND_MIN_M_FP64_LONG
                                                   : FDE_BAND_MIN_M_FP64;
      band = band && h->m >= mmin;
    }
    route = band ? FDE_BLOCKS_BAND : FDE_BLOCKS_LU;
  }
  for (fde_bvm *h : P->hs) {
    if (route == FDE_BLOCKS_HESSENBERG && h->m > hess_reduce_max_m())
      return fail(FDE_EUNSUPPORTED, "the Hessenberg route takes m <= %d (m = %d)", hess_reduce_max_m(), h->m);
  }
  for (fde_bvm *h : P->hs) {
    h->pc = FDE_PC_STRANG;
    if (h->blk_route != route && h->self) h->self->desc_dirty = true;
    h->blk_route = route;
    if (route == FDE_BLOCKS_HESSENBERG) STCHK(hess_alloc(h));
    if (route == FDE_BLOCKS_BAND) STCHK(band_alloc(h));
  }
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
  // plan_prepare uploads the descriptors only if one of them changed (a refactorisation of
  // the same shape keeps them, and needs no host round trip here)
  STCHK(plan_prepare(P, std::max(P->R, 1), prec));
  hipEvent_t e0 = get_event(L), e1 = get_event(L);
  HIPCHK(hipMemsetAsync(P->d_flag, 0, sizeof(int), L->stream));
  HIPCHK(hipEventRecord(e0, L->stream));
  if (route == FDE_BLOCKS_HESSENBERG) {
    TraceRange tr("blocks: Hessenberg route");
    STCHK(prec == FDE_FP64 ? hess_factor<double>(P) : hess_factor<float>(P));
  } else if (route == FDE_BLOCKS_BAND) {
    TraceRange tr("blocks: band route");
    STCHK(prec == FDE_FP64 ? band_factor<double>(P) : band_factor<float>(P));
  } else {
    TraceRange tr("blocks: block LU");
    STCHK(prec == FDE_FP64 ? factor_plan_impl<double>(P) : factor_plan_impl<float>(P));
  }
  HIPCHK(hipEventRecord(e1, L->stream));
  int *flag_pin = (int *)((char *)P->pin + P->pin_err) + 1;  // pinned: no staging copy
  HIPCHK(hipMemcpyAsync(flag_pin, P->d_flag, sizeof(int), hipMemcpyDeviceToHost, L->stream));
  std::vector<int> herr(P->hs.size(), 0);
  if (route == FDE_BLOCKS_HESSENBERG)
    for (size_t i = 0; i < P->hs.size(); ++i)
      HIPCHK(hipMemcpyAsync(&herr[i], P->hs[i]->hwk.err, sizeof(int), hipMemcpyDeviceToHost, L->stream));
  if (route == FDE_BLOCKS_BAND)
    for (size_t i = 0; i < P->hs.size(); ++i)
      HIPCHK(hipMemcpyAsync(&herr[i], P->hs[i]->d_berr, sizeof(int), hipMemcpyDeviceToHost, L->stream));
  STCHK(sync_and_flush(L));
  for (size_t i = 0; i < herr.size(); ++i)
    if (herr[i]) {
      if (route == FDE_BLOCKS_BAND) (void)hipMemset(P->hs[i]->d_berr, 0, sizeof(int));
      return fail(FDE_EDEVICE, "the Hessenberg or band reduction of instance %zu did not complete", i);
    }
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  L->evpool.push_back(e0);
  L->evpool.push_back(e1);
  if (*flag_pin) return fail(FDE_ESINGULAR, "zero or non-finite pivot in a preconditioner block");
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
// Maps over every instance of the plan (gates select the instances of a launch), uploaded
// into the plan's own buffer.  Rebuilt only when the item counts change (block-solve W or
// precision); recorded graphs refer to this buffer, so a rebuild drops them.
static fde_status ensure_full_maps(Plan *P) {
  const int count = (int)P->hs.size();
  const int prec = P->hs[0]->prec;
  if (P->full_ok && P->full.prec == prec && P->full.pc == P->hs[0]->pc &&
      P->full.route == P->hs[0]->blk_route)
    return FDE_OK;
  std::vector<int> slots(count), a(count), b(count), c(count), d(count), e(count), f(count), g(count),
      qq(count);
  SolveMaps S;
  {
    long long total_mp = 0;
    for (int q = 0; q < count; ++q) total_mp += P->hs[q]->mp;
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    S.tfft_cols = time_fft_cols_per_item(total_mp, std::max(cus, 1));
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned_cols.find(plan_shape_key(P, prec));
    if (it != g_tuned_cols.end()) S.tfft_cols = it->second;
  }
  for (int q = 0; q < count; ++q) {
    fde_bvm *h = P->hs[q];
    slots[q] = q;
    g[q] = h->nb;
    a[q] = h->s;
    b[q] = h->mp / S.tfft_cols;
    c[q] = h->nb * P->desc[q].W;
    d[q] = h->nblk;
    e[q] = h->s;
    f[q] = h->need_Ju0 ? 1 : 0;
    S.max_log2L = std::max(S.max_log2L, h->log2L);
    S.max_log2s = std::max(S.max_log2s, h->log2s);
    S.max_mp = std::max(S.max_mp, h->mp);
    qq[q] = qgemm_items(h->nb, h->mp);
    const double esz = h->prec == FDE_FP64 ? 16.0 : 8.0;
    const double fac = h->blk_route != FDE_BLOCKS_LU ? 0.5 * h->m * (h->m + 1.0)
                                                             : (double)h->m * h->m;
    S.trsv_bytes += (double)h->nb * fac * esz + 32.0 * h->nb * h->m;
    S.qg_flops += 2.0 * (2.0 * (h->nb - 1)) * h->m * h->m;  // 2 (nb - 1) real rows times Q
    S.vec_bytes += 8.0 * h->n();
    S.tfft_bytes += 8.0 * h->n() + 16.0 * h->nb * h->m;
    S.bccb_bytes += 32.0 * h->nb * h->m;  // one complex read and write per (frequency, node)
    // band L solve: the band's L11^{-1} and L21 pieces (2 x 64 x 64 per panel) and the vector
    S.band_l_bytes += (double)h->nb * h->npan * 2.0 * 64.0 * 64.0 * esz + 32.0 * h->nb * h->m;
  }
  const std::vector<HostMap> hm = {make_map(slots, a), make_map(slots, b), make_map(slots, c),
                                   make_map(slots, d), make_map(slots, e), make_map(slots, f),
                                   make_map(slots, g), make_map(slots, qq)};
  size_t need = 0;
  for (const HostMap &m : hm) need += m.ids.size() + m.pre.size();
  HIPCHK(hipStreamSynchronize(P->lead->stream));
  graphs_invalidate(P);
  if (need > P->fullmaps_ints) {
    if (P->d_fullmaps) {
      auto it = std::find(P->allocs.begin(), P->allocs.end(), (void *)P->d_fullmaps);
      if (it != P->allocs.end()) P->allocs.erase(it);
      (void)hipFree(P->d_fullmaps);
      P->d_fullmaps = nullptr;
      P->fullmaps_ints = 0;
    }
    void *p = nullptr;
    STCHK(plan_alloc(P, &p, need * sizeof(int)));
    P->d_fullmaps = (int *)p;
    P->fullmaps_ints = need;
  }
  P->fullmaps_host.clear();
  std::vector<ItemMap> dm;
  for (const HostMap &m : hm) {
    const size_t oi = P->fullmaps_host.size();
    P->fullmaps_host.insert(P->fullmaps_host.end(), m.ids.begin(), m.ids.end());
    const size_t op = P->fullmaps_host.size();
    P->fullmaps_host.insert(P->fullmaps_host.end(), m.pre.begin(), m.pre.end());
    dm.push_back(ItemMap{P->d_fullmaps + oi, P->d_fullmaps + op, (int)m.ids.size(), nullptr});
  }
  HIPCHK(hipMemcpy(P->d_fullmaps, P->fullmaps_host.data(), P->fullmaps_host.size() * sizeof(int),
                   hipMemcpyHostToDevice));
  S.mv = dm[0];
  S.tfft = dm[1];
  S.trsv = dm[2];
  S.kry = dm[3];
  S.rhs = dm[4];
  S.ju0 = dm[5];
  S.blk = dm[6];
  S.n_blk = hm[6].items;
  S.qg = dm[7];
  S.n_qg = hm[7].items;
  S.pc = P->hs[0]->pc;
  S.route = P->hs[0]->blk_route;
  S.n_mv = hm[0].items;
  S.n_tfft = hm[1].items;
  S.n_trsv = hm[2].items;
  S.n_kry = hm[3].items;
  S.n_rhs = hm[4].items;
  S.n_ju0 = hm[5].items;
  S.prec = prec;
  S.trsv_solo = P->trsv_solo ? 1 : 0;
  S.kry_one_n = 0;
  for (fde_bvm *h : P->hs) S.kry_one_n = std::max(S.kry_one_n, h->n());
  for (fde_bvm *h : P->hs)
    if (h->nblk != 1) S.kry_one_n = 0;
  S.npan_u = P->hs[0]->npan;
  for (fde_bvm *h : P->hs)
    if (h->npan != S.npan_u) S.npan_u = 0;
  P->full = S;
  P->full_ok = true;
  return FDE_OK;
}

static fde_status op_matvec(Plan *P, const SolveMaps &S, int src, int sj, int dst, int dj) {
  fde_bvm *L = P->lead;
  HIPCHK(run(L, "bvm_matvec", 2.0 * S.vec_bytes, [&] {
    return launch_bvm_matvec(P->d_desc, S.mv, S.n_mv, S.max_log2L, src, sj, dst, dj, 0, L->stream);
  }));
  return FDE_OK;
}

// Cooperative block solves are used unless the device refuses cooperative launches (then the
// ordinary launch, k_trsv); decided once per process, never while recording.
static bool g_coop_ok = true;

// The block solve (both sweeps, or the U sweep only for first_sweep = 1) in the plan's launch
// form; a device that refuses the cooperative launch gets the ordinary one.
static hipError_t block_solve(Plan *P, const SolveMaps &S, int first_sweep, hipStream_t st) {
  if (!S.trsv_solo && g_coop_ok) {
    const hipError_t e =
        S.prec == FDE_FP64
            ? launch_trsv_coop<double>(P->d_desc, S.trsv, S.n_trsv, P->d_epoch, P->d_err, st, first_sweep,
                                       &S.blk, S.n_blk, S.npan_u)
            : launch_trsv_coop<float>(P->d_desc, S.trsv, S.n_trsv, P->d_epoch, P->d_err, st, first_sweep,
                                      &S.blk, S.n_blk, S.npan_u);
    if (e == hipSuccess || g_capture) return e;  // a refusal while recording ends the recording
    (void)hipGetLastError();
    g_coop_ok = false;
  }
  return S.prec == FDE_FP64 ? launch_trsv<double>(P->d_desc, S.trsv, S.n_trsv, first_sweep, st)
                            : launch_trsv<float>(P->d_desc, S.trsv, S.n_trsv, first_sweep, st);
}

static fde_status op_precond(Plan *P, const SolveMaps &S, int src, int sj, int dst, int dj) {
  fde_bvm *L = P->lead;
  hipStream_t st = L->stream;
  if (S.pc == FDE_PC_NONE) {  // identity
    if (src == dst && sj == dj) return FDE_OK;
    HIPCHK(run(L, "copy", 2.0 * S.vec_bytes, [&] {
      return launch_copy(P->d_desc, S.kry, S.n_kry, src, sj, dst, dj, st);
    }));
    return FDE_OK;
  }
  if (S.pc != FDE_PC_STRANG) {  // BCCB: time DFT, space-Fourier diagonal solve, inverse time DFT
    HIPCHK(run(L, "time_rfft", S.tfft_bytes, [&] {
      return launch_time_rfft(P->d_desc, S.tfft, S.n_tfft, S.max_log2s, S.tfft_cols, src, sj, st);
    }));
    HIPCHK(run(L, "bccb_solve", S.bccb_bytes, [&] {
      return launch_bccb_solve(P->d_desc, S.blk, S.n_blk, S.max_log2L, st);
    }));
    HIPCHK(run(L, "time_irfft", S.tfft_bytes, [&] {
      return launch_time_irfft(P->d_desc, S.tfft, S.n_tfft, S.max_log2s, S.tfft_cols, dst, dj, st);
    }));
    return FDE_OK;
  }
  unsigned long long *ctr = nullptr;
  STCHK(epoch_counter(&ctr));
  HIPCHK(run(L, "time_rfft", S.tfft_bytes, [&] {
    return launch_time_rfft(P->d_desc, S.tfft, S.n_tfft, S.max_log2s, S.tfft_cols, src, sj, st, ctr, P->d_epoch);
  }));
  if (S.route == FDE_BLOCKS_BAND) {
    // Q^T v_k (the frequency vectors are rows: the row v_k^T Q), the band L solve, U^{-1}, Q
    HIPCHK(run(L, "qgemm", S.qg_flops, [&] { return launch_qgemm(P->d_desc, S.qg, S.n_qg, 0, 0, st); }));
    HIPCHK(run(L, "band_lsolve", S.band_l_bytes, [&] {
      return S.prec == FDE_FP64 ? launch_band_lsolve<double>(P->d_desc, S.blk, S.n_blk, st)
                                : launch_band_lsolve<float>(P->d_desc, S.blk, S.n_blk, st);
    }));
    HIPCHK(run(L, "trsv", S.trsv_bytes, [&] { return block_solve(P, S, 1, st); }));
    HIPCHK(run(L, "qgemm", S.qg_flops, [&] { return launch_qgemm(P->d_desc, S.qg, S.n_qg, 1, 1, st); }));
    HIPCHK(run(L, "time_irfft", S.tfft_bytes, [&] {
      return launch_time_irfft(P->d_desc, S.tfft, S.n_tfft, S.max_log2s, S.tfft_cols, dst, dj, st);
    }));
    return FDE_OK;
  }
  if (S.route == FDE_BLOCKS_HESSENBERG) {
    // Q^T v_k, the row exchanges and eliminations, U^{-1}, then Q (the frequency vectors are
    // rows, so Q^T v_k is the row v_k^T Q)
    HIPCHK(run(L, "qgemm", S.qg_flops, [&] { return launch_qgemm(P->d_desc, S.qg, S.n_qg, 0, 0, st); }));
    HIPCHK(run(L, "hess_lsolve", S.bccb_bytes, [&] {
      return launch_hess_lsolve(P->d_desc, S.blk, S.n_blk, S.max_mp, st);
    }));
    HIPCHK(run(L, "trsv", S.trsv_bytes, [&] { return block_solve(P, S, 1, st); }));
    HIPCHK(run(L, "qgemm", S.qg_flops, [&] { return launch_qgemm(P->d_desc, S.qg, S.n_qg, 1, 1, st); }));
    HIPCHK(run(L, "time_irfft", S.tfft_bytes, [&] {
      return launch_time_irfft(P->d_desc, S.tfft, S.n_tfft, S.max_log2s, S.tfft_cols, dst, dj, st);
    }));
    return FDE_OK;
  }
  HIPCHK(run(L, "trsv", S.trsv_bytes, [&] { return block_solve(P, S, 0, st); }));
  HIPCHK(run(L, "time_irfft", S.tfft_bytes, [&] {
    return launch_time_irfft(P->d_desc, S.tfft, S.n_tfft, S.max_log2s, S.tfft_cols, dst, dj, st);
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
// GMRES over a plan: restart cycles in lockstep (right preconditioning, flexible form, MGS
// Arnoldi, Givens rotations; convergence only on the recomputed true residual).
//
// The host sets up (right-hand sides, norms, the projected initial guess), then alternates
// two fixed launch sequences until every instance has finished:
//   restart step: r = b - M x, beta = ||r||, v_0 = r / beta, and the device decides per
//                 instance: converged, out of iterations, or a new cycle;
//   cycle:        R Arnoldi steps (S^{-1}, M, MGS, normalisation, Givens on the device),
//                 then y = H^{-1} g and x += Z y.
// Instances that finish stop contributing items through the gate arrays, so the sequences
// never change and are recorded once as hipGraphs and replayed (unless recording fails,
// then they are launched directly).  The host reads the control records once per cycle.
// ====================================================================================
struct InstState {
  double truer = 0, est = 0;
  int its = 0, restarts = 0;
  bool conv = false, fail = false;
};

// Sum of an instance's chunk partials (part0 or part1) in index order.
static double part_sum(const Plan *P, const std::vector<double> &parts, int i, int psel) {
  double t = 0.0;
  const size_t base = P->part_off[i] + (psel ? P->hs[i]->nblk : 0);
  for (int q = 0; q < P->hs[i]->nblk; ++q) t += parts[base + q];
  return t;
}

// Records emit()'s launches on the lead stream into g.  On any failure nothing has run and g
// stays empty.
static fde_status record_segment(Plan *P, GraphSeg &g, const std::function<fde_status()> &emit) {
  hipStream_t st = P->lead->stream;
  graph_release(P, g);
  if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipGetLastError();
    return FDE_EUNSUPPORTED;
  }
  g_capture = &g;
  const std::string saved = g_err;
  const fde_status s = emit();
  g_capture = nullptr;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &graph);
  hipError_t ei = hipErrorUnknown;
  if (s == FDE_OK && e == hipSuccess && graph) ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    (void)hipGetLastError();
    g.exec = nullptr;
    graph_release(P, g);
    g_err = saved;
    return FDE_EUNSUPPORTED;
  }
  return FDE_OK;
}

// Runs a segment: replays its graph (recording it first if needed) or launches it directly.
static fde_status run_segment(Plan *P, GraphSeg &g, bool use_graph,
                              const std::function<fde_status()> &emit) {
  fde_bvm *L = P->lead;
  if (use_graph && !g.exec && record_segment(P, g, emit) != FDE_OK) P->graph_off = true;
  if (use_graph && g.exec) {
    HIPCHK(hipGraphLaunch(g.exec, L->stream));
    for (const Pending &p : g.prof) L->pend.push_back(p);
    return FDE_OK;
  }
  return emit();
}

static fde_status gmres_plan(Plan *P, const fde_solve_opts &o, const std::vector<char> &has_x0,
                             std::vector<InstState> &st) {
  fde_bvm *L = P->lead;
  const int count = (int)P->hs.size();
  const int R = o.restart;
  hipStream_t stream = L->stream;
  STCHK(ensure_full_maps(P));
  unsigned long long *ctr = nullptr;
  STCHK(epoch_counter(&ctr));  // allocated (once) before anything is recorded
  const SolveMaps &S = P->full;
  int *g_live = P->d_gates + GATE_LIVE * count;
  int *g_act = P->d_gates + GATE_ACTIVE * count;
  int *g_x0 = P->d_gates + GATE_X0 * count;
  const SolveMaps Slive = gated(S, g_live), Sact = gated(S, g_act), Sx0 = gated(S, g_x0);

  // right-hand sides and their norms
  STCHK(op_rhs(P, S));
  HIPCHK(run(L, "dot", S.vec_bytes, [&] { return launch_dot_partial(P->d_desc, S.kry, S.n_kry, VS_B, VS_B, 0, stream); }));
  // part0 and part1 of the last instance end the range the host sums (each instance's block
  // also holds its Gram-Schmidt partials after part1)
  const size_t nparts = P->part_off.back() + 2 * (size_t)P->hs.back()->nblk;
  std::vector<double> parts(nparts);
  // the partials through pinned staging (a read into pageable memory would stage and block)
  auto fetch_parts = [&]() -> fde_status {
    HIPCHK(hipMemcpyAsync(P->pin_parts, P->d_part, nparts * sizeof(double), hipMemcpyDeviceToHost, stream));
    STCHK(sync_and_flush(L));
    std::memcpy(parts.data(), P->pin_parts, nparts * sizeof(double));
    return FDE_OK;
  };
  // Left preconditioning measures residuals after the preconditioner: the reference norm of
  // the stopping test is ||P^{-1} b||.  (With no preconditioner both sides are the same.)
  const bool left = L->opt_side == FDE_SIDE_LEFT && S.pc != FDE_PC_NONE;
  bool any_x0 = false;
  for (int i = 0; i < count; ++i) any_x0 = any_x0 || has_x0[i];
  // A zero start with right preconditioning needs nothing from the host before the first
  // cycle: the control records are set up on the device (k_gm_init) and the host first reads
  // them after the first stretch of Arnoldi steps.
  const bool dev_init = !left && !any_x0;
  std::vector<double> bnorm(count, 0.0);
  if (!dev_init) {
    STCHK(fetch_parts());
    for (int i = 0; i < count; ++i) {
      bnorm[i] = std::sqrt(part_sum(P, parts, i, 0));
      if (!std::isfinite(bnorm[i])) return fail(FDE_EINVAL, "right-hand side %d is not finite", i);
    }
  }
  const std::vector<double> bnorm_true = bnorm;
  if (left) {
    STCHK(op_precond(P, S, VS_B, 0, VS_TMP, 0));
    HIPCHK(run(L, "dot", S.vec_bytes, [&] { return launch_dot_partial(P->d_desc, S.kry, S.n_kry, VS_TMP, VS_TMP, 0, stream); }));
    STCHK(fetch_parts());
    STCHK(check_trsv_err(P));
    for (int i = 0; i < count; ++i) {
      bnorm[i] = bnorm_true[i] == 0.0 ? 0.0 : std::sqrt(part_sum(P, parts, i, 0));
      if (!std::isfinite(bnorm[i])) return fail(FDE_ESINGULAR, "P^{-1} b of instance %d is not finite", i);
    }
  }
  // An initial guess is first scaled by the gamma minimising ||b - gamma M x0|| (one step of
  // minimal residual along x0), so that ||r_0|| <= ||b||: a poor guess never starts worse
  // than the zero start.  A guess that leaves ||b - gamma M x0|| above the gate (the lead
  // handle's FDE_OPT_X0_GATE, millionths of ||b||) gets gamma = 0: the zero start.
  std::vector<int> &gh = P->gates_host;
  gh.assign(GATE_COUNT * count, 0);
  for (int i = 0; i < count; ++i) gh[GATE_X0 * count + i] = has_x0[i] ? 1 : 0;
  if (any_x0) {
    HIPCHK(hipMemcpyAsync(P->d_gates, gh.data(), gh.size() * sizeof(int), hipMemcpyHostToDevice, stream));
    if (o.x0_kind == FDE_X0_LOWRANK) {  // x holds c: start from S^{-1}(b + c)
      HIPCHK(run(L, "axpy", 3.0 * S.vec_bytes, [&] { return launch_axpy(P->d_desc, Sx0.kry, S.n_kry, VS_X, VS_B, 1.0, stream); }));
      STCHK(op_precond(P, Sx0, VS_X, 0, VS_X, 0));
    }
    STCHK(op_matvec(P, Sx0, VS_X, 0, VS_TMP, 0));
    HIPCHK(run(L, "dot", S.vec_bytes, [&] { return launch_dot_partial(P->d_desc, Sx0.kry, S.n_kry, VS_B, VS_TMP, 0, stream); }));
    HIPCHK(run(L, "dot", S.vec_bytes, [&] { return launch_dot_partial(P->d_desc, Sx0.kry, S.n_kry, VS_TMP, VS_TMP, 1, stream); }));
    STCHK(fetch_parts());
    std::vector<double> ybuf((size_t)count * (R + 1), 0.0);
    const double gate = L->opt_x0_gate * 1e-6;
    for (int i = 0; i < count; ++i) {
      if (!has_x0[i]) continue;
      const double bm = part_sum(P, parts, i, 0), mm = part_sum(P, parts, i, 1);
      double g = (mm > 0.0 && std::isfinite(bm / mm)) ? bm / mm : 0.0;
      const double bb = bnorm_true[i] * bnorm_true[i];
      // ||b - g M x0||^2 = ||b||^2 - <b, M x0>^2 / ||M x0||^2
      const double rr = bb > 0.0 && mm > 0.0 ? std::max(0.0, bb - bm * (bm / mm)) : bb;
      if (L->opt_x0_gate > 0 && !(rr <= gate * gate * bb)) g = 0.0;
      ybuf[(size_t)i * (R + 1)] = g;
      P->hs[i]->x0_kept = g != 0.0 ? 1 : 0;
    }
    HIPCHK(hipMemcpy(P->d_y, ybuf.data(), ybuf.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(run(L, "scale_x", 2.0 * S.vec_bytes, [&] { return launch_scale_x(P->d_desc, Sx0.kry, S.n_kry, stream); }));
  }
  // control records and gates
  std::vector<GmresCtl> &ctl = P->ctl_host;
  ctl.assign(count, GmresCtl{});
  if (dev_init) HIPCHK(launch_gm_init(P->d_desc, P->d_ctl, P->d_gates, count, o.rtol, o.maxit, stream));
  for (int i = 0; !dev_init && i < count; ++i) {
    GmresCtl &c = ctl[i];
    c.bnorm = bnorm[i];
    c.tol = o.rtol;
    c.maxit = o.maxit;
    if (bnorm[i] == 0.0) {  // u = 0 exactly
      HIPCHK(hipMemsetAsync(P->hs[i]->d_x, 0, P->hs[i]->n() * sizeof(double), stream));
      c.done = c.conv = 1;
    }
    gh[GATE_LIVE * count + i] = c.done ? 0 : 1;
    gh[GATE_ACTIVE * count + i] = 0;
  }
  if (!dev_init) {  // from pinned staging (an upload from pageable memory would block the host)
    GmresCtl *cu = (GmresCtl *)((char *)P->pin + P->pin_ctl_up);
    int *gu = (int *)((char *)P->pin + P->pin_gates_up);
    std::memcpy(cu, ctl.data(), count * sizeof(GmresCtl));
    std::memcpy(gu, gh.data(), gh.size() * sizeof(int));
    HIPCHK(hipMemcpyAsync(P->d_ctl, cu, count * sizeof(GmresCtl), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(P->d_gates, gu, gh.size() * sizeof(int), hipMemcpyHostToDevice, stream));
  }

  // Timing events are not recorded into graphs: a profiled solve launches directly.
  const bool use_graph = L->opt_graphs != 0 && !P->graph_off && !L->prof;
  const int ortho = L->opt_ortho;
  if (P->graph_R != R || P->graph_prec != S.prec || P->graph_side != (int)left ||
      P->graph_ortho != ortho) {
    HIPCHK(hipStreamSynchronize(stream));
    graphs_invalidate(P);
    P->graph_R = R;
    P->graph_prec = S.prec;
    P->graph_side = (int)left;
    P->graph_ortho = ortho;
  }
  // v_0 = r / ||r|| with r = b - M x (right) or P^{-1}(b - M x) (left); the norm goes to the
  // control record's restart test.
  auto restart_step = [&]() -> fde_status {
    STCHK(op_matvec(P, Slive, VS_X, 0, VS_TMP, 0));
    if (S.kry_one_n > 0 && !left) {  // one chunk per instance: residual, norm, v_0, decision
      HIPCHK(run(L, "residual", 3.0 * S.vec_bytes, [&] {
        return launch_restart1(P->d_desc, S.kry, S.n_kry, S.kry_one_n, P->d_ctl, P->d_work, P->d_gates,
                               count, stream);
      }));
      return FDE_OK;
    }
    HIPCHK(run(L, "residual", 3.0 * S.vec_bytes, [&] { return launch_residual(P->d_desc, Slive.kry, S.n_kry, stream); }));
    if (left) {
      STCHK(op_precond(P, Slive, VS_V, 0, VS_V, 0));
      HIPCHK(run(L, "dot", S.vec_bytes, [&] { return launch_dot_partial(P->d_desc, Slive.kry, S.n_kry, VS_V, VS_V, 0, stream); }));
    }
    HIPCHK(run(L, "normalize", 2.0 * S.vec_bytes, [&] {
      return launch_normalize(P->d_desc, Slive.kry, S.n_kry, VS_V, 0, VS_V, 0, 0, -1, stream);
    }));
    HIPCHK(launch_gm_restart(P->d_desc, P->d_ctl, P->d_work, P->d_gates, count, stream));
    return FDE_OK;
  };
  // Arnoldi step j: w = M P^{-1} v_j (right; z_j = P^{-1} v_j is kept) or P^{-1} M v_j (left).
  auto steps = [&](int j0, int j1) -> fde_status {
    for (int j = j0; j < j1; ++j) {
      g_step = j;
      if (left) {
        STCHK(op_matvec(P, Sact, VS_V, j, VS_TMP, 0));
        STCHK(op_precond(P, Sact, VS_TMP, 0, VS_W, 0));
      } else {
        STCHK(op_precond(P, Sact, VS_V, j, VS_Z, j));
        STCHK(op_matvec(P, Sact, VS_Z, j, VS_W, 0));
      }
      if (ortho == FDE_ORTHO_MGS && S.kry_one_n > 0) {
        // one chunk per instance: the projections, the norm and the Givens update in one launch
        HIPCHK(run(L, "arnoldi", (j + 4.0) * S.vec_bytes, [&] {
          return launch_arnoldi1(P->d_desc, Sact.kry, S.n_kry, S.kry_one_n, j, P->d_ctl, P->d_work,
                                 P->d_gates, count, R, stream);
        }));
        continue;
      }
      if (ortho == FDE_ORTHO_CGS2) {
        // classical Gram-Schmidt twice: V^T w, w -= V h, V^T w, w -= V h', column h + h'
        HIPCHK(run(L, "cgs", (j + 2.0) * S.vec_bytes,
                   [&] { return launch_cgs_dot(P->d_desc, Sact.kry, S.n_kry, j, stream); }));
        HIPCHK(run(L, "cgs", (2.0 * j + 5.0) * S.vec_bytes,
                   [&] { return launch_cgs_update(P->d_desc, Sact.kry, S.n_kry, j, 0, stream); }));
        HIPCHK(run(L, "cgs", (j + 3.0) * S.vec_bytes,
                   [&] { return launch_cgs_update(P->d_desc, Sact.kry, S.n_kry, j, 1, stream); }));
      } else {
        for (int i = 0; i <= j + 1; ++i) {
          HIPCHK(run(L, "mgs", (i == 0 ? 2.0 : 4.0) * S.vec_bytes,
                     [&] { return launch_mgs_step(P->d_desc, Sact.kry, S.n_kry, i, j, stream); }));
        }
      }
      HIPCHK(run(L, "normalize", 2.0 * S.vec_bytes, [&] {
        return launch_normalize(P->d_desc, Sact.kry, S.n_kry, VS_W, 0, VS_V, j + 1, (j + 1) & 1, j + 1, stream);
      }));
      HIPCHK(launch_gm_givens(P->d_desc, P->d_ctl, P->d_work, P->d_gates, count, j, R, stream));
    }
    g_step = -1;
    return FDE_OK;
  };
  auto finish_and_restart = [&]() -> fde_status {
    if (S.kry_one_n > 0) {  // one chunk per instance: back substitution and x += Q y together
      HIPCHK(run(L, "update_x", 3.0 * S.vec_bytes, [&] {
        return launch_finish1(P->d_desc, S.kry, S.n_kry, S.kry_one_n, P->d_ctl, P->d_work, P->d_gates,
                              count, left ? VS_V : VS_Z, stream);
      }));
      return restart_step();
    }
    HIPCHK(launch_gm_backsolve(P->d_desc, P->d_ctl, P->d_work, count, stream));
    HIPCHK(run(L, "update_x", 3.0 * S.vec_bytes, [&] {
      return launch_update_x(P->d_desc, Slive.kry, S.n_kry, left ? VS_V : VS_Z, stream);
    }));
    return restart_step();
  };
  // Reads the control records.  Launches of Arnoldi steps >= j0 + (steps taken since the
  // snapshot its0) were gated off for every instance; the profile does not count them.
  std::vector<int> its0(count, 0);
  int j0 = 0;
  GmresCtl *ctl_pin = (GmresCtl *)P->pin;
  int *err_pin = (int *)((char *)P->pin + P->pin_err);
  *err_pin = 0;
  auto read_ctl = [&]() -> fde_status {
    HIPCHK(hipMemcpyAsync(ctl_pin, P->d_ctl, count * sizeof(GmresCtl), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipMemcpyAsync(err_pin, P->d_err, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    std::memcpy(ctl.data(), ctl_pin, count * sizeof(GmresCtl));
    for (int i = 0; i < count; ++i)
      if (ctl[i].badrhs) return fail(FDE_EINVAL, "right-hand side %d is not finite", i);
    int taken = 0;
    for (int i = 0; i < count; ++i) taken = std::max(taken, ctl[i].its - its0[i]);
    L->prof_step_limit = j0 + taken;
    const fde_status sf = sync_and_flush(L);
    L->prof_step_limit = 1 << 30;
    for (int i = 0; i < count; ++i) its0[i] = ctl[i].its;
    return sf;
  };
  auto segment = [&](GraphSeg &g, const std::function<fde_status()> &emit) -> fde_status {
    const fde_status r = run_segment(P, g, use_graph && !P->graph_off, emit);
    g_step = -1;
    return r;
  };
  // Cycle c runs its first stretch of Arnoldi steps up to the length of cycle c of the
  // previous solve (the whole cycle if unknown), then checks on the host and continues in
  // stretches of four steps while some instance is still active.
  constexpr int kStretch = 4;
  std::vector<int> taken_per_cycle;
  STCHK(segment(P->seg_restart, restart_step));
  // From a zero start the first restart step can end only the instances the host already
  // marked done (b = 0) or that fail (then their gated steps launch nothing), so the host
  // goes straight on to the cycle and reads the records after its first stretch.
  if (any_x0 || o.maxit <= 0) STCHK(read_ctl());
  for (int c = 0;; ++c) {
    bool any = false;
    for (int i = 0; i < count; ++i) any = any || !ctl[i].done;
    if (!any) break;
    TraceRange tr_cycle("gmres restart cycle");
    std::vector<int> its_cycle(count);
    for (int i = 0; i < count; ++i) its_cycle[i] = ctl[i].its;
    const int pred = c < (int)P->pred_steps.size() ? P->pred_steps[c] : 0;
    int j = 0, len = pred > 0 ? std::min(pred, R) : R;
    for (;;) {
      const int j1 = std::min(R, j + len);
      j0 = j;
      STCHK(segment(P->seg_steps[{j, j1}], [&] { return steps(j, j1); }));
      j = j1;
      if (j >= R) break;
      STCHK(read_ctl());
      bool active = false;
      for (int i = 0; i < count; ++i) active = active || ctl[i].active;
      if (!active) break;
      len = kStretch;
    }
    STCHK(segment(P->seg_finish, finish_and_restart));
    STCHK(read_ctl());
    int cyc = 0;
    for (int i = 0; i < count; ++i) cyc = std::max(cyc, ctl[i].its - its_cycle[i]);
    taken_per_cycle.push_back(cyc);
  }
  P->pred_steps = taken_per_cycle;
  if (left) {  // the control records hold preconditioned residuals: report the true one
    STCHK(op_matvec(P, S, VS_X, 0, VS_TMP, 0));
    HIPCHK(run(L, "residual", 3.0 * S.vec_bytes, [&] { return launch_residual(P->d_desc, S.kry, S.n_kry, stream); }));
    STCHK(fetch_parts());
    for (int i = 0; i < count; ++i)
      ctl[i].truer = bnorm_true[i] > 0.0 ? std::sqrt(part_sum(P, parts, i, 0)) / bnorm_true[i] : 0.0;
  }
  for (int i = 0; i < count; ++i) {
    st[i].truer = ctl[i].truer;
    st[i].est = ctl[i].est;
    st[i].its = ctl[i].its;
    st[i].restarts = ctl[i].restarts;
    st[i].conv = ctl[i].conv != 0;
    st[i].fail = ctl[i].fail != 0;
  }
  if (*err_pin) {  // read with the last control records (no block solve ran after them)
    (void)hipMemset(P->d_err, 0, sizeof(int));
    return fail(FDE_EDEVICE, "block solve abandoned a dependency wait");
  }
  for (int i = 0; i < count; ++i)
    if (st[i].fail) return fail(FDE_ENOCONV, "instance %d produced a non-finite residual", i);
  return FDE_OK;
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

// ---- autotuner of the block-solve launch shape ------------------------------------------
// On the first solve of a plan shape (instance sizes + precision) the block solve is timed in
// each launch form: the ordinary one-workgroup-per-block launch (recorded as W = -1; blocks of
// up to four panels) and the cooperative one for each candidate W (workgroups per block)
// within the co-residency limit, on the factored blocks (the values in the work vectors do
// not matter for the timing); the fastest is kept for the life of the process.  Every form
// gives the same bits.  Skipped when the form is forced by an option, when autotuning is off,
// or when cooperative launches are unavailable.
static fde_status autotune_trsv(Plan *P, int prec) {
  fde_bvm *L = P->lead;
  if (!L->opt_autotune || L->opt_trsv_w != 0 || !g_coop_ok || L->pc != FDE_PC_STRANG) return FDE_OK;
  const std::string key = plan_shape_key(P, prec);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (g_tuned_w.count(key)) return FDE_OK;
  }
  int wtop = 1;
  for (fde_bvm *h : P->hs) wtop = std::max(wtop, trsv_wmax(P, h, prec));
  // -1: the ordinary one-workgroup-per-block launch, a candidate for blocks of at most
  // four panels (one workgroup streams a whole factor: beyond that it cannot win, and timing
  // it would cost more than the solves it could speed up)
  int npan_max = 0;
  for (fde_bvm *h : P->hs) npan_max = std::max(npan_max, h->npan);
  std::vector<int> cands;
  if (npan_max <= 4) cands.push_back(-1);
  for (int w = 1; w <= wtop; w = w < 4 ? w + 1 : w + w / 2) cands.push_back(w);
  if (cands.back() != wtop) cands.push_back(wtop);
  const bool prof = L->prof;
  L->prof = false;
  auto set_w = [&](int w) -> fde_status {
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      g_tuned_w[key] = w;
    }
    STCHK(plan_prepare(P, std::max(P->R, 1), prec));
    return ensure_full_maps(P);
  };
  hipEvent_t e0 = get_event(L), e1 = get_event(L);
  int best_w = cands.back();
  float best = 1e30f;
  fde_status s = FDE_OK;
  for (int w : cands) {
    if ((s = set_w(w)) != FDE_OK) break;
    float tmin = 1e30f;
    for (int rep = 0; rep < 4 && s == FDE_OK; ++rep) {
      (void)hipEventRecord(e0, L->stream);
      s = op_precond(P, P->full, VS_TMP, 0, VS_TMP, 0);
      (void)hipEventRecord(e1, L->stream);
      if (s != FDE_OK) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        s = fail(FDE_EDEVICE, "autotuner timing failed");
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) tmin = std::min(tmin, ms);  // the first repetition warms up
    }
    if (s != FDE_OK) break;
    if (tmin < best) {
      best = tmin;
      best_w = w;
    }
  }
  L->evpool.push_back(e0);
  L->evpool.push_back(e1);
  L->prof = prof;
  if (s == FDE_OK) s = check_trsv_err(P);
  const fde_status s2 = set_w(best_w);
  return s != FDE_OK ? s : s2;
}

// The time FFTs' column groups (4, 8 or 16 spatial columns per workgroup; every choice gives
// the same bits, each column's transform being the same), timed on the first solve of a plan
// shape like the block solve: the forward and inverse transform pair, fastest of three
// repetitions after a warm-up, kept for the process.  The heuristic choice
// (time_fft_cols_per_item) stands when autotuning is off.
static fde_status autotune_tfft(Plan *P, int prec) {
  fde_bvm *L = P->lead;
  if (!L->opt_autotune || L->pc == FDE_PC_NONE) return FDE_OK;
  const std::string key = plan_shape_key(P, prec);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (g_tuned_cols.count(key)) return FDE_OK;
  }
  const bool prof = L->prof;
  L->prof = false;
  auto set_cols = [&](int c) -> fde_status {
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      g_tuned_cols[key] = c;
    }
    P->full_ok = false;  // new item counts: new maps (and graphs)
    return ensure_full_maps(P);
  };
  hipEvent_t e0 = get_event(L), e1 = get_event(L);
  int best_c = 16;
  float best = 1e30f;
  fde_status s = FDE_OK;
  for (int c : {4, 8, 16}) {
    if ((s = set_cols(c)) != FDE_OK) break;
    const SolveMaps &S = P->full;
    float tmin = 1e30f;
    for (int rep = 0; rep < 4 && s == FDE_OK; ++rep) {
      (void)hipEventRecord(e0, L->stream);
      hipError_t e = launch_time_rfft(P->d_desc, S.tfft, S.n_tfft, S.max_log2s, S.tfft_cols, VS_TMP, 0, L->stream);
      if (e == hipSuccess)
        e = launch_time_irfft(P->d_desc, S.tfft, S.n_tfft, S.max_log2s, S.tfft_cols, VS_TMP, 0, L->stream);
      (void)hipEventRecord(e1, L->stream);
      if (e != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        s = fail(FDE_EDEVICE, "autotuner timing of the time FFTs failed");
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) tmin = std::min(tmin, ms);
    }
    if (s != FDE_OK) break;
    if (tmin < best) {
      best = tmin;
      best_c = c;
    }
  }
  L->evpool.push_back(e0);
  L->evpool.push_back(e1);
  L->prof = prof;
  const fde_status s2 = set_cols(best_c);
  return s != FDE_OK ? s : s2;
}

static fde_status solve_plan(Plan *P, const double *const *u0, const double *const *f,
                             double *const *u, const double *const *x0, const fde_solve_opts &o,
                             fde_solve_info *info) {
  TraceRange tr_solve("fde_bvm_solve");
  fde_bvm *L = P->lead;
  const int count = (int)P->hs.size();
  const int prec = P->hs[0]->prec;
  for (int i = 0; i < count; ++i) {
    fde_bvm *h = P->hs[i];
    if (h->prec < 0) return fail(FDE_EINVAL, "fde_precond_factor must succeed before solving (instance %d)", i);
    if (h->prec != prec) return fail(FDE_EINVAL, "all instances of a batch need the same precision");
    if (h->pc != P->hs[0]->pc) return fail(FDE_EINVAL, "all instances of a batch need the same preconditioner");
    if (!u0[i] || !f[i] || !u[i]) return fail(FDE_EINVAL, "u0, f and u are required (instance %d)", i);
    if (h->stream != L->stream) HIPCHK(hipStreamSynchronize(h->stream));
  }
  STCHK(plan_prepare(P, o.restart, prec));
  STCHK(autotune_trsv(P, prec));
  STCHK(autotune_tfft(P, prec));
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
  for (int i = 0; i < count; ++i) {
    has_x0[i] = (x0 && x0[i]) ? 1 : 0;
    P->hs[i]->x0_kept = 0;
  }
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
  STCHK(plan_prepare(h->self, std::max(h->self->R, 1), h->prec));
  STCHK(ensure_full_maps(h->self));
  S = h->self->full;
  return FDE_OK;
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

// ---- allocation-free preconditioner apply --------------------------------------------------
// Working memory of fde_apply_precond_noalloc: one file-scope device array per GPU, held until
// the process ends.  Layout: the launch head (descriptor, item maps, epoch counter and slots,
// error flag) in the first NA_HEAD bytes, the block-solve flags [nb][npan][2] in the next
// NA_FLAGS bytes (a region of their own, so no other use of the array ever overwrites them:
// every apply draws a larger epoch from the array's own counter, and flags only ever hold
// earlier epochs), then the frequency-domain vector [nb][mp] complex FP64.
static constexpr size_t NA_BYTES = (size_t)FDE_NOALLOC_SCRATCH_BYTES;
static constexpr size_t NA_HEAD = 4096;
static constexpr size_t NA_FLAGS = 512u << 10;
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

struct NoallocHead {
  InstDesc desc;
  int ids[1];
  int pre_tfft[2], pre_trsv[2], pre_blk[2];
  int err;
  unsigned long long ctr;       // epochs drawn by the applies that used this array
  unsigned long long epoch[2];  // epoch of the current apply, claimed-unit counter
};
static_assert(sizeof(NoallocHead) <= NA_HEAD, "launch head exceeds its region");

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {};

// Device address of this GPU's array (the name `scratch` is a host-side stand-in): looked up
// once per device, with that device current, and kept.
static fde_status noalloc_scratch(void **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(FDE_EDEVICE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FDE_OK;
}

// Writes the launch head of one apply (the counter is left as it is); the block solve's error
// flag starts at zero.
__global__ void k_noalloc_head(NoallocHead *hd, InstDesc d, int n_tfft, int n_trsv, int n_blk) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  hd->desc = d;
  hd->ids[0] = 0;
  hd->pre_tfft[0] = 0;
  hd->pre_tfft[1] = n_tfft;
  hd->pre_trsv[0] = 0;
  hd->pre_trsv[1] = n_trsv;
  hd->pre_blk[0] = 0;
  hd->pre_blk[1] = n_blk;
  hd->err = 0;
}

extern "C" fde_status fde_apply_precond_noalloc(fde_bvm *h, const double *v, double *z) {
  if (!h || !v || !z) return fail(FDE_EINVAL, "NULL argument");
  const size_t flag_bytes = (size_t)h->nb * h->npan * 2 * sizeof(unsigned long long);
  const size_t vh_bytes = (size_t)h->nb * h->mp * sizeof(double2);
  if (flag_bytes > NA_FLAGS || vh_bytes > NA_BYTES - NA_HEAD - NA_FLAGS)
    return fail(FDE_EUNSUPPORTED,
                "m = %d, s = %d needs %zu bytes of working memory; the allocation-free apply has %zu",
                h->m, h->s, NA_HEAD + NA_FLAGS + vh_bytes, NA_BYTES);
  if (h->prec < 0) return fail(FDE_EINVAL, "fde_precond_factor must succeed first");
  if (h->pc != FDE_PC_STRANG || h->blk_route != FDE_BLOCKS_LU)
    return fail(FDE_EUNSUPPORTED, "the allocation-free apply takes the Strang preconditioner with block LU factors");
  void *base = nullptr;
  STCHK(noalloc_scratch(&base));
  unsigned char *b = (unsigned char *)base;
  NoallocHead *hd = (NoallocHead *)b;
  // launch shapes as the handle's own apply takes them (same kernels, same bits)
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int cols = time_fft_cols_per_item(h->mp, std::max(cus, 1));
  const int W = trsv_workgroups(h->self, h, h->prec);
  const int n_tfft = h->mp / cols, n_trsv = h->nb * W, n_blk = h->nb;
  InstDesc d = make_desc(h);
  d.W = W;
  d.sio = const_cast<double *>(v);  // read by the time FFT
  d.tmp = z;                        // written by the inverse time FFT
  d.tsflags = (unsigned long long *)(b + NA_HEAD);
  d.Vh = (double2 *)(b + NA_HEAD + NA_FLAGS);
  d.Vts = d.Vh;
  hipStream_t st = h->stream;
  hipLaunchKernelGGL(k_noalloc_head, dim3(1), dim3(64), 0, st, hd, d, n_tfft, n_trsv, n_blk);
  HIPCHK(hipGetLastError());
  const InstDesc *D = &hd->desc;
  const ItemMap tfft{hd->ids, hd->pre_tfft, 1, nullptr};
  const ItemMap trsv{hd->ids, hd->pre_trsv, 1, nullptr};
  const ItemMap blk{hd->ids, hd->pre_blk, 1, nullptr};
  HIPCHK(launch_time_rfft(D, tfft, n_tfft, h->log2s, cols, VS_SIO, 0, st, &hd->ctr, hd->epoch));
  if (h->self->trsv_solo)  // the handle's plan takes the ordinary one-workgroup launch (same bits)
    HIPCHK(h->prec == FDE_FP64 ? launch_trsv<double>(D, trsv, n_trsv, 0, st) : launch_trsv<float>(D, trsv, n_trsv, 0, st));
  else
    HIPCHK(h->prec == FDE_FP64
               ? launch_trsv_coop<double>(D, trsv, n_trsv, hd->epoch, &hd->err, st, 0, &blk, n_blk, h->npan)
               : launch_trsv_coop<float>(D, trsv, n_trsv, hd->epoch, &hd->err, st, 0, &blk, n_blk, h->npan));
  HIPCHK(launch_time_irfft(D, tfft, n_tfft, h->log2s, cols, VS_TMP, 0, st));
  int err = 0;
  HIPCHK(hipMemcpyAsync(&err, &hd->err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (err) return fail(FDE_EDEVICE, "block solve abandoned a dependency wait");
  return FDE_OK;
}

extern "C" fde_status fde_time_rfft(fde_bvm *h, const double *v, double *vhat, int mem_space) {
  if (!h || !v || !vhat) return fail(FDE_EINVAL, "NULL argument");
  if (mem_space != FDE_MEM_HOST && mem_space != FDE_MEM_DEVICE) return fail(FDE_EINVAL, "bad mem_space");
  SolveMaps S;
  STCHK(self_maps(h, S));
  STCHK(copy_in(h, h->d_sio, v, h->n(), mem_space));
  HIPCHK(launch_time_rfft(h->self->d_desc, S.tfft, S.n_tfft, S.max_log2s, S.tfft_cols, VS_SIO, 0, h->stream));
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

extern "C" fde_status fde_get_hessenberg(fde_bvm *h, double *H, double *Q) {
  if (!h || !H || !Q) return fail(FDE_EINVAL, "NULL argument");
  const bool band = h->blk_route == FDE_BLOCKS_BAND;
  if (h->prec < 0 || h->blk_route == FDE_BLOCKS_LU || !(band ? (void *)h->d_bAQ : (void *)h->d_hH))
    return fail(FDE_EINVAL, "no Hessenberg or band factorization stored");
  const size_t m = h->m, mp = h->mp;
  const double *dH = band ? h->d_bAQ : h->d_hH;
  const double *dQ = band ? h->d_bAQ + mp * mp : h->d_hQ;
  HIPCHK(hipMemcpy2DAsync(H, m * sizeof(double), dH, mp * sizeof(double), m * sizeof(double), m,
                          hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpy2DAsync(Q, m * sizeof(double), dQ, mp * sizeof(double), m * sizeof(double), m,
                          hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return FDE_OK;
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
