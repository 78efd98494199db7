// homg_capi.cpp -- C ABI, planner and cycle driver of the MI355X HOMG library.
//
// The driver sequences the steps of the method (arXiv:1108.2045, Sec. 2) on
// one HIP stream:
//   residual r_0 = f - A u and its norm           (residual equation)
//   restriction pyramid r_1 .. r_M                (nested partial reductions)
//   the MFMG schedule of whole-grid iterations    (fused relax+interpolate)
//   u += e, fused into the last iteration; next residual
// and restarts cycles until the relative residual reaches the tolerance.
//
// Control stays on the device: every kernel of a cycle first reads a
// device-side `done` flag that the norm kernel sets when the tolerance is
// met, so the host can enqueue several cycles ahead without a round trip;
// it synchronises only to read the residual history, sizing each batch of
// cycles from the contraction observed so far.  Cycles enqueued past
// convergence do no work and leave u untouched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/homg.h"
#include "homg_internal.h"

using namespace homg;

namespace {

thread_local std::string g_err;

}  // namespace

void homg::set_last_error(const char* msg) { g_err = msg; }

namespace {

enum Kind {
  K_NORM = 0, K_RESIDUAL = 1, K_FINALIZE = 2, K_RESTRICT = 3, K_SWEEP = 4,
  K_GATHER = 5, K_LATTICE = 6, K_LEVEL_WRITE = 7, K_LEARNED = 8, K_TRANSFER = 9, K_TAIL = 10
};

// Event-pair timing of individual launches, harvested at the end of a solve.
struct Profiler {
  using Key = std::tuple<int, int, int>;  // kind, level, mode
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<Key, size_t>> pending;  // key, index of the start event
  std::map<Key, std::pair<long long, double>> acc;
};

}  // namespace

struct homg_ctx {
  int d = 0, n = 0, k = 0, levels = 0;
  int stencil = 0, prec = 0;
  double omega = 0.8;
  int max_i = 4, max_cycles = 200, temporal = 0;
  std::vector<int> sched;  // (level, iterations) pairs
  int top_level = 0;       // coarsest level the schedule visits
  int total_sweeps = 0;
  Lay dl;                  // caller's dense FP64 arrays (side n)
  Lay el;                  // internal e arrays
  std::vector<Lay> rl;     // internal residual pyramid, per level
  std::vector<Lay> al;     // internal coefficient pyramid (FP64), per level
  std::vector<Lay> cdl;    // dense layouts of the compact levels (step entry points)
  void* e[2] = {nullptr, nullptr};
  std::vector<void*> r;
  std::vector<double*> a;
  std::vector<void*> xc;   // level-blocked path: compact x_{t-1}, x_t pairs per level (2m, 2m+1)
  std::vector<void*> xp3;  // Laplacian: third compact array per level (x_{it-1} of a multi-iteration pass)
  size_t lds_limit = 65536;
  bool has_coef = false;
  double* partials = nullptr;
  int npart = 0;
  DevState* st = nullptr;
  double* hist = nullptr;
  int* zero_flag = nullptr;
  DevState* h_st = nullptr;  // pinned mirrors
  double* h_hist = nullptr;
  int device = 0;
  std::string err;
  long long launches = 0;
  Profiler prof;
  // learned relaxation (2D): 0 damped Jacobi, 1 the network with weights w
  int chain_ready = -1;        // chained path: level whose x_0 the previous level already wrote
  // chained path: the compact final state of level lat_level + 1, which
  // the first pass of level lat_level interpolates itself (no hand-over or
  // whole-grid write in between); -1: none pending
  int lat_level = -1;
  L1State lat;
  int smoother = 0;
  int active_smoother = 0;     // smoother of the solve in progress (after any fallback)
  double fallback_ratio = 1.0; // per-cycle contraction at which a solve falls back to Jacobi
  double rho_ref = 0.0;        // damped-Jacobi reference contraction from the last gate (0: none)
  uint16_t* wbf = nullptr;     // the 576 weights in BF16
  float* w32 = nullptr;        // their FP32 values (what the kernels read)
  // FP32/BF16 cycles: the coarsest level (top_level) in FP64 -- its
  // right-hand side and iterate pair, compact, layout l64
  double* r64 = nullptr;
  double* x64[2] = {nullptr, nullptr};
  Lay l64;
  // in-cycle restriction (Sec. 2): one extra array, two halves rbuf[0]
  // (odd levels) and rbuf[1] (even levels), instead of the pyramid; r[m]
  // (m >= 1) aliases them.  rhs_ready: the highest level of the current
  // chain (its level and the one below are valid); rhs_top64: the FP64
  // coarsest right-hand side of this cycle is computed.
  size_t ws_bytes = 0;          // device bytes allocated by the handle
  bool incycle = false;
  void* rbuf[2] = {nullptr, nullptr};
  int rhs_ready = 0;
  bool rhs_top64 = false;
  // power-of-two layout (Sec. 3): the quadrants' restriction families,
  // level m >= 1 of quadrant q at fam[4 m + q], layout faml[m]
  bool pow2 = false;
  std::vector<double*> fam;
  std::vector<Lay> faml;
  // L1 error (Sec. 4): partial sums and per-iteration results (allocated on first use)
  double* l1part = nullptr;
  double* l1out = nullptr;
  int l1cap = 0;
};

namespace {

homg_status fail(homg_ctx* h, homg_status s, const std::string& msg) {
  g_err = msg;
  if (h) h->err = msg;
  return s;
}

#define HIPCHK(h, call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(h, HOMG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

// Launch with optional event-pair timing under the class (kind, level, mode).
#define LAUNCH_K(h, s, kind, level, mode, call)                                 \
  do {                                                                          \
    size_t ev_ = 0;                                                             \
    if ((h)->prof.on) {                                                         \
      if (homg_status pe_ = prof_begin(h, &ev_)) return pe_;                    \
    }                                                                           \
    hipError_t le_ = (call);                                                    \
    set_launch_events(nullptr, nullptr);                                        \
    HIPCHK(h, le_);                                                             \
    ++(h)->launches;                                                            \
    if ((h)->prof.on)                                                           \
      (h)->prof.pending.push_back({Profiler::Key(kind, level, mode), ev_});     \
  } while (0)

#define LAUNCH(h, call)          \
  do {                           \
    HIPCHK(h, call);             \
    ++(h)->launches;             \
  } while (0)

// Reserve an event pair and arm it for the next launch: the launch stamps
// the pair with its own start and end (hipExtLaunchKernelGGL), so the
// elapsed time is the kernel's execution alone.
homg_status prof_begin(homg_ctx* h, size_t* ev) {
  Profiler& p = h->prof;
  while (p.pool.size() < p.used + 2) {
    hipEvent_t e;
    HIPCHK(h, hipEventCreate(&e));
    p.pool.push_back(e);
  }
  *ev = p.used;
  p.used += 2;
  set_launch_events(p.pool[*ev], p.pool[*ev + 1]);
  return HOMG_OK;
}

// Accumulate the elapsed times of all recorded pairs (waits for them).
homg_status prof_harvest(homg_ctx* h) {
  Profiler& p = h->prof;
  for (auto& kv : p.pending) {
    float ms = 0.f;
    HIPCHK(h, hipEventSynchronize(p.pool[kv.second + 1]));
    HIPCHK(h, hipEventElapsedTime(&ms, p.pool[kv.second], p.pool[kv.second + 1]));
    auto& a = p.acc[kv.first];
    a.first += 1;
    a.second += double(ms);
  }
  p.pending.clear();
  p.used = 0;
  return HOMG_OK;
}

// Keeps the handle's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int side_exponent(int64_t n) {
  if (n < 3) return -1;
  int k = 0;
  while ((int64_t(1) << (k + 1)) + 1 <= n) ++k;
  return ((int64_t(1) << k) + 1 == n) ? k : -1;
}

void free_ctx(homg_ctx* h) {
  if (!h) return;
  (void)hipFree(h->e[0]);
  (void)hipFree(h->e[1]);
  if (h->incycle) {
    if (!h->r.empty()) (void)hipFree(h->r[0]);
    (void)hipFree(h->rbuf[0]);
    (void)hipFree(h->rbuf[1]);
  } else {
    for (void* p : h->r) (void)hipFree(p);
  }
  for (double* p : h->a) (void)hipFree(p);
  for (void* p : h->xc) (void)hipFree(p);
  for (void* p : h->xp3) (void)hipFree(p);
  for (double* p : h->fam) (void)hipFree(p);
  (void)hipFree(h->partials);
  (void)hipFree(h->st);
  (void)hipFree(h->hist);
  (void)hipFree(h->zero_flag);
  (void)hipFree(h->wbf);
  (void)hipFree(h->w32);
  (void)hipFree(h->l1part);
  (void)hipFree(h->l1out);
  (void)hipFree(h->r64);
  (void)hipFree(h->x64[0]);
  (void)hipFree(h->x64[1]);
  if (h->h_st) (void)hipHostFree(h->h_st);
  if (h->h_hist) (void)hipHostFree(h->h_hist);
  for (hipEvent_t e : h->prof.pool) (void)hipEventDestroy(e);
  delete h;
}

homg_status dev_alloc(homg_ctx* h, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(h, HOMG_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  h->ws_bytes += bytes;
  return HOMG_OK;
}

// `it` iterations of level m on the whole-grid state e[*cur] (Sec. 2, fused
// relax+interpolate task), leaving the result in e[*cur] (or added into acc
// when `last`).  `first`: the state is e = 0 (first level of a cycle).
homg_status run_level_learned(homg_ctx* h, int m, int it, bool first, bool last, int next_m,
                              int* cur, double* acc, const int* done, hipStream_t s);
homg_status finish_level(homg_ctx* h, int m, bool last, int next_m, int wmode, void* xprev,
                         void* xcur, int* cur, double* acc, const int* done, hipStream_t s);

// Whether the coarsest level of this cycle runs in FP64: FP32/BF16 storage
// with damped Jacobi.  Its right-hand side is restricted in FP64 from the
// stored values of the level below, its iterations run in FP64 on the
// compact lattice, and only the final pair is rounded to the storage type
// for the hand-over (the residual, the update of u and the norms are FP64
// in every mode).
bool top64(const homg_ctx* h) {
  return h->prec != PREC_F64 && h->active_smoother == 0 && h->top_level >= 1 && h->r64;
}

// Whether level mt's iterations (chained execution, Laplacian, damped
// Jacobi) run as multi-iteration passes whose first pass takes its input
// iterate from level mt + 1's compact state: level 0, or in 2D a compact
// lattice too large for one workgroup.  In 3D the hand-over kernel plus a
// plain pass measured as fast or faster on the compact lattices (MI355X,
// 257^3: 31 against 31 us at 129^3, 13 against 16 us at 65^3, 12 against
// 16 us at 33^3: at these sizes the pass is latency-bound and the extra
// loads sit on its critical path).
bool lat_target(const homg_ctx* h, int mt) {
  if (h->temporal != 2 || h->active_smoother != 0 || h->has_coef || mt < 0 || h->pow2) return false;
  if (top64(h) && mt == h->top_level) return false;  // starts from an FP64 x_0
  const int nm = (h->n - 1) / (1 << mt) + 1;
  if (nm < 5 || mt + 1 >= h->levels) return false;
  if (mt == 0) return true;
  return lattice_small_lds(h->prec, h->d, nm, false) > h->lds_limit && mt < int(h->xp3.size()) &&
         h->xp3[mt];
}

// `it` FP64 iterations of the coarsest level m (see top64) on its compact
// lattice: x_0 is 0, the compact hand-over of the previous level, or the
// whole grid sampled on the lattice, widened exactly; the final pair is
// rounded to the storage type (into the level's compact pair) and handed
// over as any blocked level's (same contract as run_level).
homg_status run_top64(homg_ctx* h, int m, int it, bool first, bool last, int next_m, int* cur,
                      double* acc, const int* done, hipStream_t s) {
  const Lay none;
  const double* am = h->has_coef ? h->a[m] : nullptr;
  const Lay& alm = am ? h->al[m] : none;
  const int l = 1 << m, nm = (h->n - 1) / l + 1;
  const bool chained_in = !first && h->chain_ready == m;
  h->chain_ready = -1;
  h->lat_level = -1;
  double* X[2] = {h->x64[0], h->x64[1]};
  if (!first)
    LAUNCH_K(h, s, K_GATHER, m, 1,
             launch_widen(h->prec, h->d, chained_in ? h->xc[2 * m] : h->e[*cur], chained_in ? h->rl[m] : h->el,
                          chained_in ? 1 : l, X[0], h->l64, done, s));
  double* xprev;
  double* xcur;
  if (lattice_small_lds(PREC_F64, h->d, nm, am != nullptr) <= h->lds_limit) {
    LAUNCH_K(h, s, K_LATTICE, m, 4 | (first ? 1 : 0) | 256,
             launch_lattice_small(PREC_F64, h->d, nm, 1, it, h->omega, first, X[0], h->l64, h->r64, h->l64, am,
                                  alm, X[0], X[1], h->l64, done, s));
    xprev = X[0];
    xcur = X[1];
  } else {
    int src = 0;
    for (int t = 1; t <= it; ++t) {
      const int mode = (first && t == 1) ? SW_ZERO_OLD : 0;
      LAUNCH_K(h, s, K_LATTICE, m, mode | 256,
               launch_sweep(PREC_F64, h->d, nm, 0, h->omega, X[src], X[1 - src], h->l64, h->r64, h->l64, am,
                            alm, nullptr, none, mode, done, s, true));
      src = 1 - src;
    }
    xcur = X[src];
    xprev = X[1 - src];
  }
  int wmode = last ? SW_ACCUM : 0;
  if (first && it == 1) wmode |= SW_ZERO_OLD;  // x_0 = 0
  void* tp = h->xc[2 * m];
  void* tc = h->xc[2 * m + 1];
  if (!(wmode & SW_ZERO_OLD))
    LAUNCH_K(h, s, K_GATHER, m, 2, launch_narrow(h->prec, h->d, xprev, h->l64, tp, h->rl[m], done, s));
  LAUNCH_K(h, s, K_GATHER, m, 2, launch_narrow(h->prec, h->d, xcur, h->l64, tc, h->rl[m], done, s));
  return finish_level(h, m, last, next_m, wmode, tp, tc, cur, acc, done, s);
}

homg_status run_level(homg_ctx* h, int m, int it, bool first, bool last, int next_m, int* cur,
                      double* acc, const int* done, hipStream_t s) {
  if (h->active_smoother == 1) return run_level_learned(h, m, it, first, last, next_m, cur, acc, done, s);
  if (top64(h) && m == h->top_level) return run_top64(h, m, it, first, last, next_m, cur, acc, done, s);
  if (h->pow2 && m >= 1) {
    // power-of-two layout: one whole-grid launch per iteration
    const double* fm[4] = {h->fam[4 * m], h->fam[4 * m + 1], h->fam[4 * m + 2], h->fam[4 * m + 3]};
    for (int t = 0; t < it; ++t) {
      int mode = 0;
      if (first && t == 0) mode |= SW_ZERO_OLD;
      if (last && t == it - 1) mode |= SW_ACCUM;
      LAUNCH_K(h, s, K_SWEEP, m, mode | 256,
               launch_p2_sweep(h->n, m, h->omega, static_cast<const double*>(h->e[*cur]),
                               static_cast<double*>(h->e[1 - *cur]), h->el, fm, h->faml[m], acc, h->dl, mode,
                               done, s));
      *cur = 1 - *cur;
    }
    return HOMG_OK;
  }
  const Lay none;
  const double* am = h->has_coef ? h->a[m] : nullptr;
  const Lay& alm = am ? h->al[m] : none;
  // One launch per iteration: level 0 always (every node is a lattice
  // node), every level when blocking is off, and a coarse last level in
  // reduced precision (its iterate goes into u unrounded).
  // chained path: the first pass reads the next coarser level's compact state
  const L1State* l1 = h->lat_level == m ? &h->lat : nullptr;
  h->lat_level = -1;
  if (m == 0 && h->d == 3 && h->temporal) {
    // level 0 in 3D: up to TB3_MAX_IT iterations per pass, same iterates
    for (int t0 = 0; t0 < it; t0 += TB3_MAX_IT) {
      const int g = std::min(TB3_MAX_IT, it - t0);
      const bool zero = first && t0 == 0, accum = last && t0 + g == it;
      const L1State* src = t0 == 0 ? l1 : nullptr;
      const int mode = SW_TBLOCK | (zero ? SW_ZERO_OLD : 0) | (accum ? SW_ACCUM : 0) | ((g - 1) << 4) |
                       (src ? 128 : 0);
      LAUNCH_K(h, s, K_SWEEP, 0, mode,
               launch_tb_3d(h->prec, h->n, g, h->omega, h->e[*cur], h->e[1 - *cur], nullptr, h->el,
                            h->r[0], h->rl[0], acc, h->dl, zero, accum, false, done, s, 0, src));
      *cur = 1 - *cur;
    }
    return HOMG_OK;
  }
  if (m == 0 && h->d == 2 && !am && h->temporal) {
    // level 0 of a 2D constant-coefficient grid: up to TB_MAX_IT iterations
    // per pass (temporally blocked), the same iterates bit for bit
    for (int t0 = 0; t0 < it; t0 += TB_MAX_IT) {
      const int g = std::min(TB_MAX_IT, it - t0);
      const bool zero = first && t0 == 0, accum = last && t0 + g == it;
      const L1State* src = t0 == 0 ? l1 : nullptr;
      const int mode = SW_TBLOCK | (zero ? SW_ZERO_OLD : 0) | (accum ? SW_ACCUM : 0) | ((g - 1) << 4) |
                       (src ? 128 : 0);
      LAUNCH_K(h, s, K_SWEEP, 0, mode,
               launch_sweep_2d_l0_tb(h->prec, h->n, g, h->omega, h->e[*cur], h->e[1 - *cur], h->el,
                                     h->r[0], h->rl[0], acc, h->dl, zero, accum, done, s, 0, src));
      *cur = 1 - *cur;
    }
    return HOMG_OK;
  }
  if (l1 && (m == 0 || !h->temporal || (last && h->prec != PREC_F64)))
    return fail(h, HOMG_ERR_UNSUPPORTED, "the coarser level left no state for this level's iterations");
  if (m == 0 || !h->temporal || (last && h->prec != PREC_F64)) {
    for (int t = 0; t < it; ++t) {
      int mode = 0;
      if (first && t == 0) mode |= SW_ZERO_OLD;
      if (last && t == it - 1) mode |= SW_ACCUM;
      LAUNCH_K(h, s, K_SWEEP, m, mode,
               launch_sweep(h->prec, h->d, h->n, m, h->omega, h->e[*cur], h->e[1 - *cur], h->el,
                            h->r[m], h->rl[m], am, alm, acc, h->dl, mode, done, s));
      *cur = 1 - *cur;
    }
    return HOMG_OK;
  }
  // Level-blocked: iterations on the compact lattice, one whole-grid pass.
  const int l = 1 << m, nm = (h->n - 1) / l + 1;
  const Lay& cl = h->rl[m];
  void* X0 = h->xc[2 * m];
  void* X1 = h->xc[2 * m + 1];
  void* xprev;
  void* xcur;
  int wmode = last ? SW_ACCUM : 0;
  // chained path: the previous level already left x_0 in X0
  const bool chained_in = !first && h->chain_ready == m;
  h->chain_ready = -1;
  if (l1 && !lat_target(h, m))
    return fail(h, HOMG_ERR_UNSUPPORTED, "the coarser level left no state for this level's iterations");
  if (lattice_small_lds(h->prec, h->d, nm, am != nullptr) <= h->lds_limit) {
    LAUNCH_K(h, s, K_LATTICE, m, 4 | (first ? 1 : 0),
             launch_lattice_small(h->prec, h->d, nm, chained_in ? 1 : l, it, h->omega, first,
                                  chained_in ? X0 : h->e[*cur], chained_in ? cl : h->el,
                                  h->r[m], h->rl[m], am, alm, X0, X1, cl, done, s));
    xprev = X0;
    xcur = X1;
  } else if (!am && m < int(h->xp3.size()) && h->xp3[m]) {
    // Laplacian: several iterations per pass over the lattice
    if (!first && !chained_in && !l1)
      LAUNCH_K(h, s, K_GATHER, m, 0, launch_gather(h->prec, h->d, h->e[*cur], h->el, l, X0, cl, done, s));
    void* X[2] = {X0, X1};
    int src = 0;
    xprev = nullptr;
    const int gmax = h->d == 2 ? TB_MAX_IT : TB3_MAX_IT;
    const bool tiled = (h->d == 3 && nm <= LT_MAX_SIDE &&
                        lattice_3d_tiled_lds(h->prec, std::min(it, LT_MAX_IT)) <= h->lds_limit) ||
                       (h->d == 2 && nm <= LT2_MAX_SIDE);
    for (int t0 = 0; tiled && t0 < it; t0 += LT_MAX_IT) {
      // small lattice: up to four iterations per launch on LDS tiles (x_{it-1}
      // of every launch into the third array; the last one's is kept)
      const int g = std::min(LT_MAX_IT, it - t0);
      const bool zero = first && t0 == 0;
      const L1State* ls = t0 == 0 ? l1 : nullptr;
      LAUNCH_K(h, s, K_LATTICE, m,
               SW_TBLOCK | (zero ? SW_ZERO_OLD : 0) | ((g - 1) << 4) | 64 | (ls ? 128 : 0) | 256,
               h->d == 3 ? launch_lattice_3d_tiled(h->prec, nm, g, h->omega, (zero || ls) ? nullptr : X[src],
                                                   X[1 - src], h->xp3[m], cl, h->r[m], h->rl[m], zero, ls, done, s)
                         : launch_lattice_2d_tiled(h->prec, nm, g, h->omega, (zero || ls) ? nullptr : X[src],
                                                   X[1 - src], h->xp3[m], cl, h->r[m], h->rl[m], zero, ls, done, s));
      xprev = h->xp3[m];
      src = 1 - src;
    }
    for (int t0 = 0; !tiled && t0 < it; t0 += gmax) {
      const int g = std::min(gmax, it - t0);
      const bool zero = first && t0 == 0, lastg = t0 + g == it;
      // the first pass may take x_0 from the coarser level's state (x_0 is
      // then never stored: a single-iteration last pass stores it as x_{it-1})
      const L1State* ls = t0 == 0 ? l1 : nullptr;
      void* pv = (lastg && (g > 1 || ls)) ? h->xp3[m] : nullptr;
      const Lay none;
      LAUNCH_K(h, s, K_LATTICE, m,
               SW_TBLOCK | (zero ? SW_ZERO_OLD : 0) | ((g - 1) << 4) | (pv ? 64 : 0) | (ls ? 128 : 0),
               h->d == 2 ? launch_lattice_2d_tb(h->prec, nm, g, h->omega, X[src], X[1 - src], pv, cl,
                                                h->r[m], h->rl[m], zero, done, s, 0, ls)
                         : launch_tb_3d(h->prec, nm, g, h->omega, X[src], X[1 - src], pv, cl, h->r[m],
                                        h->rl[m], nullptr, none, zero, false, true, done, s, 0, ls));
      if (lastg) xprev = pv ? pv : X[src];
      src = 1 - src;
    }
    xcur = X[src];
    if (first && it == 1) wmode |= SW_ZERO_OLD;  // x_0 = 0 was never stored
  } else {
    if (!first && !chained_in)
      LAUNCH_K(h, s, K_GATHER, m, 0, launch_gather(h->prec, h->d, h->e[*cur], h->el, l, X0, cl, done, s));
    void* X[2] = {X0, X1};
    int src = 0;
    for (int t = 1; t <= it; ++t) {
      const int mode = (first && t == 1) ? SW_ZERO_OLD : 0;
      LAUNCH_K(h, s, K_LATTICE, m, mode,
               launch_sweep(h->prec, h->d, nm, 0, h->omega, X[src], X[1 - src], cl, h->r[m],
                            h->rl[m], am, alm, nullptr, none, mode, done, s, true));
      src = 1 - src;
    }
    xcur = X[src];
    xprev = X[1 - src];
    if (first && it == 1) wmode |= SW_ZERO_OLD;  // x_0 = 0 was never stored
  }
  return finish_level(h, m, last, next_m, wmode, xprev, xcur, cur, acc, done, s);
}

// The end of a blocked coarse level: one whole-grid pass, or -- on the
// chained path, when the next level is a different coarse level -- only
// that level's x_0 (the same values the whole-grid pass would leave at its
// lattice nodes).  Level 0 reads every node, so the pass before it is
// always whole-grid.
homg_status finish_level(homg_ctx* h, int m, bool last, int next_m, int wmode, void* xprev,
                         void* xcur, int* cur, double* acc, const int* done, hipStream_t s) {
  // chained path into the next finer level's multi-iteration passes: its
  // first pass interpolates this level's compact state itself
  if (!last && next_m == m - 1 && lat_target(h, next_m)) {
    h->lat.prev = (wmode & SW_ZERO_OLD) ? nullptr : xprev;
    h->lat.cur = xcur;
    h->lat.cl = h->rl[m];
    h->lat.zero_old = (wmode & SW_ZERO_OLD) != 0;
    h->lat_level = next_m;
    return HOMG_OK;
  }
  if (h->temporal == 2 && !last && next_m >= 1 && next_m != m) {
    LAUNCH_K(h, s, K_TRANSFER, next_m, wmode & SW_ZERO_OLD,
             launch_level_transfer(h->prec, h->d, m, xprev, xcur, h->rl[m], next_m, h->xc[2 * next_m],
                                   h->rl[next_m], (wmode & SW_ZERO_OLD) != 0, done, s));
    h->chain_ready = next_m;
    return HOMG_OK;
  }
  LAUNCH_K(h, s, K_LEVEL_WRITE, m, wmode,
           launch_level_write(h->prec, h->d, h->n, m, xprev, xcur, h->rl[m], h->e[1 - *cur], h->el, acc,
                              h->dl, wmode, done, s));
  *cur = 1 - *cur;
  return HOMG_OK;
}

// `it` iterations of level m with the learned relaxation (same contract as
// run_level).  A level-m iteration reads only lattice values, so the
// iterations run on the compact lattice and one whole-grid pass writes the
// level's final state (lattice nodes x_it, every other node the interpolant
// of x_{it-1}); level 0 is the whole grid.
homg_status run_level_learned(homg_ctx* h, int m, int it, bool first, bool last, int next_m,
                              int* cur, double* acc, const int* done, hipStream_t s) {
  const Lay none;
  const double* am = h->has_coef ? h->a[m] : nullptr;
  const Lay& alm = am ? h->al[m] : none;
  const int l = 1 << m, nm = (h->n - 1) / l + 1;
  const double hl = double(l) / double(h->n - 1);
  if (m == 0) {
    for (int t = 0; t < it; ++t) {
      int mode = 0;
      if (first && t == 0) mode |= SW_ZERO_OLD;
      if (last && t == it - 1) mode |= SW_ACCUM;
      LAUNCH_K(h, s, K_LEARNED, 0, mode,
               launch_learned_iter(h->prec, nm, hl, h->e[*cur], h->el, h->e[1 - *cur], h->r[0],
                                   h->rl[0], am, alm, acc, h->dl, h->w32, mode, done, s));
      *cur = 1 - *cur;
    }
    return HOMG_OK;
  }
  const Lay& cl = h->rl[m];
  void* X[2] = {h->xc[2 * m], h->xc[2 * m + 1]};
  const bool chained_in = !first && h->chain_ready == m;
  h->chain_ready = -1;
  if (nm <= LEARNED_SMALL_NM) {  // one workgroup, every iteration, x_0 read in place
    LAUNCH_K(h, s, K_LEARNED, m, 4 | (first ? 1 : 0),
             launch_learned_small(h->prec, nm, chained_in ? 1 : l, it, hl, first,
                                  chained_in ? X[0] : h->e[*cur], chained_in ? cl : h->el, h->r[m],
                                  h->rl[m], am, alm, X[0], X[1], cl, h->w32, done, s));
    return finish_level(h, m, last, next_m, last ? SW_ACCUM : 0, X[0], X[1], cur, acc, done, s);
  }
  if (!first && !chained_in)
    LAUNCH_K(h, s, K_GATHER, m, 0, launch_gather(h->prec, h->d, h->e[*cur], h->el, l, X[0], cl, done, s));
  int src = 0;
  for (int t = 1; t <= it; ++t) {
    const int mode = (first && t == 1) ? SW_ZERO_OLD : 0;
    LAUNCH_K(h, s, K_LEARNED, m, mode,
             launch_learned_iter(h->prec, nm, hl, X[src], cl, X[1 - src], h->r[m], h->rl[m], am,
                                 alm, nullptr, none, h->w32, mode, done, s));
    src = 1 - src;
  }
  int wmode = last ? SW_ACCUM : 0;
  if (first && it == 1) wmode |= SW_ZERO_OLD;  // x_0 = 0 was never stored
  return finish_level(h, m, last, next_m, wmode, X[1 - src], X[src], cur, acc, done, s);
}

// Number of leading schedule entries the coarse tail runs (0: none) and
// the finest of their levels.  They must start at the coarsest level,
// descend one level at a time, fit one workgroup's LDS, not be visited
// again, and hand over to level ms - 1 >= 1 (chained execution, Laplacian,
// damped Jacobi).
int tail_levels(const homg_ctx* h, int* ms) {
  const int np = int(h->sched.size() / 2);
  if (h->temporal != 2 || h->active_smoother != 0 || h->has_coef || np < 3 || h->pow2) return 0;
  if (h->sched[0] != h->top_level) return 0;
  int cnt = 0;
  for (int p = 0; p + 1 < np; ++p) {
    const int m = h->sched[2 * p];
    if (m != h->top_level - p || m < 2) break;
    const int nm = (h->n - 1) / (1 << m) + 1;
    if (coarse_tail_lds(h->prec, h->d, nm, p + 1, top64(h)) > h->lds_limit) break;
    if (h->sched[2 * (p + 1)] != m - 1) {  // the next entry must receive the hand-over
      cnt = p + 1;
      break;
    }
    cnt = p + 1;
  }
  // the last fused level must be followed by level ms - 1
  while (cnt >= 2 && h->sched[2 * cnt] != h->sched[2 * (cnt - 1)] - 1) --cnt;
  if (cnt < 2) return 0;
  *ms = h->sched[2 * (cnt - 1)];
  for (int p = cnt; p < np; ++p)
    if (h->sched[2 * p] > *ms) return 0;  // a fused level is visited again
  // a last coarse level in reduced precision runs whole-grid iterations
  // (its iterate goes into u unrounded) and reads the whole grid, which the
  // tail does not write
  if (cnt + 1 == np && h->prec != PREC_F64) return 0;
  return cnt;
}

// Whether a solve's residual also restricts to level 1 in the same pass
// (2D Laplacian whose schedule visits a coarse level).
bool residual_restricts(const homg_ctx* h) {
  // (an FP64 coarsest level 1 takes its restriction from the separate kernel)
  return h->d == 2 && !h->has_coef && h->top_level >= 1 && h->n >= 5 && !(top64(h) && h->top_level == 1) &&
         !h->pow2;
}

// One restriction of the cycle's pyramid, m -> m + 1 (in FP64 onto an FP64
// coarsest level).
homg_status enqueue_restrict(homg_ctx* h, int m, const int* done, hipStream_t s) {
  if (h->pow2) {  // one restriction per quadrant family
    for (int q = 0; q < 4; ++q)
      LAUNCH_K(h, s, K_RESTRICT, m, 2,
               launch_p2_restrict(m == 0 ? static_cast<const double*>(h->r[0]) : h->fam[4 * m + q],
                                  m == 0 ? h->rl[0] : h->faml[m], m == 0, h->n, q & 1, q >> 1,
                                  h->fam[4 * (m + 1) + q], h->faml[m + 1], done, s));
    return HOMG_OK;
  }
  if (top64(h) && m + 1 == h->top_level) {
    LAUNCH_K(h, s, K_RESTRICT, m, 1,
             launch_restrict_to_f64(h->prec, h->d, h->r[m], h->rl[m], h->r64, h->l64, done, s));
  } else {
    LAUNCH_K(h, s, K_RESTRICT, m, 0,
             launch_restrict(h->prec, h->d, h->r[m], h->rl[m], h->r[m + 1], h->rl[m + 1], done, s));
  }
  return HOMG_OK;
}

// The restriction chain m0 -> m0 + 1 -> ... -> m1 of the pyramid.  Its
// last P steps (2 <= P <= 4 in 2D, P = 2 in 3D, within one workgroup's LDS)
// run as one multi-level launch -- the coarse levels, where each launch
// costs its latency -- and the rest one launch each.  A last step onto an
// FP64 coarsest level keeps its own kernel.  Measured at 4097^2 / 257^3
// (FP64): 2D r_2 -> r_6 in 7.1 us against 18 us for four launches, 3D r_2 ->
// r_4 in 6.8 against 9.6 us; wider tiles (2D five levels, 3D three) or
// blocks of two nodes in 2D were slower (13-32 us, 21 us): the redundant
// halo loads of a deep tile outweigh the launches saved.
constexpr int MR_B2 = 4, MR_B3 = 4;  // owned nodes per axis of the coarsest level
constexpr int MR_P2 = 4, MR_P3 = 2;  // levels per launch at most
homg_status enqueue_restrict_chain(homg_ctx* h, int m0, int m1, const int* done, hipStream_t s) {
  if (m1 <= m0) return HOMG_OK;
  if (h->pow2 || (top64(h) && m1 == h->top_level)) {
    const int last = h->pow2 ? m0 : m1 - 1;  // power-of-two grids: one launch per step
    if (!h->pow2)
      if (homg_status e = enqueue_restrict_chain(h, m0, last, done, s)) return e;
    for (int m = last; m < m1; ++m)
      if (homg_status e = enqueue_restrict(h, m, done, s)) return e;
    return HOMG_OK;
  }
  const int B = h->d == 2 ? MR_B2 : MR_B3;
  int P = 0;
  for (int p = std::min(m1 - m0, h->d == 2 ? MR_P2 : MR_P3); p >= 2 && !P; --p)
    if (restrict_multi_lds(h->prec, h->d, p, B) <= h->lds_limit) P = p;
  for (int m = m0; m < m1 - P; ++m)
    if (homg_status e = enqueue_restrict(h, m, done, s)) return e;
  if (P) {
    const int a = m1 - P;
    void* r[MR_MAX + 1];
    Lay l[MR_MAX + 1];
    for (int k = 0; k <= P; ++k) {
      r[k] = h->r[a + k];
      l[k] = h->rl[a + k];
    }
    LAUNCH_K(h, s, K_RESTRICT, a, 3, launch_restrict_multi(h->prec, h->d, P, B, r, l, done, s));
  }
  return HOMG_OK;
}

// In-cycle restriction (Sec. 2, restrictions done inside the cycle with one
// extra array): before level m runs, make r_m valid -- continue the chain of
// nested restrictions from the last level computed, or restart it from r_0
// when the level lies below the two the array still holds.  The same
// restriction kernels run on the same values, so the result equals the
// pyramid's bit for bit.  No-op for the pyramid.
homg_status prepare_rhs(homg_ctx* h, int m, const int* done, hipStream_t s) {
  if (!h->incycle || m <= 0) return HOMG_OK;
  const bool t64 = top64(h) && m == h->top_level;
  if (t64 && h->rhs_top64) return HOMG_OK;
  const int target = t64 ? m - 1 : m;
  if (target >= 1 && !(target <= h->rhs_ready && target >= h->rhs_ready - 1)) {
    const int from = target > h->rhs_ready ? h->rhs_ready : 0;
    for (int j = from; j < target; ++j)
      if (homg_status e = enqueue_restrict(h, j, done, s)) return e;
    h->rhs_ready = target;
  }
  if (t64) {
    if (homg_status e = enqueue_restrict(h, m - 1, done, s)) return e;
    h->rhs_top64 = true;
  }
  return HOMG_OK;
}

// r_0 = f - A u in the handle's precision with its norm partials (and, see
// residual_restricts, r_1 = R r_0).
homg_status enqueue_residual(homg_ctx* h, const double* f, const double* u, int* count,
                             const int* done, hipStream_t s) {
  h->rhs_ready = residual_restricts(h) ? 1 : 0;
  h->rhs_top64 = false;
  if (residual_restricts(h)) {
    LAUNCH_K(h, s, K_RESIDUAL, 0, 1,
             launch_residual_restrict_2d(h->prec, h->n, u, h->dl, f, h->dl, h->r[0], h->rl[0], h->r[1],
                                         h->rl[1], h->partials, count, done, s));
    return HOMG_OK;
  }
  const Lay none;
  const double* a0 = h->has_coef ? h->a[0] : nullptr;
  LAUNCH_K(h, s, K_RESIDUAL, 0, 0,
           launch_residual(h->prec, h->d, h->n, u, h->dl, f, h->dl, a0, a0 ? h->al[0] : none, h->r[0],
                           h->rl[0], h->partials, count, done, s));
  return HOMG_OK;
}

// Enqueue one MFMG cycle (Sec. 2): restriction pyramid of r_0, the
// schedule's whole-grid iterations with the last one adding e into acc,
// then (if f != null) the new residual and its norm as history[cycle].
homg_status enqueue_cycle(homg_ctx* h, const double* f, double* acc, int cycle, const int* done,
                          hipStream_t s) {
  int ms = 0;
  const int ntail = tail_levels(h, &ms);
  // in a solve (f given) the residual that precedes every cycle already
  // restricted r_0 to level 1
  if (!h->incycle)
    if (homg_status e = enqueue_restrict_chain(h, f && residual_restricts(h) ? 1 : 0, ntail ? ms : h->top_level,
                                               done, s))
      return e;
  if (!f) {  // a step cycle: r_0 was just given, nothing restricted yet
    h->rhs_ready = 0;
    h->rhs_top64 = false;
  }
  if (ntail)
    if (homg_status e = prepare_rhs(h, ms, done, s)) return e;
  int cur = 0;
  const size_t np = h->sched.size() / 2;
  h->chain_ready = -1;
  h->lat_level = -1;
  size_t p0 = 0;
  if (ntail) {
    int its[BATCH_MAX_LEVELS];
    for (int k = 0; k < ntail; ++k) its[k] = h->sched[2 * (ntail - 1 - k) + 1];
    const int nms = (h->n - 1) / (1 << ms) + 1;
    const bool next_last = size_t(ntail) + 1 == np;
    const bool lat = lat_target(h, ms - 1) && !(next_last && h->prec != PREC_F64);
    if (lat || h->d == 3) {
      // the tail leaves level ms's state; level ms - 1's first pass
      // interpolates it, or else (3D) the multi-workgroup hand-over kernel
      // does: the tail's own one-workgroup hand-over to 33^3 took 16 of its
      // 37 us
      LAUNCH_K(h, s, K_TAIL, ms, 1,
               launch_coarse_tail(h->prec, h->d, nms, ntail, its, h->omega, h->r[ms], h->rl[ms], nullptr,
                                  Lay(), done, s, h->xc[2 * ms], h->xc[2 * ms + 1], h->rl[ms], top64(h)));
      if (lat) {
        h->lat.prev = h->xc[2 * ms];
        h->lat.cur = h->xc[2 * ms + 1];
        h->lat.cl = h->rl[ms];
        h->lat.zero_old = false;
        h->lat_level = ms - 1;
      } else {
        LAUNCH_K(h, s, K_TRANSFER, ms - 1, 0,
                 launch_level_transfer(h->prec, h->d, ms, h->xc[2 * ms], h->xc[2 * ms + 1], h->rl[ms], ms - 1,
                                       h->xc[2 * (ms - 1)], h->rl[ms - 1], false, done, s));
        h->chain_ready = ms - 1;
      }
    } else {
      LAUNCH_K(h, s, K_TAIL, ms, 0,
               launch_coarse_tail(h->prec, h->d, nms, ntail, its, h->omega, h->r[ms], h->rl[ms],
                                  h->xc[2 * (ms - 1)], h->rl[ms - 1], done, s, nullptr, nullptr, Lay(),
                                  top64(h)));
      h->chain_ready = ms - 1;
    }
    p0 = size_t(ntail);
  }
  for (size_t p = p0; p < np; ++p) {
    const int m = h->sched[2 * p], it = h->sched[2 * p + 1];
    // the next level, if it starts from a compact x_0 (blocked coarse level)
    int next_m = -1;
    if (p + 1 < np) {
      const int mn = h->sched[2 * (p + 1)];
      const bool next_last = p + 2 == np;
      if (mn == 0)
        next_m = 0;
      else if (h->active_smoother == 1 || !(next_last && h->prec != PREC_F64))
        next_m = mn;
    }
    if (homg_status e = prepare_rhs(h, m, done, s)) return e;
    if (homg_status e = run_level(h, m, it, p == 0, p + 1 == np, next_m, &cur, acc, done, s)) return e;
  }
  if (f) {
    int count = 0;
    if (homg_status e = enqueue_residual(h, f, acc, &count, done, s)) return e;
    LAUNCH_K(h, s, K_FINALIZE, 0, 1, launch_finalize(h->partials, count, h->st, h->hist, cycle, 1, s));
  }
  return HOMG_OK;
}

homg_status check_ready(homg_ctx* h) {
  if (h->stencil == HOMG_DIFFUSION_5PT_2D && !h->has_coef)
    return fail(h, HOMG_ERR_INVALID_ARG, "diffusion stencil needs homg_set_coefficient first");
  return HOMG_OK;
}

homg_status solve_impl(homg_ctx* h, const double* f, double* u, double tol, int fixed_cycles,
                       void* stream, homg_info* info) {
  if (!h) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null handle");
  if (!f || !u) return fail(h, HOMG_ERR_INVALID_ARG, "null f or u");
  const bool stop_on_tol = fixed_cycles < 0;
  if (stop_on_tol && !(tol > 0.0)) return fail(h, HOMG_ERR_INVALID_ARG, "tol must be > 0");
  if (!stop_on_tol && fixed_cycles > h->max_cycles)
    return fail(h, HOMG_ERR_INVALID_ARG, "cycles exceeds max_cycles of the handle");
  if (homg_status c = check_ready(h)) return c;
  DeviceGuard guard(h->device);
  if (!guard.ok) return fail(h, HOMG_ERR_HIP, "cannot select the handle's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long launches0 = h->launches;
  const int* done = &h->st->done;
  h->active_smoother = h->smoother;
  int fell_back = 0;

  LAUNCH(h, launch_init_state(h->st, stop_on_tol ? tol : 0.0, stop_on_tol ? 1 : 0, s));
  int count = 0;
  LAUNCH_K(h, s, K_NORM, 0, 0, launch_norm2(h->d, h->n, f, h->dl, h->partials, &count, s));
  LAUNCH_K(h, s, K_FINALIZE, 0, 0, launch_finalize(h->partials, count, h->st, h->hist, 0, 0, s));
  if (homg_status e = enqueue_residual(h, f, u, &count, done, s)) return e;
  LAUNCH_K(h, s, K_FINALIZE, 0, 1, launch_finalize(h->partials, count, h->st, h->hist, 0, 1, s));

  const int limit = stop_on_tol ? h->max_cycles : fixed_cycles;
  int enqueued = 0, syncs = 0;
  int batch = stop_on_tol ? 2 : limit;
  for (;;) {
    const int upto = std::min(limit, enqueued + std::max(batch, 0));
    for (int c = enqueued + 1; c <= upto; ++c)
      if (homg_status e = enqueue_cycle(h, f, u, c, done, s)) return e;
    enqueued = upto;
    HIPCHK(h, hipMemcpyAsync(h->h_st, h->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(h->h_hist, h->hist, sizeof(double) * (enqueued + 1),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    ++syncs;
    if (h->h_st->done || enqueued >= limit) break;
    const int c = h->h_st->cycles;
    // learned relaxation: fall back to damped Jacobi for the rest of the solve
    // once a cycle contracts the residual by less than fallback_ratio, or --
    // with a Jacobi reference from the gate -- once the geometric-mean
    // contraction over three or more cycles is worse than the reference
    if (h->active_smoother == 1) {
      for (int i = 1; i <= c; ++i)
        if (!(h->h_hist[i] < h->fallback_ratio * h->h_hist[i - 1])) {
          h->active_smoother = 0;
          fell_back = 1;
          break;
        }
      if (h->active_smoother == 1 && h->rho_ref > 0.0 && c >= 3 && h->h_hist[0] > 0.0) {
        const double rho = std::pow(h->h_hist[c] / h->h_hist[0], 1.0 / c);
        if (!(rho <= h->rho_ref)) {
          h->active_smoother = 0;
          fell_back = 1;
        }
      }
    }
    // size the next batch from the observed contraction
    double q = 0.5;
    if (c >= 2 && h->h_hist[c - 1] > 0) q = h->h_hist[c] / h->h_hist[c - 1];
    q = std::min(std::max(q, 1e-3), 0.95);
    const double need = std::log(tol / h->h_hist[c]) / std::log(q);
    batch = int(std::ceil(std::max(1.0, std::min(need, 16.0))));
  }
  // launch times are read once per solve, so timing adds no host work
  // between the batches of cycles
  if (h->prof.on)
    if (homg_status pe = prof_harvest(h)) return pe;
  const int cycles = std::max(h->h_st->cycles, 0);
  const double final_rel = h->h_hist[cycles];
  if (info) {
    info->cycles = cycles;
    info->relres0 = h->h_hist[0];
    info->final_relres = final_rel;
    info->converged = (h->h_st->done == 1) ? 1 : 0;
    if (info->history && info->history_cap > 0) {
      const int nh = std::min(info->history_cap, cycles + 1);
      std::memcpy(info->history, h->h_hist, sizeof(double) * nh);
    }
    info->sweeps = (long long)cycles * h->total_sweeps;
    info->launches = h->launches - launches0;
    info->host_syncs = syncs;
    info->smoother_fell_back = fell_back;
  }
  h->active_smoother = h->smoother;
  if (h->h_st->done == 2) return fail(h, HOMG_ERR_NUMERICAL, "non-finite residual norm");
  if (stop_on_tol && h->h_st->done != 1)
    return fail(h, HOMG_ERR_NOT_CONVERGED, "max_cycles reached above tol");
  return HOMG_OK;
}

}  // namespace

namespace homg {

void ctx_view(const homg_ctx* h, CtxView* v) {
  v->d = h->d;
  v->n = h->n;
  v->levels = h->levels;
  v->stencil = h->stencil;
  v->prec = h->prec;
  v->has_coef = h->has_coef ? 1 : 0;
  v->smoother = h->smoother;
  v->pow2 = h->pow2 ? 1 : 0;
  v->fallback_ratio = h->fallback_ratio;
  v->sched = h->sched;
}

hipError_t ctx_level_coefficient(const homg_ctx* h, int m, double* dense, hipStream_t s) {
  if (!h->has_coef || m < 0 || m >= h->levels) return hipErrorInvalidValue;
  return launch_unpack(PREC_F64, h->d, h->a[m], h->al[m], dense, h->cdl[m], s);
}

}  // namespace homg

extern "C" {

void homg_options_init(homg_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->struct_size = sizeof(homg_options);
  opt->omega = 0.0;
  opt->max_i = 4;
  opt->max_cycles = 200;
  opt->precision = HOMG_FP64;
  opt->temporal_block = 2;
}

homg_status homg_create(homg_handle* out, int ndim, const int64_t* dims, int levels,
                        homg_stencil stencil, const homg_options* opt) {
  if (!out) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (ndim != 2 && ndim != 3) return fail(nullptr, HOMG_ERR_INVALID_ARG, "ndim must be 2 or 3");
  if (!dims) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null dims");
  for (int i = 1; i < ndim; ++i)
    if (dims[i] != dims[0]) return fail(nullptr, HOMG_ERR_UNSUPPORTED, "all sides must be equal");
  const bool pow2 = opt && opt->struct_size == sizeof(homg_options) && opt->grid_layout == HOMG_GRID_POW2;
  if (opt && opt->struct_size == sizeof(homg_options) && opt->grid_layout != HOMG_GRID_NESTED && !pow2)
    return fail(nullptr, HOMG_ERR_INVALID_ARG, "unknown grid_layout");
  int k = side_exponent(dims[0]);
  if (pow2) {
    k = -1;
    if (dims[0] >= 4 && (dims[0] & (dims[0] - 1)) == 0)
      for (k = 0; (int64_t(1) << k) < dims[0]; ++k) {
      }
    if (k < 2) return fail(nullptr, HOMG_ERR_INVALID_ARG, "power-of-two layout: side must be 2^k with k >= 2");
    if (ndim != 2 || stencil != HOMG_LAPLACE_5PT_2D)
      return fail(nullptr, HOMG_ERR_UNSUPPORTED, "power-of-two layout: 2D Laplacian only");
    if (opt->precision != HOMG_FP64)
      return fail(nullptr, HOMG_ERR_UNSUPPORTED, "power-of-two layout: FP64 only");
  }
  if (k < 1) return fail(nullptr, HOMG_ERR_INVALID_ARG, "side must be 2^k + 1 with k >= 1");
  if ((ndim == 2 && k > 15) || (ndim == 3 && k > 10))
    return fail(nullptr, HOMG_ERR_UNSUPPORTED, "grid too large");
  if (levels == 0) levels = k;
  if (levels < 1 || levels > k) return fail(nullptr, HOMG_ERR_INVALID_ARG, "levels must be in [1, k]");
  const bool st_ok = (stencil == HOMG_LAPLACE_5PT_2D && ndim == 2) ||
                     (stencil == HOMG_LAPLACE_7PT_3D && ndim == 3) ||
                     (stencil == HOMG_DIFFUSION_5PT_2D && ndim == 2);
  if (!st_ok) {
    if (stencil == HOMG_LAPLACE_5PT_2D || stencil == HOMG_LAPLACE_7PT_3D || stencil == HOMG_DIFFUSION_5PT_2D)
      return fail(nullptr, HOMG_ERR_UNSUPPORTED, "stencil does not match ndim");
    return fail(nullptr, HOMG_ERR_INVALID_ARG, "unknown stencil");
  }
  homg_options o;
  homg_options_init(&o);
  if (opt) {
    if (opt->struct_size != sizeof(homg_options))
      return fail(nullptr, HOMG_ERR_INVALID_ARG, "homg_options.struct_size mismatch");
    o = *opt;
    for (int i = 0; i < 5; ++i)
      if (o.reserved[i] != 0) return fail(nullptr, HOMG_ERR_INVALID_ARG, "reserved options must be 0");
  }
  double omega = o.omega > 0 ? o.omega : (ndim == 2 ? 4.0 / 5.0 : 6.0 / 7.0);
  if (!(omega > 0.0 && omega <= 1.0)) return fail(nullptr, HOMG_ERR_INVALID_ARG, "omega must be in (0, 1]");
  const int max_i = o.max_i > 0 ? o.max_i : 4;
  const int max_cycles = o.max_cycles > 0 ? o.max_cycles : 200;
  if (max_cycles > 100000) return fail(nullptr, HOMG_ERR_INVALID_ARG, "max_cycles too large");
  if (o.precision < HOMG_FP64 || o.precision > HOMG_BF16_IR)
    return fail(nullptr, HOMG_ERR_INVALID_ARG, "unknown precision");
  if (o.temporal_block < 0 || o.temporal_block > 2)
    return fail(nullptr, HOMG_ERR_INVALID_ARG, "temporal_block must be 0, 1 or 2");
  if (o.restriction != HOMG_RESTRICT_PYRAMID && o.restriction != HOMG_RESTRICT_IN_CYCLE)
    return fail(nullptr, HOMG_ERR_INVALID_ARG, "unknown restriction mode");
  if (o.restriction == HOMG_RESTRICT_IN_CYCLE && pow2)
    return fail(nullptr, HOMG_ERR_UNSUPPORTED, "in-cycle restriction: nested grids only");

  std::vector<int> sched;
  if (o.schedule) {
    if (o.schedule_len < 1 || o.schedule_len > 4096)
      return fail(nullptr, HOMG_ERR_INVALID_ARG, "schedule_len must be in [1, 4096]");
    for (int i = 0; i < o.schedule_len; ++i) {
      const int m = o.schedule[2 * i], it = o.schedule[2 * i + 1];
      if (m < 0 || m >= levels) return fail(nullptr, HOMG_ERR_INVALID_ARG, "schedule level out of range");
      if (it < 1 || it > 1 << 20) return fail(nullptr, HOMG_ERR_INVALID_ARG, "schedule iterations must be >= 1");
      sched.push_back(m);
      sched.push_back(it);
    }
  } else {
    // MFMG (Sec. 2, Fig. 1): two iterations on the coarsest level, doubling
    // per finer level, capped at MaxI.
    const int M = levels - 1;
    for (int m = M; m >= 0; --m) {
      const int64_t want = int64_t(1) << std::min(M - m + 1, 30);
      sched.push_back(m);
      sched.push_back(int(std::min<int64_t>(want, max_i)));
    }
  }

  homg_ctx* h = new (std::nothrow) homg_ctx;
  if (!h) return fail(nullptr, HOMG_ERR_OOM, "host allocation failed");
  h->d = ndim;
  h->n = int(dims[0]);
  h->k = k;
  h->levels = levels;
  h->stencil = stencil;
  h->prec = o.precision;
  h->omega = omega;
  h->max_i = max_i;
  h->max_cycles = max_cycles;
  h->temporal = o.temporal_block;
  h->pow2 = pow2;
  h->incycle = o.restriction == HOMG_RESTRICT_IN_CYCLE;
  h->sched = sched;
  h->top_level = 0;
  h->total_sweeps = 0;
  for (size_t p = 0; p < sched.size(); p += 2) {
    h->top_level = std::max(h->top_level, sched[p]);
    h->total_sweeps += sched[p + 1];
  }
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(nullptr, HOMG_ERR_HIP, "hipGetDevice failed");
  }
  const int eb = prec_bytes(h->prec);
  h->dl = dense_layout(ndim, h->n);
  h->el = padded_layout(ndim, h->n, eb);
  for (int m = 0; m < levels; ++m) {
    const int side = pow2 ? (m == 0 ? h->n : h->n >> m) : (h->n - 1) / (1 << m) + 1;
    h->rl.push_back(padded_layout(ndim, side, eb));
    h->al.push_back(padded_layout(ndim, side, 8));
    h->cdl.push_back(dense_layout(ndim, side));
  }
  homg_status stt = HOMG_OK;
  for (int b = 0; b < 2 && !stt; ++b) stt = dev_alloc(h, &h->e[b], size_t(h->el.alloc) * eb);
  h->r.assign(levels, nullptr);
  const int rown = (pow2 || h->incycle) ? 1 : levels;  // arrays the pyramid owns
  for (int m = 0; m < rown && !stt; ++m) stt = dev_alloc(h, &h->r[m], size_t(h->rl[m].alloc) * eb);
  if (h->incycle) {
    // the one extra array: odd levels in the first half (level 1's size),
    // even levels in the second (level 2's size)
    for (int b = 0; b < 2 && b + 1 < levels && !stt; ++b)
      stt = dev_alloc(h, &h->rbuf[b], size_t(h->rl[b + 1].alloc) * eb);
    for (int m = 1; m < levels && !stt; ++m) h->r[m] = h->rbuf[(m - 1) & 1];
  }
  if (pow2) {
    // four restriction families, levels 1 .. levels-1 (side n >> m)
    h->fam.assign(4 * levels, nullptr);
    h->faml = h->rl;
    for (int m = 1; m < levels && !stt; ++m)
      for (int q = 0; q < 4 && !stt; ++q)
        stt = dev_alloc(h, reinterpret_cast<void**>(&h->fam[4 * m + q]), sizeof(double) * size_t(h->faml[m].alloc));
  }
  if (h->temporal && !pow2) {
    h->xc.assign(2 * levels, nullptr);
    for (int m = 1; m < levels && !stt; ++m)
      for (int b = 0; b < 2 && !stt; ++b)
        stt = dev_alloc(h, &h->xc[2 * m + b], size_t(h->rl[m].alloc) * eb);
    if (h->stencil != HOMG_DIFFUSION_5PT_2D) {
      h->xp3.assign(levels, nullptr);
      for (int m = 1; m < levels && !stt; ++m) {
        const int nm = (h->n - 1) / (1 << m) + 1;
        if (nm >= (ndim == 2 ? 65 : 33))  // lattices that may be too large for one workgroup's LDS
          stt = dev_alloc(h, &h->xp3[m], size_t(h->rl[m].alloc) * eb);
      }
    }
  }
  if (h->prec != PREC_F64 && h->top_level >= 1 && !stt) {
    // FP64 coarsest level of reduced-precision cycles, and the compact pair
    // its rounded state is handed over from (also without level blocking)
    const int mt = h->top_level;
    h->l64 = padded_layout(ndim, (h->n - 1) / (1 << mt) + 1, 8);
    stt = dev_alloc(h, reinterpret_cast<void**>(&h->r64), sizeof(double) * size_t(h->l64.alloc));
    for (int b = 0; b < 2 && !stt; ++b)
      stt = dev_alloc(h, reinterpret_cast<void**>(&h->x64[b]), sizeof(double) * size_t(h->l64.alloc));
    if (h->xc.empty()) h->xc.assign(2 * levels, nullptr);
    for (int b = 0; b < 2 && !stt; ++b)
      if (!h->xc[2 * mt + b]) stt = dev_alloc(h, &h->xc[2 * mt + b], size_t(h->rl[mt].alloc) * eb);
  }
  h->npart = partials_bound(ndim, h->n);
  if (!stt) stt = dev_alloc(h, reinterpret_cast<void**>(&h->partials), sizeof(double) * h->npart);
  if (!stt) stt = dev_alloc(h, reinterpret_cast<void**>(&h->st), sizeof(DevState));
  if (!stt) stt = dev_alloc(h, reinterpret_cast<void**>(&h->hist), sizeof(double) * (max_cycles + 1));
  if (!stt) stt = dev_alloc(h, reinterpret_cast<void**>(&h->zero_flag), sizeof(int) * 64);
  if (stt) {
    std::string msg = h->err;
    free_ctx(h);
    return fail(nullptr, stt, msg);
  }
  bool ok = hipHostMalloc(reinterpret_cast<void**>(&h->h_st), sizeof(DevState), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&h->h_hist), sizeof(double) * (max_cycles + 1), hipHostMallocDefault) == hipSuccess;
  // e's boundary nodes are never written: zero both buffers once.
  ok = ok && hipMemset(h->e[0], 0, size_t(h->el.alloc) * eb) == hipSuccess &&
       hipMemset(h->e[1], 0, size_t(h->el.alloc) * eb) == hipSuccess &&
       hipMemset(h->zero_flag, 0, sizeof(int) * 64) == hipSuccess;
  for (int m = 0; m < rown && ok; ++m)
    if (h->r[m]) ok = hipMemset(h->r[m], 0, size_t(h->rl[m].alloc) * eb) == hipSuccess;
  for (int b = 0; b < 2 && ok; ++b)
    if (h->rbuf[b]) ok = hipMemset(h->rbuf[b], 0, size_t(h->rl[b + 1].alloc) * eb) == hipSuccess;
  for (int m = 1; m < int(h->fam.size()) / 4 && ok; ++m)
    for (int q = 0; q < 4 && ok; ++q)
      ok = hipMemset(h->fam[4 * m + q], 0, sizeof(double) * size_t(h->faml[m].alloc)) == hipSuccess;
  // compact lattices: boundary nodes are read as 0 and never written
  for (size_t m = 1; 2 * m + 1 < h->xc.size() && ok; ++m)
    for (int b = 0; b < 2 && ok; ++b)
      if (h->xc[2 * m + b]) ok = hipMemset(h->xc[2 * m + b], 0, size_t(h->rl[m].alloc) * eb) == hipSuccess;
  if (h->r64) {
    const size_t b64 = sizeof(double) * size_t(h->l64.alloc);
    ok = ok && hipMemset(h->r64, 0, b64) == hipSuccess && hipMemset(h->x64[0], 0, b64) == hipSuccess &&
         hipMemset(h->x64[1], 0, b64) == hipSuccess;
  }
  for (size_t m = 0; m < h->xp3.size() && ok; ++m)
    if (h->xp3[m]) ok = hipMemset(h->xp3[m], 0, size_t(h->rl[m].alloc) * eb) == hipSuccess;
  if (ok) {
    int optin = 0, base = 0;
    (void)hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, h->device);
    (void)hipDeviceGetAttribute(&base, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device);
    h->lds_limit = size_t(std::max(std::max(optin, base), 16384));
  }
  ok = ok && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    free_ctx(h);
    return fail(nullptr, HOMG_ERR_HIP, "workspace initialisation failed");
  }
  *out = h;
  return HOMG_OK;
}

homg_status homg_destroy(homg_handle h) {
  if (!h) return HOMG_OK;
  DeviceGuard guard(h->device);
  (void)hipDeviceSynchronize();
  free_ctx(h);
  return HOMG_OK;
}

homg_status homg_set_coefficient(homg_handle h, const double* a, void* stream) {
  if (!h) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null handle");
  if (!a) return fail(h, HOMG_ERR_INVALID_ARG, "null coefficient");
  if (h->stencil != HOMG_DIFFUSION_5PT_2D)
    return fail(h, HOMG_ERR_INVALID_ARG, "coefficient only applies to the diffusion stencil");
  DeviceGuard guard(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->a.empty()) {
    h->a.assign(h->levels, nullptr);
    for (int m = 0; m < h->levels; ++m)
      if (homg_status e = dev_alloc(h, reinterpret_cast<void**>(&h->a[m]), sizeof(double) * h->al[m].alloc))
        return e;
    for (int m = 0; m < h->levels; ++m)
      HIPCHK(h, hipMemsetAsync(h->a[m], 0, sizeof(double) * h->al[m].alloc, s));
  }
  // level-m lattice coefficients: the nodal values sampled every 2^m nodes
  for (int m = 0; m < h->levels; ++m)
    LAUNCH(h, launch_sample(h->d, a, h->dl, 1 << m, h->a[m], h->al[m], s));
  h->has_coef = true;
  return HOMG_OK;
}

homg_status homg_solve(homg_handle h, const double* f, double* u, double tol, void* stream,
                       homg_info* info) {
  return solve_impl(h, f, u, tol, -1, stream, info);
}

homg_status homg_solve_cycles(homg_handle h, const double* f, double* u, int cycles, void* stream,
                              homg_info* info) {
  if (cycles < 0) return fail(h, HOMG_ERR_INVALID_ARG, "cycles must be >= 0");
  return solve_impl(h, f, u, 1.0, cycles, stream, info);
}

homg_status homg_residual(homg_handle h, const double* f, const double* u, double* r,
                          double* relres_out, void* stream) {
  if (!h) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null handle");
  if (!f || !u) return fail(h, HOMG_ERR_INVALID_ARG, "null f or u");
  if (homg_status c = check_ready(h)) return c;
  DeviceGuard guard(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int count = 0;
  LAUNCH(h, launch_init_state(h->st, 0.0, 0, s));
  LAUNCH(h, launch_norm2(h->d, h->n, f, h->dl, h->partials, &count, s));
  LAUNCH(h, launch_finalize(h->partials, count, h->st, h->hist, 0, 0, s));
  const double* a0 = h->has_coef ? h->a[0] : nullptr;
  const Lay none;
  if (r)
    LAUNCH(h, launch_residual(PREC_F64, h->d, h->n, u, h->dl, f, h->dl, a0, a0 ? h->al[0] : none,
                              r, h->dl, h->partials, &count, h->zero_flag, s));
  else
    LAUNCH(h, launch_residual(h->prec, h->d, h->n, u, h->dl, f, h->dl, a0, a0 ? h->al[0] : none,
                              h->r[0], h->rl[0], h->partials, &count, h->zero_flag, s));
  LAUNCH(h, launch_finalize(h->partials, count, h->st, h->hist, 0, 1, s));
  HIPCHK(h, hipMemcpyAsync(h->h_hist, h->hist, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (relres_out) *relres_out = h->h_hist[0];
  return HOMG_OK;
}

homg_status homg_workspace_bytes(homg_handle h, size_t* bytes) {
  if (!h || !bytes) return fail(h, HOMG_ERR_INVALID_ARG, "null argument");
  *bytes = h->ws_bytes;
  return HOMG_OK;
}

homg_status homg_get_schedule(homg_handle h, int* pairs, int cap, int* len) {
  if (!h || !len) return fail(h, HOMG_ERR_INVALID_ARG, "null argument");
  const int np = int(h->sched.size() / 2);
  *len = np;
  if (pairs) {
    if (cap < np) return fail(h, HOMG_ERR_WORKSPACE, "schedule buffer too small");
    for (int i = 0; i < 2 * np; ++i) pairs[i] = h->sched[i];
  }
  return HOMG_OK;
}

homg_status homg_step_restrict(homg_handle h, int level, const double* r_fine, double* r_coarse,
                               void* stream) {
  if (!h) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null handle");
  if (!r_fine || !r_coarse) return fail(h, HOMG_ERR_INVALID_ARG, "null array");
  if (level < 0 || level >= h->levels - 1) return fail(h, HOMG_ERR_INVALID_ARG, "level out of range");
  if (h->pow2) return fail(h, HOMG_ERR_UNSUPPORTED, "step_restrict: nested grids only");
  DeviceGuard guard(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  h->active_smoother = h->smoother;
  LAUNCH(h, launch_pack(h->prec, h->d, r_fine, h->cdl[level], h->r[level], h->rl[level], s));
  if (top64(h) && level + 1 == h->top_level) {
    LAUNCH(h, launch_restrict_to_f64(h->prec, h->d, h->r[level], h->rl[level], h->r64, h->l64, h->zero_flag, s));
    LAUNCH(h, launch_unpack(PREC_F64, h->d, h->r64, h->l64, r_coarse, h->cdl[level + 1], s));
    return HOMG_OK;
  }
  LAUNCH(h, launch_restrict(h->prec, h->d, h->r[level], h->rl[level], h->r[level + 1], h->rl[level + 1],
                            h->zero_flag, s));
  LAUNCH(h, launch_unpack(h->prec, h->d, h->r[level + 1], h->rl[level + 1], r_coarse, h->cdl[level + 1], s));
  return HOMG_OK;
}

homg_status homg_step_sweeps(homg_handle h, int level, int iters, const double* e_old,
                             const double* r_level, double* e_new, void* stream) {
  if (!h) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null handle");
  if (!e_old || !r_level || !e_new) return fail(h, HOMG_ERR_INVALID_ARG, "null array");
  if (level < 0 || level >= h->levels) return fail(h, HOMG_ERR_INVALID_ARG, "level out of range");
  if (iters < 1) return fail(h, HOMG_ERR_INVALID_ARG, "iters must be >= 1");
  if (h->pow2) return fail(h, HOMG_ERR_UNSUPPORTED, "step_sweeps: nested grids only");
  if (homg_status c = check_ready(h)) return c;
  DeviceGuard guard(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  h->active_smoother = h->smoother;
  LAUNCH(h, launch_pack(h->prec, h->d, e_old, h->dl, h->e[0], h->el, s));
  if (top64(h) && level == h->top_level)
    LAUNCH(h, launch_pack(PREC_F64, h->d, r_level, h->cdl[level], h->r64, h->l64, s));
  else
    LAUNCH(h, launch_pack(h->prec, h->d, r_level, h->cdl[level], h->r[level], h->rl[level], s));
  int cur = 0;
  h->chain_ready = -1;
  h->lat_level = -1;
  if (homg_status e = run_level(h, level, iters, false, false, -1, &cur, nullptr, h->zero_flag, s)) return e;
  LAUNCH(h, launch_unpack(h->prec, h->d, h->e[cur], h->el, e_new, h->dl, s));
  // the solver relies on zero boundaries in both e buffers
  const size_t eb = size_t(prec_bytes(h->prec));
  HIPCHK(h, hipMemsetAsync(h->e[0], 0, size_t(h->el.alloc) * eb, s));
  HIPCHK(h, hipMemsetAsync(h->e[1], 0, size_t(h->el.alloc) * eb, s));
  return HOMG_OK;
}

homg_status homg_step_cycle(homg_handle h, const double* r0, double* acc, void* stream) {
  if (!h) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null handle");
  if (!r0 || !acc) return fail(h, HOMG_ERR_INVALID_ARG, "null array");
  if (homg_status c = check_ready(h)) return c;
  DeviceGuard guard(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  h->active_smoother = h->smoother;
  LAUNCH(h, launch_pack(h->prec, h->d, r0, h->dl, h->r[0], h->rl[0], s));
  return enqueue_cycle(h, nullptr, acc, 1, h->zero_flag, s);
}

homg_status homg_set_profiling(homg_handle h, int enable) {
  if (!h) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null handle");
  DeviceGuard guard(h->device);
  if (homg_status e = prof_harvest(h)) return e;
  h->prof.acc.clear();
  h->prof.on = enable != 0;
  return HOMG_OK;
}

homg_status homg_get_profile(homg_handle h, homg_kernel_time* out, int cap, int* len) {
  if (!h || !len) return fail(h, HOMG_ERR_INVALID_ARG, "null argument");
  DeviceGuard guard(h->device);
  if (homg_status e = prof_harvest(h)) return e;
  *len = int(h->prof.acc.size());
  if (out) {
    if (cap < *len) return fail(h, HOMG_ERR_WORKSPACE, "profile buffer too small");
    int i = 0;
    for (auto& kv : h->prof.acc) {
      out[i].kind = std::get<0>(kv.first);
      out[i].level = std::get<1>(kv.first);
      out[i].mode = std::get<2>(kv.first);
      out[i].reserved = 0;
      out[i].launches = kv.second.first;
      out[i].ms = kv.second.second;
      ++i;
    }
  }
  return HOMG_OK;
}

homg_status homg_set_smoother(homg_handle h, int smoother, const float* w, double fallback_ratio,
                              void* stream) {
  if (!h) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null handle");
  if (smoother != HOMG_SMOOTHER_JACOBI && smoother != HOMG_SMOOTHER_LEARNED)
    return fail(h, HOMG_ERR_INVALID_ARG, "unknown smoother");
  if (smoother == HOMG_SMOOTHER_LEARNED && (h->d != 2 || h->pow2))
    return fail(h, HOMG_ERR_UNSUPPORTED, "the learned smoother is 2D only, on nested grids");
  if (smoother == HOMG_SMOOTHER_LEARNED && !w && !h->w32)
    return fail(h, HOMG_ERR_INVALID_ARG, "the learned smoother needs weights");
  DeviceGuard guard(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (w) {
    if (!h->w32) {
      if (homg_status e = dev_alloc(h, reinterpret_cast<void**>(&h->w32), sizeof(float) * NW)) return e;
      if (homg_status e = dev_alloc(h, reinterpret_cast<void**>(&h->wbf), sizeof(uint16_t) * NW)) return e;
    }
    LAUNCH(h, launch_round_weights(w, h->wbf, h->w32, s));
  }
  if (smoother == HOMG_SMOOTHER_LEARNED && h->xc.empty()) {
    // compact lattice pairs of every coarse level (boundary nodes stay 0)
    const int eb = prec_bytes(h->prec);
    h->xc.assign(2 * h->levels, nullptr);
    for (int m = 1; m < h->levels; ++m)
      for (int b = 0; b < 2; ++b) {
        if (homg_status e = dev_alloc(h, &h->xc[2 * m + b], size_t(h->rl[m].alloc) * eb)) return e;
        HIPCHK(h, hipMemsetAsync(h->xc[2 * m + b], 0, size_t(h->rl[m].alloc) * eb, s));
      }
  }
  h->smoother = smoother;
  h->active_smoother = smoother;
  h->fallback_ratio = fallback_ratio > 0.0 ? fallback_ratio : 1.0;
  return HOMG_OK;
}

homg_status homg_get_smoother_weights(homg_handle h, float* w_out, void* stream) {
  if (!h || !w_out) return fail(h, HOMG_ERR_INVALID_ARG, "null argument");
  if (!h->w32) return fail(h, HOMG_ERR_INVALID_ARG, "no weights set");
  DeviceGuard guard(h->device);
  HIPCHK(h, hipMemcpyAsync(w_out, h->w32, sizeof(float) * NW, hipMemcpyDeviceToDevice,
                           static_cast<hipStream_t>(stream)));
  return HOMG_OK;
}

homg_status homg_smoother_gate(homg_handle h, int count, const double* const* f, int cycles,
                               void* stream, double* rho_learned, double* rho_jacobi,
                               int* accepted) {
  if (!h || !f || count < 1 || cycles < 1 || !accepted)
    return fail(h, HOMG_ERR_INVALID_ARG, "invalid gate arguments");
  if (!h->w32) return fail(h, HOMG_ERR_INVALID_ARG, "no learned weights set");
  if (cycles > h->max_cycles) return fail(h, HOMG_ERR_INVALID_ARG, "cycles exceeds max_cycles");
  DeviceGuard guard(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* u = nullptr;
  const size_t bytes = sizeof(double) * size_t(h->dl.alloc);
  if (homg_status e = dev_alloc(h, reinterpret_cast<void**>(&u), bytes)) return e;
  const int keep = h->smoother;
  const double keep_ratio = h->fallback_ratio;
  homg_status st = HOMG_OK;
  int ok = 1;
  double rho_max = 0.0;  // the Jacobi reference the runtime fallback compares against
  std::vector<double> hist(cycles + 1);
  for (int i = 0; i < count && st == HOMG_OK; ++i) {
    double rho[2] = {0.0, 0.0};
    for (int which = 0; which < 2 && st == HOMG_OK; ++which) {
      h->smoother = which == 0 ? HOMG_SMOOTHER_JACOBI : HOMG_SMOOTHER_LEARNED;
      h->fallback_ratio = 1e300;  // measure the smoother as it is
      if (hipMemsetAsync(u, 0, bytes, s) != hipSuccess) {
        st = fail(h, HOMG_ERR_HIP, "hipMemsetAsync failed");
        break;
      }
      homg_info info{};
      info.history = hist.data();
      info.history_cap = cycles + 1;
      st = solve_impl(h, f[i], u, 1.0, cycles, stream, &info);
      if (st != HOMG_OK) break;
      // geometric mean of the per-cycle contraction
      rho[which] = (hist[0] > 0.0) ? std::pow(hist[cycles] / hist[0], 1.0 / cycles) : 0.0;
    }
    if (st != HOMG_OK) break;
    rho_max = std::max(rho_max, rho[0]);
    if (rho_jacobi) rho_jacobi[i] = rho[0];
    if (rho_learned) rho_learned[i] = rho[1];
    if (!(rho[1] <= rho[0])) ok = 0;
  }
  h->smoother = keep;
  h->active_smoother = keep;
  h->fallback_ratio = keep_ratio;
  (void)hipStreamSynchronize(s);
  (void)hipFree(u);
  h->ws_bytes -= bytes;
  if (st != HOMG_OK) return st;
  *accepted = ok;
  h->rho_ref = rho_max;
  return HOMG_OK;
}

}  // extern "C"

namespace {

// Workspace of the L1 error for up to `slots` results.
homg_status l1_ready(homg_ctx* h, int slots) {
  if (!h->l1part)
    if (homg_status e = dev_alloc(h, reinterpret_cast<void**>(&h->l1part), sizeof(double) * l1_partials())) return e;
  if (h->l1cap < slots) {
    (void)hipFree(h->l1out);
    h->ws_bytes -= sizeof(double) * size_t(h->l1cap);
    h->l1out = nullptr;
    h->l1cap = 0;
    if (homg_status e = dev_alloc(h, reinterpret_cast<void**>(&h->l1out), sizeof(double) * slots)) return e;
    h->l1cap = slots;
  }
  return HOMG_OK;
}

}  // namespace

extern "C" {

homg_status homg_l1_error(homg_handle h, const double* u_ref, const double* v, double* err_out, void* stream) {
  if (!h) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null handle");
  if (!u_ref || !v || !err_out) return fail(h, HOMG_ERR_INVALID_ARG, "null argument");
  DeviceGuard guard(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (homg_status e = l1_ready(h, 1)) return e;
  LAUNCH(h, launch_l1(PREC_F64, h->d, h->n, u_ref, v, nullptr, h->el, h->l1part, h->l1out, s));
  HIPCHK(h, hipMemcpyAsync(err_out, h->l1out, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return HOMG_OK;
}

homg_status homg_trace_cycle(homg_handle h, const double* f, double* u, const double* u_ref, double* err_out,
                             int cap, int* count, void* stream) {
  if (!h) return fail(nullptr, HOMG_ERR_INVALID_ARG, "null handle");
  if (!f || !u || !u_ref || !err_out || !count) return fail(h, HOMG_ERR_INVALID_ARG, "null argument");
  if (h->prec != PREC_F64 || h->smoother != HOMG_SMOOTHER_JACOBI)
    return fail(h, HOMG_ERR_UNSUPPORTED, "the cycle trace runs FP64 damped-Jacobi handles");
  if (cap < h->total_sweeps) return fail(h, HOMG_ERR_WORKSPACE, "err_out holds fewer entries than the cycle's iterations");
  if (homg_status c = check_ready(h)) return c;
  DeviceGuard guard(h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (homg_status e = l1_ready(h, h->total_sweeps)) return e;
  h->active_smoother = 0;
  const int* done = h->zero_flag;
  // r_0 = f - A u and its pyramid, as at the start of a solve's cycle
  int pcount = 0;
  const Lay none;
  const double* a0 = h->has_coef ? h->a[0] : nullptr;
  LAUNCH(h, launch_residual(h->prec, h->d, h->n, u, h->dl, f, h->dl, a0, a0 ? h->al[0] : none, h->r[0], h->rl[0],
                            h->partials, &pcount, done, s));
  h->rhs_ready = 0;
  h->rhs_top64 = false;
  for (int m = 0; !h->incycle && m < h->top_level; ++m)
    if (homg_status e = enqueue_restrict(h, m, done, s)) return e;
  // the schedule one whole-grid iteration at a time (the form in which
  // every iterate exists on the whole grid), the L1 error of u + e after
  // each; the last iteration adds e into u
  const int keep = h->temporal;
  h->temporal = 0;
  h->chain_ready = -1;
  h->lat_level = -1;
  int cur = 0, k = 0;
  homg_status st = HOMG_OK;
  const size_t np = h->sched.size() / 2;
  for (size_t p = 0; p < np && st == HOMG_OK; ++p) {
    const int m = h->sched[2 * p], it = h->sched[2 * p + 1];
    st = prepare_rhs(h, m, done, s);
    for (int t = 0; t < it && st == HOMG_OK; ++t, ++k) {
      const bool first = p == 0 && t == 0, last = p + 1 == np && t + 1 == it;
      st = run_level(h, m, 1, first, last, -1, &cur, u, done, s);
      if (st != HOMG_OK) break;
      hipError_t le = launch_l1(h->prec, h->d, h->n, u_ref, u, last ? nullptr : h->e[cur], h->el, h->l1part,
                                h->l1out + k, s);
      ++h->launches;
      if (le != hipSuccess) st = fail(h, HOMG_ERR_HIP, std::string("launch_l1: ") + hipGetErrorString(le));
    }
  }
  h->temporal = keep;
  if (st != HOMG_OK) return st;
  HIPCHK(h, hipMemcpyAsync(err_out, h->l1out, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  *count = k;
  return HOMG_OK;
}

const char* homg_last_error(homg_handle h) {
  if (h) return h->err.c_str();
  return g_err.c_str();
}

const char* homg_version(void) { return "homg-mi355x 0.1 (gfx950)"; }

}  // extern "C"
