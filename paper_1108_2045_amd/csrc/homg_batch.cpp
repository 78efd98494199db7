// homg_batch.cpp -- batched HOMG solver: C ABI, arena, graph.
//
// Many independent 2D problems of uneven size advance together: every
// problem walks its own MFMG sequence (Sec. 2 of arXiv:1108.2045: residual,
// restriction pyramid, fused relax+interpolate iterations, restart) one
// stage per step, and one launch runs a step for all problems at once (the
// tiles of every active problem's stage, one workgroup each).  A HIP graph
// of 64 step launches and the advance of the step counter is built once
// and replayed on the caller's stream until no problem is active; the
// per-call inputs (array pointers, tolerance) live in device descriptors
// uploaded before each solve, so the graph never changes.  (A persistent
// kernel with a grid barrier per step was measured slower on MI355X: one
// barrier costs 40-170 us against a few us per graph node.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/homg.h"
#include "homg_internal.h"

using namespace homg;

struct homg_batch_ctx {
  int count = 0, prec = 0, max_i = 4, max_cycles = 200;
  double omega = 0.8;
  std::vector<int> sides, levels;
  std::vector<int> sweep_levels;  // concatenated per-problem iteration levels
  std::map<int, int> tile_rows;   // side -> rows per tile (absent: default)
  std::map<int, int> pass_iters;  // side -> iterations per level-0 pass (absent: TB_MAX_IT)
  size_t sched_cap = 0;           // capacity of d_sweep_levels (ints)
  BatchProblem* h_probs = nullptr;
  BatchProblem* d_probs = nullptr;
  BatchRun* h_run = nullptr;
  BatchRun* d_run = nullptr;
  BatchState* h_state = nullptr;
  BatchState* d_state = nullptr;
  int* h_done = nullptr;
  int* d_done = nullptr;
  int* d_sweep_levels = nullptr;
  BatchSync* h_sync = nullptr;
  BatchSync* d_sync = nullptr;
  void* arena = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int grid = 0, device = 0;
  int max_steps = 0;
  std::string err;
};

namespace {

homg_status bfail(homg_batch_ctx* b, homg_status s, const std::string& msg) {
  set_last_error(msg.c_str());
  if (b) b->err = msg;
  return s;
}

#define BHIP(b, call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return bfail(b, HOMG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

int side_k(int64_t n) {
  if (n < 3) return -1;
  int k = 0;
  while ((int64_t(1) << (k + 1)) + 1 <= n) ++k;
  return ((int64_t(1) << k) + 1 == n) ? k : -1;
}

void free_batch(homg_batch_ctx* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  (void)hipFree(b->arena);
  (void)hipFree(b->d_probs);
  (void)hipFree(b->d_run);
  (void)hipFree(b->d_state);
  (void)hipFree(b->d_done);
  (void)hipFree(b->d_sweep_levels);
  (void)hipFree(b->d_sync);
  if (b->h_probs) (void)hipHostFree(b->h_probs);
  if (b->h_run) (void)hipHostFree(b->h_run);
  if (b->h_state) (void)hipHostFree(b->h_state);
  if (b->h_done) (void)hipHostFree(b->h_done);
  if (b->h_sync) (void)hipHostFree(b->h_sync);
  delete b;
}

// Tile rows (the walked length of a tile) of the fine-grid stages.
// The iteration stages of one cycle (levels M .. 0, n_m = min(2^(M-m+1),
// MaxI) iterations each, chained as in the single-problem solver): each
// coarse level's iterations on its compact lattice -- one multi-iteration
// pass (BST_LTB) below the top when the lattice side is at least
// BATCH_LTB_MIN_SIDE and n_m <= TB_MAX_IT, else one stage per iteration --
// and its hand-over to the next finer level's lattice (to the whole grid
// before level 0), then level 0 in passes of up to `depth` (<= TB_MAX_IT)
// iterations, the last adding into u.
std::vector<int> stage_codes(int n, int L, int max_i, int depth) {
  std::vector<int> codes;
  const int M = L - 1;
  auto iters = [&](int m) { return std::min(1 << std::min(M - m + 1, 30), max_i); };
  for (int m = M; m >= 1; --m) {
    const int it = iters(m);
    if (m < M && it <= TB_MAX_IT && (n - 1) / (1 << m) + 1 >= BATCH_LTB_MIN_SIDE) {
      // the level's iterations in one pass, then the hand-over from its outputs
      codes.push_back(bst_code(BST_LTB, m, it, 0, false, false));
      codes.push_back(bst_code(BST_XFER, m, it, 1, false, false));
      continue;
    }
    for (int t = 1; t <= it; ++t) codes.push_back(bst_code(BST_SWEEP, m, 1, t, m == M && t == 1, false));
    codes.push_back(bst_code(BST_XFER, m, it, 0, m == M && it == 1, false));
  }
  const int it0 = iters(0);
  int q = 0;
  for (int t0 = 0; t0 < it0; t0 += depth, ++q) {
    const int g = std::min(depth, it0 - t0);
    codes.push_back(bst_code(BST_L0, 0, g, q, M == 0 && t0 == 0, t0 + g == it0));
  }
  return codes;
}

int rows_for(const homg_batch_ctx* b, int side) {
  auto it = b->tile_rows.find(side);
  if (it != b->tile_rows.end() && it->second > 0) return std::min(it->second, side - 2);
  return default_walk_len(2, side);
}

int depth_for(const homg_batch_ctx* b, int side) {
  auto it = b->pass_iters.find(side);
  return (it != b->pass_iters.end() && it->second > 0) ? std::min(it->second, TB_MAX_IT) : TB_MAX_IT;
}

// Stage table of every problem for the current pass depths (host copy; the
// upload happens in run_once), and the step bound that follows from it.
void build_schedule(homg_batch_ctx* b) {
  b->sweep_levels.clear();
  int max_cycle_len = 0;
  for (int i = 0; i < b->count; ++i) {
    BatchProblem& q = b->h_probs[i];
    const std::vector<int> codes = stage_codes(b->sides[i], b->levels[i], b->max_i, depth_for(b, b->sides[i]));
    q.sched_off = int(b->sweep_levels.size());
    q.sweeps = int(codes.size());
    b->sweep_levels.insert(b->sweep_levels.end(), codes.begin(), codes.end());
    max_cycle_len = std::max(max_cycle_len, q.top + q.sweeps + 2);
  }
  // each problem's tiles per stage of a cycle, filled on the device
  // (launch_batch_tile_table) so that a step looks its tile count up
  for (int i = 0; i < b->count; ++i) {
    BatchProblem& q = b->h_probs[i];
    q.tile_off = int(b->sweep_levels.size());
    b->sweep_levels.insert(b->sweep_levels.end(), size_t(q.top + q.sweeps + 2), 0);
  }
  b->max_steps = 4 + (b->max_cycles + 1) * max_cycle_len;
}

void apply_tiles(homg_batch_ctx* b) {
  for (int i = 0; i < b->count; ++i) b->h_probs[i].len[0] = rows_for(b, b->sides[i]);
  build_schedule(b);
}

homg_status run_once(homg_batch_ctx* b, const double* const* f, double* const* u, double tol,
                     hipStream_t s) {
  for (int i = 0; i < b->count; ++i) {
    if (!f[i] || !u[i]) return bfail(b, HOMG_ERR_INVALID_ARG, "null f or u pointer");
    b->h_probs[i].f = f[i];
    b->h_probs[i].u = u[i];
  }
  *b->h_run = BatchRun{tol, b->omega, b->count, b->max_cycles, b->max_steps, 0};
  if (b->sweep_levels.size() > b->sched_cap)
    return bfail(b, HOMG_ERR_INVALID_ARG, "stage table exceeds its allocation");
  BHIP(b, hipMemcpyAsync(b->d_sweep_levels, b->sweep_levels.data(), sizeof(int) * b->sweep_levels.size(),
                         hipMemcpyHostToDevice, s));
  BHIP(b, hipMemcpyAsync(b->d_probs, b->h_probs, sizeof(BatchProblem) * b->count,
                         hipMemcpyHostToDevice, s));
  BHIP(b, hipMemcpyAsync(b->d_run, b->h_run, sizeof(BatchRun), hipMemcpyHostToDevice, s));
  if (!b->exec) {
    hipGraph_t g = nullptr;
    hipError_t ge = build_batch_graph(b->prec, b->count, b->grid, b->d_probs, b->d_state, b->d_done,
                                      b->d_sweep_levels, b->d_run, b->d_sync, &g);
    if (ge != hipSuccess)
      return bfail(b, HOMG_ERR_HIP, std::string("graph construction failed: ") + hipGetErrorString(ge));
    b->graph = g;
    BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  BHIP(b, launch_batch_tile_table(b->count, b->d_probs, b->d_sweep_levels, s));
  BHIP(b, launch_batch_init(b->count, b->d_state, b->d_done, b->d_sync, s));
  // replays of 64 steps until a step finds no active problem (or the step
  // bound of max_cycles is reached)
  for (int done_steps = 0; done_steps < b->max_steps; done_steps += BATCH_STEPS_PER_REPLAY) {
    BHIP(b, hipGraphLaunch(b->exec, s));
    BHIP(b, hipMemcpyAsync(b->h_sync, b->d_sync, sizeof(BatchSync), hipMemcpyDeviceToHost, s));
    BHIP(b, hipStreamSynchronize(s));
    if (b->h_sync->idle) break;
  }
  BHIP(b, hipMemcpyAsync(b->h_state, b->d_state, sizeof(BatchState) * b->count, hipMemcpyDeviceToHost, s));
  BHIP(b, hipMemcpyAsync(b->h_done, b->d_done, sizeof(int) * b->count, hipMemcpyDeviceToHost, s));
  BHIP(b, hipStreamSynchronize(s));
  return HOMG_OK;
}

}  // namespace

extern "C" {

homg_status homg_batch_create(homg_batch* out, int count, const int64_t* sides, const homg_options* opt) {
  if (!out) return bfail(nullptr, HOMG_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (count < 1 || count > 16000) return bfail(nullptr, HOMG_ERR_INVALID_ARG, "count must be in [1, 16000]");
  if (!sides) return bfail(nullptr, HOMG_ERR_INVALID_ARG, "null sides");
  homg_options o;
  homg_options_init(&o);
  if (opt) {
    if (opt->struct_size != sizeof(homg_options))
      return bfail(nullptr, HOMG_ERR_INVALID_ARG, "homg_options.struct_size mismatch");
    o = *opt;
    if (o.grid_layout != HOMG_GRID_NESTED || o.restriction != HOMG_RESTRICT_PYRAMID)
      return bfail(nullptr, HOMG_ERR_UNSUPPORTED,
                   "the batched solver runs nested grids with the restriction pyramid only");
  }
  for (int i = 0; i < count; ++i) {
    const int k = side_k(sides[i]);
    if (k < 1 || k > 15) return bfail(nullptr, HOMG_ERR_INVALID_ARG, "every side must be 2^k + 1, 1 <= k <= 15");
  }
  const double omega = o.omega > 0 ? o.omega : 0.8;
  if (!(omega > 0.0 && omega <= 1.0)) return bfail(nullptr, HOMG_ERR_INVALID_ARG, "omega must be in (0, 1]");
  if (o.precision < HOMG_FP64 || o.precision > HOMG_BF16_IR)
    return bfail(nullptr, HOMG_ERR_INVALID_ARG, "unknown precision");
  homg_batch_ctx* b = new (std::nothrow) homg_batch_ctx;
  if (!b) return bfail(nullptr, HOMG_ERR_OOM, "host allocation failed");
  b->count = count;
  b->prec = o.precision;
  b->omega = omega;
  b->max_i = o.max_i > 0 ? o.max_i : 4;
  b->max_cycles = o.max_cycles > 0 ? o.max_cycles : 200;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return bfail(nullptr, HOMG_ERR_HIP, "hipGetDevice failed");
  }
  const int eb = prec_bytes(b->prec);
  // arena layout: per problem e0, e1, r_0..r_M (storage type), partials, history
  std::vector<size_t> off;
  size_t total = 0;
  auto take = [&](size_t bytes) {
    const size_t o2 = total;
    total += (bytes + 255) & ~size_t(255);
    return o2;
  };
  struct Plan {
    size_t e[2], r[BATCH_MAX_LEVELS], x[BATCH_MAX_LEVELS][2], x3[BATCH_MAX_LEVELS] = {}, part, hist, r64 = 0,
        x64[2] = {0, 0};
    Lay el, rl[BATCH_MAX_LEVELS], l64;
  };
  std::vector<Plan> plans(count);
  for (int i = 0; i < count; ++i) {
    const int n = int(sides[i]);
    const int L = side_k(n);
    b->sides.push_back(n);
    b->levels.push_back(L);
    Plan& p = plans[i];
    p.el = padded_layout(2, n, eb);
    p.e[0] = take(size_t(p.el.alloc) * eb);
    p.e[1] = take(size_t(p.el.alloc) * eb);
    for (int m = 0; m < L; ++m) {
      p.rl[m] = padded_layout(2, (n - 1) / (1 << m) + 1, eb);
      p.r[m] = take(size_t(p.rl[m].alloc) * eb);
      for (int c = 0; c < 2 && m >= 1; ++c) p.x[m][c] = take(size_t(p.rl[m].alloc) * eb);
      if (m >= 1 && (n - 1) / (1 << m) + 1 >= BATCH_LTB_MIN_SIDE) p.x3[m] = take(size_t(p.rl[m].alloc) * eb);
    }
    if (b->prec != PREC_F64 && L >= 2) {
      // the FP64 coarsest level of reduced-precision cycles
      p.l64 = padded_layout(2, (n - 1) / (1 << (L - 1)) + 1, 8);
      p.r64 = take(sizeof(double) * size_t(p.l64.alloc));
      p.x64[0] = take(sizeof(double) * size_t(p.l64.alloc));
      p.x64[1] = take(sizeof(double) * size_t(p.l64.alloc));
    }
    p.part = take(sizeof(double) * size_t(batch_tiles(n, 1)));
    p.hist = take(sizeof(double) * size_t(b->max_cycles + 1));
    // the stage table is sized for one iteration per level-0 pass, the
    // longest sequence any pass depth gives: the codes and the row of
    // tiles per stage (restrictions, codes, residual, finalize)
    b->sched_cap += 2 * stage_codes(n, L, b->max_i, 1).size() + size_t(L - 1) + 2;
  }
  homg_status st = HOMG_OK;
  if (hipMalloc(&b->arena, total) != hipSuccess) {
    (void)hipGetLastError();
    free_batch(b);
    return bfail(nullptr, HOMG_ERR_OOM, "batch arena allocation of " + std::to_string(total) + " bytes failed");
  }
  bool ok = hipMemset(b->arena, 0, total) == hipSuccess;  // e boundaries stay 0 forever
  ok = ok && hipMalloc(reinterpret_cast<void**>(&b->d_probs), sizeof(BatchProblem) * count) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&b->d_run), sizeof(BatchRun)) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&b->d_state), sizeof(BatchState) * count) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&b->d_done), sizeof(int) * count) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&b->d_sync), sizeof(BatchSync)) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->h_probs), sizeof(BatchProblem) * count, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->h_run), sizeof(BatchRun), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->h_state), sizeof(BatchState) * count, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->h_done), sizeof(int) * count, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->h_sync), sizeof(BatchSync), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_batch(b);
    return bfail(nullptr, HOMG_ERR_OOM, "batch workspace allocation failed");
  }
  char* base = static_cast<char*>(b->arena);
  for (int i = 0; i < count; ++i) {
    BatchProblem& q = b->h_probs[i];
    std::memset(&q, 0, sizeof(q));
    const Plan& p = plans[i];
    const int n = b->sides[i], L = b->levels[i];
    q.e[0] = base + p.e[0] + size_t(p.el.off) * eb;
    q.e[1] = base + p.e[1] + size_t(p.el.off) * eb;
    q.ep = p.el.pitch;
    for (int m = 0; m < L; ++m) {
      q.r[m] = base + p.r[m] + size_t(p.rl[m].off) * eb;
      for (int c = 0; c < 2 && m >= 1; ++c) q.x[m][c] = base + p.x[m][c] + size_t(p.rl[m].off) * eb;
      if (m >= 1 && (n - 1) / (1 << m) + 1 >= BATCH_LTB_MIN_SIDE) q.x3[m] = base + p.x3[m] + size_t(p.rl[m].off) * eb;
      q.rp[m] = p.rl[m].pitch;
      q.len[m] = default_walk_len(2, (n - 1) / (1 << m) + 1);
    }
    if (p.r64 || p.x64[0]) {
      q.r64 = reinterpret_cast<double*>(base + p.r64) + p.l64.off;
      q.x64[0] = reinterpret_cast<double*>(base + p.x64[0]) + p.l64.off;
      q.x64[1] = reinterpret_cast<double*>(base + p.x64[1]) + p.l64.off;
      q.p64 = p.l64.pitch;
    }
    q.partials = reinterpret_cast<double*>(base + p.part);
    q.history = reinterpret_cast<double*>(base + p.hist);
    q.n = n;
    q.levels = L;
    q.top = L - 1;
    q.id = i;
  }
  build_schedule(b);
  if (hipMalloc(reinterpret_cast<void**>(&b->d_sweep_levels), sizeof(int) * b->sched_cap) != hipSuccess ||
      hipMemcpy(b->d_sweep_levels, b->sweep_levels.data(), sizeof(int) * b->sweep_levels.size(),
                hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    free_batch(b);
    return bfail(nullptr, HOMG_ERR_OOM, "schedule table allocation failed");
  }
  int per_cu = 0, cus = 0;
  size_t lds = 0;
  if (batch_occupancy(b->prec, count, &per_cu, &lds) != hipSuccess || per_cu < 1 ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
    (void)hipGetLastError();
    free_batch(b);
    return bfail(nullptr, HOMG_ERR_HIP, "cannot size the step launches");
  }
  // one resident wave of workgroups per step launch; they take the step's
  // tiles round-robin
  b->grid = per_cu * cus;
  (void)st;
  if (hipDeviceSynchronize() != hipSuccess) {
    free_batch(b);
    return bfail(nullptr, HOMG_ERR_HIP, "batch initialisation failed");
  }
  *out = b;
  return HOMG_OK;
}

homg_status homg_batch_destroy(homg_batch b) {
  if (!b) return HOMG_OK;
  (void)hipDeviceSynchronize();
  free_batch(b);
  return HOMG_OK;
}

homg_status homg_batch_set_tile_rows(homg_batch b, int64_t side, int rows) {
  if (!b) return bfail(nullptr, HOMG_ERR_INVALID_ARG, "null batch handle");
  if (rows < 0 || rows > 4096) return bfail(b, HOMG_ERR_INVALID_ARG, "rows must be in [0, 4096]");
  if (rows == 0) b->tile_rows.erase(int(side));
  else b->tile_rows[int(side)] = rows;
  return HOMG_OK;
}

homg_status homg_batch_set_pass_iters(homg_batch b, int64_t side, int iters) {
  if (!b) return bfail(nullptr, HOMG_ERR_INVALID_ARG, "null batch handle");
  if (iters < 0 || iters > TB_MAX_IT) return bfail(b, HOMG_ERR_INVALID_ARG, "iters must be in [0, 4]");
  if (iters == 0) b->pass_iters.erase(int(side));
  else b->pass_iters[int(side)] = iters;
  return HOMG_OK;
}

homg_status homg_batch_solve(homg_batch b, const double* const* f, double* const* u, double tol,
                             void* stream, double* relres_out, int* cycles_out, int* status_out) {
  if (!b) return bfail(nullptr, HOMG_ERR_INVALID_ARG, "null batch handle");
  if (!f || !u) return bfail(b, HOMG_ERR_INVALID_ARG, "null f or u array");
  if (!(tol > 0.0)) return bfail(b, HOMG_ERR_INVALID_ARG, "tol must be > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  apply_tiles(b);
  if (homg_status e = run_once(b, f, u, tol, s)) return e;
  homg_status worst = HOMG_OK;
  for (int i = 0; i < b->count; ++i) {
    const int dn = b->h_done[i];
    homg_status si = dn == 1 ? HOMG_OK : (dn == 2 ? HOMG_ERR_NUMERICAL : HOMG_ERR_NOT_CONVERGED);
    if (relres_out) relres_out[i] = b->h_state[i].final_rel;
    if (cycles_out) cycles_out[i] = b->h_state[i].cycles;
    if (status_out) status_out[i] = si;
    if (si == HOMG_ERR_NUMERICAL) worst = si;
    else if (si != HOMG_OK && worst == HOMG_OK) worst = si;
  }
  if (worst != HOMG_OK) return bfail(b, worst, "some problems did not converge");
  return HOMG_OK;
}

homg_status homg_batch_tune(homg_batch b, const double* const* f, double* const* u, double tol,
                            void* stream, const char* cache_path) {
  if (!b) return bfail(nullptr, HOMG_ERR_INVALID_ARG, "null batch handle");
  if (!f || !u) return bfail(b, HOMG_ERR_INVALID_ARG, "null f or u array");
  if (!(tol > 0.0)) return bfail(b, HOMG_ERR_INVALID_ARG, "tol must be > 0");
  for (int i = 0; i < b->count; ++i)
    if (!f[i] || !u[i]) return bfail(b, HOMG_ERR_INVALID_ARG, "null f or u pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<int> distinct = b->sides;
  std::sort(distinct.begin(), distinct.end());
  distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
  const char* pname = b->prec == PREC_F64 ? "fp64" : (b->prec == PREC_F32 ? "fp32" : "bf16");
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
  char key[128];
  std::snprintf(key, sizeof key, "gfx950/cu%d/%s/maxi%d/rows+iters", cus, pname, b->max_i);
  // cache: lines of the form   <key> <side> <rows> <iterations per level-0 pass>
  if (cache_path) {
    if (FILE* fp = std::fopen(cache_path, "r")) {
      char line[256], k2[128];
      int side = 0, rows = 0, its = 0, hits = 0;
      while (std::fgets(line, sizeof line, fp))
        if (std::sscanf(line, "%127s %d %d %d", k2, &side, &rows, &its) == 4 && std::strcmp(k2, key) == 0 &&
            std::find(distinct.begin(), distinct.end(), side) != distinct.end() && rows > 0 && its > 0 &&
            its <= TB_MAX_IT) {
          b->tile_rows[side] = rows;
          b->pass_iters[side] = its;
          ++hits;
        }
      std::fclose(fp);
      if (hits >= int(distinct.size())) return HOMG_OK;
    }
  }
  // Every candidate starts from the caller's initial guesses: they are saved
  // here and restored (outside the timed region) before each run, and
  // restored once more at the end, so u is left as given.
  std::vector<size_t> uoff(b->count + 1, 0);
  for (int i = 0; i < b->count; ++i) uoff[i + 1] = uoff[i] + size_t(b->sides[i]) * b->sides[i];
  double* saved = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&saved), sizeof(double) * uoff[b->count]) != hipSuccess) {
    (void)hipGetLastError();
    return bfail(b, HOMG_ERR_OOM, "tuner copy of the initial guesses could not be allocated");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  homg_status st = HOMG_OK;
  auto hip_ok = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && st == HOMG_OK) st = bfail(b, HOMG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return st == HOMG_OK;
  };
  auto copy_u = [&](bool save) {
    for (int i = 0; i < b->count && st == HOMG_OK; ++i) {
      const size_t bytes = sizeof(double) * (uoff[i + 1] - uoff[i]);
      hip_ok(save ? hipMemcpyAsync(saved + uoff[i], u[i], bytes, hipMemcpyDeviceToDevice, s)
                  : hipMemcpyAsync(u[i], saved + uoff[i], bytes, hipMemcpyDeviceToDevice, s),
             "hipMemcpyAsync");
    }
  };
  // one run of the current tiles: restore u, time the solve, check that it
  // did work (a run whose problems all meet tol at cycle 0 times nothing)
  auto once = [&](float* ms) {
    copy_u(false);
    apply_tiles(b);
    if (!hip_ok(hipEventRecord(e0, s), "hipEventRecord")) return false;
    if (homg_status e = run_once(b, f, u, tol, s)) {
      st = e;
      return false;
    }
    if (!hip_ok(hipEventRecord(e1, s), "hipEventRecord") || !hip_ok(hipEventSynchronize(e1), "hipEventSynchronize") ||
        !hip_ok(hipEventElapsedTime(ms, e0, e1), "hipEventElapsedTime"))
      return false;
    int most = 0;
    for (int i = 0; i < b->count; ++i) most = std::max(most, b->h_state[i].cycles);
    if (most < 1) {
      st = bfail(b, HOMG_ERR_INVALID_ARG, "the initial guesses already meet tol: no cycle to time");
      return false;
    }
    return true;
  };
  // a candidate's time: the median of three runs
  auto timed = [&](float* ms) {
    float t[3];
    for (int r = 0; r < 3; ++r)
      if (!once(&t[r])) return false;
    std::sort(t, t + 3);
    *ms = t[1];
    return true;
  };
  hip_ok(hipEventCreate(&e0), "hipEventCreate");
  hip_ok(hipEventCreate(&e1), "hipEventCreate");
  copy_u(true);
  float best = 0.f, warm = 0.f;
  bool ok = st == HOMG_OK && once(&warm) && timed(&best);
  // coordinate descent over the sides, largest first: tile rows, then the
  // iterations per level-0 pass
  for (auto it = distinct.rbegin(); ok && it != distinct.rend(); ++it) {
    const int side = *it;
    const int keep = rows_for(b, side);
    int best_rows = keep;
    for (int rows : {4, 8, 16, 32, 64, 128}) {
      if (rows == keep || rows > side - 2) continue;
      b->tile_rows[side] = rows;
      float ms = 0.f;
      if (!(ok = timed(&ms))) break;
      if (ms < best) {
        best = ms;
        best_rows = rows;
      }
    }
    b->tile_rows[side] = best_rows;
    const int keep_it = depth_for(b, side);
    int best_it = keep_it;
    for (int its = 1; ok && its <= TB_MAX_IT; ++its) {
      if (its == keep_it) continue;
      b->pass_iters[side] = its;
      float ms = 0.f;
      if (!(ok = timed(&ms))) break;
      if (ms < best) {
        best = ms;
        best_it = its;
      }
    }
    b->pass_iters[side] = best_it;
  }
  copy_u(false);
  hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(saved);
  if (st != HOMG_OK) return st;
  if (cache_path) {
    if (FILE* fp = std::fopen(cache_path, "a")) {
      for (int side : distinct) std::fprintf(fp, "%s %d %d %d\n", key, side, rows_for(b, side), depth_for(b, side));
      std::fclose(fp);
    }
  }
  return HOMG_OK;
}

}  // extern "C"
