// homg_internal.h -- declarations shared by the C-ABI driver (homg_capi.cpp)
// and the HIP kernels (homg_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

struct homg_ctx;

namespace homg {

enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };

inline int prec_bytes(int p) { return p == PREC_F64 ? 8 : (p == PREC_F32 ? 4 : 2); }

// Layout of one d-dimensional array of side `side`, in elements.  Node
// (k,j,i) sits at base + off + k*plane + j*pitch + i.  Internal arrays are
// padded so that node (.,.,1) -- the first interior node of every row --
// starts a 128-byte line and every row starts on the same phase; dense
// arrays (the caller's) have off = 0, pitch = side, plane = side*side.
struct Lay {
  int side = 0;
  int64_t off = 0, pitch = 0, plane = 0, alloc = 0;
};

Lay dense_layout(int d, int side);
Lay padded_layout(int d, int side, int elem_bytes);

// Per-solve device state (one per handle).
struct DevState {
  int done;      // 0 running, 1 converged, 2 non-finite norm
  int cycles;    // last cycle whose residual was recorded
  int stop_on_tol;
  int pad;
  double fnorm;  // ||f||_2 over interior nodes (1 if f == 0)
  double tol;
};

enum SweepMode { SW_ZERO_OLD = 1, SW_ACCUM = 2, SW_TBLOCK = 8 };

// Upper bound on the number of per-block partial sums written by the norm /
// residual launches for a grid of side n.
int partials_bound(int d, int n);

// ||f||^2 over interior nodes -> partials; *count receives the number.
hipError_t launch_norm2(int d, int n, const double* f, const Lay& fl, double* partials,
                        int* count, hipStream_t s);
// r0 = f - A u (FP64) stored in the precision `prec`; per-block sums of r^2.
// `a` (nullable) is the nodal coefficient for the diffusion operator, in the
// layout al.
hipError_t launch_residual(int prec, int d, int n, const double* u, const Lay& ul,
                           const double* f, const Lay& fl, const double* a, const Lay& al,
                           void* r0, const Lay& rl, double* partials, int* count,
                           const int* done, hipStream_t s);
// 2D Laplacian (n >= 5): the residual of launch_residual and, in the same
// pass, its full-weighting restriction to level 1 (rc, layout cl of side
// (n-1)/2+1), equal bit for bit to launch_restrict applied to the stored r0.
// Per-wave sums of r^2 (their number in *count).
hipError_t launch_residual_restrict_2d(int prec, int n, const double* u, const Lay& ul,
                                       const double* f, const Lay& fl, void* r0, const Lay& rl,
                                       void* rc, const Lay& cl, double* partials, int* count,
                                       const int* done, hipStream_t s);
// Sums `count` partials in a fixed order.  mode 0: fnorm = sqrt(sum) and
// resets the state; mode 1: history[cycle] = sqrt(sum)/fnorm and updates done.
hipError_t launch_finalize(const double* partials, int count, DevState* st, double* history,
                           int cycle, int mode, hipStream_t s);
hipError_t launch_init_state(DevState* st, double tol, int stop_on_tol, hipStream_t s);
// Normalised L1 error (Sec. 4, discrete): *out (device) = sum |uref - v| /
// sum |uref| over all n^d nodes, v = u + e (e: internal iterate of type
// prec, layout el) or v = u when e is null; uref and u dense FP64.  part:
// l1_partials() doubles of workspace.
int l1_partials();
hipError_t launch_l1(int prec, int d, int n, const double* uref, const double* u, const void* e,
                     const Lay& el, double* part, double* out, hipStream_t s);
// One full-weighting restriction: fine level (side nf) -> coarse (side (nf-1)/2+1).
hipError_t launch_restrict(int prec, int d, const void* rf, const Lay& fl, void* rc,
                           const Lay& cl, const int* done, hipStream_t s);
// P consecutive restrictions r_a -> ... -> r_{a+P} in one launch (r[k],
// l[k]: the array and layout of level a + k, k = 0 .. P): the same bits as
// P launch_restrict calls.  Workgroups own blocks of B nodes per axis of
// level a + P; restrict_multi_lds: the LDS bytes that needs.
constexpr int MR_MAX = 6;
size_t restrict_multi_lds(int prec, int d, int P, int B);
hipError_t launch_restrict_multi(int prec, int d, int P, int B, void* const* r, const Lay* l, const int* done,
                                 hipStream_t s);
// One whole-grid relax+interpolate iteration at level m.  eo/en: fine
// arrays (layout el); rm: compact level-m residual (layout rl); am: compact
// level-m nodal coefficient (FP64, layout al) or null; mode: SweepMode bits;
// with SW_ACCUM the iterate is added to u (FP64, layout ul) instead of
// being stored in en.  compact: a level-0 iteration on the compact lattice
// of a coarse level (same arithmetic, a kernel symbol of its own).
hipError_t launch_sweep(int prec, int d, int n, int m, double omega, const void* eo, void* en,
                        const Lay& el, const void* rm, const Lay& rl, const double* am,
                        const Lay& al, double* u, const Lay& ul, int mode, const int* done,
                        hipStream_t s, bool compact = false);
// Level 0 of a 2D constant-coefficient grid: `it` (<= TB_MAX_IT) iterations
// in one pass (temporal blocking), equal bit for bit to `it` launch_sweep
// calls; reads e (unless zero) and r once, writes en or adds into u once.
// A wave walks a band of `len` rows (0: tb_band's choice).  Short bands
// re-read more halo rows (from L2) but put more waves in flight: tb_band
// returns the longest band (64, 32, 16 or 8 rows) that still gives
// TB_MIN_WAVES waves, else 4 (measured on MI355X, FP64: the pass beats the
// single-iteration kernels from 129^2 up, 1.4-2.8x; on the small lattices
// of a 4097^2 solve, 4-row bands took 10 -> 7.6 us per pass at 257^2).
constexpr int TB_MAX_IT = 4;
constexpr int TB_MIN_WAVES = 4096;
__host__ __device__ inline int tb_waves(int n, int it, int len) {
  const int valid = 64 - 2 * it;
  return ((n - 2 + valid - 1) / valid) * ((n - 2 + len - 1) / len);
}
// Workgroups of a pass: each takes one column tile on four consecutive bands
// (one wave per band), so its four waves write different rows.
__host__ __device__ inline int tb_blocks(int n, int it, int len) {
  const int valid = 64 - 2 * it;
  return ((n - 2 + valid - 1) / valid) * ((n - 2 + 4 * len - 1) / (4 * len));
}
int tb_band(int n, int it);
// A coarse level's final compact state (layout cl, side (n-1)/2+1 for a
// pass over side n): x_it in cur and x_{it-1} in prev (unread when
// zero_old: x_{it-1} = 0).  A pass given one -- level 0 after level 1, or
// the compact lattice of level m after level m + 1, which sits in it the
// same way -- takes its input iterate from it: lattice nodes of the
// coarser level x_it, every other interior node the multilinear
// interpolant of x_{it-1}, exactly as the coarser level's whole-grid write
// (or hand-over) would have stored them, instead of reading eo.
struct L1State {
  const void* prev = nullptr;
  const void* cur = nullptr;
  Lay cl;
  bool zero_old = false;
};
hipError_t launch_sweep_2d_l0_tb(int prec, int n, int it, double omega, const void* eo, void* en,
                                 const Lay& el, const void* rm, const Lay& rl, double* u,
                                 const Lay& ul, bool zero, bool accum, const int* done, hipStream_t s,
                                 int len = 0, const L1State* l1 = nullptr);
// 3D compact lattice of side n (Laplacian, damped Jacobi): it (<= LT_MAX_IT)
// iterations in one launch, blocks of 8^3 owned nodes iterating with a halo
// of `it` nodes in LDS.  x_0: 0 (zero), the compact array xo, or the next
// coarser level's state (l1); x_it into xn and x_{it-1} into xprev (layout
// cl; neither may alias xo).  lattice_3d_tiled_lds: its LDS bytes.
constexpr int LT_MAX_IT = 4;
constexpr int LT_MAX_SIDE = 65;  // the solver uses it on lattices up to this side
size_t lattice_3d_tiled_lds(int prec, int it);
hipError_t launch_lattice_3d_tiled(int prec, int n, int it, double omega, const void* xo, void* xn, void* xprev,
                                   const Lay& cl, const void* rm, const Lay& rl, bool zero, const L1State* l1,
                                   const int* done, hipStream_t s);
// The same on a 2D compact lattice (blocks of 24^2 owned nodes).
constexpr int LT2_MAX_SIDE = 513;  // the solver uses it on lattices up to this side
hipError_t launch_lattice_2d_tiled(int prec, int n, int it, double omega, const void* xo, void* xn, void* xprev,
                                   const Lay& cl, const void* rm, const Lay& rl, bool zero, const L1State* l1,
                                   const int* done, hipStream_t s);
// The same on the compact lattice of a coarse level (side nm): x_it into en
// and, when eprev is not null, x_{it-1} into eprev (layout cl); l1: x_0
// from the next coarser level's state.
hipError_t launch_lattice_2d_tb(int prec, int nm, int it, double omega, const void* eo, void* en,
                                void* eprev, const Lay& cl, const void* rm, const Lay& rl, bool zero,
                                const int* done, hipStream_t s, int len = 0, const L1State* l1 = nullptr);
// 3D (7-point Laplacian) counterpart: `it` (<= TB3_MAX_IT) iterations in one
// pass over the level-0 grid or (compact) a coarse level's lattice of side
// n (layout el for eo, en, eprev; r in rl); accum (level 0 only): add x_it
// into u (dense FP64, ul) instead of storing it; eprev (compact only): also
// store x_{it-1}; l1: the input iterate from the next coarser level's
// state (not with zero).  A block walks
// `len` planes (0: tb3_band's choice: the longest of 32, 16, 8 planes that
// still gives TB3_MIN_BLOCKS blocks, else 4; at 257^3 that is 16 planes in
// 1760 blocks, measured 5% faster per pass than 32 planes in 880 -- 119
// against 126 us for the pass that adds into u -- and at 513^3 level 0
// keeps 32 planes).
constexpr int TB3_MAX_IT = 2;
constexpr int TB3_MIN_BLOCKS = 1536;
int tb3_blocks(int n, int it, int len);
int tb3_band(int n, int it);
hipError_t launch_tb_3d(int prec, int n, int it, double omega, const void* eo, void* en, void* eprev,
                        const Lay& el, const void* rm, const Lay& rl, double* u, const Lay& ul,
                        bool zero, bool accum, bool compact, const int* done, hipStream_t s, int len = 0,
                        const L1State* l1 = nullptr);
// Convert between a dense FP64 array and an internal array of `prec`.
hipError_t launch_pack(int prec, int d, const double* src, const Lay& sl, void* dst,
                       const Lay& dl, hipStream_t s);
hipError_t launch_unpack(int prec, int d, const void* src, const Lay& sl, double* dst,
                         const Lay& dl, hipStream_t s);
// Copy an FP64 array between layouts, sampling every `stride`-th node of the
// source (stride 1: plain copy; stride l: the level-l lattice).
hipError_t launch_sample(int d, const double* src, const Lay& sl, int stride, double* dst,
                         const Lay& dl, hipStream_t s);

// Level-blocked path (same results as one launch per iteration):
// x_0 = the whole grid sampled on the level-l lattice (all compact nodes).
hipError_t launch_gather(int prec, int d, const void* src, const Lay& sl, int l, void* dst,
                         const Lay& dl, const int* done, hipStream_t s);
// LDS bytes the single-workgroup lattice kernel needs for a compact side nm.
size_t lattice_small_lds(int prec, int d, int nm, bool var);
// All `it` iterations of a level on a compact lattice of side nm held by one
// workgroup; x_0 gathered from e (layout el, stride l) unless zero; writes
// x_{it-1} to xprev and x_it to xcur (compact layout cl).
hipError_t launch_lattice_small(int prec, int d, int nm, int l, int it, double omega, bool zero,
                                const void* e, const Lay& el, const void* rm, const Lay& rl,
                                const double* am, const Lay& al, void* xprev, void* xcur,
                                const Lay& cl, const int* done, hipStream_t s);
// Coarse tail (chained execution, Laplacian, damped Jacobi): levels ms ..
// ms + nlev - 1 of a schedule that starts at the coarsest of them and
// descends one level at a time, run by one workgroup in LDS: restriction
// of r_ms (side nms, layout rl) to the coarser levels, its[k] iterations of
// level ms + k, and the hand-over of level ms's final state to the compact
// x_0 of level ms - 1 (dst, layout tl) -- or, given scur, level ms's final
// x_it and x_{it-1} at every node into scur and sprev (layout sl, side nms)
// for a next pass that interpolates them itself.  coarse_tail_lds: its LDS
// bytes.
// top64 (FP32/BF16 cycles): the coarsest level of the tail in FP64 (its
// restriction, iterates and arithmetic), rounded to the storage type only
// for the hand-over.
size_t coarse_tail_lds(int prec, int d, int nms, int nlev, bool top64 = false);
hipError_t launch_coarse_tail(int prec, int d, int nms, int nlev, const int* its, double omega,
                              const void* rms, const Lay& rl, void* dst, const Lay& tl,
                              const int* done, hipStream_t s, void* sprev = nullptr,
                              void* scur = nullptr, const Lay& sl = Lay(), bool top64 = false);
// FP64 coarsest level of a reduced-precision cycle: the restriction to it
// (input in the storage type of prec, widened exactly, FP64 sums and
// output); the exact widening of the level-l lattice of an array in the
// storage type into an FP64 compact array (every node of dl.side); and the
// rounding of an FP64 compact array to the storage type (to FP32, then BF16).
hipError_t launch_restrict_to_f64(int prec, int d, const void* rf, const Lay& fl, double* rc,
                                  const Lay& cl, const int* done, hipStream_t s);
hipError_t launch_widen(int prec, int d, const void* src, const Lay& sl, int l, double* dst,
                        const Lay& dl, const int* done, hipStream_t s);
hipError_t launch_narrow(int prec, int d, const double* src, const Lay& sl, void* dst, const Lay& dl,
                         const int* done, hipStream_t s);
// LDS bytes of the whole-grid pass of level m.
size_t level_write_lds(int prec, int d, int n, int m);
// Whole-grid pass of level m from compact x_{it-1} (xprev) and x_it (xcur):
// mode SW_ZERO_OLD = x_{it-1} is 0, SW_ACCUM = add into u instead of storing.
hipError_t launch_level_write(int prec, int d, int n, int m, const void* xprev, const void* xcur,
                              const Lay& cl, void* en, const Lay& el, double* u, const Lay& ul,
                              int mode, const int* done, hipStream_t s);
// Chained path: the state the level-m write would produce, sampled at the
// interior nodes of the level-mt lattice into that level's compact array
// (layout tl); zero_old: x_{it-1} = 0.
hipError_t launch_level_transfer(int prec, int d, int m, const void* xprev, const void* xcur,
                                 const Lay& cl, int mt, void* dst, const Lay& tl, bool zero_old,
                                 const int* done, hipStream_t s);
// ---- power-of-two grids (Sec. 3; 2D Laplacian, FP64), N = 2^k nodes per side
// Family restriction of quadrant (sx, sy): level 1 from the whole-grid r_0
// (from_r0; F in layout fl of side N, read from that quadrant's corner) or
// level j from level j - 1 (compact, side 2 * cl.side).
hipError_t launch_p2_restrict(const double* F, const Lay& fl, bool from_r0, int N, int sx, int sy, double* C,
                              const Lay& cl, const int* done, hipStream_t s);
// One whole-grid iteration at level m >= 1; fam[q] (q = 2 sy + sx) is the
// level-m family array of quadrant q (layout fl, side N >> m); mode: SW_ZERO_OLD
// / SW_ACCUM (add into u, layout ul, instead of storing en).
hipError_t launch_p2_sweep(int N, int m, double omega, const double* eo, double* en, const Lay& el,
                           const double* const* fam, const Lay& fl, double* u, const Lay& ul, int mode,
                           const int* done, hipStream_t s);

// ---- batched solver (2D, constant coefficient): graph-replayed step launches
constexpr int BATCH_MAX_LEVELS = 16;
// Iteration stages of a batched cycle, one int each in the schedule table:
// kind (bits 0-3), level (4-8), iterations (9-12), index (13-20), zero
// (21: the stage starts from e = 0, or a hand-over of a level whose
// x_{it-1} = 0 was never stored), accum (22: the pass adds into u).
//   BST_SWEEP: iteration `index` (1-based) of coarse level m on its compact
//              lattice (ping-pong x[m][0] -> x[m][1] -> ...);
//   BST_XFER:  hand-over of level m after `iterations` iterations to the
//              compact x_0 of level m - 1 (to the whole grid e[0] if m = 1);
//              index 1: the iterations ran as one BST_LTB pass (x_it in
//              x[m][1], x_{it-1} in x3[m]);
//   BST_L0:    level-0 pass `index` of `iterations` iterations (e[index & 1]
//              -> e[1 - index & 1]);
//   BST_LTB:   all `iterations` (<= TB_MAX_IT) iterations of coarse level m
//              below the top in one multi-iteration pass on its compact
//              lattice: x[m][0] -> x_it in x[m][1], x_{it-1} in x3[m].
enum { BST_SWEEP = 1, BST_XFER = 2, BST_L0 = 3, BST_LTB = 4 };
// Coarse levels whose lattice side is at least this run as one BST_LTB
// pass; smaller lattices keep one step per iteration.
constexpr int BATCH_LTB_MIN_SIDE = 17;
constexpr int BATCH_LTB_LEN = 16;  // band rows of a BST_LTB tile (wave)
__host__ __device__ inline int bst_code(int kind, int level, int count, int index, bool zero, bool accum) {
  return kind | (level << 4) | (count << 9) | (index << 13) | (zero ? 1 << 21 : 0) | (accum ? 1 << 22 : 0);
}
__host__ __device__ inline int bst_kind(int c) { return c & 15; }
__host__ __device__ inline int bst_level(int c) { return (c >> 4) & 31; }
__host__ __device__ inline int bst_count(int c) { return (c >> 9) & 15; }
__host__ __device__ inline int bst_index(int c) { return (c >> 13) & 255; }
__host__ __device__ inline bool bst_zero(int c) { return (c >> 21) & 1; }
__host__ __device__ inline bool bst_accum(int c) { return (c >> 22) & 1; }

struct BatchProblem {         // one problem, read by the step kernels
  const double* f;            // caller arrays, dense side n
  double* u;
  // FP32/BF16 batches: the coarsest level (level top) in FP64 -- its
  // right-hand side and iterate pair, compact, pitch p64; the iterations
  // also store their rounding into x[top] for the hand-over
  double* r64;
  double* x64[2];
  int64_t p64;
  void* e[2];                 // internal e ping-pong, pointer at node (0,0)
  void* r[BATCH_MAX_LEVELS];  // residual pyramid, pointer at node (0,0) of each level
  void* x[BATCH_MAX_LEVELS][2];  // compact iterate pair of each coarse level (layout of r)
  void* x3[BATCH_MAX_LEVELS];    // third compact array: x_{it-1} of a BST_LTB pass
  int64_t ep;                 // pitch of e
  int64_t rp[BATCH_MAX_LEVELS];
  int len[BATCH_MAX_LEVELS];  // rows walked per tile on level-m grids (tile shape)
  double* partials;           // per-tile norm sums
  double* history;            // relres after cycles 0..max_cycles
  int n, levels, top, sweeps; // side, levels, coarsest level visited, iteration stages per cycle
  int sched_off, id;           // offset of the stage codes in the table; problem index
  int tile_off, pad1;          // offset of the tiles-per-stage row (one cycle) in the table
};
struct BatchState {
  int cycles;
  int retired;                // step in which the problem finished (INT32_MAX while active)
  double fnorm;
  double final_rel;
};
struct BatchRun {
  double tol, omega;
  int count, max_cycles, max_steps, pad;
};
// Step counter of a batched solve: step kernel j of a replay runs step
// base + j; the replay's last node advances base.  idle: a step found no
// active problem (every later step returns at once).
struct BatchSync {
  int base, steps, idle, pad;
};
// Workgroups of one step launch; graph nodes (steps) per replay.
constexpr int BATCH_STEPS_PER_REPLAY = 64;
hipError_t batch_occupancy(int prec, int P, int* blocks_per_cu, size_t* lds);
int default_walk_len(int d, int n);
int batch_tiles(int side, int len);
// Reset of the per-solve state (problem states, done flags, step counter).
hipError_t launch_batch_init(int P, BatchState* bs, int* done, BatchSync* sync, hipStream_t s);
// Fill every problem's tiles-per-stage row of the table (stages 4 .. of one
// cycle, at table[tile_off ..]) from its stage codes and tile shapes; run
// after the table and the problems are uploaded, before the steps.
hipError_t launch_batch_tile_table(int P, const BatchProblem* probs, int* table, hipStream_t s);
// Graph of BATCH_STEPS_PER_REPLAY step kernels (steps base .. base + S - 1 of
// every problem's sequence, each tile of a step one workgroup) and the
// advance of base.
hipError_t build_batch_graph(int prec, int P, int grid, const BatchProblem* probs, BatchState* bs,
                             int* done, const int* levels_of_sweep, const BatchRun* run,
                             BatchSync* sync, hipGraph_t* out);

// ---- learned lattice smoother (2D)
constexpr int HID = 16;                 // hidden channels
constexpr int NW1 = HID * 3 * 9;        // first layer: 16 x 3 channels x 3x3 taps
constexpr int NW = NW1 + HID * 9;       // + second layer: 16 x 3x3 taps = 576 weights
constexpr int TRAIN_MAX_ROWS = 1024;    // workgroups (partial-sum rows) of one backward launch
constexpr int ENERGY_MAX_PARTS = 1024;  // workgroups of one energy launch

// One learned relaxation of every interior node of a compact lattice of
// side nm and spacing hl: xo = xi + y.  Layouts: xl for xi/xo, rl for r,
// al for the FP64 nodal coefficient a (null: constant coefficient); mode
// SW_ZERO_OLD (xi = 0, not read) / SW_ACCUM (u += xi + y instead of the store).
// w: the 576 weights as FP32 values.
// Lattices of side <= LEARNED_SMALL_NM: all `it` learned relaxations in one
// workgroup (x_0 from e with stride l, or 0 when zero); writes x_{it-1} to
// xprev and x_it to xcur.
constexpr int LEARNED_SMALL_NM = 16;
hipError_t launch_learned_small(int prec, int nm, int l, int it, double hl, bool zero, const void* e,
                                const Lay& el, const void* r, const Lay& rl, const double* a,
                                const Lay& al, void* xprev, void* xcur, const Lay& cl,
                                const float* w, const int* done, hipStream_t s);
hipError_t launch_learned_iter(int prec, int nm, double hl, const void* xi, const Lay& xl,
                               void* xo, const void* r, const Lay& rl, const double* a,
                               const Lay& al, double* u, const Lay& ul, const float* w, int mode,
                               const int* done, hipStream_t s);
// Training on dense FP32 compact arrays of side nm.  fwd: z = delta - y (y if
// delta is null).  bwd: per-workgroup partial sums of dL/dw (576) and E(z)
// into part[j * pstride + row], rows = train_bwd_rows(nm); e0 = &E(delta).
hipError_t launch_train_fwd(int nm, float hl2, const float* x, const float* r, const float* a,
                            const float* delta, float* z, const float* w, hipStream_t s);
int train_bwd_rows(int nm);
hipError_t launch_train_bwd(int nm, float hl2, const float* x, const float* r, const float* a,
                            const float* z, const double* e0, const float* w, float* part,
                            int64_t pstride, hipStream_t s);
// out[j] = sum of part[j][0..rows) (FP64, fixed order), j = 0..NW.
hipError_t launch_train_reduce(const float* part, int64_t pstride, int rows, double* out,
                               hipStream_t s);
hipError_t launch_train_adam(const double* sums, int batch, const double* e0s, const int* idx,
                             float* theta, float* m1, float* m2, uint16_t* wbf, float* w32,
                             int step, double lr, double beta1, double beta2, double eps,
                             double* loss, hipStream_t s);
// *out = E(v) = v^T A v over interior nodes (part: ENERGY_MAX_PARTS doubles).
hipError_t launch_energy(const float* v, const float* a, int nm, double* part, double* out,
                         hipStream_t s);
hipError_t launch_round_weights(const float* src, uint16_t* wbf, float* w32, hipStream_t s);
// dst (dense FP32, side nm) = src on the l-lattice, or sub - src when sub != null.
hipError_t launch_lattice_f32(const double* src, int64_t sp, int l, const double* sub, int64_t bp,
                              int nm, float* dst, hipStream_t s);

hipError_t launch_add_dense(double* v, const double* e, int64_t count, hipStream_t s);

// What the trainer needs to know about a solver handle.
struct CtxView {
  int d = 0, n = 0, levels = 0, stencil = 0, prec = 0, has_coef = 0, smoother = 0, pow2 = 0;
  double fallback_ratio = 1.0;
  std::vector<int> sched;  // (level, iterations) pairs
};
void ctx_view(const homg_ctx* h, CtxView* v);
// The handle's level-m nodal coefficient as a dense FP64 array (side (n-1)/2^m + 1).
hipError_t ctx_level_coefficient(const homg_ctx* h, int m, double* dense, hipStream_t s);

// Record the text of the calling thread's last error (homg_last_error(NULL)).
void set_last_error(const char* msg);

// Start/stop events stamped on the next launch of this thread (null: none).
void set_launch_events(hipEvent_t start, hipEvent_t stop);
void current_launch_events(hipEvent_t* start, hipEvent_t* stop);

}  // namespace homg
