// homg_internal.h -- declarations shared by the C-ABI driver (homg_capi.cpp)
// and the HIP kernels (homg_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

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

enum SweepMode { SW_ZERO_OLD = 1, SW_ACCUM = 2 };

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
// Sums `count` partials in a fixed order.  mode 0: fnorm = sqrt(sum) and
// resets the state; mode 1: history[cycle] = sqrt(sum)/fnorm and updates done.
hipError_t launch_finalize(const double* partials, int count, DevState* st, double* history,
                           int cycle, int mode, hipStream_t s);
hipError_t launch_init_state(DevState* st, double tol, int stop_on_tol, hipStream_t s);
// One full-weighting restriction: fine level (side nf) -> coarse (side (nf-1)/2+1).
hipError_t launch_restrict(int prec, int d, const void* rf, const Lay& fl, void* rc,
                           const Lay& cl, const int* done, hipStream_t s);
// One whole-grid relax+interpolate iteration at level m.  eo/en: fine
// arrays (layout el); rm: compact level-m residual (layout rl); am: compact
// level-m nodal coefficient (FP64, layout al) or null; mode: SweepMode bits;
// with SW_ACCUM the iterate is added to u (FP64, layout ul) instead of
// being stored in en.
hipError_t launch_sweep(int prec, int d, int n, int m, double omega, const void* eo, void* en,
                        const Lay& el, const void* rm, const Lay& rl, const double* am,
                        const Lay& al, double* u, const Lay& ul, int mode, const int* done,
                        hipStream_t s);
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
// LDS bytes of the whole-grid pass of level m.
size_t level_write_lds(int prec, int d, int n, int m);
// Whole-grid pass of level m from compact x_{it-1} (xprev) and x_it (xcur):
// mode SW_ZERO_OLD = x_{it-1} is 0, SW_ACCUM = add into u instead of storing.
hipError_t launch_level_write(int prec, int d, int n, int m, const void* xprev, const void* xcur,
                              const Lay& cl, void* en, const Lay& el, double* u, const Lay& ul,
                              int mode, const int* done, hipStream_t s);
// ---- batched persistent solver (2D, constant coefficient)
constexpr int BATCH_MAX_LEVELS = 16;
struct BatchProblem {         // one problem, read by the persistent kernel
  const double* f;            // caller arrays, dense side n
  double* u;
  void* e[2];                 // internal e ping-pong, pointer at node (0,0)
  void* r[BATCH_MAX_LEVELS];  // residual pyramid, pointer at node (0,0) of each level
  int64_t ep;                 // pitch of e
  int64_t rp[BATCH_MAX_LEVELS];
  int len[BATCH_MAX_LEVELS];  // rows walked per tile on level-m grids (tile shape)
  double* partials;           // per-tile norm sums
  double* history;            // relres after cycles 0..max_cycles
  int n, levels, top, sweeps; // side, levels, coarsest level visited, iterations per cycle
  int sched_off, id, pad0, pad1;
};
struct BatchState {
  int cycles;
  int pad;
  double fnorm;
  double final_rel;
};
struct BatchRun {
  double tol, omega;
  int count, max_cycles, max_steps, pad;
  uint64_t barrier_ticks;     // wall-clock limit of one barrier wait (100 MHz ticks)
};
struct BatchSync {
  unsigned count, gen;
  int abort, steps;
};
hipError_t batch_occupancy(int prec, int P, int* blocks_per_cu, size_t* lds);
int default_walk_len(int d, int n);
int batch_tiles(int side, int len);
hipError_t launch_batch(int prec, int P, int grid, const BatchProblem* probs, BatchState* bs, int* done,
                        const int* levels_of_sweep, const BatchRun* run, BatchSync* sync,
                        hipStream_t s);

// Record the text of the calling thread's last error (homg_last_error(NULL)).
void set_last_error(const char* msg);

// Start/stop events stamped on the next launch of this thread (null: none).
void set_launch_events(hipEvent_t start, hipEvent_t stop);

}  // namespace homg
