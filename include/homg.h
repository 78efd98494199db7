/*
 * homg.h -- C ABI of the MI355X (gfx950) high occupancy multigrid library.
 *
 * The method is the high occupancy multigrid (HOMG) of Becerra-Sagredo,
 * Malaga and Mandujano, "A novel and scalable multigrid algorithm for
 * many-core architectures" (arXiv:1108.2045).  It solves A u = f (Sec. 2)
 * for the discretised Poisson problem -Laplace u = f (5-point in 2D, 7-point
 * in 3D) or the diffusion problem -div(a grad u) = f, with Dirichlet data on
 * the boundary of the unit square/cube, on nested grids of n = 2^k + 1 nodes
 * per side.  Every iteration is one whole-grid task: the nodes of the
 * current level's lattice relax (damped Jacobi, Sec. 2 level-m relaxation)
 * while every other node interpolates from that lattice (Sec. 2, fused
 * relaxation and interpolation).  Levels follow the modified full multigrid
 * schedule (Sec. 2, Fig. 1) and cycles restart on the residual equation
 * until the requested relative residual (Sec. 2, last paragraph).
 *
 * Conventions shared by every entry point
 *  - Arrays passed in are DEVICE pointers (hipMalloc'd or PyTorch tensors on
 *    the GPU), dense, C order with x fastest: 2D node (j,i) at j*n + i, 3D
 *    node (k,j,i) at (k*n + j)*n + i, boundary nodes included.  The caller
 *    owns them; the library never keeps them after a call returns.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *    of a call is enqueued on it.
 *  - Every call returns a homg_status; nothing aborts and no C++ exception
 *    leaves the library.  Arguments are validated before any device work.
 *    The text of the last error is available from homg_last_error.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef HOMG_H
#define HOMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct homg_ctx *homg_handle;

typedef enum homg_status {
    HOMG_OK = 0,
    HOMG_ERR_INVALID_ARG = 1,   /* bad size, level, pointer, tolerance, option */
    HOMG_ERR_UNSUPPORTED = 2,   /* valid but not implemented combination */
    HOMG_ERR_OOM = 3,           /* device allocation failed */
    HOMG_ERR_WORKSPACE = 4,     /* caller-provided buffer too small */
    HOMG_ERR_HIP = 5,           /* a HIP runtime call failed (text in homg_last_error) */
    HOMG_ERR_NUMERICAL = 6,     /* NaN or Inf in the residual norm */
    HOMG_ERR_NOT_CONVERGED = 7  /* max_cycles reached above tol; u holds the last iterate */
} homg_status;

/* Discrete operator (Sec. 2 and Sec. 4: A from the Poisson equation; the
 * diffusion form -div(a grad) uses the harmonic mean of the nodal
 * coefficient on each face). */
typedef enum homg_stencil {
    HOMG_LAPLACE_5PT_2D = 0,
    HOMG_LAPLACE_7PT_3D = 1,
    HOMG_DIFFUSION_5PT_2D = 2
} homg_stencil;

/* Arithmetic of the sweeps and transfers.  The residual r = f - A u, the
 * update of u and the norms are always FP64 (iterative refinement on the
 * residual restart of Sec. 2). */
typedef enum homg_precision {
    HOMG_FP64 = 0,     /* everything in FP64 */
    HOMG_FP32_IR = 1,  /* sweeps, restriction and stored e, r in FP32 */
    HOMG_BF16_IR = 2   /* stored e, r in BF16 (round to nearest even), FP32 arithmetic */
} homg_precision;

typedef struct homg_options {
    size_t struct_size;    /* sizeof(homg_options); homg_options_init sets it */
    double omega;          /* damped-Jacobi weight; <= 0 selects 4/5 (2D), 6/7 (3D) */
    int max_i;             /* MaxI, the cap on iterations per level; <= 0 selects 4 */
    int max_cycles;        /* cycles per solve; <= 0 selects 200 */
    const int *schedule;   /* optional explicit schedule: schedule_len (level, iterations) pairs,
                              visited in order; NULL selects the MFMG schedule (levels M..0,
                              iterations min(2^(M-m+1), MaxI)) */
    int schedule_len;
    int precision;         /* homg_precision */
    int temporal_block;    /* 2 (default): chained -- the iterations of a coarse level run on its
                              compact lattice, a coarse level followed by another coarse level
                              hands over only that level's lattice values, and the whole grid is
                              written only before level 0 or the last level; for a Laplacian
                              with damped Jacobi, a level followed by the next finer one hands
                              over nothing: the finer level's first pass interpolates the
                              coarser level's lattice values itself (always before level 0; in
                              2D between any two lattices large enough for several workgroups;
                              in 3D after the one-workgroup coarse tail);
                              1: level-blocked -- as 2, but the whole grid is written after every
                              level;
                              0: one whole-grid launch per iteration.
                              With 1 or 2, several iterations of a Laplacian (2D: four, 3D: two)
                              run in one pass at level 0 and on large lattices.  All three give
                              the same results bit for bit. */
    int grid_layout;       /* HOMG_GRID_NESTED (0): n = 2^k + 1 nodes per side, nested level
                              lattices (Sec. 2).  HOMG_GRID_POW2 (1): the power-of-two strategy of
                              Sec. 3 -- 2D Laplacian, FP64, n = 2^k (k >= 2) nodes per side, node
                              (j,i) at (i h, j h) with h = 1/(n-1); four quadrants whose level-m
                              marks are measured from each quadrant's external corner up to the
                              points just outside it (index n/2 or n/2 - 1), every mark relaxing
                              with its quadrant's own restricted residual (one nested restriction
                              sequence per quadrant, anchored at its corner), every other node
                              interpolating bilinearly from its own quadrant's marks only.  Every
                              level-m >= 1 iteration is one whole-grid launch; level 0 runs as on
                              nested grids.  The batched, learned, step-restrict/step-sweeps and
                              variable-coefficient paths are nested-only (HOMG_ERR_UNSUPPORTED). */
    int restriction;       /* HOMG_RESTRICT_PYRAMID (0): every cycle first restricts r_0 to all its
                              levels, one compact array per level (Sec. 2, restrictions as a
                              pre-processing step in independent arrays).
                              HOMG_RESTRICT_IN_CYCLE (1): Sec. 2's memory-saving form -- the
                              restrictions run inside the cycle, before each coarse level, into one
                              extra array (two halves, sized for levels 1 and 2, holding the last
                              two levels of the chain; a level below them restarts the chain from
                              r_0).  Same results bit for bit; nested grids only. */
    int reserved[5];       /* must be 0 */
} homg_options;

enum { HOMG_GRID_NESTED = 0, HOMG_GRID_POW2 = 1 };
enum { HOMG_RESTRICT_PYRAMID = 0, HOMG_RESTRICT_IN_CYCLE = 1 };

typedef struct homg_info {
    int cycles;            /* MFMG cycles executed */
    int converged;         /* 1 if relres <= tol */
    double relres0;        /* relative residual of the initial guess */
    double final_relres;   /* ||f - A u||_2 / ||f||_2 over interior nodes after the last cycle */
    double *history;       /* optional host array: relres after cycles 0..cycles */
    int history_cap;       /* its capacity in doubles */
    long long sweeps;      /* whole-grid iterations executed */
    long long launches;    /* kernel launches enqueued */
    int host_syncs;        /* stream synchronisations to read the residual norm */
    int smoother_fell_back;/* 1 if the learned smoother was replaced by damped Jacobi
                              during this solve (see homg_set_smoother) */
} homg_info;

/* Fill *opt with the defaults and set struct_size. */
void homg_options_init(homg_options *opt);

/*
 * Create a solver for one grid.  ndim in {2,3}; dims[0..ndim-1] all equal to
 * n = 2^k + 1 with k >= 1 (power-of-two layout: n = 2^k, k >= 2); levels in
 * [1, k] (0 selects k, so the coarsest lattice is 3^d with one interior
 * unknown -- one per quadrant in the power-of-two layout); stencil must match ndim.  opt
 * may be NULL (defaults).  Allocates all device workspace on the current
 * device (padded internal copies of e and the residual pyramid); *out is set
 * only on success.
 */
homg_status homg_create(homg_handle *out, int ndim, const int64_t *dims, int levels,
                        homg_stencil stencil, const homg_options *opt);

/* Release the handle and its device memory.  NULL is accepted. */
homg_status homg_destroy(homg_handle h);

/*
 * Nodal coefficient a > 0 (dense n^d FP64 device array) for the diffusion
 * stencil.  Copied into the handle; required before homg_solve for
 * HOMG_DIFFUSION_5PT_2D.
 */
homg_status homg_set_coefficient(homg_handle h, const double *a, void *stream);

/*
 * Solve A u = f to relative residual tol (Sec. 2: MFMG cycles restarted on
 * the residual equation).  f: dense FP64 right-hand side (boundary entries
 * ignored).  u: dense FP64, in = initial guess with the Dirichlet data on the
 * boundary, out = solution; boundary entries are never written.  Returns
 * after the first cycle whose relative residual ||f - A u||_2 / ||f||_2
 * (interior nodes; ||f|| replaced by 1 if f = 0) is <= tol (HOMG_OK), or
 * HOMG_ERR_NOT_CONVERGED after max_cycles, or HOMG_ERR_NUMERICAL on a
 * non-finite norm.  tol must be > 0.  info may be NULL.
 */
homg_status homg_solve(homg_handle h, const double *f, double *u, double tol,
                       void *stream, homg_info *info);

/*
 * Run exactly `cycles` MFMG cycles (no stopping test); otherwise as
 * homg_solve.  Used to compare with a reference at equal cycle counts.
 */
homg_status homg_solve_cycles(homg_handle h, const double *f, double *u, int cycles,
                              void *stream, homg_info *info);

/*
 * Residual r = f - A u in FP64 (Sec. 2, the residual equation).  r may be
 * NULL; otherwise a dense FP64 array whose interior entries receive r (its
 * boundary entries are not written).
 * *relres_out (host) receives ||r||_2 / ||f||_2 over interior nodes.
 * Synchronises the stream.
 */
homg_status homg_residual(homg_handle h, const double *f, const double *u, double *r,
                          double *relres_out, void *stream);

/* Device memory the handle holds (its workspace; the caller's arrays not
 * included), in bytes, to *bytes (host). */
homg_status homg_workspace_bytes(homg_handle h, size_t *bytes);

/* The schedule in use: writes up to cap (level, iterations) pairs into
 * pairs (host) and returns their count in *len. */
homg_status homg_get_schedule(homg_handle h, int *pairs, int cap, int *len);

/*
 * Paper-reproduction support (Sec. 4).
 *
 * homg_l1_error: the normalised L1 error of Sec. 4 in discrete form,
 *   *err_out (host) = sum |u_ref - v| / sum |u_ref| over all n^d nodes of the
 *   dense FP64 device arrays u_ref (e.g. the analytic solution sampled at the
 *   nodes) and v (the approximation); sum |u_ref - v| itself if u_ref = 0.
 *   Fixed summation order; synchronises.
 * homg_trace_cycle: one MFMG cycle (the handle's schedule) on A e = f - A u
 *   from e = 0, run one whole-grid iteration at a time, recording after
 *   iteration k (k = 1 .. sweeps of the cycle) the normalised L1 error of
 *   u + e_k against u_ref in err_out[k-1] (host, cap entries); the last
 *   iteration adds e into u, as a solve's cycle does.  *count receives the
 *   number of iterations.  Each iteration is one work unit (WU) of Sec. 4
 *   (an operation over the entire grid).  FP64 handles with damped Jacobi
 *   only (HOMG_ERR_UNSUPPORTED otherwise); HOMG_ERR_WORKSPACE if cap is
 *   smaller than the cycle's iterations.  Synchronises.
 */
homg_status homg_l1_error(homg_handle h, const double *u_ref, const double *v, double *err_out,
                          void *stream);
homg_status homg_trace_cycle(homg_handle h, const double *f, double *u, const double *u_ref,
                             double *err_out, int cap, int *count, void *stream);

/*
 * Kernel-level entry points (the steps of one cycle, for testing and
 * measurement).  Dense FP64 device arrays in and out; inside, the data are
 * converted to the handle's precision and layout, the same kernels as in
 * homg_solve run, and the result is widened back to FP64.
 *
 * homg_step_restrict: one full-weighting restriction (Sec. 2, restrictions
 *   as weighted averages) from level `level` to level+1.  r_fine has side
 *   (n-1)/2^level + 1, r_coarse side (n-1)/2^(level+1) + 1; 0 <= level < levels-1.
 * homg_step_sweeps: `iters` whole-grid relax+interpolate iterations at level
 *   `level` (Sec. 2, fused task) starting from e_old (side n, boundary
 *   entries 0: the error vanishes on the Dirichlet boundary), with level
 *   right-hand side r_level (side (n-1)/2^level + 1); writes the final iterate
 *   to e_new (side n, boundary 0).  iters >= 1.
 * homg_step_cycle: one MFMG cycle on A e = r0 starting from e = 0; ADDS the
 *   resulting correction e to `acc` (side n, FP64), as the solver adds it to u.
 */
homg_status homg_step_restrict(homg_handle h, int level, const double *r_fine,
                               double *r_coarse, void *stream);
homg_status homg_step_sweeps(homg_handle h, int level, int iters, const double *e_old,
                             const double *r_level, double *e_new, void *stream);
homg_status homg_step_cycle(homg_handle h, const double *r0, double *acc, void *stream);

/*
 * Per-launch device timing (measurement support).  With profiling enabled,
 * every kernel the handle launches is stamped with its own start and end
 * events (recorded by the dispatch on the launch's stream), and the elapsed
 * times are accumulated per kernel class (kind, level, mode) at the end of
 * every solve and by homg_get_profile.  Enabling or disabling clears the
 * accumulated times.
 *   kind: 0 norm of f, 1 residual, 2 norm finalisation, 3 restriction from
 *   `level` to level+1, 4 whole-grid iteration at `level`, 5 sampling of the
 *   grid on the level lattice, 6 iterations on the compact lattice, 7
 *   whole-grid pass of a blocked level, 8 learned relaxation of the level
 *   lattice (level 0: of the whole grid), 9 hand-over of a finished coarse
 *   level to the lattice of `level` (chained execution), 10 the leading
 *   coarse levels down to `level` in one workgroup (chained execution).
 *   mode (kind 1): 1 = the pass also restricts the residual to level 1;
 *   mode (kinds 4, 6, 7, 8): bit 0 = starts from e = 0, bit 1 = adds into u;
 *   bit 2 (kinds 6, 8) = every iteration of the level in one workgroup that
 *   holds the whole lattice; bit 3 (kinds 4, 6) = several iterations in one
 *   temporally blocked pass, bits 4-5 their number minus one, bit 6 (kind
 *   6) = the pass also stores the iterate before its last, bit 7 (kinds 4,
 *   6) = the pass takes its first iterate from the next coarser level's
 *   compact state (chained execution: no hand-over or whole-grid write in
 *   between); mode (kind 10): 1 = the tail leaves its finest level's state
 *   for the next level's first pass instead of handing over.
 * homg_get_profile synchronises outstanding events, then writes up to cap
 * entries and their count in *len.
 */
typedef struct homg_kernel_time {
    int kind;
    int level;
    int mode;
    int reserved;
    long long launches;
    double ms;
} homg_kernel_time;

homg_status homg_set_profiling(homg_handle h, int enable);
homg_status homg_get_profile(homg_handle h, homg_kernel_time *out, int cap, int *len);

/*
 * Batched solver: many independent 2D Poisson problems (5-point, zero
 * Dirichlet) of uneven sides, solved together.  All problems advance in
 * lockstep steps of their own MFMG sequence (Sec. 2), one kernel launch per
 * step for all of them (the launches captured once in a HIP graph of 64
 * steps, replayed until every problem has retired); each retires when its
 * relative residual reaches tol.  Precision, omega, MaxI and max_cycles
 * come from opt (schedule and temporal_block are ignored: the MFMG schedule
 * runs chained -- each coarse level iterates on its compact lattice and
 * hands over only the next finer level's lattice values, the whole grid is
 * written once, before level 0 -- and level 0 runs in multi-iteration
 * passes).
 *
 * homg_batch_create: count >= 1 problems with sides[i] = 2^k + 1, 3 <= side
 *   <= 32769 and at most 16 levels; allocates one device arena for all of
 *   them.  *out set only on success.
 * homg_batch_solve: f[i], u[i] are host arrays of `count` device pointers to
 *   dense FP64 side^2 arrays (u: initial guess in, solution out; boundary
 *   entries never written).  relres_out / cycles_out / status_out (host,
 *   `count` entries each, may be NULL) receive each problem's final relative
 *   residual, cycles and homg_status.  Returns HOMG_OK if every problem
 *   converged, HOMG_ERR_NOT_CONVERGED / HOMG_ERR_NUMERICAL if any did not,
 *   HOMG_ERR_HIP on a runtime failure.  Synchronises the stream.
 * homg_batch_set_tile_rows: rows per tile (the tile shape of the
 *   fine-grid stages) for all problems of side `side`; 0 restores the
 *   default.
 * homg_batch_set_pass_iters: iterations per level-0 pass (1..4; 0 restores
 *   the default 4) for all problems of side `side`.  Every pass depth gives
 *   the same iterates bit for bit; only the traffic and the number of steps
 *   change.
 * homg_batch_tune: picks both by timing candidates on the given inputs:
 *   coordinate descent over the sides, largest first, tile rows in {4, ...,
 *   128} and then pass iterations in {1, ..., 4}, each candidate timed as
 *   the median of three solves.  Every timed solve starts from the caller's
 *   u (a device copy is saved first and restored before each run and at the
 *   end, so u is left as given); HOMG_ERR_INVALID_ARG if a run needs no
 *   cycle at all (every initial guess already meets tol).  The choice is
 *   read from / appended to the text file cache_path (lines "<arch/CUs/
 *   precision/MaxI key> <side> <rows> <iterations>"; NULL: no cache); a
 *   cache that covers every side skips the timing.
 */
typedef struct homg_batch_ctx *homg_batch;

homg_status homg_batch_create(homg_batch *out, int count, const int64_t *sides,
                              const homg_options *opt);
homg_status homg_batch_solve(homg_batch b, const double *const *f, double *const *u, double tol,
                             void *stream, double *relres_out, int *cycles_out, int *status_out);
homg_status homg_batch_set_tile_rows(homg_batch b, int64_t side, int rows);
homg_status homg_batch_set_pass_iters(homg_batch b, int64_t side, int iters);
homg_status homg_batch_tune(homg_batch b, const double *const *f, double *const *u, double tol,
                            void *stream, const char *cache_path);
homg_status homg_batch_destroy(homg_batch b);

/*
 * Learned relaxation (2D stencils).  The paper relaxes the lattice nodes of
 * the fused task with damped Jacobi (Sec. 2, level-m relaxation, the
 * explicit Euler step of the heat equation).  With HOMG_SMOOTHER_LEARNED a
 * small bias-free network replaces it; interpolation, restriction, schedule
 * and restart are unchanged.  On the compact level-m lattice (spacing
 * h_l = 2^m h) at every interior lattice node p:
 *   rho = (h_l^2 r_m(p) - sum_q a_pq (x_p - x_q)) / sum_q a_pq  (a_pq: harmonic mean
 *         of the nodal coefficient across the face to lattice neighbour q; 1 for
 *         the Laplacian; damped Jacobi is x + omega rho),
 *   X = (rho, rho (a_E - a_W)/(a_E + a_W), rho (a_N - a_S)/(a_N + a_S)),
 *   H_c = max(0, sum_ci sum_k W1[c][ci][k] X_ci(p + o_k)), c = 0..15, 0 on the boundary,
 *   x'(p) = x(p) + sum_c sum_k W2[c][k] H_c(p + o_k),
 * with the 3x3 offsets o_k = (dy, dx), k = 3(dy+1) + (dx+1) (a correlation;
 * on the whole grid, taps dilated by 2^m) and values outside the lattice 0.
 * Weights: HOMG_SMOOTHER_WEIGHTS = 576 values, W1[c][ci][k] at 27c + 9ci + k,
 * then W2[c][k] at 432 + 9c + k.  They are stored in BF16 (round to nearest
 * even) and the network computes in FP32.
 *
 * homg_set_smoother: smoother HOMG_SMOOTHER_JACOBI or _LEARNED; w = 576 FP32
 *   values on the DEVICE (NULL keeps the weights already set; required the
 *   first time LEARNED is selected), rounded to BF16 on copy.
 *   fallback_ratio (<= 0 selects 1.0): a solve that sees a cycle whose
 *   relative residual is not below fallback_ratio times the previous one
 *   switches to damped Jacobi for the rest of that solve (checked at each
 *   host synchronisation; info->smoother_fell_back = 1).  After a
 *   homg_smoother_gate call the handle also holds a damped-Jacobi reference
 *   (the worst geometric-mean per-cycle contraction of Jacobi on the gate's
 *   problems): a learned solve whose geometric-mean contraction over three
 *   or more cycles is worse than it falls back too.  HOMG_ERR_UNSUPPORTED
 *   for 3D handles.
 * homg_get_smoother_weights: copies the FP32 values of the BF16 weights (576)
 *   to the device array w_out.
 * homg_smoother_gate: for each of `count` held-out right-hand sides f[i]
 *   (device arrays of the handle's size), runs `cycles` cycles from u = 0 with
 *   damped Jacobi and with the learned weights and reports the geometric-mean
 *   per-cycle contraction (relres_cycles / relres_0)^(1/cycles) of each in
 *   rho_jacobi[i], rho_learned[i] (host arrays, may be NULL); *accepted = 1
 *   iff the learned one is not worse on any problem.  Synchronises.
 */
#define HOMG_SMOOTHER_WEIGHTS 576
enum { HOMG_SMOOTHER_JACOBI = 0, HOMG_SMOOTHER_LEARNED = 1 };

homg_status homg_set_smoother(homg_handle h, int smoother, const float *w, double fallback_ratio,
                              void *stream);
homg_status homg_get_smoother_weights(homg_handle h, float *w_out, void *stream);
homg_status homg_smoother_gate(homg_handle h, int count, const double *const *f, int cycles,
                               void *stream, double *rho_learned, double *rho_jacobi,
                               int *accepted);

/*
 * Training of the learned relaxation on pairs that plain HOMG generates.
 *
 * homg_trainer_add_problem: h is a 2D handle (its coefficient set for the
 *   diffusion stencil); runs `cycles` plain damped-Jacobi HOMG cycles on the
 *   device right-hand side f from u = 0 and records every relaxation input
 *   of every level as a sample: the compact lattice iterate x_t, the level
 *   residual r_m, the lattice coefficient and the error delta = x* - x_t
 *   against the exact level solution x* (A_m x* = h_l^2 r_m, solved by HOMG
 *   to relative residual 1e-12 on a handle of the compact side).  Samples
 *   are stored on the device in FP32.  The handle's smoother is left as it was.
 * homg_trainer_train: Adam (FP32 master weights, moments start at 0) from
 *   the device weights w0 for opt->steps steps; each step draws opt->batch
 *   samples uniformly (splitmix64 from opt->seed), and minimises the mean of
 *   L = E(delta - y)/E(delta), E(v) = v^T A_m v, the energy-norm error left by
 *   one learned relaxation relative to the error before it.  Writes the FP32
 *   values of the trained BF16 weights to the device array w_out and, if
 *   loss_hist (host, opt->steps entries) is given, each step's batch loss.
 * homg_trainer_loss: the mean of L over all samples for device weights w
 *   (used as given, no rounding), to *mean_loss (host).  Synchronises.
 */
typedef struct homg_trainer_ctx *homg_trainer;
typedef struct homg_train_options {
    size_t struct_size;    /* sizeof(homg_train_options) */
    int steps;             /* Adam steps (>= 1) */
    int batch;             /* samples per step (1..256) */
    double lr, beta1, beta2, eps;  /* Adam step size and parameters */
    uint64_t seed;
    int reserved[8];       /* must be 0 */
} homg_train_options;

void homg_train_options_init(homg_train_options *opt);  /* 300 steps, batch 8, lr 1e-3, Adam defaults */
homg_status homg_trainer_create(homg_trainer *out);
homg_status homg_trainer_add_problem(homg_trainer t, homg_handle h, const double *f, int cycles,
                                     void *stream);
homg_status homg_trainer_count(homg_trainer t, int *samples);
homg_status homg_trainer_train(homg_trainer t, const float *w0, const homg_train_options *opt,
                               float *w_out, double *loss_hist, void *stream);
homg_status homg_trainer_loss(homg_trainer t, const float *w, double *mean_loss, void *stream);
homg_status homg_trainer_destroy(homg_trainer t);

/*
 * Kernel-level entry points of the learned relaxation on one compact
 * lattice (testing and measurement).  Dense FP32 device arrays of side
 * nm >= 3 (node (J, I) at J*nm + I); x is the iterate with its boundary
 * entries 0 (they enter the flux of the nodes next to the boundary);
 * boundary entries of r and delta are not read; a = nodal coefficient
 * (NULL: Laplacian); hl = lattice spacing; w = 576 FP32 weights used as given.
 * homg_learn_forward: y (network output, interior nodes; boundary entries
 *   not written).
 * homg_learn_grad: grad (device, 577 doubles) = dL/dw for the sample, then
 *   E(delta - y); *loss (host) = L.  Allocates its own workspace; synchronises.
 * homg_learn_adam: one Adam step (Kingma and Ba) on 576 FP32 master weights
 *   theta with moments m1, m2 (device, updated in place), gradient grad
 *   (device, 576 doubles), 1-based step t; w_out (device, 576) receives the
 *   FP32 values of theta rounded to BF16.  Moments are FP32; the bias
 *   corrections and the update are formed in FP64 and theta is rounded back.
 */
homg_status homg_learn_forward(int nm, double hl, const float *x, const float *r, const float *a,
                               const float *w, float *y, void *stream);
homg_status homg_learn_grad(int nm, double hl, const float *x, const float *r, const float *a,
                            const float *delta, const float *w, double *grad, double *loss,
                            void *stream);
homg_status homg_learn_adam(float *theta, float *m1, float *m2, const double *grad, int t, double lr,
                            double beta1, double beta2, double eps, float *w_out, void *stream);

/*
 * homg_residual without a handle and without any device allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Laplacian of the handle-free
 * grid (5-point for ndim 2, 7-point for ndim 3), side n = 2^k + 1 (2D k <=
 * 15, 3D k <= 10).  f, u, r: dense FP64 device arrays of n^ndim nodes; the
 * interior entries of r (required) receive f - A u, its boundary entries are
 * not written; *relres_out (host, may
 * be NULL) receives ||r||_2 / ||f||_2 over interior nodes (the stream is
 * then synchronised).  Results equal homg_residual's bit for bit.
 * The partial sums live in a static device workspace of
 * HOMG_NOALLOC_MAX_PARTIALS doubles plus 64 bytes (about 1 MiB), which
 * every GPU that runs this call holds until the process ends; a grid that
 * needs more partial sums gets HOMG_ERR_WORKSPACE.  All calls on one GPU
 * share that workspace: calls that overlap on one GPU (different streams or
 * host threads) race; a call clears what it needs before use.
 */
#define HOMG_NOALLOC_MAX_PARTIALS 131072
homg_status homg_residual_noalloc(int ndim, int64_t n, const double *f, const double *u, double *r,
                                  double *relres_out, void *stream);

/* Text of the last error on h (or of the calling thread if h is NULL). */
const char *homg_last_error(homg_handle h);

/* Library version string. */
const char *homg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HOMG_H */
