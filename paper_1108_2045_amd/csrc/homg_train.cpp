// homg_train.cpp -- training of the learned lattice relaxation: C ABI.
//
// Samples come from plain HOMG (damped-Jacobi relaxation, Sec. 2 of
// arXiv:1108.2045): for every relaxation of every level of a cycle on the
// residual equation, the compact lattice iterate x_t that the relaxation
// reads, the level's restricted residual r_m, the lattice coefficient and
// the error delta = x* - x_t against the exact solution of the level system
// (itself solved by HOMG).  Training minimises the energy-norm error left by
// one learned relaxation, E(delta - y)/E(delta), with Adam on FP32 master
// weights; the forward, backward, reduction and optimiser steps are HIP
// kernels (homg_learned.hip), enqueued from here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/homg.h"
#include "homg_internal.h"

using namespace homg;

namespace {

struct Sample {
  const float* x;      // compact iterate (FP32, dense side nm)
  const float* delta;  // x* - x
  const float* r;      // level residual
  const float* a;      // lattice coefficient (null: Laplacian)
  int nm;
  float hl2;
};

}  // namespace

struct homg_trainer_ctx {
  std::vector<void*> blocks;   // device allocations holding the samples
  std::vector<Sample> samples;
  std::vector<double> e0;      // E(delta) per sample
  int max_nm = 0;
  std::string err;
};

namespace {

homg_status tfail(homg_trainer_ctx* t, homg_status s, const std::string& msg) {
  set_last_error(msg.c_str());
  if (t) t->err = msg;
  return s;
}

#define TCHK(t, call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return tfail(t, HOMG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

// Device buffers released at scope exit.
struct DevBufs {
  std::vector<void*> p;
  ~DevBufs() {
    for (void* q : p) (void)hipFree(q);
  }
  template <typename T>
  hipError_t alloc(T** out, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1));
    if (e != hipSuccess) {
      *out = nullptr;
      return e;
    }
    p.push_back(q);
    *out = static_cast<T*>(q);
    return hipSuccess;
  }
};

// Handles of the compact level systems, released at scope exit.
struct Handles {
  std::vector<homg_handle> h;
  ~Handles() {
    for (homg_handle q : h) (void)homg_destroy(q);
  }
};

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

void homg_train_options_init(homg_train_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->struct_size = sizeof(homg_train_options);
  opt->steps = 300;
  opt->batch = 8;
  opt->lr = 1e-3;
  opt->beta1 = 0.9;
  opt->beta2 = 0.999;
  opt->eps = 1e-8;
  opt->seed = 0;
}

homg_status homg_trainer_create(homg_trainer* out) {
  if (!out) return tfail(nullptr, HOMG_ERR_INVALID_ARG, "null output");
  *out = new (std::nothrow) homg_trainer_ctx;
  if (!*out) return tfail(nullptr, HOMG_ERR_OOM, "host allocation failed");
  return HOMG_OK;
}

homg_status homg_trainer_destroy(homg_trainer t) {
  if (!t) return HOMG_OK;
  (void)hipDeviceSynchronize();
  for (void* p : t->blocks) (void)hipFree(p);
  delete t;
  return HOMG_OK;
}

homg_status homg_trainer_count(homg_trainer t, int* samples) {
  if (!t || !samples) return tfail(t, HOMG_ERR_INVALID_ARG, "null argument");
  *samples = int(t->samples.size());
  return HOMG_OK;
}

homg_status homg_trainer_add_problem(homg_trainer t, homg_handle h, const double* f, int cycles,
                                     void* stream) {
  if (!t || !h || !f) return tfail(t, HOMG_ERR_INVALID_ARG, "null argument");
  if (cycles < 1 || cycles > 64) return tfail(t, HOMG_ERR_INVALID_ARG, "cycles must be in [1, 64]");
  CtxView v;
  ctx_view(h, &v);
  if (v.d != 2 || v.pow2) return tfail(t, HOMG_ERR_UNSUPPORTED, "training needs a 2D handle on a nested grid");
  const bool var = v.stencil == HOMG_DIFFUSION_5PT_2D;
  if (var && !v.has_coef) return tfail(t, HOMG_ERR_INVALID_ARG, "set the coefficient first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = v.n, L = v.levels;
  const size_t nn = size_t(n) * n;
  auto side = [&](int m) { return (n - 1) / (1 << m) + 1; };

  DevBufs tmp;
  double *u = nullptr, *e[2] = {nullptr, nullptr}, *part = nullptr;
  std::vector<double*> rm(L, nullptr), xs(L, nullptr), am(L, nullptr);
  std::vector<float*> af(L, nullptr);
  TCHK(t, tmp.alloc(&u, nn));
  TCHK(t, tmp.alloc(&e[0], nn));
  TCHK(t, tmp.alloc(&e[1], nn));
  TCHK(t, tmp.alloc(&part, ENERGY_MAX_PARTS));
  for (int m = 0; m < L; ++m) {
    const size_t c = size_t(side(m)) * side(m);
    TCHK(t, tmp.alloc(&rm[m], c));
    TCHK(t, tmp.alloc(&xs[m], c));
    if (var) {
      TCHK(t, tmp.alloc(&am[m], c));
      TCHK(t, tmp.alloc(&af[m], c));
    }
  }
  double* e0dev = nullptr;
  int nsamp = 0;
  for (size_t p = 0; p < v.sched.size(); p += 2) nsamp += v.sched[p + 1];
  nsamp *= cycles;
  TCHK(t, tmp.alloc(&e0dev, size_t(nsamp)));

  // exact solvers of the compact level systems (spacing h_l = 1/(side-1))
  Handles lh;
  lh.h.assign(L, nullptr);
  std::vector<bool> used(L, false);
  for (size_t p = 0; p < v.sched.size(); p += 2) used[v.sched[p]] = true;
  for (int m = 0; m < L; ++m) {
    if (!used[m]) continue;
    homg_options o;
    homg_options_init(&o);
    o.max_cycles = 400;
    const int64_t dims[2] = {side(m), side(m)};
    if (homg_status st = homg_create(&lh.h[m], 2, dims, 0, var ? HOMG_DIFFUSION_5PT_2D : HOMG_LAPLACE_5PT_2D, &o))
      return tfail(t, st, std::string("level solver: ") + homg_last_error(nullptr));
    if (var) {
      TCHK(t, ctx_level_coefficient(h, m, am[m], s));
      if (homg_status st = homg_set_coefficient(lh.h[m], am[m], stream)) return tfail(t, st, homg_last_error(lh.h[m]));
      TCHK(t, launch_lattice_f32(am[m], side(m), 1, nullptr, 0, side(m), af[m], s));
    }
  }
  // plain HOMG generates the pairs
  const int keep = v.smoother;
  if (keep != HOMG_SMOOTHER_JACOBI)
    if (homg_status st = homg_set_smoother(h, HOMG_SMOOTHER_JACOBI, nullptr, 0.0, stream)) return tfail(t, st, homg_last_error(h));
  struct Restore {
    homg_handle h;
    int keep;
    double ratio;
    void* s;
    ~Restore() {
      if (keep != HOMG_SMOOTHER_JACOBI) (void)homg_set_smoother(h, keep, nullptr, ratio, s);
    }
  } restore{h, keep, v.fallback_ratio, stream};

  TCHK(t, hipMemsetAsync(u, 0, sizeof(double) * nn, s));
  // sample storage of this call: handed to the trainer on success, else freed
  struct Pending {
    std::vector<void*> p;
    hipStream_t s;
    bool keep = false;
    ~Pending() {
      if (keep) return;
      (void)hipStreamSynchronize(s);
      for (void* q : p) (void)hipFree(q);
    }
  } pending{{}, s};
  std::vector<void*>& new_blocks = pending.p;
  std::vector<Sample> new_samples;
  int k = 0;
  for (int c = 0; c < cycles; ++c) {
    double rel = 0.0;
    homg_status st = homg_residual(h, f, u, rm[0], &rel, stream);
    for (int m = 0; m + 1 < L && st == HOMG_OK; ++m) st = homg_step_restrict(h, m, rm[m], rm[m + 1], stream);
    for (int m = 0; m < L && st == HOMG_OK; ++m) {
      if (!used[m]) continue;
      TCHK(t, hipMemsetAsync(xs[m], 0, sizeof(double) * side(m) * side(m), s));
      st = homg_solve(lh.h[m], rm[m], xs[m], 1e-11, stream, nullptr);
      if (st == HOMG_ERR_NOT_CONVERGED) st = HOMG_OK;  // FP64 floor of a large level: keep the best iterate
    }
    if (st != HOMG_OK) return tfail(t, st, std::string("pair generation: ") + homg_last_error(nullptr));
    TCHK(t, hipMemsetAsync(e[0], 0, sizeof(double) * nn, s));
    TCHK(t, hipMemsetAsync(e[1], 0, sizeof(double) * nn, s));
    int cur = 0;
    for (size_t p = 0; p < v.sched.size(); p += 2) {
      const int m = v.sched[p], it = v.sched[p + 1];
      const int l = 1 << m, nm = side(m);
      const size_t cnt = size_t(nm) * nm;
      float* blk = nullptr;
      if (hipMalloc(reinterpret_cast<void**>(&blk), sizeof(float) * cnt * (1 + 2 * size_t(it))) != hipSuccess)
        return tfail(t, HOMG_ERR_OOM, "sample allocation failed");
      new_blocks.push_back(blk);
      float* rf = blk;
      TCHK(t, launch_lattice_f32(rm[m], nm, 1, nullptr, 0, nm, rf, s));
      const double hl = 1.0 / double(nm - 1);
      for (int i = 0; i < it; ++i) {
        float* xf = blk + cnt * (1 + 2 * size_t(i));
        float* df = xf + cnt;
        TCHK(t, launch_lattice_f32(e[cur], n, l, nullptr, 0, nm, xf, s));
        TCHK(t, launch_lattice_f32(e[cur], n, l, xs[m], nm, nm, df, s));
        TCHK(t, launch_energy(df, var ? af[m] : nullptr, nm, part, e0dev + k, s));
        new_samples.push_back(Sample{xf, df, rf, nullptr, nm, float(hl * hl)});
        ++k;
        st = homg_step_sweeps(h, m, 1, e[cur], rm[m], e[1 - cur], stream);
        if (st != HOMG_OK) return tfail(t, st, std::string("pair generation: ") + homg_last_error(h));
        cur = 1 - cur;
      }
      if (var) {  // the samples keep their own copy of the lattice coefficient
        float* ab = nullptr;
        if (hipMalloc(reinterpret_cast<void**>(&ab), sizeof(float) * cnt) != hipSuccess)
          return tfail(t, HOMG_ERR_OOM, "sample allocation failed");
        new_blocks.push_back(ab);
        TCHK(t, hipMemcpyAsync(ab, af[m], sizeof(float) * cnt, hipMemcpyDeviceToDevice, s));
        for (int i = 0; i < it; ++i) new_samples[new_samples.size() - 1 - i].a = ab;
      }
      t->max_nm = std::max(t->max_nm, nm);
    }
    TCHK(t, launch_add_dense(u, e[cur], int64_t(nn), s));
  }
  std::vector<double> e0(k);
  TCHK(t, hipMemcpyAsync(e0.data(), e0dev, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  TCHK(t, hipStreamSynchronize(s));
  for (int i = 0; i < k; ++i) {
    // an iterate that already is the level solution carries no information
    if (!(e0[i] > 0.0) || !std::isfinite(e0[i])) continue;
    t->samples.push_back(new_samples[i]);
    t->e0.push_back(e0[i]);
  }
  t->blocks.insert(t->blocks.end(), new_blocks.begin(), new_blocks.end());
  pending.keep = true;
  return HOMG_OK;
}

homg_status homg_trainer_train(homg_trainer t, const float* w0, const homg_train_options* opt,
                               float* w_out, double* loss_hist, void* stream) {
  if (!t || !w0 || !opt || !w_out) return tfail(t, HOMG_ERR_INVALID_ARG, "null argument");
  if (opt->struct_size != sizeof(homg_train_options))
    return tfail(t, HOMG_ERR_INVALID_ARG, "homg_train_options.struct_size mismatch");
  for (int i = 0; i < 8; ++i)
    if (opt->reserved[i]) return tfail(t, HOMG_ERR_INVALID_ARG, "reserved options must be 0");
  if (opt->steps < 1 || opt->steps > 1000000 || opt->batch < 1 || opt->batch > 256)
    return tfail(t, HOMG_ERR_INVALID_ARG, "steps must be >= 1 and batch in [1, 256]");
  if (!(opt->lr > 0.0) || !(opt->beta1 >= 0.0 && opt->beta1 < 1.0) ||
      !(opt->beta2 >= 0.0 && opt->beta2 < 1.0) || !(opt->eps > 0.0))
    return tfail(t, HOMG_ERR_INVALID_ARG, "invalid Adam parameters");
  const int S = int(t->samples.size());
  if (S < 1) return tfail(t, HOMG_ERR_INVALID_ARG, "no samples");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int steps = opt->steps, B = opt->batch;

  DevBufs tmp;
  float *theta, *m1, *m2, *w32, *z, *part;
  uint16_t* wbf;
  int* idx;
  double *e0s, *sums, *loss;
  TCHK(t, tmp.alloc(&theta, NW));
  TCHK(t, tmp.alloc(&m1, NW));
  TCHK(t, tmp.alloc(&m2, NW));
  TCHK(t, tmp.alloc(&w32, NW));
  TCHK(t, tmp.alloc(&wbf, NW));
  TCHK(t, tmp.alloc(&z, size_t(t->max_nm) * t->max_nm));
  TCHK(t, tmp.alloc(&part, size_t(NW + 1) * TRAIN_MAX_ROWS));
  TCHK(t, tmp.alloc(&idx, size_t(steps) * B));
  TCHK(t, tmp.alloc(&e0s, S));
  TCHK(t, tmp.alloc(&sums, size_t(B) * (NW + 1)));
  TCHK(t, tmp.alloc(&loss, steps));

  std::vector<int> hidx(size_t(steps) * B);
  uint64_t st = opt->seed;
  for (auto& v : hidx) v = int(splitmix64(st) % uint64_t(S));
  TCHK(t, hipMemcpyAsync(idx, hidx.data(), sizeof(int) * hidx.size(), hipMemcpyHostToDevice, s));
  TCHK(t, hipMemcpyAsync(e0s, t->e0.data(), sizeof(double) * S, hipMemcpyHostToDevice, s));
  TCHK(t, hipMemcpyAsync(theta, w0, sizeof(float) * NW, hipMemcpyDeviceToDevice, s));
  TCHK(t, hipMemsetAsync(m1, 0, sizeof(float) * NW, s));
  TCHK(t, hipMemsetAsync(m2, 0, sizeof(float) * NW, s));
  TCHK(t, launch_round_weights(theta, wbf, w32, s));
  for (int step = 1; step <= steps; ++step) {
    for (int b = 0; b < B; ++b) {
      const int i = hidx[size_t(step - 1) * B + b];
      const Sample& q = t->samples[i];
      TCHK(t, launch_train_fwd(q.nm, q.hl2, q.x, q.r, q.a, q.delta, z, w32, s));
      TCHK(t, launch_train_bwd(q.nm, q.hl2, q.x, q.r, q.a, z, e0s + i, w32, part, TRAIN_MAX_ROWS, s));
      TCHK(t, launch_train_reduce(part, TRAIN_MAX_ROWS, train_bwd_rows(q.nm), sums + size_t(b) * (NW + 1), s));
    }
    TCHK(t, launch_train_adam(sums, B, e0s, idx + size_t(step - 1) * B, theta, m1, m2, wbf, w32, step,
                              opt->lr, opt->beta1, opt->beta2, opt->eps, loss, s));
  }
  TCHK(t, hipMemcpyAsync(w_out, w32, sizeof(float) * NW, hipMemcpyDeviceToDevice, s));
  std::vector<double> hl(steps);
  TCHK(t, hipMemcpyAsync(hl.data(), loss, sizeof(double) * steps, hipMemcpyDeviceToHost, s));
  TCHK(t, hipStreamSynchronize(s));
  if (loss_hist) std::memcpy(loss_hist, hl.data(), sizeof(double) * steps);
  return HOMG_OK;
}

homg_status homg_trainer_loss(homg_trainer t, const float* w, double* mean_loss, void* stream) {
  if (!t || !w || !mean_loss) return tfail(t, HOMG_ERR_INVALID_ARG, "null argument");
  const int S = int(t->samples.size());
  if (S < 1) return tfail(t, HOMG_ERR_INVALID_ARG, "no samples");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBufs tmp;
  float* z;
  double *part, *ez;
  TCHK(t, tmp.alloc(&z, size_t(t->max_nm) * t->max_nm));
  TCHK(t, tmp.alloc(&part, ENERGY_MAX_PARTS));
  TCHK(t, tmp.alloc(&ez, S));
  for (int i = 0; i < S; ++i) {
    const Sample& q = t->samples[i];
    TCHK(t, launch_train_fwd(q.nm, q.hl2, q.x, q.r, q.a, q.delta, z, w, s));
    // z is written at interior nodes only; E reads interior nodes only
    TCHK(t, launch_energy(z, q.a, q.nm, part, ez + i, s));
  }
  std::vector<double> h(S);
  TCHK(t, hipMemcpyAsync(h.data(), ez, sizeof(double) * S, hipMemcpyDeviceToHost, s));
  TCHK(t, hipStreamSynchronize(s));
  double acc = 0.0;
  for (int i = 0; i < S; ++i) acc += h[i] / t->e0[i];
  *mean_loss = acc / S;
  return HOMG_OK;
}

homg_status homg_learn_forward(int nm, double hl, const float* x, const float* r, const float* a,
                               const float* w, float* y, void* stream) {
  if (nm < 3 || nm > 65537 || !(hl > 0.0)) return tfail(nullptr, HOMG_ERR_INVALID_ARG, "invalid size or spacing");
  if (!x || !r || !w || !y) return tfail(nullptr, HOMG_ERR_INVALID_ARG, "null array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  TCHK(nullptr, launch_train_fwd(nm, float(hl * hl), x, r, a, nullptr, y, w, s));
  return HOMG_OK;
}

homg_status homg_learn_grad(int nm, double hl, const float* x, const float* r, const float* a,
                            const float* delta, const float* w, double* grad, double* loss,
                            void* stream) {
  if (nm < 3 || nm > 65537 || !(hl > 0.0)) return tfail(nullptr, HOMG_ERR_INVALID_ARG, "invalid size or spacing");
  if (!x || !r || !delta || !w || !grad) return tfail(nullptr, HOMG_ERR_INVALID_ARG, "null array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBufs tmp;
  float *z, *part;
  double *epart, *e0;
  TCHK(nullptr, tmp.alloc(&z, size_t(nm) * nm));
  TCHK(nullptr, tmp.alloc(&part, size_t(NW + 1) * TRAIN_MAX_ROWS));
  TCHK(nullptr, tmp.alloc(&epart, ENERGY_MAX_PARTS));
  TCHK(nullptr, tmp.alloc(&e0, 1));
  const float hl2 = float(hl * hl);
  TCHK(nullptr, launch_energy(delta, a, nm, epart, e0, s));
  TCHK(nullptr, launch_train_fwd(nm, hl2, x, r, a, delta, z, w, s));
  TCHK(nullptr, launch_train_bwd(nm, hl2, x, r, a, z, e0, w, part, TRAIN_MAX_ROWS, s));
  TCHK(nullptr, launch_train_reduce(part, TRAIN_MAX_ROWS, train_bwd_rows(nm), grad, s));
  double ez = 0.0, e0h = 0.0;
  TCHK(nullptr, hipMemcpyAsync(&ez, grad + NW, sizeof(double), hipMemcpyDeviceToHost, s));
  TCHK(nullptr, hipMemcpyAsync(&e0h, e0, sizeof(double), hipMemcpyDeviceToHost, s));
  TCHK(nullptr, hipStreamSynchronize(s));
  if (loss) *loss = e0h > 0.0 ? ez / e0h : 0.0;
  return HOMG_OK;
}

homg_status homg_learn_adam(float* theta, float* m1, float* m2, const double* grad, int t, double lr,
                            double beta1, double beta2, double eps, float* w_out, void* stream) {
  if (!theta || !m1 || !m2 || !grad || !w_out) return tfail(nullptr, HOMG_ERR_INVALID_ARG, "null array");
  if (t < 1 || !(lr > 0.0) || !(eps > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
    return tfail(nullptr, HOMG_ERR_INVALID_ARG, "invalid Adam parameters");
  hipStream_t s = static_cast<hipStream_t>(stream);
  TCHK(nullptr, launch_train_adam(grad, 1, nullptr, nullptr, theta, m1, m2, nullptr, w_out, t, lr,
                                  beta1, beta2, eps, nullptr, s));
  return HOMG_OK;
}

}  // extern "C"
