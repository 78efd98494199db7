// homg_kernels.hip -- gfx950 kernels of the high occupancy multigrid (HOMG,
// arXiv:1108.2045): residual + norm, full-weighting restriction, and the
// fused whole-grid relax+interpolate iteration (Sec. 2).
//
// All three are bandwidth-bound stencils (about 0.3 flop per byte), so the
// kernels are written for HBM streaming, not for MFMA: one lane owns one
// x column (2D) or one (x,y) column (3D) and walks the slowest axis, keeping
// the values it will reuse (the row/plane above, the corners of the current
// level-m cell) in registers.  A wavefront therefore reads and writes 64
// consecutive elements of a row per step (coalesced; the padded layout puts
// the first interior node of every row on a 128-byte line), neighbours along
// x come from the L1 through unaligned reloads, and at coarse levels the
// only global reads are the few lattice corners per cell -- the sweep is
// write-dominated there.
//
// Arithmetic is written with explicit fused multiply-adds and the file is
// compiled with -ffp-contract=off, so every kernel that evaluates the same
// node formula produces the same bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "homg_internal.h"

namespace homg {

// ------------------------------------------------------------ storage types

struct bf16 {
  uint16_t bits;
};

template <typename T> struct Tr;
template <> struct Tr<double> { using C = double; };
template <> struct Tr<float> { using C = float; };
template <> struct Tr<bf16> { using C = float; };

__device__ __forceinline__ double ld(const double* p) { return *p; }
__device__ __forceinline__ float ld(const float* p) { return *p; }
__device__ __forceinline__ float ld(const bf16* p) {
  return __uint_as_float(uint32_t(p->bits) << 16);
}
__device__ __forceinline__ void st(double* p, double v) { *p = v; }
__device__ __forceinline__ void st(float* p, float v) { *p = v; }
// FP32 -> BF16, round to nearest even; NaN stays NaN.
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ void st(bf16* p, float v) { p->bits = f2bf(v); }

__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ------------------------------------------------------------ node formulas
// Shared by every kernel that evaluates a node, so results agree bit for bit.

// Damped Jacobi at a lattice node, constant coefficient (Sec. 2, level-m
// relaxation with the sign that converges): c + w (h_l^2 r - (2d c - sum nb)),
// w = omega / 2d.  q is the neighbour sum, added pairwise per axis.
template <typename C>
__device__ __forceinline__ C relax_const(C c, C q, C r, C w, C hl2, C two_d) {
  C lap = fmac(two_d, c, -q);           // 2d c - sum nb
  C res = fmac(hl2, r, -lap);           // h_l^2 r - (2d c - sum nb)
  return fmac(w, res, c);
}

// Harmonic mean of two nodal coefficients (the face coefficient).
__device__ __forceinline__ double harm(double a, double b) { return 2.0 * a * b / (a + b); }

// Linear interpolation a + t (b - a), t in [0, 1).
template <typename C>
__device__ __forceinline__ C lerp(C a, C b, C t) { return fmac(t, b - a, a); }

// ------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic block sum (fixed order for a fixed block size); result valid
// in thread 0.  Every thread of the block must call it.
template <int NT>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[NT / 64];
  v = wave_sum(v);
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w];
  }
  return s;
}

// ------------------------------------------------------------ launch shapes

constexpr int BX2 = 256;          // 2D: lanes along x per block
constexpr int BX3 = 64, BY3 = 4;  // 3D: lanes along x and y per block

// Rows (2D) or planes (3D) walked by one block: enough blocks to fill the
// 256 CUs several times over, long enough walks to amortise the halo reloads.
static int walk_len(int d, int n) {
  const int64_t inner = n - 2;
  const int64_t columns = d == 2 ? inner : inner * inner;
  const int64_t lanes_per_block = d == 2 ? BX2 : BX3 * BY3;
  const int64_t col_blocks = (columns + lanes_per_block - 1) / lanes_per_block;
  const int64_t target_blocks = 4096;
  int64_t len = (inner * col_blocks + target_blocks - 1) / target_blocks;
  if (len < 4) len = 4;
  if (len > 64) len = 64;
  if (len > inner) len = inner;
  return int(len);
}

static dim3 grid_of(int d, int n, int len) {
  const int inner = n - 2;
  const int walks = (inner + len - 1) / len;
  if (d == 2) return dim3((inner + BX2 - 1) / BX2, walks, 1);
  return dim3((inner + BX3 - 1) / BX3, (inner + BY3 - 1) / BY3, walks);
}

int partials_bound(int d, int n) {
  if (n < 3) return 1;
  dim3 g = grid_of(d, n, walk_len(d, n));
  return int(g.x * g.y * g.z);
}

Lay dense_layout(int d, int side) {
  Lay L;
  L.side = side;
  L.off = 0;
  L.pitch = side;
  L.plane = d == 3 ? int64_t(side) * side : 0;
  L.alloc = d == 3 ? int64_t(side) * side * side : int64_t(side) * side;
  return L;
}

Lay padded_layout(int d, int side, int elem_bytes) {
  const int64_t a = 128 / elem_bytes;  // elements per 128-byte line
  Lay L;
  L.side = side;
  L.pitch = ((side + a - 1) / a) * a;
  L.off = a - 1;  // node (.,.,1) of row 0 on a line boundary; pitch keeps the phase
  L.plane = d == 3 ? L.pitch * side : 0;
  const int64_t rows = d == 3 ? int64_t(side) * side : side;
  L.alloc = L.off + rows * L.pitch + a;  // tail slack: whole final line
  return L;
}

// ------------------------------------------------------------ norm of f

__global__ __launch_bounds__(256) void k_norm2_2d(const double* __restrict__ f, int64_t fp, int n,
                                                  int len, double* __restrict__ partials) {
  const int x = 1 + blockIdx.x * BX2 + threadIdx.x;
  const int y0 = 1 + blockIdx.y * len;
  const int y1 = min(n - 1, y0 + len);
  double s = 0.0;
  if (x <= n - 2)
    for (int y = y0; y < y1; ++y) {
      double v = f[int64_t(y) * fp + x];
      s = fmac(v, v, s);
    }
  s = block_sum<256>(s);
  if (threadIdx.x == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_norm2_3d(const double* __restrict__ f, int64_t fp,
                                                  int64_t fpl, int n, int len,
                                                  double* __restrict__ partials) {
  const int x = 1 + blockIdx.x * BX3 + threadIdx.x;
  const int y = 1 + blockIdx.y * BY3 + threadIdx.y;
  const int z0 = 1 + blockIdx.z * len;
  const int z1 = min(n - 1, z0 + len);
  double s = 0.0;
  if (x <= n - 2 && y <= n - 2)
    for (int z = z0; z < z1; ++z) {
      double v = f[int64_t(z) * fpl + int64_t(y) * fp + x];
      s = fmac(v, v, s);
    }
  s = block_sum<256>(s);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    partials[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

// ------------------------------------------------------------ residual
// r = f - A u on interior nodes (Sec. 2, residual equation), FP64
// arithmetic; r stored in the cycle precision T; per-block sum of r^2 of the
// FP64 values.

template <typename T, bool VAR>
__global__ __launch_bounds__(256) void k_residual_2d(
    const double* __restrict__ u, int64_t up, const double* __restrict__ f, int64_t fp,
    const double* __restrict__ a, int64_t ap, T* __restrict__ r, int64_t rp, int n, int len,
    double inv_h2, double* __restrict__ partials, const int* __restrict__ done) {
  if (*done) return;
  const int x = 1 + blockIdx.x * BX2 + threadIdx.x;
  const int y0 = 1 + blockIdx.y * len;
  const int y1 = min(n - 1, y0 + len);
  double s = 0.0;
  if (x <= n - 2) {
    double ym = u[int64_t(y0 - 1) * up + x];
    double c = u[int64_t(y0) * up + x];
    double aym = 0.0, ac = 0.0;
    if (VAR) {
      aym = a[int64_t(y0 - 1) * ap + x];
      ac = a[int64_t(y0) * ap + x];
    }
    for (int y = y0; y < y1; ++y) {
      const double* row = u + int64_t(y) * up;
      const double yp = row[up + x];
      const double xm = row[x - 1], xp = row[x + 1];
      double au;
      if (VAR) {
        const double* arow = a + int64_t(y) * ap;
        const double ayp = arow[ap + x];
        const double axm = arow[x - 1], axp = arow[x + 1];
        const double cxm = harm(ac, axm), cxp = harm(ac, axp);
        const double cym = harm(ac, aym), cyp = harm(ac, ayp);
        au = fmac(cxm, c - xm, cxp * (c - xp)) + fmac(cym, c - ym, cyp * (c - yp));
        aym = ac;
        ac = ayp;
      } else {
        au = fmac(4.0, c, -((xm + xp) + (ym + yp)));
      }
      const double rv = fmac(-inv_h2, au, f[int64_t(y) * fp + x]);
      st(r + int64_t(y) * rp + x, typename Tr<T>::C(rv));
      s = fmac(rv, rv, s);
      ym = c;
      c = yp;
    }
  }
  s = block_sum<256>(s);
  if (threadIdx.x == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_residual_3d(
    const double* __restrict__ u, int64_t up, int64_t upl, const double* __restrict__ f,
    int64_t fp, int64_t fpl, T* __restrict__ r, int64_t rp, int64_t rpl, int n, int len,
    double inv_h2, double* __restrict__ partials, const int* __restrict__ done) {
  if (*done) return;
  const int x = 1 + blockIdx.x * BX3 + threadIdx.x;
  const int y = 1 + blockIdx.y * BY3 + threadIdx.y;
  const int z0 = 1 + blockIdx.z * len;
  const int z1 = min(n - 1, z0 + len);
  double s = 0.0;
  if (x <= n - 2 && y <= n - 2) {
    const int64_t col = int64_t(y) * up + x;
    double zm = u[int64_t(z0 - 1) * upl + col];
    double c = u[int64_t(z0) * upl + col];
    for (int z = z0; z < z1; ++z) {
      const double* pl = u + int64_t(z) * upl + col;
      const double zp = pl[upl];
      const double xm = pl[-1], xp = pl[1], ym = pl[-up], yp = pl[up];
      const double au = fmac(6.0, c, -(((xm + xp) + (ym + yp)) + (zm + zp)));
      const double rv = fmac(-inv_h2, au, f[int64_t(z) * fpl + int64_t(y) * fp + x]);
      st(r + int64_t(z) * rpl + int64_t(y) * rp + x, typename Tr<T>::C(rv));
      s = fmac(rv, rv, s);
      zm = c;
      c = zp;
    }
  }
  s = block_sum<256>(s);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    partials[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

// ------------------------------------------------------------ finalize

__global__ __launch_bounds__(256) void k_init_state(DevState* st, double tol, int stop_on_tol) {
  if (threadIdx.x == 0) {
    st->done = 0;
    st->cycles = -1;
    st->stop_on_tol = stop_on_tol;
    st->fnorm = 1.0;
    st->tol = tol;
  }
}

__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partials, int count,
                                                  DevState* st, double* __restrict__ history,
                                                  int cycle, int mode) {
  if (mode == 1 && st->done) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) s += partials[i];
  s = block_sum<256>(s);
  if (threadIdx.x == 0) {
    if (mode == 0) {
      const double fn = sqrt(s);
      st->fnorm = fn > 0.0 ? fn : 1.0;
    } else {
      const double rel = sqrt(s) / st->fnorm;
      history[cycle] = rel;
      st->cycles = cycle;
      if (!(rel <= 1.7976931348623157e308)) st->done = 2;  // NaN or Inf
      else if (st->stop_on_tol && rel <= st->tol) st->done = 1;
    }
  }
}

// ------------------------------------------------------------ restriction
// Full weighting (Sec. 2: linearly weighted averages as nested partial
// reductions): coarse node = (1/4)[1 2 1] per axis of the fine neighbours.

template <typename T>
__global__ __launch_bounds__(256) void k_restrict_2d(const T* __restrict__ rf, int64_t fp,
                                                     T* __restrict__ rc, int64_t cp, int nc,
                                                     int len, const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  const int I = 1 + blockIdx.x * BX2 + threadIdx.x;
  if (I > nc - 2) return;
  const int J0 = 1 + blockIdx.y * len;
  const int J1 = min(nc - 1, J0 + len);
  const int xi = 2 * I;
  auto rowsum = [&](int yf) {
    const T* row = rf + int64_t(yf) * fp + xi;
    return fmac(C(2), ld(row), ld(row - 1) + ld(row + 1));
  };
  C top = rowsum(2 * J0 - 1);
  for (int J = J0; J < J1; ++J) {
    const C mid = rowsum(2 * J);
    const C bot = rowsum(2 * J + 1);
    st(rc + int64_t(J) * cp + I, fmac(C(2), mid, top + bot) * C(0.0625));
    top = bot;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_restrict_3d(const T* __restrict__ rf, int64_t fp,
                                                     int64_t fpl, T* __restrict__ rc, int64_t cp,
                                                     int64_t cpl, int nc, int len,
                                                     const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  const int I = 1 + blockIdx.x * BX3 + threadIdx.x;
  const int J = 1 + blockIdx.y * BY3 + threadIdx.y;
  if (I > nc - 2 || J > nc - 2) return;
  const int K0 = 1 + blockIdx.z * len;
  const int K1 = min(nc - 1, K0 + len);
  const int64_t col = int64_t(2 * J) * fp + 2 * I;
  auto planesum = [&](int zf) {
    const T* p = rf + int64_t(zf) * fpl + col;
    auto rs = [&](const T* q) { return fmac(C(2), ld(q), ld(q - 1) + ld(q + 1)); };
    return fmac(C(2), rs(p), rs(p - fp) + rs(p + fp));
  };
  C top = planesum(2 * K0 - 1);
  for (int K = K0; K < K1; ++K) {
    const C mid = planesum(2 * K);
    const C bot = planesum(2 * K + 1);
    st(rc + int64_t(K) * cpl + int64_t(J) * cp + I, fmac(C(2), mid, top + bot) * C(0.015625));
    top = bot;
  }
}

// ------------------------------------------------------------ fused sweep
// One HOMG iteration at level m over the whole grid (Sec. 2): interior
// lattice nodes (every index a multiple of l = 2^m) relax, every other
// interior node takes the multilinear interpolant of the previous iterate's
// lattice values at the corners of its level-m cell (the interpolation is
// delayed one iteration, Sec. 4).  Boundary nodes of e are 0 and never
// written.  ZERO: the previous iterate is 0 (first iteration of a cycle; no
// reads of e).  ACCUM: the new iterate is added to u instead of stored (last
// iteration of a cycle).

template <typename T, int MODE, bool VAR>
__device__ __forceinline__ void emit_2d(T* en, int64_t eoff, double* u, int64_t uoff,
                                        typename Tr<T>::C v) {
  if (MODE & SW_ACCUM) {
    u[uoff] += double(v);
  } else {
    st(en + eoff, v);
  }
}

// Level 0: every interior node relaxes (plain damped Jacobi).
template <typename T, int MODE, bool VAR>
__global__ __launch_bounds__(256) void k_sweep_2d_l0(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, const T* __restrict__ r,
    int64_t rp, const double* __restrict__ a, int64_t ap, double* __restrict__ u, int64_t up,
    int n, int len, typename Tr<T>::C w, typename Tr<T>::C hl2, const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  const int x = 1 + blockIdx.x * BX2 + threadIdx.x;
  if (x > n - 2) return;
  const int y0 = 1 + blockIdx.y * len;
  const int y1 = min(n - 1, y0 + len);
  C ym = C(0), c = C(0);
  if (!(MODE & SW_ZERO_OLD)) {
    ym = ld(eo + int64_t(y0 - 1) * ep + x);
    c = ld(eo + int64_t(y0) * ep + x);
  }
  double aym = 0.0, ac = 0.0;
  if (VAR) {
    aym = a[int64_t(y0 - 1) * ap + x];
    ac = a[int64_t(y0) * ap + x];
  }
  for (int y = y0; y < y1; ++y) {
    const C rv = ld(r + int64_t(y) * rp + x);
    C xm = C(0), xp = C(0), yp = C(0);
    if (!(MODE & SW_ZERO_OLD)) {
      const T* row = eo + int64_t(y) * ep;
      yp = ld(row + ep + x);
      xm = ld(row + x - 1);
      xp = ld(row + x + 1);
    }
    C v;
    if (VAR) {
      const double* arow = a + int64_t(y) * ap;
      const double ayp = arow[ap + x];
      const C cxm = C(harm(ac, arow[x - 1])), cxp = C(harm(ac, arow[x + 1]));
      const C cym = C(harm(ac, aym)), cyp = C(harm(ac, ayp));
      const C sa = (cxm + cxp) + (cym + cyp);
      const C flux = fmac(cxm, c - xm, cxp * (c - xp)) + fmac(cym, c - ym, cyp * (c - yp));
      v = fmac(w / sa, fmac(hl2, rv, -flux), c);
      aym = ac;
      ac = ayp;
    } else {
      v = relax_const<C>(c, (xm + xp) + (ym + yp), rv, w, hl2, C(4));
    }
    emit_2d<T, MODE, VAR>(en, int64_t(y) * ep + x, u, int64_t(y) * up + x, v);
    ym = c;
    c = yp;
  }
}

// Levels m >= 1: lattice nodes relax, the rest interpolate.  The lane keeps
// the four corners of its current level-m cell; they change every l rows.
template <typename T, int MODE, bool VAR>
__global__ __launch_bounds__(256) void k_sweep_2d_coarse(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, const T* __restrict__ rm,
    int64_t rp, const double* __restrict__ am, int64_t ap, double* __restrict__ u, int64_t up,
    int n, int len, int m, typename Tr<T>::C w, typename Tr<T>::C hl2,
    const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  const int x = 1 + blockIdx.x * BX2 + threadIdx.x;
  if (x > n - 2) return;
  const int l = 1 << m;
  const int mask = l - 1;
  const C inv_l = C(1) / C(l);
  const int y0 = 1 + blockIdx.y * len;
  const int y1 = min(n - 1, y0 + len);
  const int xa = x & ~mask, xb = xa + l;
  const C tx = C(x - xa) * inv_l;
  const bool latc = (x == xa);
  int ya = y0 & ~mask;
  C t0 = C(0), t1 = C(0), b0 = C(0), b1 = C(0);
  if (!(MODE & SW_ZERO_OLD)) {
    t0 = ld(eo + int64_t(ya) * ep + xa);
    t1 = ld(eo + int64_t(ya) * ep + xb);
    b0 = ld(eo + int64_t(ya + l) * ep + xa);
    b1 = ld(eo + int64_t(ya + l) * ep + xb);
  }
  C top = lerp(t0, t1, tx), bot = lerp(b0, b1, tx);
  for (int y = y0; y < y1; ++y) {
    if (y - ya == l) {
      ya += l;
      t0 = b0;
      t1 = b1;
      top = bot;
      if (!(MODE & SW_ZERO_OLD)) {
        b0 = ld(eo + int64_t(ya + l) * ep + xa);
        b1 = ld(eo + int64_t(ya + l) * ep + xb);
      }
      bot = lerp(b0, b1, tx);
    }
    C v;
    if (latc && y == ya) {
      const C rv = ld(rm + int64_t(ya >> m) * rp + (xa >> m));
      C xm = C(0), ym = C(0);
      if (!(MODE & SW_ZERO_OLD)) {
        xm = ld(eo + int64_t(ya) * ep + xa - l);
        ym = ld(eo + int64_t(ya - l) * ep + xa);
      }
      if (VAR) {
        const int I = xa >> m, J = ya >> m;
        const double* arow = am + int64_t(J) * ap + I;
        const double ac = arow[0];
        const C cxm = C(harm(ac, arow[-1])), cxp = C(harm(ac, arow[1]));
        const C cym = C(harm(ac, arow[-ap])), cyp = C(harm(ac, arow[ap]));
        const C sa = (cxm + cxp) + (cym + cyp);
        const C flux = fmac(cxm, t0 - xm, cxp * (t0 - t1)) + fmac(cym, t0 - ym, cyp * (t0 - b0));
        v = fmac(w / sa, fmac(hl2, rv, -flux), t0);
      } else {
        v = relax_const<C>(t0, (xm + t1) + (ym + b0), rv, w, hl2, C(4));
      }
    } else {
      v = lerp(top, bot, C(y - ya) * inv_l);
    }
    emit_2d<T, MODE, VAR>(en, int64_t(y) * ep + x, u, int64_t(y) * up + x, v);
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_sweep_3d_l0(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, int64_t epl,
    const T* __restrict__ r, int64_t rp, int64_t rpl, double* __restrict__ u, int64_t up,
    int64_t upl, int n, int len, typename Tr<T>::C w, typename Tr<T>::C hl2,
    const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  const int x = 1 + blockIdx.x * BX3 + threadIdx.x;
  const int y = 1 + blockIdx.y * BY3 + threadIdx.y;
  if (x > n - 2 || y > n - 2) return;
  const int z0 = 1 + blockIdx.z * len;
  const int z1 = min(n - 1, z0 + len);
  const int64_t col = int64_t(y) * ep + x;
  C zm = C(0), c = C(0);
  if (!(MODE & SW_ZERO_OLD)) {
    zm = ld(eo + int64_t(z0 - 1) * epl + col);
    c = ld(eo + int64_t(z0) * epl + col);
  }
  for (int z = z0; z < z1; ++z) {
    const C rv = ld(r + int64_t(z) * rpl + int64_t(y) * rp + x);
    C zp = C(0), xm = C(0), xp = C(0), ym = C(0), yp = C(0);
    if (!(MODE & SW_ZERO_OLD)) {
      const T* p = eo + int64_t(z) * epl + col;
      zp = ld(p + epl);
      xm = ld(p - 1);
      xp = ld(p + 1);
      ym = ld(p - ep);
      yp = ld(p + ep);
    }
    const C v = relax_const<C>(c, ((xm + xp) + (ym + yp)) + (zm + zp), rv, w, hl2, C(6));
    if (MODE & SW_ACCUM)
      u[int64_t(z) * upl + int64_t(y) * up + x] += double(v);
    else
      st(en + int64_t(z) * epl + col, v);
    zm = c;
    c = zp;
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_sweep_3d_coarse(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, int64_t epl,
    const T* __restrict__ rm, int64_t rp, int64_t rpl, double* __restrict__ u, int64_t up,
    int64_t upl, int n, int len, int m, typename Tr<T>::C w, typename Tr<T>::C hl2,
    const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  const int x = 1 + blockIdx.x * BX3 + threadIdx.x;
  const int y = 1 + blockIdx.y * BY3 + threadIdx.y;
  if (x > n - 2 || y > n - 2) return;
  const int l = 1 << m;
  const int mask = l - 1;
  const C inv_l = C(1) / C(l);
  const int z0 = 1 + blockIdx.z * len;
  const int z1 = min(n - 1, z0 + len);
  const int xa = x & ~mask, xb = xa + l;
  const int ya = y & ~mask, yb = ya + l;
  const C tx = C(x - xa) * inv_l, ty = C(y - ya) * inv_l;
  const bool latxy = (x == xa) && (y == ya);
  const int64_t c00 = int64_t(ya) * ep + xa, c01 = int64_t(ya) * ep + xb;
  const int64_t c10 = int64_t(yb) * ep + xa, c11 = int64_t(yb) * ep + xb;
  int za = z0 & ~mask;
  // corners of the top (za) and bottom (za + l) planes of the current cell
  C t00 = C(0), t01 = C(0), t10 = C(0), t11 = C(0);
  C b00 = C(0), b01 = C(0), b10 = C(0), b11 = C(0);
  if (!(MODE & SW_ZERO_OLD)) {
    const T* pt = eo + int64_t(za) * epl;
    const T* pb = pt + int64_t(l) * epl;
    t00 = ld(pt + c00); t01 = ld(pt + c01); t10 = ld(pt + c10); t11 = ld(pt + c11);
    b00 = ld(pb + c00); b01 = ld(pb + c01); b10 = ld(pb + c10); b11 = ld(pb + c11);
  }
  C top = lerp(lerp(t00, t01, tx), lerp(t10, t11, tx), ty);
  C bot = lerp(lerp(b00, b01, tx), lerp(b10, b11, tx), ty);
  for (int z = z0; z < z1; ++z) {
    if (z - za == l) {
      za += l;
      t00 = b00; t01 = b01; t10 = b10; t11 = b11;
      top = bot;
      if (!(MODE & SW_ZERO_OLD)) {
        const T* pb = eo + int64_t(za + l) * epl;
        b00 = ld(pb + c00); b01 = ld(pb + c01); b10 = ld(pb + c10); b11 = ld(pb + c11);
      }
      bot = lerp(lerp(b00, b01, tx), lerp(b10, b11, tx), ty);
    }
    C v;
    if (latxy && z == za) {
      const C rv = ld(rm + int64_t(za >> m) * rpl + int64_t(ya >> m) * rp + (xa >> m));
      C xm = C(0), ym = C(0), zm = C(0);
      if (!(MODE & SW_ZERO_OLD)) {
        const T* p = eo + int64_t(za) * epl + c00;
        xm = ld(p - l);
        ym = ld(p - int64_t(l) * ep);
        zm = ld(p - int64_t(l) * epl);
      }
      v = relax_const<C>(t00, ((xm + t01) + (ym + t10)) + (zm + b00), rv, w, hl2, C(6));
    } else {
      v = lerp(top, bot, C(z - za) * inv_l);
    }
    if (MODE & SW_ACCUM)
      u[int64_t(z) * upl + int64_t(y) * up + x] += double(v);
    else
      st(en + int64_t(z) * epl + int64_t(y) * ep + x, v);
  }
}

// ------------------------------------------------------------ pack / unpack

template <typename T>
__global__ __launch_bounds__(256) void k_pack(const double* __restrict__ src, int64_t sp,
                                              int64_t spl, T* __restrict__ dst, int64_t dp,
                                              int64_t dpl, int side, int nz) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= side || z >= nz) return;
  st(dst + int64_t(z) * dpl + int64_t(y) * dp + x,
     typename Tr<T>::C(src[int64_t(z) * spl + int64_t(y) * sp + x]));
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack(const T* __restrict__ src, int64_t sp,
                                                int64_t spl, double* __restrict__ dst, int64_t dp,
                                                int64_t dpl, int side, int nz) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= side || z >= nz) return;
  dst[int64_t(z) * dpl + int64_t(y) * dp + x] = double(ld(src + int64_t(z) * spl + int64_t(y) * sp + x));
}

__global__ __launch_bounds__(256) void k_sample(const double* __restrict__ src, int64_t sp,
                                                int64_t spl, int stride, double* __restrict__ dst,
                                                int64_t dp, int64_t dpl, int side, int nz) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= side || z >= nz) return;
  dst[int64_t(z) * dpl + int64_t(y) * dp + x] =
      src[int64_t(z) * stride * spl + int64_t(y) * stride * sp + int64_t(x) * stride];
}

// ------------------------------------------------------------ launchers

#define HOMG_LAUNCH(kernel, grid, block, stream, ...)               \
  do {                                                              \
    hipLaunchKernelGGL(kernel, grid, block, 0, stream, __VA_ARGS__); \
    return hipGetLastError();                                       \
  } while (0)

hipError_t launch_norm2(int d, int n, const double* f, const Lay& fl, double* partials,
                        int* count, hipStream_t s) {
  const int len = walk_len(d, n);
  const dim3 g = grid_of(d, n, len);
  *count = int(g.x * g.y * g.z);
  if (d == 2) HOMG_LAUNCH(k_norm2_2d, g, dim3(BX2), s, f + fl.off, fl.pitch, n, len, partials);
  HOMG_LAUNCH(k_norm2_3d, g, dim3(BX3, BY3), s, f + fl.off, fl.pitch, fl.plane, n, len, partials);
}

template <typename T>
static hipError_t residual_t(int d, int n, const double* u, const Lay& ul, const double* f,
                             const Lay& fl, const double* a, const Lay& al, void* r0,
                             const Lay& rl, double* partials, int* count, const int* done,
                             hipStream_t s) {
  const int len = walk_len(d, n);
  const dim3 g = grid_of(d, n, len);
  *count = int(g.x * g.y * g.z);
  const double h = 1.0 / double(n - 1);
  const double inv_h2 = 1.0 / (h * h);
  T* r = static_cast<T*>(r0) + rl.off;
  if (d == 2) {
    if (a)
      HOMG_LAUNCH((k_residual_2d<T, true>), g, dim3(BX2), s, u + ul.off, ul.pitch, f + fl.off,
                  fl.pitch, a + al.off, al.pitch, r, rl.pitch, n, len, inv_h2, partials, done);
    HOMG_LAUNCH((k_residual_2d<T, false>), g, dim3(BX2), s, u + ul.off, ul.pitch, f + fl.off,
                fl.pitch, (const double*)nullptr, int64_t(0), r, rl.pitch, n, len, inv_h2,
                partials, done);
  }
  HOMG_LAUNCH((k_residual_3d<T>), g, dim3(BX3, BY3), s, u + ul.off, ul.pitch, ul.plane,
              f + fl.off, fl.pitch, fl.plane, r, rl.pitch, rl.plane, n, len, inv_h2, partials,
              done);
}

hipError_t launch_residual(int prec, int d, int n, const double* u, const Lay& ul,
                           const double* f, const Lay& fl, const double* a, const Lay& al,
                           void* r0, const Lay& rl, double* partials, int* count,
                           const int* done, hipStream_t s) {
  switch (prec) {
    case PREC_F64: return residual_t<double>(d, n, u, ul, f, fl, a, al, r0, rl, partials, count, done, s);
    case PREC_F32: return residual_t<float>(d, n, u, ul, f, fl, a, al, r0, rl, partials, count, done, s);
    default: return residual_t<bf16>(d, n, u, ul, f, fl, a, al, r0, rl, partials, count, done, s);
  }
}

hipError_t launch_finalize(const double* partials, int count, DevState* st, double* history,
                           int cycle, int mode, hipStream_t s) {
  HOMG_LAUNCH(k_finalize, dim3(1), dim3(256), s, partials, count, st, history, cycle, mode);
}

hipError_t launch_init_state(DevState* st, double tol, int stop_on_tol, hipStream_t s) {
  HOMG_LAUNCH(k_init_state, dim3(1), dim3(256), s, st, tol, stop_on_tol);
}

template <typename T>
static hipError_t restrict_t(int d, const void* rf, const Lay& fl, void* rc, const Lay& cl,
                             const int* done, hipStream_t s) {
  const int nc = cl.side;
  const int len = walk_len(d, nc);
  const dim3 g = grid_of(d, nc, len);
  const T* f = static_cast<const T*>(rf) + fl.off;
  T* c = static_cast<T*>(rc) + cl.off;
  if (d == 2) HOMG_LAUNCH((k_restrict_2d<T>), g, dim3(BX2), s, f, fl.pitch, c, cl.pitch, nc, len, done);
  HOMG_LAUNCH((k_restrict_3d<T>), g, dim3(BX3, BY3), s, f, fl.pitch, fl.plane, c, cl.pitch,
              cl.plane, nc, len, done);
}

hipError_t launch_restrict(int prec, int d, const void* rf, const Lay& fl, void* rc,
                           const Lay& cl, const int* done, hipStream_t s) {
  if (cl.side < 3) return hipSuccess;
  switch (prec) {
    case PREC_F64: return restrict_t<double>(d, rf, fl, rc, cl, done, s);
    case PREC_F32: return restrict_t<float>(d, rf, fl, rc, cl, done, s);
    default: return restrict_t<bf16>(d, rf, fl, rc, cl, done, s);
  }
}

template <typename T, int MODE>
static hipError_t sweep_tm(int d, int n, int m, double omega, const void* eo_, void* en_,
                           const Lay& el, const void* rm_, const Lay& rl, const double* am,
                           const Lay& al, double* u, const Lay& ul, const int* done,
                           hipStream_t s) {
  using C = typename Tr<T>::C;
  const int len = walk_len(d, n);
  const dim3 g = grid_of(d, n, len);
  const T* eo = eo_ ? static_cast<const T*>(eo_) + el.off : nullptr;
  T* en = en_ ? static_cast<T*>(en_) + el.off : nullptr;
  const T* rm = static_cast<const T*>(rm_) + rl.off;
  const double hl = double(1 << m) / double(n - 1);
  const C hl2 = C(hl * hl);
  double* uu = u ? u + ul.off : nullptr;
  if (d == 2) {
    const C w = am ? C(omega) : C(omega / 4.0);
    const double* a = am ? am + al.off : nullptr;
    if (m == 0) {
      if (am)
        HOMG_LAUNCH((k_sweep_2d_l0<T, MODE, true>), g, dim3(BX2), s, eo, en, el.pitch, rm,
                    rl.pitch, a, al.pitch, uu, ul.pitch, n, len, w, hl2, done);
      HOMG_LAUNCH((k_sweep_2d_l0<T, MODE, false>), g, dim3(BX2), s, eo, en, el.pitch, rm,
                  rl.pitch, a, al.pitch, uu, ul.pitch, n, len, w, hl2, done);
    }
    if (am)
      HOMG_LAUNCH((k_sweep_2d_coarse<T, MODE, true>), g, dim3(BX2), s, eo, en, el.pitch, rm,
                  rl.pitch, a, al.pitch, uu, ul.pitch, n, len, m, w, hl2, done);
    HOMG_LAUNCH((k_sweep_2d_coarse<T, MODE, false>), g, dim3(BX2), s, eo, en, el.pitch, rm,
                rl.pitch, a, al.pitch, uu, ul.pitch, n, len, m, w, hl2, done);
  }
  const C w = C(omega / 6.0);
  if (m == 0)
    HOMG_LAUNCH((k_sweep_3d_l0<T, MODE>), g, dim3(BX3, BY3), s, eo, en, el.pitch, el.plane, rm,
                rl.pitch, rl.plane, uu, ul.pitch, ul.plane, n, len, w, hl2, done);
  HOMG_LAUNCH((k_sweep_3d_coarse<T, MODE>), g, dim3(BX3, BY3), s, eo, en, el.pitch, el.plane,
              rm, rl.pitch, rl.plane, uu, ul.pitch, ul.plane, n, len, m, w, hl2, done);
}

template <typename T>
static hipError_t sweep_t(int d, int n, int m, double omega, const void* eo, void* en,
                          const Lay& el, const void* rm, const Lay& rl, const double* am,
                          const Lay& al, double* u, const Lay& ul, int mode, const int* done,
                          hipStream_t s) {
  switch (mode & 3) {
    case 0: return sweep_tm<T, 0>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, done, s);
    case 1: return sweep_tm<T, 1>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, done, s);
    case 2: return sweep_tm<T, 2>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, done, s);
    default: return sweep_tm<T, 3>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, done, s);
  }
}

hipError_t launch_sweep(int prec, int d, int n, int m, double omega, const void* eo, void* en,
                        const Lay& el, const void* rm, const Lay& rl, const double* am,
                        const Lay& al, double* u, const Lay& ul, int mode, const int* done,
                        hipStream_t s) {
  switch (prec) {
    case PREC_F64: return sweep_t<double>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, mode, done, s);
    case PREC_F32: return sweep_t<float>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, mode, done, s);
    default: return sweep_t<bf16>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, mode, done, s);
  }
}

static dim3 copy_grid(int d, int side) {
  return dim3((side + 255) / 256, side, d == 3 ? side : 1);
}

hipError_t launch_pack(int prec, int d, const double* src, const Lay& sl, void* dst,
                       const Lay& dl, hipStream_t s) {
  const int side = sl.side, nz = d == 3 ? side : 1;
  const dim3 g = copy_grid(d, side);
  switch (prec) {
    case PREC_F64:
      HOMG_LAUNCH((k_pack<double>), g, dim3(256), s, src + sl.off, sl.pitch, sl.plane,
                  static_cast<double*>(dst) + dl.off, dl.pitch, dl.plane, side, nz);
    case PREC_F32:
      HOMG_LAUNCH((k_pack<float>), g, dim3(256), s, src + sl.off, sl.pitch, sl.plane,
                  static_cast<float*>(dst) + dl.off, dl.pitch, dl.plane, side, nz);
    default:
      HOMG_LAUNCH((k_pack<bf16>), g, dim3(256), s, src + sl.off, sl.pitch, sl.plane,
                  static_cast<bf16*>(dst) + dl.off, dl.pitch, dl.plane, side, nz);
  }
}

hipError_t launch_unpack(int prec, int d, const void* src, const Lay& sl, double* dst,
                         const Lay& dl, hipStream_t s) {
  const int side = sl.side, nz = d == 3 ? side : 1;
  const dim3 g = copy_grid(d, side);
  switch (prec) {
    case PREC_F64:
      HOMG_LAUNCH((k_unpack<double>), g, dim3(256), s, static_cast<const double*>(src) + sl.off,
                  sl.pitch, sl.plane, dst + dl.off, dl.pitch, dl.plane, side, nz);
    case PREC_F32:
      HOMG_LAUNCH((k_unpack<float>), g, dim3(256), s, static_cast<const float*>(src) + sl.off,
                  sl.pitch, sl.plane, dst + dl.off, dl.pitch, dl.plane, side, nz);
    default:
      HOMG_LAUNCH((k_unpack<bf16>), g, dim3(256), s, static_cast<const bf16*>(src) + sl.off,
                  sl.pitch, sl.plane, dst + dl.off, dl.pitch, dl.plane, side, nz);
  }
}

hipError_t launch_sample(int d, const double* src, const Lay& sl, int stride, double* dst,
                         const Lay& dl, hipStream_t s) {
  const int side = dl.side, nz = d == 3 ? side : 1;
  HOMG_LAUNCH(k_sample, copy_grid(d, side), dim3(256), s, src + sl.off, sl.pitch, sl.plane,
              stride, dst + dl.off, dl.pitch, dl.plane, side, nz);
}

}  // namespace homg
