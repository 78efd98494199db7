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
#include <hip/hip_ext.h>
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
// Stores are streaming (non-temporal): every kernel here writes each output
// element once and the next kernel reads it from memory, so the written
// lines need not stay in the caches (on MI355X this lifts a read+write
// stream from about 5.2 to 7.5 TB/s).
__device__ __forceinline__ void st(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st(float* p, float v) { __builtin_nontemporal_store(v, p); }
// FP32 -> BF16, round to nearest even; NaN stays NaN (quieted: the upper
// half of its bits with bit 6 set).  One v_cvt_pk_bf16_f32: on MI355X it
// gives exactly that result for every one of the 2^32 FP32 bit patterns,
// where the same rounding done with integer operations took five or six
// instructions per value.
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, __bf16(f)); }
__device__ __forceinline__ void st(bf16* p, float v) { __builtin_nontemporal_store(f2bf(v), &p->bits); }
// Write-only passes (a level's whole-grid write, the coarse-level sweeps)
// keep ordinary stores: on MI355X a pure write stream runs faster with them
// (5.6 against 4.5 TB/s), while streams that also read gain from streaming
// stores.
__device__ __forceinline__ void st_w(double* p, double v) { *p = v; }
__device__ __forceinline__ void st_w(float* p, float v) { *p = v; }
__device__ __forceinline__ void st_w(bf16* p, float v) { p->bits = f2bf(v); }
// u += v on the caller's FP64 array (the last iteration of a cycle).
__device__ __forceinline__ void add_to(double* p, double v) { __builtin_nontemporal_store(*p + v, p); }

// Value as it reads back after a store in storage type T.
template <typename T> __device__ __forceinline__ typename Tr<T>::C rnd(typename Tr<T>::C v) { return v; }
template <> __device__ __forceinline__ float rnd<bf16>(float v) {
  return __uint_as_float(uint32_t(f2bf(v)) << 16);
}

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

// Damped Jacobi for -div(a grad) at a lattice node: c + w (h_l^2 r - flux) / sum_a
// with face coefficients the harmonic means of the nodal coefficient
// (w = omega here).  Neighbours in the order -x, +x, -y, +y.
template <typename C>
__device__ __forceinline__ C relax_var(C c, C xm, C xp, C ym, C yp, double ac, double axm,
                                       double axp, double aym, double ayp, C r, C w, C hl2) {
  const C cxm = C(harm(ac, axm)), cxp = C(harm(ac, axp));
  const C cym = C(harm(ac, aym)), cyp = C(harm(ac, ayp));
  const C sa = (cxm + cxp) + (cym + cyp);
  const C flux = fmac(cxm, c - xm, cxp * (c - xp)) + fmac(cym, c - ym, cyp * (c - yp));
  return fmac(w / sa, fmac(hl2, r, -flux), c);
}

// Linear interpolation a + t (b - a), t in [0, 1).
template <typename C>
__device__ __forceinline__ C lerp(C a, C b, C t) { return fmac(t, b - a, a); }

// ------------------------------------------------------------ lane exchange
// The value of the previous / next lane of the wave (lane i gets lane i - 1
// / i + 1) by a DPP wave shift (a VALU move; no LDS round trip as with
// __shfl_up / __shfl_down).  The lane at the wave's end reads 0; every
// caller discards what those lanes compute.
__device__ __forceinline__ int dpp_prev(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true);  // wave_shr:1
}
__device__ __forceinline__ int dpp_next(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true);  // wave_shl:1
}
__device__ __forceinline__ float lane_prev(float v) { return __int_as_float(dpp_prev(__float_as_int(v))); }
__device__ __forceinline__ float lane_next(float v) { return __int_as_float(dpp_next(__float_as_int(v))); }
__device__ __forceinline__ double lane_prev(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = unsigned(dpp_prev(int(b))), hi = unsigned(dpp_prev(int(b >> 32)));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double lane_next(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = unsigned(dpp_next(int(b))), hi = unsigned(dpp_next(int(b >> 32)));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// The same shifts where the end lane takes `edge` instead: the DPP move
// leaves a lane without a source lane at its old value (bound_ctrl off), so
// no lane-dependent select follows the shift (the compiler may turn such a
// select into a branch that runs the shift with the end lane switched off,
// and an inactive source lane reads 0).
__device__ __forceinline__ double lane_prev_or(double edge, double v) {
  const long long b = __double_as_longlong(v), e = __double_as_longlong(edge);
  const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(int(e), int(b), 0x138, 0xf, 0xf, false));
  const unsigned hi = unsigned(__builtin_amdgcn_update_dpp(int(e >> 32), int(b >> 32), 0x138, 0xf, 0xf, false));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double lane_next_or(double edge, double v) {
  const long long b = __double_as_longlong(v), e = __double_as_longlong(edge);
  const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(int(e), int(b), 0x130, 0xf, 0xf, false));
  const unsigned hi = unsigned(__builtin_amdgcn_update_dpp(int(e >> 32), int(b >> 32), 0x130, 0xf, 0xf, false));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float lane_prev_or(float edge, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_next_or(float edge, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130, 0xf, 0xf, false));
}

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

constexpr int BX2 = 256;          // 2D: lanes per block
// 2D tiles: a block's four waves take TW2 = 64 columns each on four
// consecutive bands of `len` rows (wave w of block row `by` walks band
// 4 by + w), so the waves of one block write different rows.  Measured on
// MI355X with a padded 4097^2 FP64 array: a pure write stream runs at 5.9
// TB/s this way against 4.2 TB/s with the four waves side by side on the
// same rows, and a two-read one-write stream with streaming stores at 7.8
// against 6.9 TB/s.
constexpr int TW2 = 64;
__device__ __forceinline__ int t2_x(int bx) { return 1 + bx * TW2 + int(threadIdx.x & 63); }
__device__ __forceinline__ int t2_y0(int by, int len) { return 1 + (by * 4 + int(threadIdx.x >> 6)) * len; }
__host__ __device__ inline int t2_gx(int n) { return (n - 2 + TW2 - 1) / TW2; }
__host__ __device__ inline int t2_gy(int n, int len) { return (n - 2 + 4 * len - 1) / (4 * len); }
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
  (void)walks;
  if (d == 2) return dim3(t2_gx(n), t2_gy(n, len), 1);
  return dim3((inner + BX3 - 1) / BX3, (inner + BY3 - 1) / BY3, walks);
}

// The fused 2D residual + restriction (k_residual_restrict_2d): owned
// columns per wave, waves for a band length, and its band length -- the
// longest even band of at most 32 rows that still gives 4096 waves (else 2
// rows), lengthened while that keeps the same number of full rounds of
// resident waves (MI355X: 256 CUs x 32 waves), so that no short last round
// of waves runs alone.
constexpr int RR_W = 62;
constexpr int RR_SLOTS = 256 * 32;
static int rr_waves(int n, int len) {
  return ((n - 2 + RR_W - 1) / RR_W) * ((n - 2 + len - 1) / len);
}
static int rr_band(int n) {
  int len = 2;
  for (int l : {32, 16, 8, 4})
    if (rr_waves(n, l) >= 4096) {
      len = l;
      break;
    }
  const int rounds = rr_waves(n, len) / RR_SLOTS;
  if (rounds >= 1)
    while (rr_waves(n, len) > rounds * RR_SLOTS) len += 2;
  return len;
}

int partials_bound(int d, int n) {
  if (n < 3) return 1;
  dim3 g = grid_of(d, n, walk_len(d, n));
  int64_t count = int64_t(g.x) * g.y * g.z;
  if (d == 2) {  // the fused residual + restriction: one partial per wave
    const int64_t w = rr_waves(n, rr_band(n));
    if (w > count) count = w;
  }
  if (d == 3) {  // the 3D residual's grid: 4 rows per lane, walks of 8 planes
    const int64_t inner = n - 2, len3 = inner < 8 ? inner : 8;
    const int64_t c3 = ((inner + BX3 - 1) / BX3) * ((inner + 4 * BY3 - 1) / (4 * BY3)) * ((inner + len3 - 1) / len3);
    if (c3 > count) count = c3;
  }
  return int(count);
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

// Workgroups of a launch are dealt to the 8 XCDs round-robin (workgroup h
// runs on XCD h % 8).  xcd_order maps h to a logical index so that each XCD
// receives one contiguous range of logical workgroups (a bijection on
// [0, count)).
__device__ __forceinline__ unsigned xcd_order(unsigned h, unsigned count) {
  const unsigned q = count / 8, rem = count % 8, x = h % 8;
  return x * q + min(x, rem) + h / 8;
}

// ------------------------------------------------------------ norm of f

__device__ __forceinline__ void tile_norm2_2d(const double* __restrict__ f, int64_t fp, int n,
                                                  int len, double* __restrict__ partials, int bx, int by, int pidx) {
  const int x = t2_x(bx);
  const int y0 = t2_y0(by, len);
  const int y1 = min(n - 1, y0 + len);
  double s = 0.0;
  if (x <= n - 2)
    for (int y = y0; y < y1; ++y) {
      double v = f[int64_t(y) * fp + x];
      s = fmac(v, v, s);
    }
  s = block_sum<256>(s);
  if (threadIdx.x == 0) partials[pidx] = s;
}

__global__ __launch_bounds__(256) void k_norm2_2d(const double* __restrict__ f, int64_t fp, int n,
                                                  int len, double* __restrict__ partials) {
  tile_norm2_2d(f, fp, n, len, partials, blockIdx.x, blockIdx.y, blockIdx.y * gridDim.x + blockIdx.x);
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
__device__ __forceinline__ void tile_residual_2d(
    const double* __restrict__ u, int64_t up, const double* __restrict__ f, int64_t fp,
    const double* __restrict__ a, int64_t ap, T* __restrict__ r, int64_t rp, int n, int len,
    double inv_h2, double* __restrict__ partials, int bx, int by, int pidx) {
  const int x = t2_x(bx);
  const int y0 = t2_y0(by, len);
  const int y1 = min(n - 1, y0 + len);
  double s = 0.0;
  if (x <= n - 2 && y0 <= n - 2) {
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
  if (threadIdx.x == 0) partials[pidx] = s;
}

template <typename T, bool VAR>
__global__ __launch_bounds__(256) void k_residual_2d(
    const double* __restrict__ u, int64_t up, const double* __restrict__ f, int64_t fp,
    const double* __restrict__ a, int64_t ap, T* __restrict__ r, int64_t rp, int n, int len,
    double inv_h2, double* __restrict__ partials, const int* __restrict__ done) {
  if (*done) return;
  tile_residual_2d<T, VAR>(u, up, f, fp, a, ap, r, rp, n, len, inv_h2, partials, blockIdx.x, blockIdx.y, blockIdx.y * gridDim.x + blockIdx.x);
}

// 3D residual: a lane owns R3Y consecutive y rows (as the level-0 sweep),
// walks of RES3_LEN planes.  The x neighbours come from the neighbour lanes
// (DPP wave shifts; lanes past the grid hold the boundary column); only
// lanes 0 and 63 load the column just outside the tile.  The grid is 1D and
// XCD-ordered (x tiles fastest, then y, then z), so the tiles that share
// halo rows and cache lines run on the same XCD and its L2.
constexpr int RES3_LEN = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_residual_3d(
    const double* __restrict__ u, int64_t up, int64_t upl, const double* __restrict__ f,
    int64_t fp, int64_t fpl, T* __restrict__ r, int64_t rp, int64_t rpl, int n, int len,
    double inv_h2, double* __restrict__ partials, const int* __restrict__ done) {
  if (*done) return;
  constexpr int R = 4;  // = R3Y (declared with the sweeps below)
  const int gx = (n - 2 + BX3 - 1) / BX3, gy = (n - 2 + BY3 * R - 1) / (BY3 * R);
  const int lg = int(xcd_order(blockIdx.x, gridDim.x));
  const int bx = lg % gx, by = (lg / gx) % gy, bz = lg / (gx * gy);
  const int lane = threadIdx.x;
  const int x = 1 + bx * BX3 + lane;
  const int yb = 1 + (by * BY3 + __builtin_amdgcn_readfirstlane(int(threadIdx.y))) * R;
  const int z0 = 1 + bz * len;
  const int z1 = min(n - 1, z0 + len);
  const bool xin = x <= n - 2;
  const int xc = min(x, n - 1);
  const bool edge = lane == 0 || lane == BX3 - 1;
  const int xe = lane == 0 ? x - 1 : min(x + 1, n - 1);  // the edge lanes' outside column
  double s = 0.0;
  if (yb <= n - 2) {
    double c[R], zm[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int64_t col = int64_t(min(yb + k, n - 2)) * up + xc;
      zm[k] = u[int64_t(z0 - 1) * upl + col];
      c[k] = u[int64_t(z0) * upl + col];
    }
    const int64_t ylo = int64_t(yb - 1) * up + xc;
    const int64_t yhi = int64_t(min(yb + R, n - 1)) * up + xc;
    for (int z = z0; z < z1; ++z) {
      double zp[R], fv[R], ev[R];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int yk = min(yb + k, n - 2);
        const double* q = u + int64_t(z) * upl + int64_t(yk) * up;
        zp[k] = q[upl + xc];
        fv[k] = f[int64_t(z) * fpl + int64_t(yk) * fp + xc];
        ev[k] = 0.0;
        if (edge) ev[k] = q[xe];
      }
      const double below = u[int64_t(z) * upl + ylo];
      const double above = u[int64_t(z) * upl + yhi];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        // u's boundary rows carry the Dirichlet data, so the row above the
        // last interior row is read from memory, never assumed 0
        const double ym = k == 0 ? below : c[k - 1];
        const double yp = k == R - 1 ? above : (yb + k + 1 <= n - 2 ? c[k + 1] : u[int64_t(z) * upl + int64_t(n - 1) * up + xc]);
        const double xm = lane_prev_or(ev[k], c[k]);  // lane 0: ev
        const double xp = lane_next_or(ev[k], c[k]);  // lane 63: ev
        const double au = fmac(6.0, c[k], -(((xm + xp) + (ym + yp)) + (zm[k] + zp[k])));
        const double rv = fmac(-inv_h2, au, fv[k]);
        if (xin && yb + k <= n - 2) {
          st(r + int64_t(z) * rpl + int64_t(yb + k) * rp + x, typename Tr<T>::C(rv));
          s = fmac(rv, rv, s);
        }
      }
#pragma unroll
      for (int k = 0; k < R; ++k) {
        zm[k] = c[k];
        c[k] = zp[k];
      }
    }
  }
  s = block_sum<256>(s);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[lg] = s;
}

// 2D residual with the restriction to level 1 fused in.  Each wave walks a
// band of rows over 64 columns and owns the inner 62 (lanes 1..62; lane 63
// is a halo whose residual only feeds the restriction, lane 0 idles); it
// also computes the first row of the next band, so that every level-1 node
// whose fine rows start in the band (x = 2I on an owned even column, y = 2J
// with 2J - 1 in the band) finds its 3 x 3 fine residuals in the wave: the
// x neighbours by lane shuffles, the rows in a three-row window.  The fine
// residual is rounded to T before it is restricted, as the separate
// restriction would read it back, and the weights and their order are
// those of tile_restrict_2d.
template <typename T>
__global__ __launch_bounds__(256) void k_residual_restrict_2d(
    const double* __restrict__ u, int64_t up, const double* __restrict__ f, int64_t fp,
    T* __restrict__ r, int64_t rp, T* __restrict__ rc, int64_t cp, int n, int len, double inv_h2,
    double* __restrict__ partials, const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  const int wv = __builtin_amdgcn_readfirstlane(int(xcd_order(blockIdx.x, gridDim.x)) * 4 +
                                                int(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int gx = (n - 2 + RR_W - 1) / RR_W;
  // (the four waves of a workgroup side by side on the same band measured
  // faster here than on four bands: 87 against 103 us at 4097^2)
  if (wv >= gx * ((n - 2 + len - 1) / len)) return;  // the whole wave
  const int pidx = wv;
  const int x = (wv % gx) * RR_W + lane;
  const int Y0 = 1 + (wv / gx) * len, Y1 = min(n - 1, Y0 + len);  // len even: Y0 odd
  const bool xin = x >= 1 && x <= n - 2;
  const bool own = xin && lane >= 1 && lane <= RR_W;
  const bool emit = (x & 1) == 0 && lane >= 2 && lane <= RR_W && x <= n - 3;
  const int xc = min(x, n - 1);
  double ym = u[int64_t(Y0 - 1) * up + xc], c = u[int64_t(Y0) * up + xc];
  C rs2 = C(0), rs1 = C(0);  // row sums of rows y - 2, y - 1
  double s = 0.0;
  const int ylast = min(Y1, n - 2);  // the next band's first row, if interior
  for (int y = Y0; y <= ylast; ++y) {
    const double* row = u + int64_t(y) * up;
    const double yp = row[up + xc];
    // x neighbours from the neighbour lanes (lane 0's own residual is not
    // used); lane 63's right neighbour lies past the wave
    const double xm = __shfl_up(c, 1);
    double xp = __shfl_down(c, 1);
    if (lane == 63) xp = row[min(xc + 1, n - 1)];
    const double au = fmac(4.0, c, -((xm + xp) + (ym + yp)));
    const double rv = fmac(-inv_h2, au, f[int64_t(y) * fp + xc]);
    const C rt = xin ? rnd<T>(C(rv)) : C(0);
    if (own && y < Y1) {
      st(r + int64_t(y) * rp + x, C(rv));
      s = fmac(rv, rv, s);
    }
    const C rs = fmac(C(2), rt, __shfl_up(rt, 1) + __shfl_down(rt, 1));
    if ((y & 1) && y >= Y0 + 2 && emit)  // y = 2J + 1: level-1 node (x / 2, J) complete
      st(rc + int64_t(y >> 1) * cp + (x >> 1), fmac(C(2), rs1, rs2 + rs) * C(0.0625));
    rs2 = rs1;
    rs1 = rs;
    ym = c;
    c = yp;
  }
  s = wave_sum(s);
  if (lane == 0) partials[pidx] = s;
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

// One workgroup of 1024 lanes (a per-wave partial count of ~8k, as the
// fused 2D residual gives at 4097^2, is then 8 loads per lane).
constexpr int FIN_NT = 1024;
__global__ __launch_bounds__(FIN_NT) void k_finalize(const double* __restrict__ partials, int count,
                                                     DevState* st, double* __restrict__ history,
                                                     int cycle, int mode) {
  if (mode == 1 && st->done) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += FIN_NT) s += partials[i];
  s = block_sum<FIN_NT>(s);
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

// ------------------------------------------------------------ L1 error
// The normalised L1 error of Sec. 4 in its discrete form, sum |u_ref - v| /
// sum |u_ref| over all nodes, with v = u (+ e, an internal iterate in its
// storage type and padded layout, when given).  A fixed grid of L1_BLOCKS
// workgroups walks the rows; each writes its two partial sums, and one
// workgroup adds them in a fixed order -- the result does not depend on
// timing.
constexpr int L1_BLOCKS = 1024;
constexpr int P2_ROWS = 8;  // rows walked per block by the power-of-two sweep

template <typename T, bool HAS_E>
__global__ __launch_bounds__(256) void k_l1_partial(const double* __restrict__ uref, const double* __restrict__ u,
                                                    const T* __restrict__ e, int64_t ep, int64_t epl, int n,
                                                    int d, double* __restrict__ part) {
  const int64_t rows = d == 3 ? int64_t(n) * n : int64_t(n);
  double s1 = 0.0, s2 = 0.0;
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const int64_t j = d == 3 ? row % n : row, k = d == 3 ? row / n : 0;
    const int64_t o = row * n;
    for (int i = threadIdx.x; i < n; i += 256) {
      double v = u[o + i];
      if (HAS_E) v += double(ld(e + k * epl + j * ep + i));
      const double a = uref[o + i];
      s1 += fabs(a - v);
      s2 += fabs(a);
    }
  }
  s1 = block_sum<256>(s1);
  __syncthreads();
  s2 = block_sum<256>(s2);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1;
    part[2 * blockIdx.x + 1] = s2;
  }
}

__global__ __launch_bounds__(256) void k_l1_finish(const double* __restrict__ part, int nb, double* __restrict__ out) {
  double s1 = 0.0, s2 = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    s1 += part[2 * b];
    s2 += part[2 * b + 1];
  }
  s1 = block_sum<256>(s1);
  __syncthreads();
  s2 = block_sum<256>(s2);
  if (threadIdx.x == 0) *out = s2 > 0.0 ? s1 / s2 : s1;
}

// ------------------------------------------------------------ restriction
// Full weighting (Sec. 2: linearly weighted averages as nested partial
// reductions): coarse node = (1/4)[1 2 1] per axis of the fine neighbours.

// TO: the coarse level's storage type, whose arithmetic the restriction
// uses; TI (the fine level's) is TO except for the restriction to an FP64
// coarsest level of a reduced-precision cycle, which widens the stored
// values exactly and sums in FP64.
template <typename TI, typename TO = TI>
__device__ __forceinline__ void tile_restrict_2d(const TI* __restrict__ rf, int64_t fp,
                                                     TO* __restrict__ rc, int64_t cp, int nc,
                                                     int len, int bx, int by) {
  using C = typename Tr<TO>::C;
  const int I = t2_x(bx);
  const int J0 = t2_y0(by, len);
  if (I > nc - 2 || J0 > nc - 2) return;
  const int J1 = min(nc - 1, J0 + len);
  const int xi = 2 * I;
  auto rowsum = [&](int yf) {
    const TI* row = rf + int64_t(yf) * fp + xi;
    return fmac(C(2), C(ld(row)), C(ld(row - 1)) + C(ld(row + 1)));
  };
  C top = rowsum(2 * J0 - 1);
  for (int J = J0; J < J1; ++J) {
    const C mid = rowsum(2 * J);
    const C bot = rowsum(2 * J + 1);
    st(rc + int64_t(J) * cp + I, fmac(C(2), mid, top + bot) * C(0.0625));
    top = bot;
  }
}

template <typename TI, typename TO = TI>
__global__ __launch_bounds__(256) void k_restrict_2d(const TI* __restrict__ rf, int64_t fp,
                                                     TO* __restrict__ rc, int64_t cp, int nc,
                                                     int len, const int* __restrict__ done) {
  if (*done) return;
  tile_restrict_2d<TI, TO>(rf, fp, rc, cp, nc, len, blockIdx.x, blockIdx.y);
}

template <typename TI, typename TO = TI>
__global__ __launch_bounds__(256) void k_restrict_3d(const TI* __restrict__ rf, int64_t fp,
                                                     int64_t fpl, TO* __restrict__ rc, int64_t cp,
                                                     int64_t cpl, int nc, int len,
                                                     const int* __restrict__ done) {
  using C = typename Tr<TO>::C;
  if (*done) return;
  const int I = 1 + blockIdx.x * BX3 + threadIdx.x;
  const int J = 1 + blockIdx.y * BY3 + threadIdx.y;
  if (I > nc - 2 || J > nc - 2) return;
  const int K0 = 1 + blockIdx.z * len;
  const int K1 = min(nc - 1, K0 + len);
  const int64_t col = int64_t(2 * J) * fp + 2 * I;
  auto planesum = [&](int zf) {
    const TI* p = rf + int64_t(zf) * fpl + col;
    auto rs = [&](const TI* q) { return fmac(C(2), C(ld(q)), C(ld(q - 1)) + C(ld(q + 1))); };
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

template <typename T, int MODE, bool VAR, bool WRITE_ONLY = false>
__device__ __forceinline__ void emit_2d(T* en, int64_t eoff, double* u, int64_t uoff,
                                        typename Tr<T>::C v) {
  if (MODE & SW_ACCUM) {
    add_to(u + uoff, double(v));
  } else if (WRITE_ONLY) {
    st_w(en + eoff, v);
  } else {
    st(en + eoff, v);
  }
}

// Level 0: every interior node relaxes (plain damped Jacobi).  The walk
// takes U rows per step and issues all their loads before any arithmetic,
// so each lane keeps several rows of memory traffic in flight.  Constant
// coefficient: the x neighbours come from the neighbour lanes (DPP wave
// shifts; the wave is 64 consecutive columns), the end lanes load their
// outside column; lanes past the last interior column (xc clamped) walk
// along and store nothing.
template <typename T, int MODE, bool VAR, int U>
__device__ __forceinline__ void rows_2d_l0(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, const T* __restrict__ r,
    int64_t rp, const double* __restrict__ a, int64_t ap, double* __restrict__ u, int64_t up,
    int x, int xc, int xe, bool edge, bool xin, int y, typename Tr<T>::C w, typename Tr<T>::C hl2,
    typename Tr<T>::C& ym, typename Tr<T>::C& c, double& aym, double& ac) {
  using C = typename Tr<T>::C;
  C rv[U], xm[U], xp[U], yp[U], ev[U];
  double axm[U], axp[U], ayp[U];
#pragma unroll
  for (int k = 0; k < U; ++k) {
    rv[k] = ld(r + int64_t(y + k) * rp + xc);
    xm[k] = xp[k] = yp[k] = ev[k] = C(0);
    if (!(MODE & SW_ZERO_OLD)) {
      const T* row = eo + int64_t(y + k) * ep;
      yp[k] = ld(row + ep + xc);
      if (VAR) {
        xm[k] = ld(row + x - 1);
        xp[k] = ld(row + x + 1);
      } else if (edge) {
        ev[k] = ld(row + xe);
      }
    }
    if (VAR) {
      const double* arow = a + int64_t(y + k) * ap;
      ayp[k] = arow[ap + x];
      axm[k] = arow[x - 1];
      axp[k] = arow[x + 1];
    }
  }
#pragma unroll
  for (int k = 0; k < U; ++k) {
    C v;
    if (VAR) {
      v = relax_var<C>(c, xm[k], xp[k], ym, yp[k], ac, axm[k], axp[k], aym, ayp[k], rv[k], w, hl2);
      aym = ac;
      ac = ayp[k];
    } else {
      const C xl = lane_prev_or(ev[k], c), xr = lane_next_or(ev[k], c);  // lane 0 / 63: ev
      v = relax_const<C>(c, (xl + xr) + (ym + yp[k]), rv[k], w, hl2, C(4));
    }
    if (xin) emit_2d<T, MODE, VAR>(en, int64_t(y + k) * ep + x, u, int64_t(y + k) * up + x, v);
    ym = c;
    c = yp[k];
  }
}

template <typename T, int MODE, bool VAR>
__device__ __forceinline__ void tile_sweep_2d_l0(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, const T* __restrict__ r,
    int64_t rp, const double* __restrict__ a, int64_t ap, double* __restrict__ u, int64_t up,
    int n, int len, typename Tr<T>::C w, typename Tr<T>::C hl2, int bx, int by) {
  using C = typename Tr<T>::C;
  const int x = t2_x(bx);
  const int y0 = t2_y0(by, len);
  // (the last block row may hold empty bands; with a variable coefficient
  // the lanes past the grid leave too, the x neighbours being loaded)
  if (y0 > n - 2 || (VAR && x > n - 2)) return;
  const int y1 = min(n - 1, y0 + len);
  const bool xin = x <= n - 2;
  const int xc = min(x, n - 1);
  const int lane = threadIdx.x & 63;
  const bool edge = lane == 0 || lane == 63;
  const int xe = lane == 0 ? x - 1 : min(x + 1, n - 1);
  C ym = C(0), c = C(0);
  if (!(MODE & SW_ZERO_OLD)) {
    ym = ld(eo + int64_t(y0 - 1) * ep + xc);
    c = ld(eo + int64_t(y0) * ep + xc);
  }
  double aym = 0.0, ac = 0.0;
  if (VAR) {
    aym = a[int64_t(y0 - 1) * ap + x];
    ac = a[int64_t(y0) * ap + x];
  }
  constexpr int U = 4;
  int y = y0;
  for (; y + U <= y1; y += U)
    rows_2d_l0<T, MODE, VAR, U>(eo, en, ep, r, rp, a, ap, u, up, x, xc, xe, edge, xin, y, w, hl2, ym, c, aym, ac);
  for (; y < y1; ++y)
    rows_2d_l0<T, MODE, VAR, 1>(eo, en, ep, r, rp, a, ap, u, up, x, xc, xe, edge, xin, y, w, hl2, ym, c, aym, ac);
}

template <typename T, int MODE, bool VAR>
__global__ __launch_bounds__(256) void k_sweep_2d_l0(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, const T* __restrict__ r,
    int64_t rp, const double* __restrict__ a, int64_t ap, double* __restrict__ u, int64_t up,
    int n, int len, typename Tr<T>::C w, typename Tr<T>::C hl2, const int* __restrict__ done) {
  if (*done) return;
  // one-dimensional grid in XCD order: the walks of one XCD form one band of
  // rows, so the rows shared by vertically adjacent walks stay in its L2
  const unsigned lg = xcd_order(blockIdx.x, gridDim.x);
  const int gx = t2_gx(n);
  tile_sweep_2d_l0<T, MODE, VAR>(eo, en, ep, r, rp, a, ap, u, up, n, len, w, hl2, int(lg % gx), int(lg / gx));
}

// Level 1's final state seen from level 0 (chained path): the value the
// level-1 whole-grid write would leave at a level-0 node, computed from the
// compact arrays instead of read back from a whole grid.  Lattice nodes
// (every index even) take x_it, every other interior node the multilinear
// interpolant of x_{it-1} over its level-1 cell, boundary nodes 0; the
// formula, its order of operations and the rounding to T are those of the
// whole-grid write (k_level_write_2d/3d with m = 1), so both give the same
// bits.  The compact lattice of level m sits in that of level m + 1 the
// same way (and the hand-over kernels and the coarse tail evaluate the same
// formula), so the passes over a compact lattice use it too: "level 1" is
// then level m + 1 and "level 0" level m.
template <typename T>
struct L1Src {
  const T* prev;    // x_{it-1}, unread when zero_old
  const T* cur;     // x_it
  int64_t cp, cpl;  // compact row pitch, plane pitch
  int zero_old;
};

// One lane's column (2D): node x, rows visited in increasing order.  The
// x-interpolants of the two level-1 rows around the current row are kept
// and shifted as the walk enters the next level-1 row.
template <typename T>
struct L1Col2 {
  using C = typename Tr<T>::C;
  const T* p;
  const T* q;
  int64_t cp;
  int I, band;
  C tx, top, bot;
  bool live, latx, zold;
  __device__ __forceinline__ void init(const L1Src<T>& s, int x, int n) {
    live = x >= 1 && x <= n - 2;
    latx = (x & 1) == 0;
    I = live ? x >> 1 : 0;
    tx = C(x & 1) * (C(1) / C(2));
    p = s.prev;
    q = s.cur;
    cp = s.cp;
    zold = s.zero_old != 0;
    band = -2;
    top = bot = C(0);
  }
  __device__ __forceinline__ C xl(int J) const {
    if (zold) return lerp(C(0), C(0), tx);
    const T* a = p + int64_t(J) * cp + I;
    return lerp(ld(a), ld(a + 1), tx);
  }
  // Rows ys..ys+3 of a walk in steps of four rows (ys keeps its parity, so
  // the level-1 rows advance by two per step): the x-interpolants of level-1
  // rows j0, j0+1 come from the previous step (prime() before the first),
  // rows j0+2, j0+3 are loaded, with no branch between the loads.
  C w0, w1;
  __device__ __forceinline__ void prime(int ys, int n) {
    const int j0 = ys >> 1, nm1 = (n - 1) >> 1;
    w0 = xl(min(j0, nm1));
    w1 = xl(min(j0 + 1, nm1));
  }
  __device__ __forceinline__ void rows4(int ys, int n, C (&v)[4]) {
    const int j0 = ys >> 1, nm1 = (n - 1) >> 1;
    const bool odd = (ys & 1) != 0;
    // rows past the lattice only feed rows off the grid
    const C x2 = xl(min(j0 + 2, nm1)), x3 = xl(min(j0 + 3, nm1));
    C qv[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) qv[e] = ld(q + int64_t(min(j0 + int(odd) + e, nm1)) * cp + I);
    const C h = C(1) / C(2);
    // row k lies in level-1 row j0 + (k + odd) / 2; its even rows are k = odd, odd + 2
    const C t[4] = {lerp(w0, w1, C(ys & 1) * h),
                    odd ? lerp(w1, x2, C((ys + 1) & 1) * h) : lerp(w0, w1, C((ys + 1) & 1) * h),
                    lerp(w1, x2, C((ys + 2) & 1) * h),
                    odd ? lerp(x2, x3, C((ys + 3) & 1) * h) : lerp(w1, x2, C((ys + 3) & 1) * h)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int y = ys + k;
      const C val = (latx && (y & 1) == 0) ? qv[k >> 1] : t[k];
      v[k] = (live && y >= 1 && y <= n - 2) ? rnd<T>(val) : C(0);
    }
    w0 = x2;
    w1 = x3;
  }
  __device__ __forceinline__ C at(int y, int n) {
    if (!live || y < 1 || y > n - 2) return C(0);
    const int J = y >> 1;
    if (J != band) {
      top = J == band + 1 ? bot : xl(J);
      bot = xl(J + 1);
      band = J;
    }
    const C v = (latx && (y & 1) == 0) ? ld(q + int64_t(J) * cp + I)
                                       : lerp(top, bot, C(y & 1) * (C(1) / C(2)));
    return rnd<T>(v);
  }
};

// One lane's R consecutive rows yb.. of one x (3D), planes visited in
// increasing order.  Per level-1 plane the lane forms the x-interpolants of
// the (at most four) level-1 rows its rows touch, then each row's
// y-interpolant; the two planes around the current plane are kept.  yb is
// the same for the whole wave, so everything derived from it stays scalar.
template <typename T, int R>
struct L1Col3 {
  using C = typename Tr<T>::C;
  const T* p;
  const T* q;
  int64_t cp, cpl;
  int I, yb, n, band;
  bool xin, xeven, zold;
  C top[R], bot[R];
  __device__ __forceinline__ void init(const L1Src<T>& s, int x, int yb_, int n_) {
    static_assert(R == 4, "four rows per lane");
    n = n_;
    yb = __builtin_amdgcn_readfirstlane(yb_);
    xin = x >= 1 && x <= n - 2;
    xeven = (x & 1) == 0;
    I = xin ? x >> 1 : 0;
    p = s.prev;
    q = s.cur;
    cp = s.cp;
    cpl = s.cpl;
    zold = s.zero_old != 0;
    band = -2;
#pragma unroll
    for (int k = 0; k < R; ++k) top[k] = bot[k] = C(0);
  }
  __device__ __forceinline__ C tx() const { return xeven ? C(0) : C(1) / C(2); }
  // y-interpolants of the lane's rows on level-1 plane K
  __device__ __forceinline__ void plane(int K, C (&out)[R]) const {
    const int j0 = yb >> 1, nm1 = (n - 1) >> 1;  // arithmetic shift: yb may be -1
    const bool odd = (yb & 1) != 0;
    C xv[R];
    if (zold) {
#pragma unroll
      for (int d = 0; d < R; ++d) xv[d] = lerp(C(0), C(0), tx());
    } else {
      // the uniform test stays outside the row loop, so the rows' loads
      // are issued together
      C a0[R], a1[R];
#pragma unroll
      for (int d = 0; d < R; ++d) {
        // rows past the lattice only feed rows off the grid
        const int J = min(max(j0 + d, 0), nm1);
        const T* a = p + int64_t(K) * cpl + int64_t(J) * cp + I;
        a0[d] = ld(a);
        a1[d] = ld(a + 1);
      }
#pragma unroll
      for (int d = 0; d < R; ++d) xv[d] = lerp(a0[d], a1[d], tx());
    }
    // row k lies in level-1 row j0 + (k + odd) / 2
    const C h = C(1) / C(2);
    out[0] = lerp(xv[0], xv[1], C(yb & 1) * h);
    out[1] = odd ? lerp(xv[1], xv[2], C((yb + 1) & 1) * h) : lerp(xv[0], xv[1], C((yb + 1) & 1) * h);
    out[2] = lerp(xv[1], xv[2], C((yb + 2) & 1) * h);
    out[3] = odd ? lerp(xv[2], xv[3], C((yb + 3) & 1) * h) : lerp(xv[1], xv[2], C((yb + 3) & 1) * h);
  }
  __device__ __forceinline__ void at(int z, C (&v)[R]) {
    if (z < 1 || z > n - 2) {
#pragma unroll
      for (int k = 0; k < R; ++k) v[k] = C(0);
      return;
    }
    const int K = z >> 1;
    // x_it at the lane's lattice position of each row, loaded for every
    // lane (the index is in range for all) and kept only at level-1
    // lattice nodes: no divergent branch around the loads
    C lat[R];
#pragma unroll
    for (int k = 0; k < R; ++k)
      lat[k] = ld(q + int64_t(K) * cpl + int64_t(min(max((yb + k) >> 1, 0), (n - 1) >> 1)) * cp + I);
    if (K != band) {
      if (K == band + 1) {
#pragma unroll
        for (int k = 0; k < R; ++k) top[k] = bot[k];
      } else {
        plane(K, top);
      }
      plane(K + 1, bot);
      band = K;
    }
    const C tz = C(z & 1) * (C(1) / C(2));
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int y = yb + k;
      const bool node = xeven && (y & 1) == 0 && (z & 1) == 0;  // a level-1 lattice node
      const C t = node ? lat[k] : lerp(top[k], bot[k], tz);
      v[k] = (xin && y >= 1 && y <= n - 2) ? rnd<T>(t) : C(0);
    }
  }
};

// Level 0, IT <= 4 iterations in one pass (temporal blocking).  Each wave
// owns 64 consecutive columns and walks a band of rows; the
// iterations form a pipeline down the band: iteration t is computed t rows
// behind the row just loaded, from a three-row window of iteration t-1 in
// registers (the y neighbours) and the neighbour lanes' values (the x
// neighbours, by cross-lane shuffles).  A lane's value after t iterations is
// only right if both neighbours' values after t-1 were, so the valid lanes
// shrink by one per iteration at each wave edge: a wave emits its inner
// 64 - 2 IT columns and waves overlap by 2 IT columns; the band is entered
// IT rows early and left IT rows late for the same reason.  Every
// intermediate iterate is rounded as a store would round it, and the last
// one goes to memory exactly as the single-iteration kernel sends it, so
// the result equals IT single sweeps bit for bit while e and r are read
// once and the result written (or added into u) once.

template <typename T, bool ZERO, bool ACCUM, bool PREV, int IT, int U, bool LAT>
__device__ __forceinline__ void tb_steps(const T* __restrict__ eo, T* __restrict__ en,
                                         T* __restrict__ eprev, int64_t ep,
                                         const T* __restrict__ r, int64_t rp, double* __restrict__ u,
                                         int64_t up, int n, int x, int xc, bool xin, bool emit, int Y0,
                                         int Y1, int ys, typename Tr<T>::C w, typename Tr<T>::C hl2,
                                         typename Tr<T>::C (&win)[IT][3], typename Tr<T>::C (&rw)[IT + 1],
                                         L1Col2<T>& lc) {
  using C = typename Tr<T>::C;
  C xl[U], rl[U];
  double uo[U];
#pragma unroll
  for (int k = 0; k < U; ++k) {  // rows past the grid read the boundary row (zero)
    rl[k] = ld(r + int64_t(min(max(ys + k - 1, 0), n - 1)) * rp + xc);
    if (!LAT) xl[k] = ZERO ? C(0) : ld(eo + int64_t(min(ys + k, n - 1)) * ep + xc);
    // the old value of the u entry emitted at step k (row ys + k - IT),
    // loaded with the rows; lanes and steps that emit nothing read a row
    // of the band (clamped), so the load needs no branch
    if (ACCUM) uo[k] = u[int64_t(min(max(ys + k - IT, Y0), Y1 - 1)) * up + xc];
  }
  if (LAT) {
    if constexpr (U == 4) {
      lc.rows4(ys, n, xl);
    } else {
#pragma unroll
      for (int k = 0; k < U; ++k) xl[k] = lc.at(min(ys + k, n - 1), n);
    }
  }
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const int y0 = ys + k;
    win[0][0] = win[0][1];
    win[0][1] = win[0][2];
    win[0][2] = xl[k];
#pragma unroll
    for (int t = IT; t > 1; --t) rw[t] = rw[t - 1];
    rw[1] = rl[k];
#pragma unroll
    for (int t = 1; t <= IT; ++t) {
      const int y = y0 - t;
      const C c = win[t - 1][1];
      const C xm = lane_prev(c), xp = lane_next(c);
      const bool in = xin && y >= 1 && y <= n - 2;
      C v = relax_const<C>(c, (xm + xp) + (win[t - 1][0] + win[t - 1][2]), rw[t], w, hl2, C(4));
      if (t < IT) {
        win[t][0] = win[t][1];
        win[t][1] = win[t][2];
        win[t][2] = in ? rnd<T>(v) : C(0);
      } else if (emit && in && y >= Y0 && y < Y1) {
        if (ACCUM)
          st(u + int64_t(y) * up + x, uo[k] + double(v));
        else
          st(en + int64_t(y) * ep + x, v);
        if (PREV) st(eprev + int64_t(y) * ep + x, c);  // the iterate before the last
      }
    }
  }
}

// Wave wv of the pass (waves numbered x-band fastest).  LAT: e comes from
// level 1's compact state (L1Src) instead of eo.
template <typename T, bool ZERO, bool ACCUM, bool PREV, int IT, bool LAT = false>
__device__ __forceinline__ void tb_body(const T* __restrict__ eo, T* __restrict__ en,
                                        T* __restrict__ eprev, int64_t ep, const T* __restrict__ r,
                                        int64_t rp, double* __restrict__ u, int64_t up, int n, int len,
                                        typename Tr<T>::C w, typename Tr<T>::C hl2, int wv,
                                        const L1Src<T>& l1 = L1Src<T>{}) {
  using C = typename Tr<T>::C;
  constexpr int VALID = 64 - 2 * IT;
  const int lane = threadIdx.x & 63;
  const int gx = (n - 2 + VALID - 1) / VALID, gy = (n - 2 + len - 1) / len;
  // wave wv: workgroup wv / 4 takes column tile (wv / 4) % gx on bands
  // 4 ((wv / 4) / gx) .. + 3, one per wave (tb_blocks)
  const int q = wv >> 2, band = (q / gx) * 4 + (wv & 3);
  if (band >= gy) return;  // the whole wave
  const int x = 1 + (q % gx) * VALID - IT + lane;
  const int Y0 = 1 + band * len, Y1 = min(n - 1, Y0 + len);
  const bool xin = x >= 1 && x <= n - 2;
  const bool emit = lane >= IT && lane < 64 - IT;
  const int xc = min(max(x, 0), n - 1);  // columns off the grid read the boundary (zero)
  C win[IT][3], rw[IT + 1];
#pragma unroll
  for (int t = 0; t < IT; ++t) win[t][0] = win[t][1] = win[t][2] = C(0);
#pragma unroll
  for (int t = 0; t <= IT; ++t) rw[t] = C(0);
  L1Col2<T> lc;
  int ys = max(Y0 - IT, 0);
  if (LAT) {
    lc.init(l1, x, n);
    lc.prime(ys, n);
  }
  const int ye = Y1 + IT;  // one past the last row loaded
  for (; ys + 4 <= ye; ys += 4)
    tb_steps<T, ZERO, ACCUM, PREV, IT, 4, LAT>(eo, en, eprev, ep, r, rp, u, up, n, x, xc, xin, emit, Y0, Y1,
                                               ys, w, hl2, win, rw, lc);
  for (; ys < ye; ++ys)
    tb_steps<T, ZERO, ACCUM, PREV, IT, 1, LAT>(eo, en, eprev, ep, r, rp, u, up, n, x, xc, xin, emit, Y0, Y1,
                                               ys, w, hl2, win, rw, lc);
}

template <typename T, bool ZERO, bool ACCUM, int IT, bool LAT>
// Five waves per SIMD: the u loads issued with the rows take the pass from
// 94 to 108 VGPRs, which would leave four waves per SIMD and a second round
// of waves at 4097^2 (4736 waves, 4096 resident); held at 96 VGPRs (12 bytes
// spilled) it runs 101 us against 115 us with the dependent reads.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_sweep_2d_l0_tb(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, const T* __restrict__ r, int64_t rp,
    double* __restrict__ u, int64_t up, int n, int len, typename Tr<T>::C w, typename Tr<T>::C hl2,
    const int* __restrict__ done, L1Src<T> l1) {
  if (*done) return;
  // XCD order: the waves of one XCD are neighbours (their overlapping
  // columns and rows meet in that XCD's L2)
  const int wv = int(xcd_order(blockIdx.x, gridDim.x)) * 4 + int(threadIdx.x >> 6);
  tb_body<T, ZERO, ACCUM, false, IT, LAT>(eo, en, nullptr, ep, r, rp, u, up, n, len, w, hl2, wv, l1);
}

// The same pass over the compact lattice of a coarse level (n = its side),
// optionally also storing the iterate before the last (PREV), which the
// level's whole-grid pass interpolates.  LAT: x_0 is the next coarser
// level's final state seen on this lattice (the compact lattice of level m
// sits in that of level m + 1 as level 0 sits in level 1).
template <typename T, bool ZERO, bool PREV, int IT, bool LAT>
__global__ __launch_bounds__(256) void k_lattice_2d_tb(
    const T* __restrict__ eo, T* __restrict__ en, T* __restrict__ eprev, int64_t ep,
    const T* __restrict__ r, int64_t rp, int n, int len, typename Tr<T>::C w, typename Tr<T>::C hl2,
    const int* __restrict__ done, L1Src<T> l1) {
  if (*done) return;
  const int wv = int(xcd_order(blockIdx.x, gridDim.x)) * 4 + int(threadIdx.x >> 6);
  tb_body<T, ZERO, false, PREV, IT, LAT>(eo, en, eprev, ep, r, rp, nullptr, 0, n, len, w, hl2, wv, l1);
}

// Levels m >= 1: lattice nodes relax, the rest interpolate.  The lane keeps
// the four corners of its current level-m cell; they change every l rows.
template <typename T, int MODE, bool VAR>
__device__ __forceinline__ void tile_sweep_2d_coarse(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, const T* __restrict__ rm,
    int64_t rp, const double* __restrict__ am, int64_t ap, double* __restrict__ u, int64_t up,
    int n, int len, int m, typename Tr<T>::C w, typename Tr<T>::C hl2, int bx, int by) {
  using C = typename Tr<T>::C;
  const int x = t2_x(bx);
  const int y0 = t2_y0(by, len);
  if (x > n - 2 || y0 > n - 2) return;
  const int l = 1 << m;
  const int mask = l - 1;
  const C inv_l = C(1) / C(l);
  const int y1 = min(n - 1, y0 + len);
  const int xa = x & ~mask, xb = xa + l;
  const C tx = C(x - xa) * inv_l;
  const bool latc = (x == xa);
  int ya = y0 & ~mask;
  // corners of the current cell's top (ya) and bottom (ya + l) rows; the
  // next cell's bottom corners are loaded one cell ahead
  C t0 = C(0), t1 = C(0), b0 = C(0), b1 = C(0), n0 = C(0), n1 = C(0);
  if (!(MODE & SW_ZERO_OLD)) {
    t0 = ld(eo + int64_t(ya) * ep + xa);
    t1 = ld(eo + int64_t(ya) * ep + xb);
    b0 = ld(eo + int64_t(ya + l) * ep + xa);
    b1 = ld(eo + int64_t(ya + l) * ep + xb);
  }
  C top = lerp(t0, t1, tx), bot = lerp(b0, b1, tx);
  for (int yc = y0; yc < y1; ya += l) {
    const int ye = min(y1, ya + l);
    if (!(MODE & SW_ZERO_OLD) && ye < y1) {
      n0 = ld(eo + int64_t(ya + 2 * l) * ep + xa);
      n1 = ld(eo + int64_t(ya + 2 * l) * ep + xb);
    }
    for (int y = yc; y < ye; ++y) {
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
          v = relax_var<C>(t0, xm, t1, ym, b0, arow[0], arow[-1], arow[1], arow[-ap], arow[ap], rv,
                           w, hl2);
        } else {
          v = relax_const<C>(t0, (xm + t1) + (ym + b0), rv, w, hl2, C(4));
        }
      } else {
        v = lerp(top, bot, C(y - ya) * inv_l);
      }
      emit_2d<T, MODE, VAR, true>(en, int64_t(y) * ep + x, u, int64_t(y) * up + x, v);
    }
    yc = ye;
    t0 = b0;
    t1 = b1;
    b0 = n0;
    b1 = n1;
    top = bot;
    bot = lerp(b0, b1, tx);
  }
}

template <typename T, int MODE, bool VAR>
__global__ __launch_bounds__(256) void k_sweep_2d_coarse(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, const T* __restrict__ rm,
    int64_t rp, const double* __restrict__ am, int64_t ap, double* __restrict__ u, int64_t up,
    int n, int len, int m, typename Tr<T>::C w, typename Tr<T>::C hl2,
    const int* __restrict__ done) {
  if (*done) return;
  tile_sweep_2d_coarse<T, MODE, VAR>(eo, en, ep, rm, rp, am, ap, u, up, n, len, m, w, hl2, blockIdx.x, blockIdx.y);
}

// 3D level 0: a lane owns R3Y consecutive y rows of one x column and walks
// z, so the y neighbours of its inner rows come from its own registers and
// only the rows just below and above its group are loaded (the block's
// 64 x 4 lanes cover 64 x 16 nodes of each plane).
constexpr int R3Y = 4;

template <typename T, int MODE>
__device__ __forceinline__ void tile_sweep_3d_l0(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, int64_t epl,
    const T* __restrict__ r, int64_t rp, int64_t rpl, double* __restrict__ u, int64_t up,
    int64_t upl, int n, int len, typename Tr<T>::C w, typename Tr<T>::C hl2) {
  using C = typename Tr<T>::C;
  // one-dimensional grid in XCD order (the tiles that share halo rows and
  // planes meet in one XCD's L2), walks of len planes, as the 3D residual
  const int gx = (n - 2 + BX3 - 1) / BX3, gy = (n - 2 + BY3 * R3Y - 1) / (BY3 * R3Y);
  const int lg = int(xcd_order(blockIdx.x, gridDim.x));
  const int bx = lg % gx, by = (lg / gx) % gy, bz = lg / (gx * gy);
  const int lane = threadIdx.x;
  const int x = 1 + bx * BX3 + lane;
  const int yb = 1 + (by * BY3 + __builtin_amdgcn_readfirstlane(int(threadIdx.y))) * R3Y;
  if (yb > n - 2) return;  // the whole wave
  const int z0 = 1 + bz * len;
  const int z1 = min(n - 1, z0 + len);
  // lanes past the last interior column keep walking (their values feed the
  // neighbour lanes' x neighbours) and store nothing; x neighbours come from
  // the neighbour lanes, the end lanes load their outside column
  const bool xin = x <= n - 2;
  const int xc = min(x, n - 1);
  const bool edge = lane == 0 || lane == BX3 - 1;
  const int xe = lane == 0 ? x - 1 : min(x + 1, n - 1);
  // rows yb .. yb+R3Y-1; those past n-2 are clamped (computed, not stored)
  C c[R3Y], zm[R3Y];
#pragma unroll
  for (int k = 0; k < R3Y; ++k) {
    const int64_t col = int64_t(min(yb + k, n - 2)) * ep + xc;
    c[k] = zm[k] = C(0);
    if (!(MODE & SW_ZERO_OLD)) {
      zm[k] = ld(eo + int64_t(z0 - 1) * epl + col);
      c[k] = ld(eo + int64_t(z0) * epl + col);
    }
  }
  const int64_t ylo = int64_t(yb - 1) * ep + xc;
  const int64_t yhi = int64_t(min(yb + R3Y, n - 1)) * ep + xc;
  for (int z = z0; z < z1; ++z) {
    C zp[R3Y], ev[R3Y], rv[R3Y];
    C below = C(0), above = C(0);
#pragma unroll
    for (int k = 0; k < R3Y; ++k) {
      const int yk = min(yb + k, n - 2);
      rv[k] = ld(r + int64_t(z) * rpl + int64_t(yk) * rp + xc);
      zp[k] = ev[k] = C(0);
      if (!(MODE & SW_ZERO_OLD)) {
        const T* q = eo + int64_t(z) * epl + int64_t(yk) * ep;
        zp[k] = ld(q + epl + xc);
        if (edge) ev[k] = ld(q + xe);
      }
    }
    if (!(MODE & SW_ZERO_OLD)) {
      below = ld(eo + int64_t(z) * epl + ylo);
      above = ld(eo + int64_t(z) * epl + yhi);
    }
#pragma unroll
    for (int k = 0; k < R3Y; ++k) {
      const C ym = k == 0 ? below : c[k - 1];
      // the row above is the next owned row, or the group's upper neighbour
      // (the boundary row, 0, when the group ends at n-2)
      const C yp = k == R3Y - 1 ? above : (yb + k + 1 <= n - 2 ? c[k + 1] : C(0));
      const C xm = lane_prev_or(ev[k], c[k]);  // lane 0: ev
      const C xp = lane_next_or(ev[k], c[k]);  // lane 63: ev
      const C v = relax_const<C>(c[k], ((xm + xp) + (ym + yp)) + (zm[k] + zp[k]), rv[k], w, hl2, C(6));
      if (xin && yb + k <= n - 2) {
        if (MODE & SW_ACCUM)
          add_to(u + int64_t(z) * upl + int64_t(yb + k) * up + x, double(v));
        else
          st(en + int64_t(z) * epl + int64_t(yb + k) * ep + x, v);
      }
    }
#pragma unroll
    for (int k = 0; k < R3Y; ++k) {
      zm[k] = c[k];
      c[k] = zp[k];
    }
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_sweep_3d_l0(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, int64_t epl,
    const T* __restrict__ r, int64_t rp, int64_t rpl, double* __restrict__ u, int64_t up,
    int64_t upl, int n, int len, typename Tr<T>::C w, typename Tr<T>::C hl2,
    const int* __restrict__ done) {
  if (*done) return;
  tile_sweep_3d_l0<T, MODE>(eo, en, ep, epl, r, rp, rpl, u, up, upl, n, len, w, hl2);
}

// 3D level 0, IT <= 2 iterations in one pass.  A block of 64 x 4 lanes owns
// a 64 x 16 tile of (x, y) columns (four consecutive rows per lane) and
// walks z; iteration t is computed t planes behind the plane just loaded.
// A lane keeps, per iteration level, its four rows of the last three planes
// (the z neighbours, and the y neighbours of its inner rows); the x
// neighbours come from the neighbour lanes (DPP wave shifts: a wave is one
// 64-column row group), and the lane's first and last rows of each level's
// centre plane go to LDS, where the waves above and below read them as y
// neighbours (double-buffered: one barrier per plane).  The tile's outer IT columns and rows only feed the inner ones,
// so a block emits (64 - 2 IT) x (16 - 2 IT) columns and the band of planes
// is entered IT planes early and left IT planes late.  Every intermediate
// iterate is rounded as a store would round it, so the result equals IT
// single sweeps bit for bit.
constexpr int TB3_R = 4;                 // rows per lane
constexpr int TB3_TY = BY3 * TB3_R;      // tile rows (16)

template <typename T, bool ZERO, bool ACCUM, bool PREV, int IT, bool LAT = false>
__device__ __forceinline__ void tb3_body(const T* __restrict__ eo, T* __restrict__ en,
                                         T* __restrict__ eprev, int64_t ep, int64_t epl,
                                         const T* __restrict__ r, int64_t rp, int64_t rpl,
                                         double* __restrict__ u, int64_t up, int64_t upl, int n,
                                         int len, typename Tr<T>::C w, typename Tr<T>::C hl2,
                                         const L1Src<T>& l1 = L1Src<T>{}) {
  using C = typename Tr<T>::C;
  constexpr int VX = BX3 - 2 * IT, VY = TB3_TY - 2 * IT;
  __shared__ C P[IT][2][TB3_TY][BX3];
  const int gx = (n - 2 + VX - 1) / VX, gy = (n - 2 + VY - 1) / VY;
  const int lg = int(xcd_order(blockIdx.x, gridDim.x));
  const int bx = lg % gx, by = (lg / gx) % gy, bz = lg / (gx * gy);
  // threadIdx.y is one value per wave: keep the rows (and their offsets) scalar
  const int lx = threadIdx.x, row0 = __builtin_amdgcn_readfirstlane(int(threadIdx.y) * TB3_R);
  const int x = 1 + bx * VX - IT + lx;
  const int yb = 1 + by * VY - IT + row0;  // first of the lane's rows
  const int Z0 = 1 + bz * len, Z1 = min(n - 1, Z0 + len);
  const int xc = min(max(x, 0), n - 1);
  const bool xin = x >= 1 && x <= n - 2;
  const bool emit_x = lx >= IT && lx < BX3 - IT;
  // clamped (y, x) offsets in e and r: positions off the grid read the boundary (zero)
  int64_t col[TB3_R], rcol[TB3_R];
  bool yin[TB3_R], emit[TB3_R];
#pragma unroll
  for (int k = 0; k < TB3_R; ++k) {
    const int y = yb + k, ycl = min(max(y, 0), n - 1);
    col[k] = int64_t(ycl) * ep + xc;
    rcol[k] = int64_t(ycl) * rp + xc;
    yin[k] = xin && y >= 1 && y <= n - 2;
    emit[k] = emit_x && row0 + k >= IT && row0 + k < TB3_TY - IT && yin[k];
  }
  C win[IT][3][TB3_R], rr[IT][TB3_R];
#pragma unroll
  for (int t = 0; t < IT; ++t)
#pragma unroll
    for (int k = 0; k < TB3_R; ++k) {
      win[t][0][k] = win[t][1][k] = win[t][2][k] = C(0);
      rr[t][k] = C(0);
    }
  const int ym_row = max(row0 - 1, 0), yp_row = min(row0 + TB3_R, TB3_TY - 1);
  L1Col3<T, TB3_R> lc;
  if (LAT) lc.init(l1, x, yb, n);
  int b = 0;
  for (int zl = max(Z0 - IT, 0); zl < Z1 + IT; ++zl, b ^= 1) {
    const int zlc = min(zl, n - 1), zr = min(max(zl - 1, 0), n - 1);
    const int ze = zl - IT;  // the plane this step emits
    const bool zemit = ze >= Z0 && ze < Z1;
    C lv[TB3_R], rvs[TB3_R];
    double uo[TB3_R];
#pragma unroll
    for (int k = 0; k < TB3_R; ++k) {
      rvs[k] = ld(r + int64_t(zr) * rpl + rcol[k]);
      if (!LAT) lv[k] = ZERO ? C(0) : ld(eo + int64_t(zlc) * epl + col[k]);
      // the old values of the emitted u entries travel with the plane's
      // loads instead of one dependent read per row at the store (on
      // MI355X, 134 -> 125 us per pass at 257^3)
      uo[k] = 0.0;
      if (ACCUM && zemit && emit[k]) uo[k] = u[int64_t(ze) * upl + int64_t(yb + k) * up + x];
    }
    if (LAT) lc.at(zlc, lv);
#pragma unroll
    for (int k = 0; k < TB3_R; ++k) {
      const C v0 = lv[k];
      const C rv = rvs[k];
      win[0][0][k] = win[0][1][k];
      win[0][1][k] = win[0][2][k];
      win[0][2][k] = v0;
#pragma unroll
      for (int t = IT - 1; t > 0; --t) rr[t][k] = rr[t - 1][k];
      rr[0][k] = rv;
      // only a lane's first and last rows are read by the waves next to it
      if (k == 0 || k == TB3_R - 1) {
        P[0][b][row0 + k][lx] = win[0][1][k];
#pragma unroll
        for (int t = 1; t < IT; ++t) P[t][b][row0 + k][lx] = win[t][2][k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 1; t <= IT; ++t) {
      const int zc = zl - t;
      const bool zin = zc >= 1 && zc <= n - 2;
      const C(&pl)[TB3_TY][BX3] = P[t - 1][b];
      C v[TB3_R];
#pragma unroll
      for (int k = 0; k < TB3_R; ++k) {
        const C c = win[t - 1][1][k];
        // x neighbours by DPP wave shifts (the wave is one row of the
        // tile); the end lanes' values are never emitted
        const C xm = lane_prev(c), xp = lane_next(c);
        const C ym = k == 0 ? pl[ym_row][lx] : win[t - 1][1][k - 1];
        const C yp = k == TB3_R - 1 ? pl[yp_row][lx] : win[t - 1][1][k + 1];
        v[k] = relax_const<C>(c, ((xm + xp) + (ym + yp)) + (win[t - 1][0][k] + win[t - 1][2][k]),
                              rr[t - 1][k], w, hl2, C(6));
      }
      if (t < IT) {
#pragma unroll
        for (int k = 0; k < TB3_R; ++k) {
          win[t][0][k] = win[t][1][k];
          win[t][1][k] = win[t][2][k];
          win[t][2][k] = (yin[k] && zin) ? rnd<T>(v[k]) : C(0);
        }
      } else if (zemit) {
#pragma unroll
        for (int k = 0; k < TB3_R; ++k) {
          if (!emit[k]) continue;
          const int y = yb + k;
          if (ACCUM)
            st(u + int64_t(zc) * upl + int64_t(y) * up + x, uo[k] + double(v[k]));
          else
            st(en + int64_t(zc) * epl + int64_t(y) * ep + x, v[k]);
          if (PREV) st(eprev + int64_t(zc) * epl + int64_t(y) * ep + x, win[t - 1][1][k]);
        }
      }
    }
  }
}

template <typename T, bool ZERO, bool ACCUM, int IT, bool LAT>
__global__ __launch_bounds__(256) void k_sweep_3d_l0_tb(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, int64_t epl, const T* __restrict__ r,
    int64_t rp, int64_t rpl, double* __restrict__ u, int64_t up, int64_t upl, int n, int len,
    typename Tr<T>::C w, typename Tr<T>::C hl2, const int* __restrict__ done, L1Src<T> l1) {
  if (*done) return;
  tb3_body<T, ZERO, ACCUM, false, IT, LAT>(eo, en, nullptr, ep, epl, r, rp, rpl, u, up, upl, n, len, w, hl2,
                                           l1);
}

template <typename T, bool ZERO, bool PREV, int IT, bool LAT>
__global__ __launch_bounds__(256) void k_lattice_3d_tb(
    const T* __restrict__ eo, T* __restrict__ en, T* __restrict__ eprev, int64_t ep, int64_t epl,
    const T* __restrict__ r, int64_t rp, int64_t rpl, int n, int len, typename Tr<T>::C w,
    typename Tr<T>::C hl2, const int* __restrict__ done, L1Src<T> l1) {
  if (*done) return;
  tb3_body<T, ZERO, false, PREV, IT, LAT>(eo, en, eprev, ep, epl, r, rp, rpl, nullptr, 0, 0, n, len, w, hl2,
                                          l1);
}

// The same iteration on the compact lattice of a coarse level (the
// level-blocked path): a kernel of its own so that profiles separate it
// from the whole-grid level-0 iteration.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_lattice_sweep_3d(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, int64_t epl,
    const T* __restrict__ r, int64_t rp, int64_t rpl, double* __restrict__ u, int64_t up,
    int64_t upl, int n, int len, typename Tr<T>::C w, typename Tr<T>::C hl2,
    const int* __restrict__ done) {
  if (*done) return;
  tile_sweep_3d_l0<T, MODE>(eo, en, ep, epl, r, rp, rpl, u, up, upl, n, len, w, hl2);
}

template <typename T, int MODE, bool VAR>
__global__ __launch_bounds__(256) void k_lattice_sweep_2d(
    const T* __restrict__ eo, T* __restrict__ en, int64_t ep, const T* __restrict__ r,
    int64_t rp, const double* __restrict__ a, int64_t ap, double* __restrict__ u, int64_t up,
    int n, int len, typename Tr<T>::C w, typename Tr<T>::C hl2, const int* __restrict__ done) {
  if (*done) return;
  tile_sweep_2d_l0<T, MODE, VAR>(eo, en, ep, r, rp, a, ap, u, up, n, len, w, hl2, blockIdx.x, blockIdx.y);
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
  // corners of the top (za) and bottom (za + l) planes of the current cell;
  // the next cell's bottom corners (za + 2l) are loaded one cell ahead, so
  // their latency overlaps the stores of the current cell
  C t00 = C(0), t01 = C(0), t10 = C(0), t11 = C(0);
  C b00 = C(0), b01 = C(0), b10 = C(0), b11 = C(0);
  C n00 = C(0), n01 = C(0), n10 = C(0), n11 = C(0);
  if (!(MODE & SW_ZERO_OLD)) {
    const T* pt = eo + int64_t(za) * epl;
    const T* pb = pt + int64_t(l) * epl;
    t00 = ld(pt + c00); t01 = ld(pt + c01); t10 = ld(pt + c10); t11 = ld(pt + c11);
    b00 = ld(pb + c00); b01 = ld(pb + c01); b10 = ld(pb + c10); b11 = ld(pb + c11);
  }
  C top = lerp(lerp(t00, t01, tx), lerp(t10, t11, tx), ty);
  C bot = lerp(lerp(b00, b01, tx), lerp(b10, b11, tx), ty);
  for (int zc = z0; zc < z1; za += l) {
    const int ze = min(z1, za + l);
    if (!(MODE & SW_ZERO_OLD) && za + 2 * l <= n - 1 && ze < z1) {
      const T* pn = eo + int64_t(za + 2 * l) * epl;
      n00 = ld(pn + c00); n01 = ld(pn + c01); n10 = ld(pn + c10); n11 = ld(pn + c11);
    }
    for (int z = zc; z < ze; ++z) {
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
        add_to(u + int64_t(z) * upl + int64_t(y) * up + x, double(v));
      else
        st_w(en + int64_t(z) * epl + int64_t(y) * ep + x, v);
    }
    zc = ze;
    t00 = b00; t01 = b01; t10 = b10; t11 = b11;
    b00 = n00; b01 = n01; b10 = n10; b11 = n11;
    top = bot;
    bot = lerp(lerp(b00, b01, tx), lerp(b10, b11, tx), ty);
  }
}

// ------------------------------------------------------------ level-blocked path
// The n_m iterations of level m read only lattice values, so they run on the
// compact level-m lattice (x_0 = the whole grid sampled on the lattice,
// x_t = one damped-Jacobi step of x_{t-1}); afterwards one whole-grid pass
// writes the level's final state: interior lattice nodes take x_{n_m}, every
// other interior node the multilinear interpolant of x_{n_m - 1} (the
// one-iteration delay of the fused task).  The node formulas are the ones
// of the one-launch-per-iteration kernels above, and every iterate is
// rounded to the storage type at the same points, so both paths produce the
// same bits.

// x_0 on the compact lattice: dst[K][J][I] = src[K l][J l][I l] (all nodes).
template <typename T>
__global__ __launch_bounds__(256) void k_gather(const T* __restrict__ src, int64_t sp,
                                                int64_t spl, int l, T* __restrict__ dst,
                                                int64_t dp, int64_t dpl, int side, int nz) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= side || z >= nz) return;
  dst[int64_t(z) * dpl + int64_t(y) * dp + x] =
      src[int64_t(z) * l * spl + int64_t(y) * l * sp + int64_t(x) * l];
}

// Small lattices: one workgroup holds the whole compact level-m lattice in
// LDS and runs all `it` iterations there; writes x_{it-1} and x_it.
// ZERO: x_0 = 0 (first level of a cycle).
constexpr int SMALL_NT = 1024;

template <typename T, bool ZERO, bool VAR>
__global__ __launch_bounds__(SMALL_NT) void k_lattice_small_2d(
    const T* __restrict__ e, int64_t ep, int l, const T* __restrict__ rm, int64_t rp,
    const double* __restrict__ am, int64_t ap, T* __restrict__ xprev, T* __restrict__ xcur,
    int64_t cp, int nm, int it, typename Tr<T>::C w, typename Tr<T>::C hl2,
    const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int cnt = nm * nm;
  C* xa = reinterpret_cast<C*>(smem);
  C* xb = xa + cnt;
  C* rr = xb + cnt;
  double* aa = reinterpret_cast<double*>(smem + ((3 * cnt * sizeof(C) + 15) & ~size_t(15)));
  for (int i = threadIdx.x; i < cnt; i += SMALL_NT) {
    const int J = i / nm, I = i - J * nm;
    const bool inner = I > 0 && I < nm - 1 && J > 0 && J < nm - 1;
    xa[i] = ZERO ? C(0) : ld(e + int64_t(J) * l * ep + int64_t(I) * l);
    xb[i] = xa[i];
    rr[i] = inner ? ld(rm + int64_t(J) * rp + I) : C(0);
    if (VAR) aa[i] = am[int64_t(J) * ap + I];
  }
  __syncthreads();
  for (int t = 1; t <= it; ++t) {
    const C* src = (t & 1) ? xa : xb;
    C* dst = (t & 1) ? xb : xa;
    for (int i = threadIdx.x; i < cnt; i += SMALL_NT) {
      const int J = i / nm, I = i - J * nm;
      if (I > 0 && I < nm - 1 && J > 0 && J < nm - 1) {
        const C c = src[i], xm = src[i - 1], xp = src[i + 1], ym = src[i - nm], yp = src[i + nm];
        C v;
        if (VAR)
          v = relax_var<C>(c, xm, xp, ym, yp, aa[i], aa[i - 1], aa[i + 1], aa[i - nm], aa[i + nm],
                           rr[i], w, hl2);
        else
          v = relax_const<C>(c, (xm + xp) + (ym + yp), rr[i], w, hl2, C(4));
        dst[i] = rnd<T>(v);
      }
    }
    __syncthreads();
  }
  const C* cur = (it & 1) ? xb : xa;
  const C* prv = (it & 1) ? xa : xb;
  for (int i = threadIdx.x; i < cnt; i += SMALL_NT) {
    const int J = i / nm, I = i - J * nm;
    st(xprev + int64_t(J) * cp + I, prv[i]);
    st(xcur + int64_t(J) * cp + I, cur[i]);
  }
}

template <typename T, bool ZERO>
__global__ __launch_bounds__(SMALL_NT) void k_lattice_small_3d(
    const T* __restrict__ e, int64_t ep, int64_t epl, int l, const T* __restrict__ rm,
    int64_t rp, int64_t rpl, T* __restrict__ xprev, T* __restrict__ xcur, int64_t cp,
    int64_t cpl, int nm, int it, typename Tr<T>::C w, typename Tr<T>::C hl2,
    const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int pl = nm * nm, cnt = pl * nm;
  C* xa = reinterpret_cast<C*>(smem);
  C* xb = xa + cnt;
  C* rr = xb + cnt;
  for (int i = threadIdx.x; i < cnt; i += SMALL_NT) {
    const int K = i / pl, rem = i - K * pl, J = rem / nm, I = rem - J * nm;
    const bool inner = I > 0 && I < nm - 1 && J > 0 && J < nm - 1 && K > 0 && K < nm - 1;
    xa[i] = ZERO ? C(0) : ld(e + int64_t(K) * l * epl + int64_t(J) * l * ep + int64_t(I) * l);
    xb[i] = xa[i];
    rr[i] = inner ? ld(rm + int64_t(K) * rpl + int64_t(J) * rp + I) : C(0);
  }
  __syncthreads();
  for (int t = 1; t <= it; ++t) {
    const C* src = (t & 1) ? xa : xb;
    C* dst = (t & 1) ? xb : xa;
    for (int i = threadIdx.x; i < cnt; i += SMALL_NT) {
      const int K = i / pl, rem = i - K * pl, J = rem / nm, I = rem - J * nm;
      if (I > 0 && I < nm - 1 && J > 0 && J < nm - 1 && K > 0 && K < nm - 1) {
        const C c = src[i];
        const C q = ((src[i - 1] + src[i + 1]) + (src[i - nm] + src[i + nm])) + (src[i - pl] + src[i + pl]);
        dst[i] = rnd<T>(relax_const<C>(c, q, rr[i], w, hl2, C(6)));
      }
    }
    __syncthreads();
  }
  const C* cur = (it & 1) ? xb : xa;
  const C* prv = (it & 1) ? xa : xb;
  for (int i = threadIdx.x; i < cnt; i += SMALL_NT) {
    const int K = i / pl, rem = i - K * pl, J = rem / nm, I = rem - J * nm;
    st(xprev + int64_t(K) * cpl + int64_t(J) * cp + I, prv[i]);
    st(xcur + int64_t(K) * cpl + int64_t(J) * cp + I, cur[i]);
  }
}

// The whole-grid pass of a level: stages the compact x_{it-1} / x_it values
// under the block's tile in LDS, then every lane walks its column writing
// lattice nodes from x_it and the rest by multilinear interpolation of
// x_{it-1}.  MODE bits: SW_ZERO_OLD (x_{it-1} = 0), SW_ACCUM (add into u).
constexpr int LW_ROWS2 = 32;  // rows per 2D tile
constexpr int LW_PLANES3 = 16;  // planes per 3D tile

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_level_write_2d(
    const T* __restrict__ xprev, const T* __restrict__ xcur, int64_t cp, T* __restrict__ en,
    int64_t ep, double* __restrict__ u, int64_t up, int n, int m, const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int l = 1 << m, mask = l - 1;
  // a tile of TW2 columns and LW_ROWS2 rows; wave w writes rows
  // Y0 + w LW_ROWS2/4 .. (the four waves on different rows)
  const int X0 = 1 + blockIdx.x * TW2, X1 = min(n - 2, X0 + TW2 - 1);
  const int Y0 = 1 + blockIdx.y * LW_ROWS2, Y1 = min(n - 2, Y0 + LW_ROWS2 - 1);
  const int I0 = X0 >> m, J0 = Y0 >> m;
  const int CW = (X1 >> m) - I0 + 2, CH = (Y1 >> m) - J0 + 2;
  C* P = reinterpret_cast<C*>(smem);
  C* Q = P + CW * CH;
  for (int i = threadIdx.x; i < CW * CH; i += BX2) {
    const int j = i / CW, c = i - j * CW;
    const int64_t g = int64_t(J0 + j) * cp + (I0 + c);
    P[i] = (MODE & SW_ZERO_OLD) ? C(0) : ld(xprev + g);
    Q[i] = ld(xcur + g);
  }
  __syncthreads();
  const int x = X0 + int(threadIdx.x & 63);
  constexpr int WR = LW_ROWS2 / 4;
  const int ya = Y0 + int(threadIdx.x >> 6) * WR, yb = min(Y1, ya + WR - 1);
  if (x > X1) return;
  const C inv_l = C(1) / C(l);
  const int xi = (x >> m) - I0;
  const C tx = C(x & mask) * inv_l;
  const bool latc = (x & mask) == 0;
  int band = -1;
  C top = C(0), bot = C(0);
  for (int y = ya; y <= yb; ++y) {
    const int yj = (y >> m) - J0;
    if (yj != band) {
      band = yj;
      const C* p = P + yj * CW + xi;
      top = lerp(p[0], p[1], tx);
      bot = lerp(p[CW], p[CW + 1], tx);
    }
    C v;
    if (latc && (y & mask) == 0)
      v = Q[yj * CW + xi];
    else
      v = lerp(top, bot, C(y & mask) * inv_l);
    if (MODE & SW_ACCUM)
      add_to(u + int64_t(y) * up + x, double(v));
    else
      st_w(en + int64_t(y) * ep + x, v);
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_level_write_3d(
    const T* __restrict__ xprev, const T* __restrict__ xcur, int64_t cp, int64_t cpl,
    T* __restrict__ en, int64_t ep, int64_t epl, double* __restrict__ u, int64_t up, int64_t upl,
    int n, int m, const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int l = 1 << m, mask = l - 1;
  const int X0 = 1 + blockIdx.x * BX3, X1 = min(n - 2, X0 + BX3 - 1);
  const int Y0 = 1 + blockIdx.y * BY3, Y1 = min(n - 2, Y0 + BY3 - 1);
  const int Z0 = 1 + blockIdx.z * LW_PLANES3, Z1 = min(n - 2, Z0 + LW_PLANES3 - 1);
  const int I0 = X0 >> m, J0 = Y0 >> m, K0 = Z0 >> m;
  const int CW = (X1 >> m) - I0 + 2, CH = (Y1 >> m) - J0 + 2, CD = (Z1 >> m) - K0 + 2;
  const int CP = CW * CH;
  C* P = reinterpret_cast<C*>(smem);
  C* Q = P + CP * CD;
  const int tid = threadIdx.y * BX3 + threadIdx.x;
  for (int i = tid; i < CP * CD; i += BX3 * BY3) {
    const int k = i / CP, rem = i - k * CP, j = rem / CW, c = rem - j * CW;
    const int64_t g = int64_t(K0 + k) * cpl + int64_t(J0 + j) * cp + (I0 + c);
    P[i] = (MODE & SW_ZERO_OLD) ? C(0) : ld(xprev + g);
    Q[i] = ld(xcur + g);
  }
  __syncthreads();
  const int x = X0 + threadIdx.x, y = Y0 + threadIdx.y;
  if (x > X1 || y > Y1) return;
  const C inv_l = C(1) / C(l);
  const int xi = (x >> m) - I0, yj = (y >> m) - J0;
  const C tx = C(x & mask) * inv_l, ty = C(y & mask) * inv_l;
  const bool latxy = (x & mask) == 0 && (y & mask) == 0;
  int band = -1;
  C top = C(0), bot = C(0);
  for (int z = Z0; z <= Z1; ++z) {
    const int zk = (z >> m) - K0;
    if (zk != band) {
      band = zk;
      const C* p = P + zk * CP + yj * CW + xi;
      top = lerp(lerp(p[0], p[1], tx), lerp(p[CW], p[CW + 1], tx), ty);
      const C* q = p + CP;
      bot = lerp(lerp(q[0], q[1], tx), lerp(q[CW], q[CW + 1], tx), ty);
    }
    C v;
    if (latxy && (z & mask) == 0)
      v = Q[zk * CP + yj * CW + xi];
    else
      v = lerp(top, bot, C(z & mask) * inv_l);
    if (MODE & SW_ACCUM)
      add_to(u + int64_t(z) * upl + int64_t(y) * up + x, double(v));
    else
      st_w(en + int64_t(z) * epl + int64_t(y) * ep + x, v);
  }
}

// Chained transfer: the whole-grid state a level-m pass would write, but
// evaluated only at the interior nodes of the level-mt lattice and stored
// in that level's compact array -- what the next level would gather.  The
// node formula and its rounding are those of the level write above, so the
// chained path matches the whole-grid path bit for bit.  Boundary nodes of
// the target are never written (they stay 0).
// Interior node (I, J) of the level-mt lattice (compact, pitch dp): the
// value the level-m whole-grid pass would leave there.
template <typename T, bool ZERO>
__device__ __forceinline__ void transfer_node_2d(const T* __restrict__ xprev, const T* __restrict__ xcur,
                                                 int64_t cp, int m, T* __restrict__ dst, int64_t dp,
                                                 int mt, int I, int J) {
  using C = typename Tr<T>::C;
  const int x = I << mt, y = J << mt;
  const int l = 1 << m, mask = l - 1;
  const C inv_l = C(1) / C(l);
  const int xi = x >> m, yj = y >> m;
  const C tx = C(x & mask) * inv_l;
  C v;
  if ((x & mask) == 0 && (y & mask) == 0) {
    v = ld(xcur + int64_t(yj) * cp + xi);
  } else {
    C p00 = C(0), p01 = C(0), p10 = C(0), p11 = C(0);
    if (!ZERO) {
      const T* p = xprev + int64_t(yj) * cp + xi;
      p00 = ld(p);
      p01 = ld(p + 1);
      p10 = ld(p + cp);
      p11 = ld(p + cp + 1);
    }
    const C top = lerp(p00, p01, tx), bot = lerp(p10, p11, tx);
    v = lerp(top, bot, C(y & mask) * inv_l);
  }
  st(dst + int64_t(J) * dp + I, v);
}

template <typename T, bool ZERO>
__global__ __launch_bounds__(256) void k_level_transfer_2d(
    const T* __restrict__ xprev, const T* __restrict__ xcur, int64_t cp, int m,
    T* __restrict__ dst, int64_t dp, int nt, int mt, const int* __restrict__ done) {
  if (*done) return;
  const int I = 1 + blockIdx.x * 256 + threadIdx.x, J = 1 + blockIdx.y;
  if (I > nt - 2) return;
  transfer_node_2d<T, ZERO>(xprev, xcur, cp, m, dst, dp, mt, I, J);
}

template <typename T, bool ZERO>
__global__ __launch_bounds__(256) void k_level_transfer_3d(
    const T* __restrict__ xprev, const T* __restrict__ xcur, int64_t cp, int64_t cpl, int m,
    T* __restrict__ dst, int64_t dp, int64_t dpl, int nt, int mt, const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  // blocks of 64 x 4 lanes: a row of a small lattice does not leave most of
  // a 256-lane block idle
  const int I = 1 + blockIdx.x * BX3 + threadIdx.x, J = 1 + blockIdx.y * BY3 + threadIdx.y, K = 1 + blockIdx.z;
  if (I > nt - 2 || J > nt - 2) return;
  const int x = I << mt, y = J << mt, z = K << mt;
  const int l = 1 << m, mask = l - 1;
  const C inv_l = C(1) / C(l);
  const int xi = x >> m, yj = y >> m, zk = z >> m;
  const C tx = C(x & mask) * inv_l, ty = C(y & mask) * inv_l;
  C v;
  if ((x & mask) == 0 && (y & mask) == 0 && (z & mask) == 0) {
    v = ld(xcur + int64_t(zk) * cpl + int64_t(yj) * cp + xi);
  } else {
    C t[8] = {C(0), C(0), C(0), C(0), C(0), C(0), C(0), C(0)};
    if (!ZERO) {
      const T* p = xprev + int64_t(zk) * cpl + int64_t(yj) * cp + xi;
      t[0] = ld(p); t[1] = ld(p + 1); t[2] = ld(p + cp); t[3] = ld(p + cp + 1);
      const T* q = p + cpl;
      t[4] = ld(q); t[5] = ld(q + 1); t[6] = ld(q + cp); t[7] = ld(q + cp + 1);
    }
    const C top = lerp(lerp(t[0], t[1], tx), lerp(t[2], t[3], tx), ty);
    const C bot = lerp(lerp(t[4], t[5], tx), lerp(t[6], t[7], tx), ty);
    v = lerp(top, bot, C(z & mask) * inv_l);
  }
  st(dst + int64_t(K) * dpl + int64_t(J) * dp + I, v);
}

// ------------------------------------------------------------ coarse tail
// The schedule's leading coarse levels ms .. M (descending one level at a
// time, each visited once) in one workgroup, everything in LDS: the
// restriction of r_ms to the coarser levels, each level's iterations from
// the state the previous level hands over (0 on the coarsest), and the
// hand-over itself -- the values the level's whole-grid pass would leave at
// the lattice nodes of the next finer level.  The last hand-over goes to
// the compact x_0 of level ms - 1 in memory.  The node formulas and the
// rounding points are those of the restriction, small-lattice and transfer
// kernels, so the result is theirs bit for bit.  Level ms + k has side
// nk = ((nms - 1) >> k) + 1; LDS holds, per level, r and two iterates.
// Per-level constants of the tail, worked out on the host (the reciprocals
// and h^2 are the correctly rounded values the device division would give),
// so that no level of the kernel starts with a division or a walk over the
// coarser levels' sizes.
struct TailLevel {
  int it;        // iterations of level ms + k
  int off;       // element offset of the level's R, P, Q arrays in LDS
  float inv_ni;  // 1 / (nk - 2): splits the level's interior nodes
  float inv_nt;  // 1 / (2 nk - 3): splits the next finer level's interior nodes
  double hl2;    // h^2 = (1 / (nk - 1))^2
};
struct TailPlan {
  TailLevel lv[BATCH_MAX_LEVELS];
  float inv_side;  // 1 / nms: splits every node of level ms
};

template <int D>
__device__ __forceinline__ int tail_count(int nk) { return D == 2 ? nk * nk : nk * nk * nk; }

// i -> (I, J, K) in a box of side s (x fastest); a single-precision
// reciprocal is exact here: i < 2^24 and (i + 1/2) / s stays at least
// 1/(2 s) away from an integer.
template <int D>
__device__ __forceinline__ void tail_split(int i, int s, float inv_s, int& I, int& J, int& K) {
  const int q = int((float(i) + 0.5f) * inv_s);
  I = i - q * s;
  if (D == 2) {
    J = q;
    K = 0;
  } else {
    K = int((float(q) + 0.5f) * inv_s);
    J = q - K * s;
  }
}

// TOP64 (reduced-precision cycles): the coarsest level of the tail runs in
// FP64 -- its right-hand side restricted in FP64 from the stored values of
// the level below, its iterates FP64 -- and only its final pair is rounded
// to the storage type before the hand-over, as the separate launches do
// (FP64 restriction, FP64 small-lattice iterations, rounding, transfer).
template <typename T, int D, bool TOP64>
__global__ __launch_bounds__(SMALL_NT) void k_coarse_tail(
    const T* __restrict__ rms, int64_t rp, int64_t rpl, T* __restrict__ dst, int64_t dp, int64_t dpl,
    int nms, int nlev, TailPlan tp, typename Tr<T>::C w, double w64, const int* __restrict__ done,
    T* __restrict__ sprev, T* __restrict__ scur, int64_t sp, int64_t spl) {
  using C = typename Tr<T>::C;
  if (*done) return;
  extern __shared__ __align__(16) unsigned char smem[];
  C* base = reinterpret_cast<C*>(smem);
  auto side = [&](int k) { return ((nms - 1) >> k) + 1; };
  // per level: R (r), P (x_0 and odd-numbered iterates' sources), Q
  auto lvl = [&](int k, int which) { return base + tp.lv[k].off + which * tail_count<D>(side(k)); };
  // FP64 arrays of the coarsest level (TOP64): R, P, Q after all C arrays
  const int ktop = nlev - 1, ctop = tail_count<D>(side(ktop));
  double* top64 = nullptr;
  if (TOP64) {
    const size_t used = size_t(lvl(ktop, 3) - base) * sizeof(C);
    top64 = reinterpret_cast<double*>(smem + ((used + 15) & ~size_t(15)));
    for (int i = threadIdx.x; i < 3 * ctop; i += SMALL_NT) top64[i] = 0.0;
  }
  // Level ms: r is loaded (0 on the boundary) and the iterates' boundary
  // nodes cleared; their interiors are written before they are read (the
  // hand-over from level ms + 1, the first iteration).  The coarser levels'
  // arrays start at 0 (x_0 = 0 on the coarsest level, and every boundary
  // node).  Each thread issues its loads of r (clamped in-range addresses,
  // the boundary's values dropped) before any LDS write, so the global
  // latency is paid once per chunk of TAIL_LB nodes, not once per node.
  constexpr int TAIL_LB = 8;
  const int cnt0 = tail_count<D>(nms);
  for (int i0 = 0; i0 < cnt0; i0 += TAIL_LB * SMALL_NT) {
    C rv[TAIL_LB];
    bool inner[TAIL_LB];
#pragma unroll
    for (int j = 0; j < TAIL_LB; ++j) {
      const int i = min(i0 + j * SMALL_NT + int(threadIdx.x), cnt0 - 1);
      int I, J, K;
      tail_split<D>(i, nms, tp.inv_side, I, J, K);
      inner[j] = I > 0 && I < nms - 1 && J > 0 && J < nms - 1 && (D == 2 || (K > 0 && K < nms - 1));
      rv[j] = ld(rms + int64_t(K) * rpl + int64_t(J) * rp + I);
    }
    if (i0 == 0) {
      const int z0 = tp.lv[nlev > 1 ? 1 : 0].off, z1 = tp.lv[ktop].off + 3 * ctop;
      for (int i = z0 + threadIdx.x; nlev > 1 && i < z1; i += SMALL_NT) base[i] = C(0);
    }
    C* R = lvl(0, 0);
    C* P = lvl(0, 1);
    C* Q = lvl(0, 2);
#pragma unroll
    for (int j = 0; j < TAIL_LB; ++j) {
      const int i = i0 + j * SMALL_NT + int(threadIdx.x);
      if (i < cnt0) {
        R[i] = inner[j] ? rv[j] : C(0);
        if (!inner[j]) P[i] = Q[i] = C(0);
      }
    }
  }
  __syncthreads();
  // restriction pyramid (full weighting, as k_restrict_*)
  for (int k = 1; k < nlev; ++k) {
    const int nf = side(k - 1), nc = side(k), ni = nc - 2, cnt = tail_count<D>(ni);
    const float inv = tp.lv[k].inv_ni;
    const C* F = lvl(k - 1, 0);
    C* R = lvl(k, 0);  // boundary nodes stay 0
    const int fp = nf, fpl = nf * nf;
    for (int i = threadIdx.x; i < cnt; i += SMALL_NT) {
      int I, J, K;
      tail_split<D>(i, ni, inv, I, J, K);
      ++I, ++J, K += D == 3;
      const int o = (D == 3 ? K * nc * nc : 0) + J * nc + I;
      if (TOP64 && k == ktop) {
        // as k_restrict_*<T, double>: the stored values widened, FP64 sums
        auto rs = [&](int q) { return fmac(2.0, double(F[q]), double(F[q - 1]) + double(F[q + 1])); };
        double v;
        if (D == 2) {
          const int q = 2 * J * fp + 2 * I;
          const double top = rs(q - fp), mid = rs(q), bot = rs(q + fp);
          v = fmac(2.0, mid, top + bot) * 0.0625;
        } else {
          auto ps = [&](int q) { return fmac(2.0, rs(q), rs(q - fp) + rs(q + fp)); };
          const int q = 2 * K * fpl + 2 * J * fp + 2 * I;
          const double top = ps(q - fpl), mid = ps(q), bot = ps(q + fpl);
          v = fmac(2.0, mid, top + bot) * 0.015625;
        }
        top64[o] = v;
        continue;
      }
      auto rs = [&](int q) { return fmac(C(2), F[q], F[q - 1] + F[q + 1]); };
      C v;
      if (D == 2) {
        const int q = 2 * J * fp + 2 * I;
        const C top = rs(q - fp), mid = rs(q), bot = rs(q + fp);
        v = fmac(C(2), mid, top + bot) * C(0.0625);
      } else {
        auto ps = [&](int q) { return fmac(C(2), rs(q), rs(q - fp) + rs(q + fp)); };
        const int q = 2 * K * fpl + 2 * J * fp + 2 * I;
        const C top = ps(q - fpl), mid = ps(q), bot = ps(q + fpl);
        v = fmac(C(2), mid, top + bot) * C(0.015625);
      }
      R[o] = rnd<T>(v);
    }
    __syncthreads();
  }
  // levels from the coarsest down
  for (int k = nlev - 1; k >= 0; --k) {
    const int nk = side(k), pl = nk * nk;
    const C hl2 = C(tp.lv[k].hl2);
    const C* R = lvl(k, 0);
    C* xa = lvl(k, 1);
    C* xb = lvl(k, 2);
    const int it = tp.lv[k].it;
    const int ni = nk - 2, icnt = tail_count<D>(ni);
    const float inv = tp.lv[k].inv_ni;
    if (TOP64 && k == ktop) {
      // FP64 iterations (as the FP64 small-lattice kernel), then the final
      // pair rounded to the storage type into xa (x_{it-1}) and xb (x_it)
      const double* R64 = top64;
      double* ya = top64 + ctop;
      double* yb = top64 + 2 * ctop;
      const double hl2d = tp.lv[k].hl2;
      for (int t = 1; t <= it; ++t) {
        const double* src = (t & 1) ? ya : yb;
        double* dstl = (t & 1) ? yb : ya;
        for (int j = threadIdx.x; j < icnt; j += SMALL_NT) {
          int I, J, K;
          tail_split<D>(j, ni, inv, I, J, K);
          const int i = (D == 3 ? (K + 1) * pl : 0) + (J + 1) * nk + (I + 1);
          const double c = src[i];
          double v;
          if (D == 2)
            v = relax_const<double>(c, (src[i - 1] + src[i + 1]) + (src[i - nk] + src[i + nk]), R64[i], w64,
                                    hl2d, 4.0);
          else
            v = relax_const<double>(
                c, ((src[i - 1] + src[i + 1]) + (src[i - nk] + src[i + nk])) + (src[i - pl] + src[i + pl]),
                R64[i], w64, hl2d, 6.0);
          dstl[i] = v;
        }
        __syncthreads();
      }
      const double* cur64 = (it & 1) ? yb : ya;
      const double* prv64 = (it & 1) ? ya : yb;
      for (int j = threadIdx.x; j < tail_count<D>(nk); j += SMALL_NT) {
        xa[j] = rnd<T>(C(prv64[j]));
        xb[j] = rnd<T>(C(cur64[j]));
      }
      __syncthreads();
    }
    for (int t = 1; t <= it && !(TOP64 && k == ktop); ++t) {
      const C* src = (t & 1) ? xa : xb;
      C* dstl = (t & 1) ? xb : xa;
      for (int j = threadIdx.x; j < icnt; j += SMALL_NT) {
        int I, J, K;
        tail_split<D>(j, ni, inv, I, J, K);
        const int i = (D == 3 ? (K + 1) * pl : 0) + (J + 1) * nk + (I + 1);
        const C c = src[i];
        C v;
        if (D == 2)
          v = relax_const<C>(c, (src[i - 1] + src[i + 1]) + (src[i - nk] + src[i + nk]), R[i], w, hl2, C(4));
        else
          v = relax_const<C>(c, ((src[i - 1] + src[i + 1]) + (src[i - nk] + src[i + nk])) + (src[i - pl] + src[i + pl]),
                             R[i], w, hl2, C(6));
        dstl[i] = rnd<T>(v);
      }
      __syncthreads();
    }
    const C* cur = (TOP64 && k == ktop) ? xb : ((it & 1) ? xb : xa);
    const C* prv = (TOP64 && k == ktop) ? xa : ((it & 1) ? xa : xb);
    if (k == 0 && scur) {
      // level ms's final state (every node) for the next level's first
      // pass, which interpolates it itself
      for (int j = threadIdx.x; j < tail_count<D>(nk); j += SMALL_NT) {
        int I, J, K;
        tail_split<D>(j, nk, tp.inv_side, I, J, K);
        const int64_t o = (D == 3 ? int64_t(K) * spl : 0) + int64_t(J) * sp + I;
        st(sprev + o, prv[j]);
        st(scur + o, cur[j]);
      }
      break;
    }
    // hand-over to level ms + k - 1 (side nt = 2 nk - 1): lattice nodes of
    // this level take x_it, the others the interpolant of x_{it-1}
    const int nt = 2 * nk - 1, ptl = nt * nt, nti = nt - 2;
    C* tgt = k > 0 ? lvl(k - 1, 1) : nullptr;
    const int tcnt = tail_count<D>(nti);
    const float tinv = tp.lv[k].inv_nt;
    for (int j = threadIdx.x; j < tcnt; j += SMALL_NT) {
      int I, J, K;
      tail_split<D>(j, nti, tinv, I, J, K);
      ++I, ++J, K += D == 3;
      const int i = (D == 3 ? K * ptl : 0) + J * nt + I;
      const int xi = I >> 1, yj = J >> 1, zk = K >> 1;
      const C tx = C(I & 1) * C(0.5), ty = C(J & 1) * C(0.5), tz = C(K & 1) * C(0.5);
      const int c0 = (D == 3 ? zk * pl : 0) + yj * nk + xi;
      C v;
      if (!(I & 1) && !(J & 1) && !(K & 1)) {
        v = cur[c0];
      } else if (D == 2) {
        const C top = lerp(prv[c0], prv[c0 + 1], tx), bot = lerp(prv[c0 + nk], prv[c0 + nk + 1], tx);
        v = lerp(top, bot, ty);
      } else {
        const C* p = prv + c0;
        const C* q = p + pl;
        const C top = lerp(lerp(p[0], p[1], tx), lerp(p[nk], p[nk + 1], tx), ty);
        const C bot = lerp(lerp(q[0], q[1], tx), lerp(q[nk], q[nk + 1], tx), ty);
        v = lerp(top, bot, tz);
      }
      if (k > 0)
        tgt[i] = rnd<T>(v);
      else
        st(dst + int64_t(K) * dpl + int64_t(J) * dp + I, v);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ tiled 3D lattice iterations
// IT (<= 4) iterations of a small 3D compact lattice in one launch: each
// workgroup holds a block of LT_B^3 owned nodes with a halo of IT nodes in
// LDS and iterates there, the region of valid values shrinking by one node
// per side and iteration, so the halo is recomputed by neighbouring blocks
// instead of exchanged between launches.  x_0 is 0 (ZERO), the compact array
// xo, or (LAT) the next coarser level's final state seen on this lattice
// (its x_it at shared lattice nodes, else the trilinear interpolant of its
// x_{it-1}); writes x_IT to xn and x_{IT-1} to xp at the owned nodes.  The
// node formula, summation order, interpolation and rounding are those of
// k_lattice_3d_tb and k_level_transfer_3d, so the bits are theirs.  Each
// lane keeps its tile nodes (up to four) for every phase, with r there in
// registers, and the coarser level's neighbourhood sits in the second
// iterate's array until the first iteration: 64 KB of LDS in FP64, two
// workgroups per CU.
constexpr int LT_B = 8;  // owned nodes per axis of a block
constexpr int LT_NT = 1024;

template <int IT>
__host__ __device__ constexpr int lt_side() { return LT_B + 2 * IT; }
__host__ __device__ constexpr int lt_cside(int S) { return S / 2 + 2; }
// tile nodes per lane (a 16^3 tile for four iterations: four)
template <int IT>
__host__ __device__ constexpr int lt_per_lane() { return (lt_side<IT>() * lt_side<IT>() * lt_side<IT>() + LT_NT - 1) / LT_NT; }

template <typename T, bool ZERO, bool LAT, int IT>
__global__ __launch_bounds__(LT_NT) void k_lattice_3d_tiled(
    const T* __restrict__ xo, T* __restrict__ xn, T* __restrict__ xp, int64_t cp, int64_t cpl,
    const T* __restrict__ r, int64_t rp, int64_t rpl, int n, int nb, typename Tr<T>::C w,
    typename Tr<T>::C hl2, const int* __restrict__ done, L1Src<T> l1) {
  using C = typename Tr<T>::C;
  if (*done) return;
  constexpr int S = lt_side<IT>(), S2 = S * S, S3 = S2 * S, SC = lt_cside(S), SC2 = SC * SC, SC3 = SC2 * SC;
  constexpr int U = lt_per_lane<IT>();
  static_assert(2 * SC3 <= S3, "the coarser level's neighbourhood fits in the second iterate's array");
  extern __shared__ __align__(16) unsigned char smem[];
  C* X0 = reinterpret_cast<C*>(smem);
  C* X1 = X0 + S3;
  C* Pc = X1;  // LAT: the coarser level's x_{it-1} and x_it around the block,
  C* Cc = Pc + SC3;  // in the second iterate's array until the first iteration
  const int lb = int(xcd_order(blockIdx.x, gridDim.x));
  const int bx = lb % nb, by = (lb / nb) % nb, bz = lb / (nb * nb);
  // tile node (i, j, k) is lattice node (gx0 + i, gy0 + j, gz0 + k)
  const int gx0 = LT_B * bx + 1 - IT, gy0 = LT_B * by + 1 - IT, gz0 = LT_B * bz + 1 - IT;
  const int hi = n - 1;
  // the lane's tile nodes q = lane + u LT_NT (fixed for every phase), their
  // coordinates, and r there (in registers: each is read by its own lane)
  int qi[U], qj[U], qk[U];
  bool live[U], in[U];
  C rv[U], xv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = int(threadIdx.x) + u * LT_NT;
    live[u] = q < S3;
    const int qc = min(q, S3 - 1);
    qk[u] = qc / S2;
    qj[u] = (qc / S) % S;
    qi[u] = qc % S;
    const int gx = gx0 + qi[u], gy = gy0 + qj[u], gz = gz0 + qk[u];
    in[u] = live[u] && gx >= 1 && gx <= n - 2 && gy >= 1 && gy <= n - 2 && gz >= 1 && gz <= n - 2;
    const int64_t cx = min(max(gx, 0), hi), cy = min(max(gy, 0), hi), cz = min(max(gz, 0), hi);
    rv[u] = ld(r + cz * rpl + cy * rp + cx);
    xv[u] = C(0);
    if (!ZERO && !LAT) xv[u] = ld(xo + cz * cpl + cy * cp + cx);
  }
  const int cx0 = max(gx0, 0) >> 1, cy0 = max(gy0, 0) >> 1, cz0 = max(gz0, 0) >> 1;
  if (LAT) {
    const int nc = (n - 1) / 2 + 1;
    const T* pp = l1.zero_old ? l1.cur : l1.prev;  // (x_{it-1} = 0: loads a valid array, drops it)
    constexpr int UC = (SC3 + LT_NT - 1) / LT_NT;
    C pv[UC], cv[UC];
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int q = min(int(threadIdx.x) + u * LT_NT, SC3 - 1);
      const int k = q / SC2, j = (q / SC) % SC, i = q % SC;
      const int64_t o = int64_t(min(cz0 + k, nc - 1)) * l1.cpl + int64_t(min(cy0 + j, nc - 1)) * l1.cp +
                        min(cx0 + i, nc - 1);
      pv[u] = ld(pp + o);
      cv[u] = ld(l1.cur + o);
    }
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int q = int(threadIdx.x) + u * LT_NT;
      if (q < SC3) {
        Pc[q] = l1.zero_old ? C(0) : pv[u];
        Cc[q] = cv[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!in[u]) continue;
      const int gx = gx0 + qi[u], gy = gy0 + qj[u], gz = gz0 + qk[u];
      const int c0 = ((gz >> 1) - cz0) * SC2 + ((gy >> 1) - cy0) * SC + ((gx >> 1) - cx0);
      C v;
      if (!(gx & 1) && !(gy & 1) && !(gz & 1)) {
        v = Cc[c0];
      } else {
        const C tx = C(gx & 1) * C(0.5), ty = C(gy & 1) * C(0.5), tz = C(gz & 1) * C(0.5);
        const C* p = Pc + c0;
        const C* q2 = p + SC2;
        const C top = lerp(lerp(p[0], p[1], tx), lerp(p[SC], p[SC + 1], tx), ty);
        const C bot = lerp(lerp(q2[0], q2[1], tx), lerp(q2[SC], q2[SC + 1], tx), ty);
        v = lerp(top, bot, tz);
      }
      xv[u] = rnd<T>(v);
    }
    // (Pc and Cc live in X1, which the first iteration writes only after the
    // barrier that follows the writes of X0 below)
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (live[u]) X0[int(threadIdx.x) + u * LT_NT] = in[u] ? xv[u] : C(0);
  __syncthreads();
#pragma unroll
  for (int t = 1; t <= IT; ++t) {
    const C* __restrict__ src = (t & 1) ? X0 : X1;
    C* __restrict__ dst = (t & 1) ? X1 : X0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // the valid region after this iteration: tile nodes t .. S - 1 - t per axis
      if (!live[u] || qi[u] < t || qi[u] >= S - t || qj[u] < t || qj[u] >= S - t || qk[u] < t || qk[u] >= S - t)
        continue;
      const int c = int(threadIdx.x) + u * LT_NT;
      C v = C(0);
      if (in[u]) {
        v = relax_const<C>(src[c], ((src[c - 1] + src[c + 1]) + (src[c - S] + src[c + S])) + (src[c - S2] + src[c + S2]),
                           rv[u], w, hl2, C(6));
        dst[c] = rnd<T>(v);
      } else {
        dst[c] = C(0);
      }
      // the last iteration's region is the owned block: x_{IT-1} (src) and x_IT
      if (t == IT && in[u]) {
        const int64_t o = int64_t(gz0 + qk[u]) * cpl + int64_t(gy0 + qj[u]) * cp + (gx0 + qi[u]);
        st(xn + o, v);
        st(xp + o, src[c]);
      }
    }
    if (t < IT) __syncthreads();
  }
}

// The same for a 2D compact lattice: blocks of LT2_B^2 owned nodes with a
// halo of IT nodes, one lane per tile node (1024 lanes for four
// iterations).  Interpolation, node formula and rounding are those of
// k_lattice_2d_tb and k_level_transfer_2d.
constexpr int LT2_B = 24;
constexpr int LT2_NT = 1024;

template <typename T, bool ZERO, bool LAT, int IT>
__global__ __launch_bounds__(LT2_NT) void k_lattice_2d_tiled(
    const T* __restrict__ xo, T* __restrict__ xn, T* __restrict__ xp, int64_t cp, const T* __restrict__ r,
    int64_t rp, int n, int nb, typename Tr<T>::C w, typename Tr<T>::C hl2, const int* __restrict__ done,
    L1Src<T> l1) {
  using C = typename Tr<T>::C;
  if (*done) return;
  constexpr int S = LT2_B + 2 * IT, S2 = S * S, SC = S / 2 + 2, SC2 = SC * SC;
  __shared__ C X0[S2], X1[S2], R[S2], Pc[LAT ? SC2 : 1], Cc[LAT ? SC2 : 1];
  const int lb = int(xcd_order(blockIdx.x, gridDim.x));
  const int bx = lb % nb, by = lb / nb;
  // tile node (i, j) is lattice node (gx0 + i, gy0 + j)
  const int gx0 = LT2_B * bx + 1 - IT, gy0 = LT2_B * by + 1 - IT;
  const int hi = n - 1;
  auto interior = [&](int gx, int gy) { return gx >= 1 && gx <= n - 2 && gy >= 1 && gy <= n - 2; };
  const int q = threadIdx.x;  // one tile node per lane (S2 <= LT2_NT)
  const int qi = q % S, qj = q / S;
  const bool live = q < S2;
  const int gx = gx0 + qi, gy = gy0 + qj;
  if (live) {  // r and (neither ZERO nor LAT) x_0: clamped loads
    const int64_t cx = min(max(gx, 0), hi), cy = min(max(gy, 0), hi);
    R[q] = ld(r + cy * rp + cx);
    if (!ZERO && !LAT) {
      const C v = ld(xo + cy * cp + cx);
      X0[q] = interior(gx, gy) ? v : C(0);
    }
    if (ZERO) X0[q] = C(0);
  }
  const int cx0 = max(gx0, 0) >> 1, cy0 = max(gy0, 0) >> 1;
  if (LAT && q < SC2) {
    const int nc = (n - 1) / 2 + 1;
    const T* pp = l1.zero_old ? l1.cur : l1.prev;  // (x_{it-1} = 0: loads a valid array, drops it)
    const int64_t o = int64_t(min(cy0 + q / SC, nc - 1)) * l1.cp + min(cx0 + q % SC, nc - 1);
    const C pv = ld(pp + o);
    Pc[q] = l1.zero_old ? C(0) : pv;
    Cc[q] = ld(l1.cur + o);
  }
  __syncthreads();
  if (LAT) {
    if (live) {
      C v = C(0);
      if (interior(gx, gy)) {
        const int c0 = ((gy >> 1) - cy0) * SC + ((gx >> 1) - cx0);
        if (!(gx & 1) && !(gy & 1)) {
          v = Cc[c0];
        } else {
          const C tx = C(gx & 1) * C(0.5), ty = C(gy & 1) * C(0.5);
          const C top = lerp(Pc[c0], Pc[c0 + 1], tx), bot = lerp(Pc[c0 + SC], Pc[c0 + SC + 1], tx);
          v = lerp(top, bot, ty);
        }
        v = rnd<T>(v);
      }
      X0[q] = v;
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 1; t <= IT; ++t) {
    const C* __restrict__ src = (t & 1) ? X0 : X1;
    C* __restrict__ dst = (t & 1) ? X1 : X0;
    // valid region after this iteration: tile nodes t .. S - 1 - t per axis
    if (live && qi >= t && qi < S - t && qj >= t && qj < S - t) {
      C v = C(0);
      const bool in = interior(gx, gy);
      if (in) {
        v = relax_const<C>(src[q], (src[q - 1] + src[q + 1]) + (src[q - S] + src[q + S]), R[q], w, hl2, C(4));
        dst[q] = rnd<T>(v);
      } else {
        dst[q] = C(0);
      }
      // the last iteration's region is the owned block: x_{IT-1} and x_IT
      if (t == IT && in) {
        const int64_t o = int64_t(gy) * cp + gx;
        st(xn + o, v);
        st(xp + o, src[q]);
      }
    }
    if (t < IT) __syncthreads();
  }
}

// ------------------------------------------------------------ multi-level restriction
// P consecutive full-weighting restrictions of the cycle's chain, r_a ->
// r_{a+1} -> ... -> r_{a+P}, in one launch: the chain's coarse end, where
// every launch is latency-bound.  Each level is rounded to the storage type
// before the next is restricted from it, as the separate launches store and
// reload it, and the node formula and summation order are those of
// k_restrict_*, so every level gets the same bits.
//
// Workgroup b (per axis) owns the interior nodes B b + 1 .. B (b + 1) of
// level a + P and, at level a + P - j, the nodes 2^j B b + 1 .. 2^j B (b + 1):
// a partition of every level's interior.  Those depend on the nodes
// 2^j B b + 1 .. 2^j B b + S_j of level a + P - j, S_j = 2^j (B + 1) - 1, and
// tile node t of one level on tile nodes 2t .. 2t + 2 of the next finer one.
// The workgroup loads its tile of r_a into LDS (each lane issues up to
// MR_LB loads before it writes any of them), restricts level by level in
// LDS and writes the nodes it owns.  A tile's nodes past the last interior node are loaded clamped or
// skipped: interior coarse nodes read interior fine nodes only.
struct MultiRestrictLevel {
  void* r;  // the level's array at node (0, 0, 0)
  int64_t pitch, plane;
  int side;  // nodes per axis
  int off;   // LDS offset of the level's tile (elements; level a + P has none)
};
struct MultiRestrictPlan {
  MultiRestrictLevel lv[MR_MAX + 1];  // lv[j]: level a + P - j; lv[P] = r_a
  int P, B, nb;                       // nb: blocks per axis
};
constexpr int MR_NT = 1024;
constexpr int MR_LB = 8;  // tile loads a lane issues before writing LDS

template <typename T, int D>
__global__ __launch_bounds__(MR_NT) void k_restrict_multi(MultiRestrictPlan mp, const int* __restrict__ done) {
  using C = typename Tr<T>::C;
  if (*done) return;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  const int P = mp.P, B = mp.B, nb = mp.nb;
  // neighbouring blocks (shared halo loads) on one XCD
  const int lb = int(xcd_order(blockIdx.x, gridDim.x));
  const int bx = lb % nb, by = (lb / nb) % nb, bz = D == 3 ? lb / (nb * nb) : 0;
  auto tside = [&](int j) { return j == 0 ? B : ((B + 1) << j) - 1; };
  {
    const MultiRestrictLevel& L = mp.lv[P];
    const int S = tside(P), cnt = D == 2 ? S * S : S * S * S, o = B << P, hi = L.side - 2;
    const T* rf = static_cast<const T*>(L.r);
    const float inv = 1.0f / float(S);
    for (int i0 = 0; i0 < cnt; i0 += MR_LB * MR_NT) {
      C v[MR_LB];
#pragma unroll
      for (int k = 0; k < MR_LB; ++k) {
        const int i = min(i0 + k * MR_NT + int(threadIdx.x), cnt - 1);
        int I, J, K;
        tail_split<D>(i, S, inv, I, J, K);
        const int gx = min(o * bx + 1 + I, hi), gy = min(o * by + 1 + J, hi), gz = D == 3 ? min(o * bz + 1 + K, hi) : 0;
        v[k] = C(ld(rf + int64_t(gz) * L.plane + int64_t(gy) * L.pitch + gx));
      }
#pragma unroll
      for (int k = 0; k < MR_LB; ++k) {
        const int i = i0 + k * MR_NT + int(threadIdx.x);
        if (i < cnt) lds[L.off + i] = v[k];
      }
    }
  }
  __syncthreads();
  for (int j = P - 1; j >= 0; --j) {
    const MultiRestrictLevel& L = mp.lv[j];
    const int Sf = tside(j + 1), Sc = tside(j), own = B << j, hi = L.side - 2;
    const int cnt = D == 2 ? Sc * Sc : Sc * Sc * Sc, fp = Sf, fpl = Sf * Sf;
    const C* F = lds + mp.lv[j + 1].off;
    C* R = lds + L.off;
    T* out = static_cast<T*>(L.r);
    const float inv = 1.0f / float(Sc);
    for (int i = threadIdx.x; i < cnt; i += MR_NT) {
      int I, J, K;
      tail_split<D>(i, Sc, inv, I, J, K);
      const int gx = own * bx + 1 + I, gy = own * by + 1 + J, gz = D == 3 ? own * bz + 1 + K : 0;
      if (gx > hi || gy > hi || (D == 3 && gz > hi)) continue;
      auto rs = [&](int q) { return fmac(C(2), F[q], F[q - 1] + F[q + 1]); };
      C v;
      if (D == 2) {
        const int q = (2 * J + 1) * fp + 2 * I + 1;
        const C top = rs(q - fp), mid = rs(q), bot = rs(q + fp);
        v = fmac(C(2), mid, top + bot) * C(0.0625);
      } else {
        auto ps = [&](int q) { return fmac(C(2), rs(q), rs(q - fp) + rs(q + fp)); };
        const int q = (2 * K + 1) * fpl + (2 * J + 1) * fp + 2 * I + 1;
        const C top = ps(q - fpl), mid = ps(q), bot = ps(q + fpl);
        v = fmac(C(2), mid, top + bot) * C(0.015625);
      }
      if (j > 0) R[i] = rnd<T>(v);
      if (I < own && J < own && (D == 2 || K < own))
        st(out + int64_t(gz) * L.plane + int64_t(gy) * L.pitch + gx, v);
    }
    if (j > 0) __syncthreads();
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

// Start/stop events of the next launch (set by the profiler, else null):
// hipExtLaunchKernelGGL stamps them with the dispatch's own start and end.
namespace {
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;
}

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_ev_start = start;
  g_ev_stop = stop;
}

void current_launch_events(hipEvent_t* start, hipEvent_t* stop) {
  *start = g_ev_start;
  *stop = g_ev_stop;
}

#define HOMG_LAUNCH_SMEM(kernel, grid, block, smem, stream, ...)                              \
  do {                                                                                        \
    hipExtLaunchKernelGGL(kernel, grid, block, smem, stream, g_ev_start, g_ev_stop, 0,        \
                          __VA_ARGS__);                                                       \
    return hipGetLastError();                                                                 \
  } while (0)

#define HOMG_LAUNCH(kernel, grid, block, stream, ...) \
  HOMG_LAUNCH_SMEM(kernel, grid, block, 0, stream, __VA_ARGS__)

// Opt a kernel in to more than 64 KB of dynamic LDS.
template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

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
  const int inner = n - 2, len3 = inner < RES3_LEN ? inner : RES3_LEN;
  const dim3 g3(((inner + BX3 - 1) / BX3) * ((inner + 4 * BY3 - 1) / (4 * BY3)) * ((inner + len3 - 1) / len3));
  *count = int(g3.x);
  HOMG_LAUNCH((k_residual_3d<T>), g3, dim3(BX3, BY3), s, u + ul.off, ul.pitch, ul.plane,
              f + fl.off, fl.pitch, fl.plane, r, rl.pitch, rl.plane, n, len3, inv_h2, partials,
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

template <typename T>
static hipError_t residual_restrict_t(int n, const double* u, const Lay& ul, const double* f,
                                      const Lay& fl, void* r0, const Lay& rl, void* rc0,
                                      const Lay& cl, double* partials, int* count, const int* done,
                                      hipStream_t s) {
  const int len = rr_band(n);
  const int waves = rr_waves(n, len);
  *count = waves;
  const double h = 1.0 / double(n - 1);
  const double inv_h2 = 1.0 / (h * h);
  HOMG_LAUNCH((k_residual_restrict_2d<T>), dim3((waves + 3) / 4), dim3(256), s, u + ul.off, ul.pitch,
              f + fl.off, fl.pitch, static_cast<T*>(r0) + rl.off, rl.pitch, static_cast<T*>(rc0) + cl.off,
              cl.pitch, n, len, inv_h2, partials, done);
}

hipError_t launch_residual_restrict_2d(int prec, int n, const double* u, const Lay& ul,
                                       const double* f, const Lay& fl, void* r0, const Lay& rl,
                                       void* rc, const Lay& cl, double* partials, int* count,
                                       const int* done, hipStream_t s) {
  if (n < 5 || (n - 1) % 2 || cl.side != (n - 1) / 2 + 1) return hipErrorInvalidValue;
  switch (prec) {
    case PREC_F64: return residual_restrict_t<double>(n, u, ul, f, fl, r0, rl, rc, cl, partials, count, done, s);
    case PREC_F32: return residual_restrict_t<float>(n, u, ul, f, fl, r0, rl, rc, cl, partials, count, done, s);
    default: return residual_restrict_t<bf16>(n, u, ul, f, fl, r0, rl, rc, cl, partials, count, done, s);
  }
}

template <typename T>
static hipError_t l1_t(int d, int n, const double* uref, const double* u, const void* e, const Lay& el,
                       double* part, double* out, hipStream_t s) {
  const int64_t rows = d == 3 ? int64_t(n) * n : int64_t(n);
  const int nb = int(rows < L1_BLOCKS ? rows : L1_BLOCKS);
  if (e)
    hipExtLaunchKernelGGL((k_l1_partial<T, true>), dim3(nb), dim3(256), 0, s, g_ev_start, g_ev_stop, 0, uref, u,
                          static_cast<const T*>(e) + el.off, el.pitch, el.plane, n, d, part);
  else
    hipExtLaunchKernelGGL((k_l1_partial<T, false>), dim3(nb), dim3(256), 0, s, g_ev_start, g_ev_stop, 0, uref,
                          u, static_cast<const T*>(nullptr), int64_t(0), int64_t(0), n, d, part);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  HOMG_LAUNCH(k_l1_finish, dim3(1), dim3(256), s, part, nb, out);
}

int l1_partials() { return 2 * L1_BLOCKS; }

hipError_t launch_l1(int prec, int d, int n, const double* uref, const double* u, const void* e,
                     const Lay& el, double* part, double* out, hipStream_t s) {
  switch (prec) {
    case PREC_F64: return l1_t<double>(d, n, uref, u, e, el, part, out, s);
    case PREC_F32: return l1_t<float>(d, n, uref, u, e, el, part, out, s);
    default: return l1_t<bf16>(d, n, uref, u, e, el, part, out, s);
  }
}

hipError_t launch_finalize(const double* partials, int count, DevState* st, double* history,
                           int cycle, int mode, hipStream_t s) {
  HOMG_LAUNCH(k_finalize, dim3(1), dim3(FIN_NT), s, partials, count, st, history, cycle, mode);
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

template <typename TI>
static hipError_t restrict_to_f64_t(int d, const void* rf, const Lay& fl, double* rc, const Lay& cl,
                                    const int* done, hipStream_t s) {
  const int nc = cl.side;
  const int len = walk_len(d, nc);
  const dim3 g = grid_of(d, nc, len);
  const TI* f = static_cast<const TI*>(rf) + fl.off;
  double* c = rc + cl.off;
  if (d == 2) HOMG_LAUNCH((k_restrict_2d<TI, double>), g, dim3(BX2), s, f, fl.pitch, c, cl.pitch, nc, len, done);
  HOMG_LAUNCH((k_restrict_3d<TI, double>), g, dim3(BX3, BY3), s, f, fl.pitch, fl.plane, c, cl.pitch,
              cl.plane, nc, len, done);
}

hipError_t launch_restrict_to_f64(int prec, int d, const void* rf, const Lay& fl, double* rc,
                                  const Lay& cl, const int* done, hipStream_t s) {
  if (cl.side < 3) return hipSuccess;
  switch (prec) {
    case PREC_F64: return restrict_to_f64_t<double>(d, rf, fl, rc, cl, done, s);
    case PREC_F32: return restrict_to_f64_t<float>(d, rf, fl, rc, cl, done, s);
    default: return restrict_to_f64_t<bf16>(d, rf, fl, rc, cl, done, s);
  }
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

size_t restrict_multi_lds(int prec, int d, int P, int B) {
  const size_t cs = prec == PREC_F64 ? 8 : 4;
  size_t cnt = 0;
  for (int j = 1; j <= P; ++j) {
    const size_t S = size_t(((B + 1) << j) - 1);
    cnt += d == 2 ? S * S : S * S * S;
  }
  return cnt * cs;
}

template <typename T>
static hipError_t restrict_multi_t(int d, int P, int B, void* const* r, const Lay* l, const int* done,
                                   hipStream_t s) {
  MultiRestrictPlan mp{};
  mp.P = P;
  mp.B = B;
  mp.nb = (l[P].side - 1 + B - 1) / B;
  int off = 0;
  for (int j = 0; j <= P; ++j) {
    const Lay& L = l[P - j];
    mp.lv[j] = MultiRestrictLevel{static_cast<T*>(r[P - j]) + L.off, L.pitch, L.plane, L.side, off};
    if (j >= 1) {
      const int S = ((B + 1) << j) - 1;
      off += d == 2 ? S * S : S * S * S;
    }
  }
  const size_t lds = restrict_multi_lds(sizeof(T) == 8 ? PREC_F64 : PREC_F32, d, P, B);
  const unsigned blocks = d == 2 ? unsigned(mp.nb * mp.nb) : unsigned(mp.nb * mp.nb * mp.nb);
  if (d == 2) {
    hipError_t a = allow_lds(k_restrict_multi<T, 2>, lds);
    if (a != hipSuccess) return a;
    HOMG_LAUNCH_SMEM((k_restrict_multi<T, 2>), dim3(blocks), dim3(MR_NT), lds, s, mp, done);
  }
  hipError_t a = allow_lds(k_restrict_multi<T, 3>, lds);
  if (a != hipSuccess) return a;
  HOMG_LAUNCH_SMEM((k_restrict_multi<T, 3>), dim3(blocks), dim3(MR_NT), lds, s, mp, done);
}

hipError_t launch_restrict_multi(int prec, int d, int P, int B, void* const* r, const Lay* l, const int* done,
                                 hipStream_t s) {
  if (P < 1 || P > MR_MAX || B < 1 || l[P].side < 3) return hipErrorInvalidValue;
  switch (prec) {
    case PREC_F64: return restrict_multi_t<double>(d, P, B, r, l, done, s);
    case PREC_F32: return restrict_multi_t<float>(d, P, B, r, l, done, s);
    default: return restrict_multi_t<bf16>(d, P, B, r, l, done, s);
  }
}

template <typename T, int MODE>
static hipError_t sweep_tm(int d, int n, int m, double omega, const void* eo_, void* en_,
                           const Lay& el, const void* rm_, const Lay& rl, const double* am,
                           const Lay& al, double* u, const Lay& ul, const int* done,
                           bool compact, hipStream_t s) {
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
    if (m == 0 && compact) {
      if (am)
        HOMG_LAUNCH((k_lattice_sweep_2d<T, MODE, true>), g, dim3(BX2), s, eo, en, el.pitch, rm,
                    rl.pitch, a, al.pitch, uu, ul.pitch, n, len, w, hl2, done);
      HOMG_LAUNCH((k_lattice_sweep_2d<T, MODE, false>), g, dim3(BX2), s, eo, en, el.pitch, rm,
                  rl.pitch, a, al.pitch, uu, ul.pitch, n, len, w, hl2, done);
    }
    if (m == 0) {
      // walks of 8 rows, one-dimensional grid in XCD order
      const int inner = n - 2, len0 = inner < 8 ? inner : 8;
      const dim3 g1(t2_gx(n) * t2_gy(n, len0));
      if (am)
        HOMG_LAUNCH((k_sweep_2d_l0<T, MODE, true>), g1, dim3(BX2), s, eo, en, el.pitch, rm,
                    rl.pitch, a, al.pitch, uu, ul.pitch, n, len0, w, hl2, done);
      HOMG_LAUNCH((k_sweep_2d_l0<T, MODE, false>), g1, dim3(BX2), s, eo, en, el.pitch, rm,
                  rl.pitch, a, al.pitch, uu, ul.pitch, n, len0, w, hl2, done);
    }
    if (am)
      HOMG_LAUNCH((k_sweep_2d_coarse<T, MODE, true>), g, dim3(BX2), s, eo, en, el.pitch, rm,
                  rl.pitch, a, al.pitch, uu, ul.pitch, n, len, m, w, hl2, done);
    HOMG_LAUNCH((k_sweep_2d_coarse<T, MODE, false>), g, dim3(BX2), s, eo, en, el.pitch, rm,
                rl.pitch, a, al.pitch, uu, ul.pitch, n, len, m, w, hl2, done);
  }
  const C w = C(omega / 6.0);
  // level 0: lanes own R3Y rows each, walks of RES3_LEN planes, one
  // XCD-ordered dimension
  const int inner = n - 2, len0 = inner < RES3_LEN ? inner : RES3_LEN;
  const dim3 g0(unsigned((inner + BX3 - 1) / BX3) * unsigned((inner + BY3 * R3Y - 1) / (BY3 * R3Y)) *
                unsigned((inner + len0 - 1) / len0));
  if (m == 0 && compact)
    HOMG_LAUNCH((k_lattice_sweep_3d<T, MODE>), g0, dim3(BX3, BY3), s, eo, en, el.pitch, el.plane,
                rm, rl.pitch, rl.plane, uu, ul.pitch, ul.plane, n, len0, w, hl2, done);
  if (m == 0)
    HOMG_LAUNCH((k_sweep_3d_l0<T, MODE>), g0, dim3(BX3, BY3), s, eo, en, el.pitch, el.plane, rm,
                rl.pitch, rl.plane, uu, ul.pitch, ul.plane, n, len0, w, hl2, done);
  HOMG_LAUNCH((k_sweep_3d_coarse<T, MODE>), g, dim3(BX3, BY3), s, eo, en, el.pitch, el.plane,
              rm, rl.pitch, rl.plane, uu, ul.pitch, ul.plane, n, len, m, w, hl2, done);
}

// Device view of a level-1 state (null: the pass reads eo).
template <typename T>
static L1Src<T> l1_src(const L1State* l1) {
  L1Src<T> v{};
  if (l1) {
    v.prev = l1->prev ? static_cast<const T*>(l1->prev) + l1->cl.off : nullptr;
    v.cur = static_cast<const T*>(l1->cur) + l1->cl.off;
    v.cp = l1->cl.pitch;
    v.cpl = l1->cl.plane;
    v.zero_old = l1->zero_old ? 1 : 0;
  }
  return v;
}

// Checks a level-1 state against a level-0 side n.
static bool l1_ok(const L1State* l1, int d, int n) {
  if (!l1) return true;
  return l1->cur && (l1->zero_old || l1->prev) && l1->cl.side == (n - 1) / 2 + 1 && n >= 5 &&
         l1->cl.pitch >= l1->cl.side && (d == 2 || l1->cl.plane >= l1->cl.pitch * l1->cl.side);
}

template <typename T, bool ZERO, bool ACCUM, bool LAT>
static hipError_t tb_t(int n, int it, int len, double omega, const void* eo_, void* en_, const Lay& el,
                       const void* rm_, const Lay& rl, double* u, const Lay& ul, const L1Src<T>& l1,
                       const int* done, hipStream_t s) {
  using C = typename Tr<T>::C;
  const T* eo = eo_ ? static_cast<const T*>(eo_) + el.off : nullptr;
  T* en = en_ ? static_cast<T*>(en_) + el.off : nullptr;
  const T* rm = static_cast<const T*>(rm_) + rl.off;
  double* uu = u ? u + ul.off : nullptr;
  const double h = 1.0 / double(n - 1);
  const C w = C(omega / 4.0), hl2 = C(h * h);
  const dim3 g(tb_blocks(n, it, len));
#define TB2_ARGS eo, en, el.pitch, rm, rl.pitch, uu, ul.pitch, n, len, w, hl2, done, l1
  switch (it) {
    case 1: HOMG_LAUNCH((k_sweep_2d_l0_tb<T, ZERO, ACCUM, 1, LAT>), g, dim3(256), s, TB2_ARGS);
    case 2: HOMG_LAUNCH((k_sweep_2d_l0_tb<T, ZERO, ACCUM, 2, LAT>), g, dim3(256), s, TB2_ARGS);
    case 3: HOMG_LAUNCH((k_sweep_2d_l0_tb<T, ZERO, ACCUM, 3, LAT>), g, dim3(256), s, TB2_ARGS);
    default: HOMG_LAUNCH((k_sweep_2d_l0_tb<T, ZERO, ACCUM, 4, LAT>), g, dim3(256), s, TB2_ARGS);
  }
#undef TB2_ARGS
}

template <typename T>
static hipError_t tb_tz(int n, int it, int len, double omega, const void* eo, void* en, const Lay& el,
                        const void* rm, const Lay& rl, double* u, const Lay& ul, bool zero, bool accum,
                        const L1State* l1, const int* done, hipStream_t s) {
  const L1Src<T> v = l1_src<T>(l1);
#define TB2_ARGS n, it, len, omega, eo, en, el, rm, rl, u, ul, v, done, s
  if (l1)  // the pass takes its e from level 1's compact state
    return accum ? tb_t<T, false, true, true>(TB2_ARGS) : tb_t<T, false, false, true>(TB2_ARGS);
  if (zero)
    return accum ? tb_t<T, true, true, false>(TB2_ARGS) : tb_t<T, true, false, false>(TB2_ARGS);
  return accum ? tb_t<T, false, true, false>(TB2_ARGS) : tb_t<T, false, false, false>(TB2_ARGS);
#undef TB2_ARGS
}

template <typename T, bool ZERO, bool PREV, bool LAT>
static hipError_t ltb_t(int nm, int it, int len, double omega, const void* eo_, void* en_, void* ep_,
                        const Lay& cl, const void* rm_, const Lay& rl, const L1Src<T>& l1, const int* done,
                        hipStream_t s) {
  using C = typename Tr<T>::C;
  const T* eo = eo_ ? static_cast<const T*>(eo_) + cl.off : nullptr;
  T* en = static_cast<T*>(en_) + cl.off;
  T* epv = ep_ ? static_cast<T*>(ep_) + cl.off : nullptr;
  const T* rm = static_cast<const T*>(rm_) + rl.off;
  const double h = 1.0 / double(nm - 1);
  const C w = C(omega / 4.0), hl2 = C(h * h);
  const dim3 g(tb_blocks(nm, it, len));
#define LTB_ARGS eo, en, epv, cl.pitch, rm, rl.pitch, nm, len, w, hl2, done, l1
  switch (it) {
    case 1: HOMG_LAUNCH((k_lattice_2d_tb<T, ZERO, PREV, 1, LAT>), g, dim3(256), s, LTB_ARGS);
    case 2: HOMG_LAUNCH((k_lattice_2d_tb<T, ZERO, PREV, 2, LAT>), g, dim3(256), s, LTB_ARGS);
    case 3: HOMG_LAUNCH((k_lattice_2d_tb<T, ZERO, PREV, 3, LAT>), g, dim3(256), s, LTB_ARGS);
    default: HOMG_LAUNCH((k_lattice_2d_tb<T, ZERO, PREV, 4, LAT>), g, dim3(256), s, LTB_ARGS);
  }
#undef LTB_ARGS
}

template <typename T>
static hipError_t ltb_tz(int nm, int it, int len, double omega, const void* eo, void* en, void* eprev,
                         const Lay& cl, const void* rm, const Lay& rl, bool zero, const L1State* l1,
                         const int* done, hipStream_t s) {
  const L1Src<T> v = l1_src<T>(l1);
#define LTB_ARGS nm, it, len, omega, eo, en, eprev, cl, rm, rl, v, done, s
  if (l1)
    return eprev ? ltb_t<T, false, true, true>(LTB_ARGS) : ltb_t<T, false, false, true>(LTB_ARGS);
  if (zero)
    return eprev ? ltb_t<T, true, true, false>(LTB_ARGS) : ltb_t<T, true, false, false>(LTB_ARGS);
  return eprev ? ltb_t<T, false, true, false>(LTB_ARGS) : ltb_t<T, false, false, false>(LTB_ARGS);
#undef LTB_ARGS
}

hipError_t launch_lattice_2d_tb(int prec, int nm, int it, double omega, const void* eo, void* en,
                                void* eprev, const Lay& cl, const void* rm, const Lay& rl, bool zero,
                                const int* done, hipStream_t s, int len, const L1State* l1) {
  if (len == 0) len = tb_band(nm, it);
  if (nm < 3 || it < 1 || it > TB_MAX_IT || len < 1 || (l1 && zero) || !l1_ok(l1, 2, nm))
    return hipErrorInvalidValue;
  switch (prec) {
    case PREC_F64: return ltb_tz<double>(nm, it, len, omega, eo, en, eprev, cl, rm, rl, zero, l1, done, s);
    case PREC_F32: return ltb_tz<float>(nm, it, len, omega, eo, en, eprev, cl, rm, rl, zero, l1, done, s);
    default: return ltb_tz<bf16>(nm, it, len, omega, eo, en, eprev, cl, rm, rl, zero, l1, done, s);
  }
}

hipError_t launch_sweep_2d_l0_tb(int prec, int n, int it, double omega, const void* eo, void* en,
                                 const Lay& el, const void* rm, const Lay& rl, double* u,
                                 const Lay& ul, bool zero, bool accum, const int* done, hipStream_t s,
                                 int len, const L1State* l1) {
  if (len == 0) len = tb_band(n, it);
  if (n < 3 || it < 1 || it > TB_MAX_IT || len < 1 || (l1 && zero) || !l1_ok(l1, 2, n))
    return hipErrorInvalidValue;
  switch (prec) {
    case PREC_F64: return tb_tz<double>(n, it, len, omega, eo, en, el, rm, rl, u, ul, zero, accum, l1, done, s);
    case PREC_F32: return tb_tz<float>(n, it, len, omega, eo, en, el, rm, rl, u, ul, zero, accum, l1, done, s);
    default: return tb_tz<bf16>(n, it, len, omega, eo, en, el, rm, rl, u, ul, zero, accum, l1, done, s);
  }
}

int tb_band(int n, int it) {
  for (int len : {64, 32, 16, 8})
    if (tb_waves(n, it, len) >= TB_MIN_WAVES) return len;
  return 4;
}

int tb3_blocks(int n, int it, int len) {
  const int vx = BX3 - 2 * it, vy = TB3_TY - 2 * it;
  return ((n - 2 + vx - 1) / vx) * ((n - 2 + vy - 1) / vy) * ((n - 2 + len - 1) / len);
}

int tb3_band(int n, int it) {
  for (int len : {32, 16, 8})
    if (tb3_blocks(n, it, len) >= TB3_MIN_BLOCKS) return len;
  return 4;
}

template <typename T, bool ZERO, bool ACCUM, bool PREV, bool LAT>
static hipError_t tb3_t(int n, int it, int len, double omega, const void* eo_, void* en_, void* ep_,
                        const Lay& el, const void* rm_, const Lay& rl, double* u, const Lay& ul,
                        bool compact, const L1Src<T>& l1, const int* done, hipStream_t s) {
  using C = typename Tr<T>::C;
  const T* eo = eo_ ? static_cast<const T*>(eo_) + el.off : nullptr;
  T* en = en_ ? static_cast<T*>(en_) + el.off : nullptr;
  T* epv = ep_ ? static_cast<T*>(ep_) + el.off : nullptr;
  const T* rm = static_cast<const T*>(rm_) + rl.off;
  double* uu = u ? u + ul.off : nullptr;
  const double h = 1.0 / double(n - 1);
  const C w = C(omega / 6.0), hl2 = C(h * h);
  const dim3 g(tb3_blocks(n, it, len)), blk(BX3, BY3);
  if (compact && !ACCUM) {  // compact lattice of a coarse level
    if (it == 1)
      HOMG_LAUNCH((k_lattice_3d_tb<T, ZERO, PREV, 1, LAT>), g, blk, s, eo, en, epv, el.pitch, el.plane, rm,
                  rl.pitch, rl.plane, n, len, w, hl2, done, l1);
    HOMG_LAUNCH((k_lattice_3d_tb<T, ZERO, PREV, 2, LAT>), g, blk, s, eo, en, epv, el.pitch, el.plane, rm,
                rl.pitch, rl.plane, n, len, w, hl2, done, l1);
  }
#define TB3_ARGS eo, en, el.pitch, el.plane, rm, rl.pitch, rl.plane, uu, ul.pitch, ul.plane, n, len, w, hl2, done, l1
  if (it == 1) HOMG_LAUNCH((k_sweep_3d_l0_tb<T, ZERO, ACCUM, 1, LAT>), g, blk, s, TB3_ARGS);
  HOMG_LAUNCH((k_sweep_3d_l0_tb<T, ZERO, ACCUM, 2, LAT>), g, blk, s, TB3_ARGS);
#undef TB3_ARGS
}

template <typename T>
static hipError_t tb3_tz(int n, int it, int len, double omega, const void* eo, void* en, void* eprev,
                         const Lay& el, const void* rm, const Lay& rl, double* u, const Lay& ul,
                         bool zero, bool accum, bool compact, const L1State* l1, const int* done,
                         hipStream_t s) {
  const L1Src<T> v = l1_src<T>(l1);
#define TB3_ARGS n, it, len, omega, eo, en, eprev, el, rm, rl, u, ul, compact, v, done, s
  if (l1 && compact)  // a compact lattice taking x_0 from the next coarser level's state
    return eprev ? tb3_t<T, false, false, true, true>(TB3_ARGS) : tb3_t<T, false, false, false, true>(TB3_ARGS);
  if (l1)  // level 0 taking its e from level 1's compact state
    return accum ? tb3_t<T, false, true, false, true>(TB3_ARGS) : tb3_t<T, false, false, false, true>(TB3_ARGS);
  if (accum)
    return zero ? tb3_t<T, true, true, false, false>(TB3_ARGS) : tb3_t<T, false, true, false, false>(TB3_ARGS);
  if (eprev)
    return zero ? tb3_t<T, true, false, true, false>(TB3_ARGS) : tb3_t<T, false, false, true, false>(TB3_ARGS);
  return zero ? tb3_t<T, true, false, false, false>(TB3_ARGS) : tb3_t<T, false, false, false, false>(TB3_ARGS);
#undef TB3_ARGS
}

template <typename T, bool ZERO, bool LAT, int IT>
static hipError_t lt2_t(int n, double omega, const void* xo_, void* xn_, void* xp_, const Lay& cl,
                        const void* rm_, const Lay& rl, const L1Src<T>& l1, const int* done, hipStream_t s) {
  using C = typename Tr<T>::C;
  const T* xo = xo_ ? static_cast<const T*>(xo_) + cl.off : nullptr;
  T* xn = static_cast<T*>(xn_) + cl.off;
  T* xp = static_cast<T*>(xp_) + cl.off;
  const T* rm = static_cast<const T*>(rm_) + rl.off;
  const double h = 1.0 / double(n - 1);
  const C w = C(omega / 4.0), hl2 = C(h * h);
  const int nb = (n - 2 + LT2_B - 1) / LT2_B;
  HOMG_LAUNCH((k_lattice_2d_tiled<T, ZERO, LAT, IT>), dim3(unsigned(nb) * nb), dim3(LT2_NT), s, xo, xn, xp,
              cl.pitch, rm, rl.pitch, n, nb, w, hl2, done, l1);
}

template <typename T, int IT>
static hipError_t lt2_it(int n, double omega, const void* xo, void* xn, void* xp, const Lay& cl, const void* rm,
                         const Lay& rl, bool zero, const L1State* l1, const int* done, hipStream_t s) {
  const L1Src<T> v = l1_src<T>(l1);
  if (l1) return lt2_t<T, false, true, IT>(n, omega, xo, xn, xp, cl, rm, rl, v, done, s);
  if (zero) return lt2_t<T, true, false, IT>(n, omega, xo, xn, xp, cl, rm, rl, v, done, s);
  return lt2_t<T, false, false, IT>(n, omega, xo, xn, xp, cl, rm, rl, v, done, s);
}

template <typename T>
static hipError_t lt2_tz(int n, int it, double omega, const void* xo, void* xn, void* xp, const Lay& cl,
                         const void* rm, const Lay& rl, bool zero, const L1State* l1, const int* done,
                         hipStream_t s) {
  switch (it) {
    case 1: return lt2_it<T, 1>(n, omega, xo, xn, xp, cl, rm, rl, zero, l1, done, s);
    case 2: return lt2_it<T, 2>(n, omega, xo, xn, xp, cl, rm, rl, zero, l1, done, s);
    case 3: return lt2_it<T, 3>(n, omega, xo, xn, xp, cl, rm, rl, zero, l1, done, s);
    default: return lt2_it<T, 4>(n, omega, xo, xn, xp, cl, rm, rl, zero, l1, done, s);
  }
}

hipError_t launch_lattice_2d_tiled(int prec, int n, int it, double omega, const void* xo, void* xn, void* xprev,
                                   const Lay& cl, const void* rm, const Lay& rl, bool zero, const L1State* l1,
                                   const int* done, hipStream_t s) {
  if (n < 3 || it < 1 || it > LT_MAX_IT || !xn || !xprev || (l1 && zero) || (!l1 && !zero && !xo) ||
      !l1_ok(l1, 2, n) || xn == xo || xprev == xo || xn == xprev)
    return hipErrorInvalidValue;
  switch (prec) {
    case PREC_F64: return lt2_tz<double>(n, it, omega, xo, xn, xprev, cl, rm, rl, zero, l1, done, s);
    case PREC_F32: return lt2_tz<float>(n, it, omega, xo, xn, xprev, cl, rm, rl, zero, l1, done, s);
    default: return lt2_tz<bf16>(n, it, omega, xo, xn, xprev, cl, rm, rl, zero, l1, done, s);
  }
}

size_t lattice_3d_tiled_lds(int prec, int it) {
  const size_t S = size_t(LT_B + 2 * it);
  return 2 * S * S * S * (prec == PREC_F64 ? 8 : 4);  // the two iterates (r stays in registers)
}

template <typename T, bool ZERO, bool LAT, int IT>
static hipError_t lt3_t(int n, double omega, const void* xo_, void* xn_, void* xp_, const Lay& cl,
                        const void* rm_, const Lay& rl, const L1Src<T>& l1, const int* done, hipStream_t s) {
  using C = typename Tr<T>::C;
  const T* xo = xo_ ? static_cast<const T*>(xo_) + cl.off : nullptr;
  T* xn = static_cast<T*>(xn_) + cl.off;
  T* xp = static_cast<T*>(xp_) + cl.off;
  const T* rm = static_cast<const T*>(rm_) + rl.off;
  const double h = 1.0 / double(n - 1);
  const C w = C(omega / 6.0), hl2 = C(h * h);
  const int nb = (n - 2 + LT_B - 1) / LT_B;
  const size_t lds = lattice_3d_tiled_lds(sizeof(T) == 8 ? PREC_F64 : PREC_F32, IT);
  hipError_t a = allow_lds(k_lattice_3d_tiled<T, ZERO, LAT, IT>, lds);
  if (a != hipSuccess) return a;
  HOMG_LAUNCH_SMEM((k_lattice_3d_tiled<T, ZERO, LAT, IT>), dim3(unsigned(nb) * nb * nb), dim3(LT_NT), lds, s, xo,
                   xn, xp, cl.pitch, cl.plane, rm, rl.pitch, rl.plane, n, nb, w, hl2, done, l1);
}

template <typename T, int IT>
static hipError_t lt3_it(int n, double omega, const void* xo, void* xn, void* xp, const Lay& cl, const void* rm,
                         const Lay& rl, bool zero, const L1State* l1, const int* done, hipStream_t s) {
  const L1Src<T> v = l1_src<T>(l1);
  if (l1) return lt3_t<T, false, true, IT>(n, omega, xo, xn, xp, cl, rm, rl, v, done, s);
  if (zero) return lt3_t<T, true, false, IT>(n, omega, xo, xn, xp, cl, rm, rl, v, done, s);
  return lt3_t<T, false, false, IT>(n, omega, xo, xn, xp, cl, rm, rl, v, done, s);
}

template <typename T>
static hipError_t lt3_tz(int n, int it, double omega, const void* xo, void* xn, void* xp, const Lay& cl,
                         const void* rm, const Lay& rl, bool zero, const L1State* l1, const int* done,
                         hipStream_t s) {
  switch (it) {
    case 1: return lt3_it<T, 1>(n, omega, xo, xn, xp, cl, rm, rl, zero, l1, done, s);
    case 2: return lt3_it<T, 2>(n, omega, xo, xn, xp, cl, rm, rl, zero, l1, done, s);
    case 3: return lt3_it<T, 3>(n, omega, xo, xn, xp, cl, rm, rl, zero, l1, done, s);
    default: return lt3_it<T, 4>(n, omega, xo, xn, xp, cl, rm, rl, zero, l1, done, s);
  }
}

hipError_t launch_lattice_3d_tiled(int prec, int n, int it, double omega, const void* xo, void* xn, void* xprev,
                                   const Lay& cl, const void* rm, const Lay& rl, bool zero, const L1State* l1,
                                   const int* done, hipStream_t s) {
  if (n < 3 || it < 1 || it > LT_MAX_IT || !xn || !xprev || (l1 && zero) || (!l1 && !zero && !xo) ||
      !l1_ok(l1, 3, n) || xn == xo || xprev == xo || xn == xprev)
    return hipErrorInvalidValue;
  switch (prec) {
    case PREC_F64: return lt3_tz<double>(n, it, omega, xo, xn, xprev, cl, rm, rl, zero, l1, done, s);
    case PREC_F32: return lt3_tz<float>(n, it, omega, xo, xn, xprev, cl, rm, rl, zero, l1, done, s);
    default: return lt3_tz<bf16>(n, it, omega, xo, xn, xprev, cl, rm, rl, zero, l1, done, s);
  }
}

hipError_t launch_tb_3d(int prec, int n, int it, double omega, const void* eo, void* en, void* eprev,
                        const Lay& el, const void* rm, const Lay& rl, double* u, const Lay& ul,
                        bool zero, bool accum, bool compact, const int* done, hipStream_t s, int len,
                        const L1State* l1) {
  if (len == 0) len = tb3_band(n, it);
  if (n < 3 || it < 1 || it > TB3_MAX_IT || len < 1 || (accum && (eprev || compact)) ||
      (l1 && (zero || (eprev && !compact))) || !l1_ok(l1, 3, n))
    return hipErrorInvalidValue;
  switch (prec) {
    case PREC_F64: return tb3_tz<double>(n, it, len, omega, eo, en, eprev, el, rm, rl, u, ul, zero, accum, compact, l1, done, s);
    case PREC_F32: return tb3_tz<float>(n, it, len, omega, eo, en, eprev, el, rm, rl, u, ul, zero, accum, compact, l1, done, s);
    default: return tb3_tz<bf16>(n, it, len, omega, eo, en, eprev, el, rm, rl, u, ul, zero, accum, compact, l1, done, s);
  }
}

template <typename T>
static hipError_t sweep_t(int d, int n, int m, double omega, const void* eo, void* en,
                          const Lay& el, const void* rm, const Lay& rl, const double* am,
                          const Lay& al, double* u, const Lay& ul, int mode, const int* done,
                          bool compact, hipStream_t s) {
  switch (mode & 3) {
    case 0: return sweep_tm<T, 0>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, done, compact, s);
    case 1: return sweep_tm<T, 1>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, done, compact, s);
    case 2: return sweep_tm<T, 2>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, done, compact, s);
    default: return sweep_tm<T, 3>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, done, compact, s);
  }
}

hipError_t launch_sweep(int prec, int d, int n, int m, double omega, const void* eo, void* en,
                        const Lay& el, const void* rm, const Lay& rl, const double* am,
                        const Lay& al, double* u, const Lay& ul, int mode, const int* done,
                        hipStream_t s, bool compact) {
  switch (prec) {
    case PREC_F64: return sweep_t<double>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, mode, done, compact, s);
    case PREC_F32: return sweep_t<float>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, mode, done, compact, s);
    default: return sweep_t<bf16>(d, n, m, omega, eo, en, el, rm, rl, am, al, u, ul, mode, done, compact, s);
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

// ------------------------------------------------------------ level-blocked launchers

// FP64 compact copy (exact widening) of the level-l lattice of an array
// stored in T; every node of the compact side, boundary included.
template <typename T>
__global__ __launch_bounds__(256) void k_widen(const T* __restrict__ src, int64_t sp, int64_t spl, int l,
                                               double* __restrict__ dst, int64_t dp, int64_t dpl, int side,
                                               int nz, const int* __restrict__ done) {
  if (*done) return;
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= side || z >= nz) return;
  dst[int64_t(z) * dpl + int64_t(y) * dp + x] =
      double(ld(src + int64_t(z) * l * spl + int64_t(y) * l * sp + int64_t(x) * l));
}

hipError_t launch_widen(int prec, int d, const void* src, const Lay& sl, int l, double* dst,
                        const Lay& dl, const int* done, hipStream_t s) {
  const int side = dl.side, nz = d == 3 ? side : 1;
  const dim3 g = copy_grid(d, side);
  switch (prec) {
    case PREC_F64:
      HOMG_LAUNCH((k_widen<double>), g, dim3(256), s, static_cast<const double*>(src) + sl.off, sl.pitch,
                  sl.plane, l, dst + dl.off, dl.pitch, dl.plane, side, nz, done);
    case PREC_F32:
      HOMG_LAUNCH((k_widen<float>), g, dim3(256), s, static_cast<const float*>(src) + sl.off, sl.pitch,
                  sl.plane, l, dst + dl.off, dl.pitch, dl.plane, side, nz, done);
    default:
      HOMG_LAUNCH((k_widen<bf16>), g, dim3(256), s, static_cast<const bf16*>(src) + sl.off, sl.pitch,
                  sl.plane, l, dst + dl.off, dl.pitch, dl.plane, side, nz, done);
  }
}

// FP64 compact array -> storage type T (rounded as k_pack rounds: to FP32,
// then, for BF16, to BF16), every node of the compact side.
template <typename T>
__global__ __launch_bounds__(256) void k_narrow(const double* __restrict__ src, int64_t sp, int64_t spl,
                                                T* __restrict__ dst, int64_t dp, int64_t dpl, int side, int nz,
                                                const int* __restrict__ done) {
  if (*done) return;
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int z = blockIdx.z;
  if (x >= side || z >= nz) return;
  st(dst + int64_t(z) * dpl + int64_t(y) * dp + x, typename Tr<T>::C(src[int64_t(z) * spl + int64_t(y) * sp + x]));
}

hipError_t launch_narrow(int prec, int d, const double* src, const Lay& sl, void* dst, const Lay& dl,
                         const int* done, hipStream_t s) {
  const int side = sl.side, nz = d == 3 ? side : 1;
  const dim3 g = copy_grid(d, side);
  switch (prec) {
    case PREC_F64:
      HOMG_LAUNCH((k_narrow<double>), g, dim3(256), s, src + sl.off, sl.pitch, sl.plane,
                  static_cast<double*>(dst) + dl.off, dl.pitch, dl.plane, side, nz, done);
    case PREC_F32:
      HOMG_LAUNCH((k_narrow<float>), g, dim3(256), s, src + sl.off, sl.pitch, sl.plane,
                  static_cast<float*>(dst) + dl.off, dl.pitch, dl.plane, side, nz, done);
    default:
      HOMG_LAUNCH((k_narrow<bf16>), g, dim3(256), s, src + sl.off, sl.pitch, sl.plane,
                  static_cast<bf16*>(dst) + dl.off, dl.pitch, dl.plane, side, nz, done);
  }
}

hipError_t launch_gather(int prec, int d, const void* src, const Lay& sl, int l, void* dst,
                         const Lay& dl, const int* done, hipStream_t s) {
  (void)done;
  const int side = dl.side, nz = d == 3 ? side : 1;
  const dim3 g = copy_grid(d, side);
  switch (prec) {
    case PREC_F64:
      HOMG_LAUNCH((k_gather<double>), g, dim3(256), s, static_cast<const double*>(src) + sl.off,
                  sl.pitch, sl.plane, l, static_cast<double*>(dst) + dl.off, dl.pitch, dl.plane, side, nz);
    case PREC_F32:
      HOMG_LAUNCH((k_gather<float>), g, dim3(256), s, static_cast<const float*>(src) + sl.off,
                  sl.pitch, sl.plane, l, static_cast<float*>(dst) + dl.off, dl.pitch, dl.plane, side, nz);
    default:
      HOMG_LAUNCH((k_gather<bf16>), g, dim3(256), s, static_cast<const bf16*>(src) + sl.off,
                  sl.pitch, sl.plane, l, static_cast<bf16*>(dst) + dl.off, dl.pitch, dl.plane, side, nz);
  }
}

size_t lattice_small_lds(int prec, int d, int nm, bool var) {
  const size_t cs = prec == PREC_F64 ? 8 : 4;
  const size_t cnt = d == 2 ? size_t(nm) * nm : size_t(nm) * nm * nm;
  size_t b = 3 * cnt * cs;
  if (var) b = ((b + 15) & ~size_t(15)) + cnt * 8;
  return b;
}

template <typename T, bool ZERO>
static hipError_t small_tz(int d, int nm, int l, int it, double omega, const void* e, const Lay& el,
                           const void* rm, const Lay& rl, const double* am, const Lay& al,
                           void* xprev, void* xcur, const Lay& cl, const int* done, hipStream_t s) {
  using C = typename Tr<T>::C;
  const double hl = 1.0 / double(nm - 1);
  const C hl2 = C(hl * hl);
  const size_t lds = lattice_small_lds(sizeof(T) == 8 ? PREC_F64 : PREC_F32, d, nm, am != nullptr);
  const T* ee = static_cast<const T*>(e) + el.off;
  const T* r = static_cast<const T*>(rm) + rl.off;
  T* xp = static_cast<T*>(xprev) + cl.off;
  T* xc = static_cast<T*>(xcur) + cl.off;
  if (d == 2) {
    if (am) {
      hipError_t a = allow_lds(k_lattice_small_2d<T, ZERO, true>, lds);
      if (a != hipSuccess) return a;
      HOMG_LAUNCH_SMEM((k_lattice_small_2d<T, ZERO, true>), dim3(1), dim3(SMALL_NT), lds, s, ee,
                       el.pitch, l, r, rl.pitch, am + al.off, al.pitch, xp, xc, cl.pitch, nm, it,
                       C(omega), hl2, done);
    }
    hipError_t a = allow_lds(k_lattice_small_2d<T, ZERO, false>, lds);
    if (a != hipSuccess) return a;
    HOMG_LAUNCH_SMEM((k_lattice_small_2d<T, ZERO, false>), dim3(1), dim3(SMALL_NT), lds, s, ee,
                     el.pitch, l, r, rl.pitch, (const double*)nullptr, int64_t(0), xp, xc, cl.pitch,
                     nm, it, C(omega / 4.0), hl2, done);
  }
  hipError_t a = allow_lds(k_lattice_small_3d<T, ZERO>, lds);
  if (a != hipSuccess) return a;
  HOMG_LAUNCH_SMEM((k_lattice_small_3d<T, ZERO>), dim3(1), dim3(SMALL_NT), lds, s, ee, el.pitch,
                   el.plane, l, r, rl.pitch, rl.plane, xp, xc, cl.pitch, cl.plane, nm, it,
                   C(omega / 6.0), hl2, done);
}

size_t coarse_tail_lds(int prec, int d, int nms, int nlev, bool top64) {
  const size_t cs = prec == PREC_F64 ? 8 : 4;
  size_t cnt = 0, ctop = 0;
  for (int k = 0; k < nlev; ++k) {
    const size_t nk = size_t((nms - 1) >> k) + 1;
    ctop = d == 2 ? nk * nk : nk * nk * nk;
    cnt += 3 * ctop;
  }
  size_t b = cnt * cs;
  if (top64 && prec != PREC_F64) b = ((b + 15) & ~size_t(15)) + 3 * ctop * 8;
  return b;
}

template <typename T, bool TOP64>
static hipError_t tail_t(int d, int nms, int nlev, const int* its, double omega, const void* rms,
                         const Lay& rl, void* dst, const Lay& tl, const int* done, hipStream_t s,
                         void* sprev, void* scur, const Lay& sl) {
  using C = typename Tr<T>::C;
  TailPlan ti{};
  int off = 0;
  for (int k = 0; k < nlev; ++k) {
    const int nk = ((nms - 1) >> k) + 1;
    const double h = 1.0 / double(nk - 1);
    ti.lv[k] = TailLevel{its[k], off, 1.0f / float(nk - 2), 1.0f / float(2 * nk - 3), h * h};
    off += 3 * (d == 2 ? nk * nk : nk * nk * nk);
  }
  ti.inv_side = 1.0f / float(nms);
  const size_t lds = coarse_tail_lds(sizeof(T) == 8 ? PREC_F64 : PREC_F32, d, nms, nlev, TOP64);
  const T* r = static_cast<const T*>(rms) + rl.off;
  T* o = dst ? static_cast<T*>(dst) + tl.off : nullptr;
  T* sp = scur ? static_cast<T*>(sprev) + sl.off : nullptr;
  T* sc = scur ? static_cast<T*>(scur) + sl.off : nullptr;
  if (d == 2) {
    hipError_t a = allow_lds(k_coarse_tail<T, 2, TOP64>, lds);
    if (a != hipSuccess) return a;
    HOMG_LAUNCH_SMEM((k_coarse_tail<T, 2, TOP64>), dim3(1), dim3(SMALL_NT), lds, s, r, rl.pitch, rl.plane, o,
                     tl.pitch, tl.plane, nms, nlev, ti, C(omega / 4.0), omega / 4.0, done, sp, sc, sl.pitch,
                     sl.plane);
  }
  hipError_t a = allow_lds(k_coarse_tail<T, 3, TOP64>, lds);
  if (a != hipSuccess) return a;
  HOMG_LAUNCH_SMEM((k_coarse_tail<T, 3, TOP64>), dim3(1), dim3(SMALL_NT), lds, s, r, rl.pitch, rl.plane, o,
                   tl.pitch, tl.plane, nms, nlev, ti, C(omega / 6.0), omega / 6.0, done, sp, sc, sl.pitch,
                   sl.plane);
}

hipError_t launch_coarse_tail(int prec, int d, int nms, int nlev, const int* its, double omega,
                              const void* rms, const Lay& rl, void* dst, const Lay& tl,
                              const int* done, hipStream_t s, void* sprev, void* scur, const Lay& sl,
                              bool top64) {
  if (nms < 5 || nlev < 2 || nlev > BATCH_MAX_LEVELS || ((nms - 1) >> (nlev - 1)) + 1 < 3 ||
      (!scur && !dst) || (scur && (!sprev || sl.side != nms)))
    return hipErrorInvalidValue;
  switch (prec) {
    case PREC_F64: return tail_t<double, false>(d, nms, nlev, its, omega, rms, rl, dst, tl, done, s, sprev, scur, sl);
    case PREC_F32:
      return top64 ? tail_t<float, true>(d, nms, nlev, its, omega, rms, rl, dst, tl, done, s, sprev, scur, sl)
                   : tail_t<float, false>(d, nms, nlev, its, omega, rms, rl, dst, tl, done, s, sprev, scur, sl);
    default:
      return top64 ? tail_t<bf16, true>(d, nms, nlev, its, omega, rms, rl, dst, tl, done, s, sprev, scur, sl)
                   : tail_t<bf16, false>(d, nms, nlev, its, omega, rms, rl, dst, tl, done, s, sprev, scur, sl);
  }
}

hipError_t launch_lattice_small(int prec, int d, int nm, int l, int it, double omega, bool zero,
                                const void* e, const Lay& el, const void* rm, const Lay& rl,
                                const double* am, const Lay& al, void* xprev, void* xcur,
                                const Lay& cl, const int* done, hipStream_t s) {
#define SMALL_CASE(T)                                                                          \
  return zero ? small_tz<T, true>(d, nm, l, it, omega, e, el, rm, rl, am, al, xprev, xcur, cl, done, s) \
              : small_tz<T, false>(d, nm, l, it, omega, e, el, rm, rl, am, al, xprev, xcur, cl, done, s)
  switch (prec) {
    case PREC_F64: SMALL_CASE(double);
    case PREC_F32: SMALL_CASE(float);
    default: SMALL_CASE(bf16);
  }
#undef SMALL_CASE
}

template <typename T>
static hipError_t transfer_t(int d, int m, const void* xprev, const void* xcur, const Lay& cl, int mt,
                             void* dst, const Lay& tl, bool zero, const int* done, hipStream_t s) {
  const T* xp = static_cast<const T*>(xprev) + cl.off;
  const T* xc = static_cast<const T*>(xcur) + cl.off;
  T* o = static_cast<T*>(dst) + tl.off;
  const int nt = tl.side;
  if (d == 2) {
    const dim3 g((nt - 2 + 255) / 256, nt - 2, 1);
    if (zero) HOMG_LAUNCH((k_level_transfer_2d<T, true>), g, dim3(256), s, xp, xc, cl.pitch, m, o, tl.pitch, nt, mt, done);
    HOMG_LAUNCH((k_level_transfer_2d<T, false>), g, dim3(256), s, xp, xc, cl.pitch, m, o, tl.pitch, nt, mt, done);
  }
  const dim3 g((nt - 2 + BX3 - 1) / BX3, (nt - 2 + BY3 - 1) / BY3, nt - 2), blk(BX3, BY3);
  if (zero)
    HOMG_LAUNCH((k_level_transfer_3d<T, true>), g, blk, s, xp, xc, cl.pitch, cl.plane, m, o, tl.pitch,
                tl.plane, nt, mt, done);
  HOMG_LAUNCH((k_level_transfer_3d<T, false>), g, blk, s, xp, xc, cl.pitch, cl.plane, m, o, tl.pitch,
              tl.plane, nt, mt, done);
}

hipError_t launch_level_transfer(int prec, int d, int m, const void* xprev, const void* xcur,
                                 const Lay& cl, int mt, void* dst, const Lay& tl, bool zero_old,
                                 const int* done, hipStream_t s) {
  if (tl.side < 3) return hipSuccess;  // no interior node
  switch (prec) {
    case PREC_F64: return transfer_t<double>(d, m, xprev, xcur, cl, mt, dst, tl, zero_old, done, s);
    case PREC_F32: return transfer_t<float>(d, m, xprev, xcur, cl, mt, dst, tl, zero_old, done, s);
    default: return transfer_t<bf16>(d, m, xprev, xcur, cl, mt, dst, tl, zero_old, done, s);
  }
}

size_t level_write_lds(int prec, int d, int n, int m) {
  const size_t cs = prec == PREC_F64 ? 8 : 4;
  if (d == 2) {
    const size_t cw = size_t(TW2 >> m) + 3, ch = size_t(LW_ROWS2 >> m) + 3;
    return 2 * cw * ch * cs;
  }
  const size_t cw = size_t(BX3 >> m) + 3, ch = size_t(BY3 >> m) + 3, cd = size_t(LW_PLANES3 >> m) + 3;
  (void)n;
  return 2 * cw * ch * cd * cs;
}

template <typename T, int MODE>
static hipError_t level_write_tm(int d, int n, int m, const void* xprev, const void* xcur,
                                 const Lay& cl, void* en, const Lay& el, double* u, const Lay& ul,
                                 const int* done, hipStream_t s) {
  const size_t lds = level_write_lds(sizeof(T) == 8 ? PREC_F64 : PREC_F32, d, n, m);
  const T* xp = static_cast<const T*>(xprev) + cl.off;
  const T* xc = static_cast<const T*>(xcur) + cl.off;
  T* e = en ? static_cast<T*>(en) + el.off : nullptr;
  double* uu = u ? u + ul.off : nullptr;
  const int inner = n - 2;
  if (d == 2) {
    const dim3 g((inner + TW2 - 1) / TW2, (inner + LW_ROWS2 - 1) / LW_ROWS2);
    HOMG_LAUNCH_SMEM((k_level_write_2d<T, MODE>), g, dim3(BX2), lds, s, xp, xc, cl.pitch, e,
                     el.pitch, uu, ul.pitch, n, m, done);
  }
  const dim3 g((inner + BX3 - 1) / BX3, (inner + BY3 - 1) / BY3, (inner + LW_PLANES3 - 1) / LW_PLANES3);
  HOMG_LAUNCH_SMEM((k_level_write_3d<T, MODE>), g, dim3(BX3, BY3), lds, s, xp, xc, cl.pitch,
                   cl.plane, e, el.pitch, el.plane, uu, ul.pitch, ul.plane, n, m, done);
}

template <typename T>
static hipError_t level_write_t(int d, int n, int m, const void* xprev, const void* xcur,
                                const Lay& cl, void* en, const Lay& el, double* u, const Lay& ul,
                                int mode, const int* done, hipStream_t s) {
  switch (mode & 3) {
    case 0: return level_write_tm<T, 0>(d, n, m, xprev, xcur, cl, en, el, u, ul, done, s);
    case 1: return level_write_tm<T, 1>(d, n, m, xprev, xcur, cl, en, el, u, ul, done, s);
    case 2: return level_write_tm<T, 2>(d, n, m, xprev, xcur, cl, en, el, u, ul, done, s);
    default: return level_write_tm<T, 3>(d, n, m, xprev, xcur, cl, en, el, u, ul, done, s);
  }
}

hipError_t launch_level_write(int prec, int d, int n, int m, const void* xprev, const void* xcur,
                              const Lay& cl, void* en, const Lay& el, double* u, const Lay& ul,
                              int mode, const int* done, hipStream_t s) {
  switch (prec) {
    case PREC_F64: return level_write_t<double>(d, n, m, xprev, xcur, cl, en, el, u, ul, mode, done, s);
    case PREC_F32: return level_write_t<float>(d, n, m, xprev, xcur, cl, en, el, u, ul, mode, done, s);
    default: return level_write_t<bf16>(d, n, m, xprev, xcur, cl, en, el, u, ul, mode, done, s);
  }
}

// ------------------------------------------------------------ power-of-two grids
// Sec. 3: a 2D grid of N = 2^k nodes per side in four quadrants.  Level-m
// marks of quadrant (sx, sy) are the nodes whose coordinates, measured from
// the quadrant's external corner (index 0 on side 0, N-1 on side 1), are
// multiples of l = 2^m no larger than N/2 -- the last one just outside the
// quadrant.  Every interior mark relaxes (5-point stencil at distance l on
// the whole grid, a neighbour outside the grid reads 0) with its quadrant's
// restricted residual; every other interior node interpolates bilinearly
// from the marks of the quadrant that owns it (no cross-quadrant reads).
// The marks of side 0 are even and those of side 1 odd on every axis, so
// each node has at most one owner lattice.  Each quadrant's residuals form
// a nested sequence anchored at its corner ("family"): level j is the full
// weighting of level j-1 on compact arrays of side N >> j whose index 0 (the
// domain boundary) stays 0.

// Mark side (0 or 1) of coordinate x at stride l = 2^m, or -1.
__device__ __forceinline__ int p2_side(int x, int N, int m) {
  const int mask = (1 << m) - 1, half = N >> 1;
  if ((x & mask) == 0 && x <= half) return 0;
  const int a = N - 1 - x;
  if ((a & mask) == 0 && a <= half) return 1;
  return -1;
}

// One iteration at level m >= 1 over the whole grid.  fam[q] points at node
// (0, 0) of family q's level-m array (pitch fp).
template <int MODE>
__global__ __launch_bounds__(256) void k_p2_sweep(const double* __restrict__ eo, double* __restrict__ en,
                                                  int64_t ep, const double* __restrict__ f0,
                                                  const double* __restrict__ f1, const double* __restrict__ f2,
                                                  const double* __restrict__ f3, int64_t fp, int N, int m,
                                                  double w, double hl2, double* __restrict__ u, int64_t up,
                                                  const int* __restrict__ done) {
  if (*done) return;
  const int x = t2_x(blockIdx.x);
  if (x > N - 2) return;
  const int l = 1 << m, half = N >> 1;
  // 1 / l is exact (l a power of two), so the weights below equal the
  // quotients (ax - cx) / l bit for bit without a division per node
  const double inv_l = 1.0 / double(l);
  const int sx = p2_side(x, N, m);
  const int tx = x >= half ? 1 : 0;
  const int ax = tx ? N - 1 - x : x, cx = (ax >> m) << m;
  const int gx0 = tx ? N - 1 - cx : cx, gx1 = tx ? N - 1 - (cx + l) : cx + l;
  const double fx = double(ax - cx) * inv_l;
  const int y0 = t2_y0(blockIdx.y, P2_ROWS), y1 = min(N - 1, y0 + P2_ROWS);
  // the corners of the lattice cell last interpolated from (the walk
  // reloads them only when a row lies in another cell)
  int cell = -1;
  double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
  for (int y = y0; y < y1; ++y) {
    const int sy = p2_side(y, N, m);
    double v;
    if (sx >= 0 && sy >= 0) {
      const double* fam = sy ? (sx ? f3 : f2) : (sx ? f1 : f0);
      const int a = sx ? N - 1 - x : x, b = sy ? N - 1 - y : y;
      const double rv = fam[int64_t(b >> m) * fp + (a >> m)];
      double c = 0.0, q = 0.0;
      if (!(MODE & SW_ZERO_OLD)) {
        const double* row = eo + int64_t(y) * ep;
        c = row[x];
        const double xm = x - l >= 0 ? row[x - l] : 0.0;
        const double xp = x + l <= N - 1 ? row[x + l] : 0.0;
        const double ym = y - l >= 0 ? eo[int64_t(y - l) * ep + x] : 0.0;
        const double yp = y + l <= N - 1 ? eo[int64_t(y + l) * ep + x] : 0.0;
        q = (xm + xp) + (ym + yp);
      }
      v = relax_const<double>(c, q, rv, w, hl2, 4.0);
    } else if (MODE & SW_ZERO_OLD) {
      v = 0.0;
    } else {
      const int ty = y >= half ? 1 : 0;
      const int ay = ty ? N - 1 - y : y, cy = (ay >> m) << m;
      const int gy0 = ty ? N - 1 - cy : cy, gy1 = ty ? N - 1 - (cy + l) : cy + l;
      const double fy = double(ay - cy) * inv_l;
      const int key = gy0 * 2 + ty;
      if (key != cell) {
        const double* r0 = eo + int64_t(gy0) * ep;
        const double* r1 = eo + int64_t(gy1) * ep;
        c00 = r0[gx0];
        c01 = r0[gx1];
        c10 = r1[gx0];
        c11 = r1[gx1];
        cell = key;
      }
      v = lerp(lerp(c00, c01, fx), lerp(c10, c11, fx), fy);
    }
    if (MODE & SW_ACCUM)
      add_to(u + int64_t(y) * up + x, v);
    else
      st_w(en + int64_t(y) * ep + x, v);
  }
}

// Family level j from level j-1 (compact, pitch fp), or -- from_r0 -- level 1
// from the whole-grid r_0 (pitch fp) seen from the corner (sx, sy).
__global__ __launch_bounds__(256) void k_p2_restrict(const double* __restrict__ F, int64_t fp,
                                                     double* __restrict__ Cc, int64_t cp, int nc, int N,
                                                     int sx, int sy, int from_r0, const int* __restrict__ done) {
  if (*done) return;
  const int A = blockIdx.x * 256 + threadIdx.x, B = blockIdx.y;
  if (A >= nc) return;
  if (A == 0 || B == 0) {
    Cc[int64_t(B) * cp + A] = 0.0;
    return;
  }
  auto at = [&](int b, int a) {
    if (from_r0) {
      const int gx = sx ? N - 1 - a : a, gy = sy ? N - 1 - b : b;
      return F[int64_t(gy) * fp + gx];
    }
    return F[int64_t(b) * fp + a];
  };
  auto rs = [&](int b) { return fmac(2.0, at(b, 2 * A), at(b, 2 * A - 1) + at(b, 2 * A + 1)); };
  const double top = rs(2 * B - 1), mid = rs(2 * B), bot = rs(2 * B + 1);
  Cc[int64_t(B) * cp + A] = fmac(2.0, mid, top + bot) * 0.0625;
}

hipError_t launch_p2_restrict(const double* F, const Lay& fl, bool from_r0, int N, int sx, int sy, double* C,
                              const Lay& cl, const int* done, hipStream_t s) {
  const int nc = cl.side;
  HOMG_LAUNCH(k_p2_restrict, dim3((nc + 255) / 256, nc), dim3(256), s, F + fl.off, fl.pitch, C + cl.off,
              cl.pitch, nc, N, sx, sy, from_r0 ? 1 : 0, done);
}

hipError_t launch_p2_sweep(int N, int m, double omega, const double* eo, double* en, const Lay& el,
                           const double* const* fam, const Lay& fl, double* u, const Lay& ul, int mode,
                           const int* done, hipStream_t s) {
  if (m < 1 || N < 4 || (N & (N - 1)) || fl.side != (N >> m)) return hipErrorInvalidValue;
  const double hl = double(1 << m) / double(N - 1);
  const dim3 g(t2_gx(N), t2_gy(N, P2_ROWS));
  const double* e = eo + el.off;
  double* o = en + el.off;
  double* uu = u ? u + ul.off : nullptr;
  const double *f0 = fam[0] + fl.off, *f1 = fam[1] + fl.off, *f2 = fam[2] + fl.off, *f3 = fam[3] + fl.off;
#define P2_CASE(MODE)                                                                                       \
  HOMG_LAUNCH((k_p2_sweep<MODE>), g, dim3(256), s, e, o, el.pitch, f0, f1, f2, f3, fl.pitch, N, m, omega / 4.0, \
              hl * hl, uu, ul.pitch, done)
  switch (mode & (SW_ZERO_OLD | SW_ACCUM)) {
    case 0: P2_CASE(0);
    case SW_ZERO_OLD: P2_CASE(SW_ZERO_OLD);
    case SW_ACCUM: P2_CASE(SW_ACCUM);
    default: P2_CASE(SW_ZERO_OLD | SW_ACCUM);
  }
#undef P2_CASE
}

// ------------------------------------------------------------ batched solver
// Many independent 2D problems of uneven size advanced together.  All
// problems move in lockstep global steps; at step k every unfinished
// problem runs the next stage of its own sequence
//     norm(f), ||f||, residual, norm      (cycle 0)
//     restriction 0..M-1, per coarse level its iterations on the compact
//     lattice and the hand-over to the next finer level (to the whole grid
//     before level 0), level 0 in multi-iteration passes, residual, norm
//                                                     (cycles 1, 2, ...)
// One launch of k_batched_step runs one step for all problems: the step's
// tiles (the same tiles, and the same tile code, as the one-problem
// kernels) are spread round-robin over the launch's workgroups, and the
// launch boundary separates steps.  The launches are recorded once in a
// HIP graph (build_batch_graph) that the host replays.  The norm stage of
// a cycle retires its problem once the relative residual reaches the
// tolerance.

// Tiles (workgroups) of a 2D stage: TW2 columns by four bands of len rows.
__device__ __forceinline__ int tiles_of(int side, int len) { return t2_gx(side) * t2_gy(side, len); }

struct StageInfo {
  int kind;   // BK_* below
  int level;  // restriction: fine level; iteration stages: level
  int code;   // iteration stages: the stage's entry of the schedule table
  int cycle;
  int step;   // step of the sequence
};
enum { BK_NONE = 0, BK_NORM = 1, BK_FNORM = 2, BK_RES = 3, BK_FIN = 4, BK_RESTRICT = 5, BK_STAGE = 6 };

__device__ __forceinline__ StageInfo stage_of(const BatchProblem& p, const int* __restrict__ table, int k) {
  StageInfo si{BK_NONE, 0, 0, 0, 0};
  if (k == 0) { si.kind = BK_NORM; return si; }
  if (k == 1) { si.kind = BK_FNORM; return si; }
  if (k == 2) { si.kind = BK_RES; return si; }
  if (k == 3) { si.kind = BK_FIN; si.cycle = 0; return si; }
  const int L = p.top + p.sweeps + 2;
  const int j = (k - 4) % L;
  si.cycle = (k - 4) / L + 1;
  if (j < p.top) { si.kind = BK_RESTRICT; si.level = j; return si; }
  if (j < p.top + p.sweeps) {
    si.kind = BK_STAGE;
    si.code = table[p.sched_off + j - p.top];
    si.level = bst_level(si.code);
    return si;
  }
  si.kind = (j == p.top + p.sweeps) ? BK_RES : BK_FIN;
  return si;
}

// Band length of a problem's multi-iteration level-0 stage: its tuned walk
// length, at least 16 rows (shorter bands re-read too many halo rows).
__host__ __device__ __forceinline__ int batch_tb_len(const BatchProblem& p) { return p.len[0] < 16 ? 16 : p.len[0]; }
constexpr int BATCH_XF_ROWS = 8;  // rows of a hand-over tile

__device__ __forceinline__ int level_side(const BatchProblem& p, int m) { return (p.n - 1) / (1 << m) + 1; }

// Level m of a batched problem is its FP64 coarsest level: reduced-precision
// storage and m the top (>= 1) level.
template <typename T>
__device__ __forceinline__ bool batch_top64(const BatchProblem& p, int m) {
  return sizeof(T) != 8 && p.top >= 1 && m == p.top;
}

__device__ __forceinline__ int stage_tiles(const BatchProblem& p, const StageInfo& si) {
  switch (si.kind) {
    case BK_STAGE: {
      const int c = si.code;
      if (bst_kind(c) == BST_L0) return tb_blocks(p.n, bst_count(c), batch_tb_len(p));
      if (bst_kind(c) == BST_LTB) return tb_blocks(level_side(p, si.level), bst_count(c), BATCH_LTB_LEN);
      if (bst_kind(c) == BST_SWEEP) return tiles_of(level_side(p, si.level), p.len[si.level]);
      const int nt = level_side(p, si.level - 1);  // hand-over target
      return nt >= 3 ? ((nt - 2 + BX2 - 1) / BX2) * ((nt - 2 + BATCH_XF_ROWS - 1) / BATCH_XF_ROWS) : 0;
    }
    case BK_NORM:
    case BK_RES: return tiles_of(p.n, p.len[0]);
    case BK_RESTRICT: {
      const int nc = (p.n - 1) / (2 << si.level) + 1;
      return nc >= 3 ? tiles_of(nc, p.len[si.level + 1]) : 0;
    }
    case BK_FNORM:
    case BK_FIN: return 1;
    default: return 0;
  }
}

template <typename T>
__device__ __forceinline__ void batch_tile(const BatchProblem& p, BatchState* __restrict__ bs,
                                           int* __restrict__ done, const StageInfo& si, int t,
                                           const BatchRun& run) {
  using C = typename Tr<T>::C;
  const int n = p.n;
  const int gx = t2_gx(n);
  const int bx = t % gx, by = t / gx;
  T* e0 = static_cast<T*>(p.e[0]);
  T* e1 = static_cast<T*>(p.e[1]);
  switch (si.kind) {
    case BK_NORM:
      tile_norm2_2d(p.f, n, n, p.len[0], p.partials, bx, by, t);
      break;
    case BK_RES: {
      const double h = 1.0 / double(n - 1);
      tile_residual_2d<T, false>(p.u, n, p.f, n, nullptr, 0, static_cast<T*>(p.r[0]), p.rp[0], n,
                                 p.len[0], 1.0 / (h * h), p.partials, bx, by, t);
      break;
    }
    case BK_FNORM:
    case BK_FIN: {
      const int count = tiles_of(n, p.len[0]);
      double s = 0.0;
      for (int i = threadIdx.x; i < count; i += 256) s += p.partials[i];
      s = block_sum<256>(s);
      if (threadIdx.x == 0) {
        BatchState& b = bs[p.id];
        if (si.kind == BK_FNORM) {
          const double fn = sqrt(s);
          b.fnorm = fn > 0.0 ? fn : 1.0;
        } else {
          const double rel = sqrt(s) / b.fnorm;
          p.history[si.cycle] = rel;
          b.cycles = si.cycle;
          b.final_rel = rel;
          int dn = 0;
          if (!(rel <= 1.7976931348623157e308)) dn = 2;
          else if (rel <= run.tol) dn = 1;
          else if (si.cycle >= run.max_cycles) dn = 3;
          if (dn) {
            // other workgroups may still be mapping this step's tiles: the
            // problem stays in this step's map and leaves it from the next
            __hip_atomic_store(&b.retired, si.step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            done[p.id] = dn;
          }
        }
      }
      break;
    }
    case BK_RESTRICT: {
      const int nc = (n - 1) / (2 << si.level) + 1;
      const int gxc = t2_gx(nc);
      if (batch_top64<T>(p, si.level + 1))
        tile_restrict_2d<T, double>(static_cast<const T*>(p.r[si.level]), p.rp[si.level], p.r64, p.p64, nc,
                                    p.len[si.level + 1], t % gxc, t / gxc);
      else
        tile_restrict_2d<T>(static_cast<const T*>(p.r[si.level]), p.rp[si.level],
                            static_cast<T*>(p.r[si.level + 1]), p.rp[si.level + 1], nc,
                            p.len[si.level + 1], t % gxc, t / gxc);
      break;
    }
    case BK_STAGE: {
      const int c = si.code, m = si.level, kind = bst_kind(c);
      const bool zero = bst_zero(c);
      if (kind == BST_SWEEP && batch_top64<T>(p, m)) {
        // the coarsest level in FP64 (the formula of the small-lattice
        // kernel), each iterate also stored rounded for the hand-over
        const int nm = level_side(p, m), it = bst_index(c);
        const double* xo = p.x64[(it - 1) & 1];
        double* xn = p.x64[it & 1];
        T* xr = static_cast<T*>(p.x[m][it & 1]);
        const double hl = 1.0 / double(nm - 1), hl2 = hl * hl, w = run.omega / 4.0;
        const int gxm = t2_gx(nm);
        const int I = t2_x(t % gxm);
        const int J0 = t2_y0(t / gxm, p.len[m]), J1 = min(nm - 1, J0 + p.len[m]);
        if (I <= nm - 2)
          for (int J = J0; J < J1; ++J) {
            const int64_t o = int64_t(J) * p.p64 + I;
            double v;
            if (zero) {
              v = relax_const<double>(0.0, (0.0 + 0.0) + (0.0 + 0.0), p.r64[o], w, hl2, 4.0);
            } else {
              v = relax_const<double>(xo[o], (xo[o - 1] + xo[o + 1]) + (xo[o - p.p64] + xo[o + p.p64]), p.r64[o],
                                      w, hl2, 4.0);
            }
            xn[o] = v;
            st(xr + int64_t(J) * p.rp[m] + I, typename Tr<T>::C(v));
          }
      } else if (kind == BST_SWEEP) {  // iteration bst_index of level m >= 1 on its compact lattice
        const int nm = level_side(p, m), it = bst_index(c);
        const T* xo = static_cast<const T*>(p.x[m][(it - 1) & 1]);
        T* xn = static_cast<T*>(p.x[m][it & 1]);
        const double hl = 1.0 / double(nm - 1);
        const C hl2 = C(hl * hl), w = C(run.omega / 4.0);
        const int gxm = t2_gx(nm);
        const T* rm = static_cast<const T*>(p.r[m]);
        if (zero)
          tile_sweep_2d_l0<T, SW_ZERO_OLD, false>(xo, xn, p.rp[m], rm, p.rp[m], nullptr, 0, nullptr, 0, nm,
                                                  p.len[m], w, hl2, t % gxm, t / gxm);
        else
          tile_sweep_2d_l0<T, 0, false>(xo, xn, p.rp[m], rm, p.rp[m], nullptr, 0, nullptr, 0, nm, p.len[m],
                                        w, hl2, t % gxm, t / gxm);
      } else if (kind == BST_LTB) {  // all iterations of level m in one pass on its compact lattice
        const int nm = level_side(p, m), cnt = bst_count(c);
        const T* xo = static_cast<const T*>(p.x[m][0]);
        T* xn = static_cast<T*>(p.x[m][1]);
        T* xq = static_cast<T*>(p.x3[m]);
        const double hl = 1.0 / double(nm - 1);
        const C hl2 = C(hl * hl), w = C(run.omega / 4.0);
        const T* rm = static_cast<const T*>(p.r[m]);
        const int wv = t * 4 + int(threadIdx.x >> 6);
        switch (cnt) {
          case 1: tb_body<T, false, false, true, 1>(xo, xn, xq, p.rp[m], rm, p.rp[m], nullptr, 0, nm, BATCH_LTB_LEN, w, hl2, wv); break;
          case 2: tb_body<T, false, false, true, 2>(xo, xn, xq, p.rp[m], rm, p.rp[m], nullptr, 0, nm, BATCH_LTB_LEN, w, hl2, wv); break;
          case 3: tb_body<T, false, false, true, 3>(xo, xn, xq, p.rp[m], rm, p.rp[m], nullptr, 0, nm, BATCH_LTB_LEN, w, hl2, wv); break;
          default: tb_body<T, false, false, true, 4>(xo, xn, xq, p.rp[m], rm, p.rp[m], nullptr, 0, nm, BATCH_LTB_LEN, w, hl2, wv); break;
        }
      } else if (kind == BST_XFER) {  // level m's final state to the lattice of level m - 1
        const int it = bst_count(c), mt = m - 1, nt = level_side(p, mt);
        const bool ltb = bst_index(c) == 1;  // from one BST_LTB pass
        const T* xc = static_cast<const T*>(ltb ? p.x[m][1] : p.x[m][it & 1]);
        const T* xp = static_cast<const T*>(ltb ? p.x3[m] : p.x[m][(it - 1) & 1]);
        T* dst = mt > 0 ? static_cast<T*>(p.x[mt][0]) : e0;
        const int64_t dp = mt > 0 ? p.rp[mt] : p.ep;
        const int gxt = (nt - 2 + BX2 - 1) / BX2;
        const int I = 1 + (t % gxt) * BX2 + threadIdx.x;
        const int J0 = 1 + (t / gxt) * BATCH_XF_ROWS, J1 = min(nt - 1, J0 + BATCH_XF_ROWS);
        if (I <= nt - 2)
          for (int J = J0; J < J1; ++J) {
            if (zero)
              transfer_node_2d<T, true>(xp, xc, p.rp[m], m, dst, dp, mt, I, J);
            else
              transfer_node_2d<T, false>(xp, xc, p.rp[m], m, dst, dp, mt, I, J);
          }
      } else {  // level-0 pass bst_index of bst_count iterations
        const int q = bst_index(c), cnt = bst_count(c);
        const T* eo = (q & 1) ? e1 : e0;
        T* en = (q & 1) ? e0 : e1;
        const double h = 1.0 / double(n - 1);
        const C hl2 = C(h * h), w = C(run.omega / 4.0);
        const T* rm = static_cast<const T*>(p.r[0]);
        const int len = batch_tb_len(p), wv = t * 4 + int(threadIdx.x >> 6);
        const bool accum = bst_accum(c);
#define BATCH_TB(Z, A, IT) \
  tb_body<T, Z, A, false, IT>(eo, en, nullptr, p.ep, rm, p.rp[0], p.u, n, n, len, w, hl2, wv)
#define BATCH_TB_IT(Z, A)             \
  switch (cnt) {                      \
    case 1: BATCH_TB(Z, A, 1); break; \
    case 2: BATCH_TB(Z, A, 2); break; \
    case 3: BATCH_TB(Z, A, 3); break; \
    default: BATCH_TB(Z, A, 4); break; \
  }
        if (zero) {
          if (accum) { BATCH_TB_IT(true, true); } else { BATCH_TB_IT(true, false); }
        } else {
          if (accum) { BATCH_TB_IT(false, true); } else { BATCH_TB_IT(false, false); }
        }
#undef BATCH_TB_IT
#undef BATCH_TB
      }
      break;
    }
    default:
      break;
  }
}

// One step of every active problem's sequence: k = base + j.  Every
// workgroup builds the same tile map (prefix sums of the active problems'
// tile counts for their stage at step k, looked up in each problem's row
// of tiles per stage) and takes the tiles g = blockIdx.x,
// blockIdx.x + gridDim.x, ...  A problem is active in step k unless it
// retired in an earlier step; the step that retires it is written by its
// finalize tile while other workgroups may be building this step's map,
// and either value they read keeps it in this step, so all maps agree.
template <typename T>
__global__ __launch_bounds__(256) void k_batched_step(const BatchProblem* __restrict__ probs,
                                                      BatchState* __restrict__ bs,
                                                      int* __restrict__ done,
                                                      const int* __restrict__ levels_of_sweep,
                                                      const BatchRun* __restrict__ runp,
                                                      BatchSync* __restrict__ sync, int j) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (sync->idle) return;
  const BatchRun run = *runp;
  const int k = sync->base + j;
  if (k >= run.max_steps) return;
  const int P = run.count;
  int* pref = reinterpret_cast<int*>(smem);  // P + 1 prefix sums of tile counts
  for (int i = threadIdx.x; i < P; i += 256) {
    const BatchProblem& p = probs[i];
    const int ret = __hip_atomic_load(&bs[i].retired, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int tiles = 0;
    if (ret >= k)  // the row of tiles per stage of a cycle (k_batch_tile_table)
      tiles = k < 4 ? stage_tiles(p, stage_of(p, levels_of_sweep, k))
                    : levels_of_sweep[p.tile_off + (k - 4) % (p.top + p.sweeps + 2)];
    pref[i + 1] = tiles;
  }
  if (threadIdx.x == 0) pref[0] = 0;
  __syncthreads();
  // scan by chunks: each thread scans its own chunk, the chunk totals are
  // scanned across the workgroup (within each wave by shuffles, then the
  // four wave totals), and each thread adds its chunk's offset
  const int chunk = (P + 255) / 256;
  const int lo = threadIdx.x * chunk + 1, hi = min(P, lo + chunk - 1);
  int acc = 0;
  for (int i = lo; i <= hi; ++i) { acc += pref[i]; pref[i] = acc; }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = acc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  __shared__ int wave_total[4];
  if (lane == 63) wave_total[wave] = incl;
  __syncthreads();
  int off = incl - acc;
  for (int q = 0; q < wave; ++q) off += wave_total[q];
  for (int i = lo; i <= hi; ++i) pref[i] += off;
  __syncthreads();
  const int total = pref[P];
  if (total == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sync->idle = 1;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) sync->steps = k + 1;
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    // problem owning global tile g: last i with pref[i] <= g
    int a = 0, b = P;
    while (b - a > 1) {
      const int mid = (a + b) >> 1;
      if (pref[mid] <= g) a = mid; else b = mid;
    }
    const BatchProblem& p = probs[a];
    StageInfo si = stage_of(p, levels_of_sweep, k);
    si.step = k;
    batch_tile<T>(p, bs, done, si, g - pref[a], run);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_batch_tile_table(const BatchProblem* __restrict__ probs, int* table) {
  const BatchProblem& p = probs[blockIdx.x];
  const int L = p.top + p.sweeps + 2;
  for (int j = threadIdx.x; j < L; j += 256) table[p.tile_off + j] = stage_tiles(p, stage_of(p, table, 4 + j));
}

__global__ __launch_bounds__(64) void k_batch_advance(BatchSync* sync, int steps) {
  if (threadIdx.x == 0) sync->base += steps;
}

__global__ __launch_bounds__(256) void k_batch_init(BatchState* bs, int* done, int P, BatchSync* sync) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < P) {
    bs[i].cycles = -1;
    bs[i].retired = 0x7fffffff;
    bs[i].fnorm = 1.0;
    bs[i].final_rel = 0.0;
    done[i] = 0;
  }
  if (i == 0) {
    sync->base = 0;
    sync->steps = 0;
    sync->idle = 0;
  }
}

int default_walk_len(int d, int n) { return walk_len(d, n); }

int batch_tiles(int side, int len) { return t2_gx(side) * t2_gy(side, len); }

hipError_t batch_occupancy(int prec, int P, int* blocks_per_cu, size_t* lds) {
  *lds = size_t(P + 1) * sizeof(int);
  switch (prec) {
    case PREC_F64: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batched_step<double>, 256, *lds);
    case PREC_F32: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batched_step<float>, 256, *lds);
    default: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batched_step<bf16>, 256, *lds);
  }
}

hipError_t launch_batch_tile_table(int P, const BatchProblem* probs, int* table, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_tile_table, dim3(P), dim3(256), 0, s, probs, table);
  return hipGetLastError();
}

// Reset of a batched solve's per-problem state and step counter (an
// ordinary launch on the caller's stream before the first replay).
hipError_t launch_batch_init(int P, BatchState* bs, int* done, BatchSync* sync, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_init, dim3((P + 255) / 256), dim3(256), 0, s, bs, done, P, sync);
  return hipGetLastError();
}

// The graph one replay runs: BATCH_STEPS_PER_REPLAY step launches in a
// chain (each `grid` workgroups of 256 lanes; step j of the replay runs
// global step base + j), then the one-lane node that advances base.
hipError_t build_batch_graph(int prec, int P, int grid, const BatchProblem* probs, BatchState* bs,
                             int* done, const int* levels_of_sweep, const BatchRun* run,
                             BatchSync* sync, hipGraph_t* out) {
  *out = nullptr;
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  void* fn = nullptr;
  switch (prec) {
    case PREC_F64: fn = reinterpret_cast<void*>(k_batched_step<double>); break;
    case PREC_F32: fn = reinterpret_cast<void*>(k_batched_step<float>); break;
    default: fn = reinterpret_cast<void*>(k_batched_step<bf16>); break;
  }
  int js[BATCH_STEPS_PER_REPLAY];
  hipGraphNode_t prev = nullptr;
  for (int j = 0; j < BATCH_STEPS_PER_REPLAY && e == hipSuccess; ++j) {
    js[j] = j;
    void* args[] = {&probs, &bs, &done, &levels_of_sweep, &run, &sync, &js[j]};
    hipKernelNodeParams kp{};
    kp.func = fn;
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = unsigned(size_t(P + 1) * sizeof(int));
    kp.kernelParams = args;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    prev = node;
  }
  if (e == hipSuccess) {
    int steps = BATCH_STEPS_PER_REPLAY;
    void* args[] = {&sync, &steps};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(k_batch_advance);
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddKernelNode(&node, g, &prev, 1, &kp);
  }
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return e;
  }
  *out = g;
  return hipSuccess;
}

}  // namespace homg
