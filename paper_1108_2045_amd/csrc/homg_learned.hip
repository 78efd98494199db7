// homg_learned.hip -- gfx950 kernels of the learned lattice smoother.
//
// The relaxation of the HOMG fused task (Sec. 2 of arXiv:1108.2045: lattice
// nodes relax, every other node interpolates) is damped Jacobi in the paper.
// Here it can be replaced, on the 2D variable-coefficient diffusion
// problem, by a small bias-free network evaluated on the compact level-m
// lattice (spacing h_l = 2^m h, so on the whole grid its 3x3 taps are
// dilated by 2^m):
//   features at an interior lattice node p (0 on the boundary):
//     rho = (h_l^2 r_m(p) - sum_q a_pq (x_p - x_q)) / sum_q a_pq
//     X = (rho, rho (a_E - a_W)/(a_E + a_W), rho (a_N - a_S)/(a_N + a_S))
//     with a_pq the harmonic mean of the nodal coefficients (W, E, S, N);
//   P_c = sum_ci sum_k W1[c][ci][k] X_ci(p + o_k),  H_c = max(P_c, 0)
//   (16 channels, interior nodes; 0 on the boundary),
//   y = sum_c sum_k W2[c][k] H_c(p + o_k),  x' = x + y,
// o_k = (dy, dx) with k = 3 (dy + 1) + (dx + 1), read as a correlation.
// Weights are stored in BF16 and used as their exact FP32 values; all
// network arithmetic is FP32 (features in the cycle's precision, then
// FP32).  Damped Jacobi is the special case y = omega rho.
//
// The work is a dense 576-MAC contraction per node over LDS-resident tiles:
// a workgroup owns a 14 x 14 block of lattice nodes and stages x and a on
// its 20 x 20 halo region, the features on 18 x 18 and the hidden layer on
// 16 x 16; both channel contractions run on the matrix cores (see the
// inference section below).
//
// Training kernels (FP32, dense compact arrays): forward writes z = delta -
// y; backward recomputes the tile's features and hidden layer, forms
// g = dL/dy = -2 A_m z / E(delta) and accumulates the 576 weight gradients
// and the energy E(z) in registers over the tiles a workgroup visits, then
// writes one row of per-workgroup partial sums; a fixed-order reduction and
// an Adam step (FP32 master weights -> BF16) follow.  Every sum has a fixed
// order, so training is deterministic.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

#include "homg_internal.h"

namespace homg {

namespace {

struct bf16s {
  uint16_t bits;
};

__device__ __forceinline__ double ldv(const double* p) { return *p; }
__device__ __forceinline__ float ldv(const float* p) { return *p; }
__device__ __forceinline__ float ldv(const bf16s* p) { return __uint_as_float(uint32_t(p->bits) << 16); }
// FP32 -> BF16 bits, round to nearest even, NaN quieted (one
// v_cvt_pk_bf16_f32, which rounds exactly so on every FP32 bit pattern).
__device__ __forceinline__ uint16_t to_bf16_bits(float f) { return __builtin_bit_cast(uint16_t, __bf16(f)); }
__device__ __forceinline__ void stv(double* p, double v) { *p = v; }
__device__ __forceinline__ void stv(float* p, float v) { *p = v; }
__device__ __forceinline__ void stv(bf16s* p, float v) { p->bits = to_bf16_bits(v); }
// v as it reads back after a store to T.
template <typename T, typename C>
__device__ __forceinline__ C stored(C v) {
  if constexpr (std::is_same<T, bf16s>::value) return __uint_as_float(uint32_t(to_bf16_bits(v)) << 16);
  else return v;
}

template <typename T> struct Acc { using C = float; };
template <> struct Acc<double> { using C = double; };

constexpr int TO = 14;          // owned tile side
constexpr int R3 = TO + 6;      // x, a staged region (halo 3)
constexpr int R2 = TO + 4;      // features (halo 2)
constexpr int R1 = TO + 2;      // hidden layer (halo 1): 16 x 16 = one node per lane
constexpr int NT = R1 * R1;     // 256 lanes
constexpr int HP = HID + 4;     // padded hidden stride in floats (16-byte aligned)
constexpr int NOWN = TO * TO;   // 196
static_assert(LEARNED_SMALL_NM == TO + 2, "one tile covers the interior of the small lattices");

template <typename C>
__device__ __forceinline__ C hmean(C a, C b) { return C(2) * a * b / (a + b); }

// Shared memory of one tile of the training kernels: features as float4
// per node (channel 3 unused), hidden layer with padded rows.
constexpr int FPL = R2 * R2;     // one feature plane
template <typename C>
struct TileLds {
  C x[R3 * R3];
  C a[R3 * R3];
  float4 f[FPL];
  float h[NT * HP];
};

// Stage x and a on the halo-3 region of the tile whose owned block starts
// at (J0, I0), then the features on the halo-2 region.  Nodes outside the
// lattice read x = 0, a = 1; features are 0 off the interior.  XT/RT/AT:
// storage of x, r_m, a (AT = void: constant coefficient).
template <typename C, typename XT, typename RT, typename AT>
__device__ __forceinline__ void stage_features(TileLds<C>& L, const XT* __restrict__ x, int64_t xp,
                                               const RT* __restrict__ r, int64_t rp,
                                               const AT* __restrict__ a, int64_t ap, int nm,
                                               int J0, int I0, C hl2) {
  const int t = threadIdx.x;
  for (int q = t; q < R3 * R3; q += NT) {
    const int J = J0 - 3 + q / R3, I = I0 - 3 + q % R3;
    const bool in = J >= 0 && J < nm && I >= 0 && I < nm;
    L.x[q] = in ? C(ldv(x + int64_t(J) * xp + I)) : C(0);
    if constexpr (!std::is_void<AT>::value) L.a[q] = in ? C(ldv(a + int64_t(J) * ap + I)) : C(1);
  }
  __syncthreads();
  for (int q = t; q < R2 * R2; q += NT) {
    const int jj = q / R2, ii = q % R2;
    const int J = J0 - 2 + jj, I = I0 - 2 + ii;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (J >= 1 && J <= nm - 2 && I >= 1 && I <= nm - 2) {
      const int c3 = (jj + 1) * R3 + (ii + 1);
      const C xc = L.x[c3];
      const C xw = L.x[c3 - 1], xe = L.x[c3 + 1], xs = L.x[c3 - R3], xn = L.x[c3 + R3];
      const C rv = C(ldv(r + int64_t(J) * rp + I));
      if constexpr (std::is_void<AT>::value) {
        const C flux = (((xc - xw) + (xc - xe)) + (xc - xs)) + (xc - xn);
        v.x = float((hl2 * rv - flux) / C(4));
      } else {
        const C ac = L.a[c3];
        const C aw = hmean(ac, L.a[c3 - 1]), ae = hmean(ac, L.a[c3 + 1]);
        const C as = hmean(ac, L.a[c3 - R3]), an = hmean(ac, L.a[c3 + R3]);
        const C sa = ((aw + ae) + as) + an;
        const C flux = ((aw * (xc - xw) + ae * (xc - xe)) + as * (xc - xs)) + an * (xc - xn);
        const C rho = (hl2 * rv - flux) / sa;
        v.x = float(rho);
        v.y = float(rho * (ae - aw) / (ae + aw));
        v.z = float(rho * (an - as) / (an + as));
      }
    }
    L.f[q] = v;
  }
  __syncthreads();
}

// Hidden layer at the lane's node of the halo-1 region (one node per lane):
// pre-activations P[16] in registers, H = max(P, 0) stored in LDS (0 off the
// interior).  Returns whether the node is interior.
template <typename C>
__device__ __forceinline__ bool stage_hidden(TileLds<C>& L, const float* __restrict__ w, int nm,
                                             int J0, int I0, float P[HID]) {
  const int t = threadIdx.x;
  const int jj = t / R1, ii = t % R1;
  const int J = J0 - 1 + jj, I = I0 - 1 + ii;
  const bool in = J >= 1 && J <= nm - 2 && I >= 1 && I <= nm - 2;
#pragma unroll
  for (int c = 0; c < HID; ++c) P[c] = 0.f;
  if (in) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int dy = k / 3 - 1, dx = k % 3 - 1;
      const float4 fv = L.f[(jj + 1 + dy) * R2 + (ii + 1 + dx)];
#pragma unroll
      for (int c = 0; c < HID; ++c) {
        float p = P[c];
        p = __builtin_fmaf(w[c * 27 + 0 * 9 + k], fv.x, p);
        p = __builtin_fmaf(w[c * 27 + 1 * 9 + k], fv.y, p);
        p = __builtin_fmaf(w[c * 27 + 2 * 9 + k], fv.z, p);
        P[c] = p;
      }
    }
  }
  float* hrow = L.h + t * HP;
#pragma unroll
  for (int c = 0; c < HID; c += 4)
    *reinterpret_cast<float4*>(hrow + c) =
        make_float4(fmaxf(P[c], 0.f), fmaxf(P[c + 1], 0.f), fmaxf(P[c + 2], 0.f), fmaxf(P[c + 3], 0.f));
  __syncthreads();
  return in;
}

// Output at owned node o (0 <= o < 196): y = sum_c sum_k W2[c][k] H_c(p + o_k).
template <typename C>
__device__ __forceinline__ float tile_output(const TileLds<C>& L, const float* __restrict__ w, int o) {
  const int oj = o / TO, oi = o % TO;
  float y = 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int dy = k / 3 - 1, dx = k % 3 - 1;
    const float* hv = L.h + ((oj + 1 + dy) * R1 + (oi + 1 + dx)) * HP;
#pragma unroll
    for (int c = 0; c < HID; c += 4) {
      const float4 h4 = *reinterpret_cast<const float4*>(hv + c);
      y = __builtin_fmaf(w[NW1 + (c + 0) * 9 + k], h4.x, y);
      y = __builtin_fmaf(w[NW1 + (c + 1) * 9 + k], h4.y, y);
      y = __builtin_fmaf(w[NW1 + (c + 2) * 9 + k], h4.z, y);
      y = __builtin_fmaf(w[NW1 + (c + 3) * 9 + k], h4.w, y);
    }
  }
  return y;
}

// ---------------------------------------------------------------- inference
// One learned relaxation of every interior node of a compact level lattice:
// xo = xi + y (or u += xi + y with ACCUM, the last iteration of a cycle).
// ZERO: xi = 0 (the first iteration of a cycle; nothing is read from xi).
//
// The two channel contractions run on the matrix cores
// (v_mfma_f32_16x16x32_bf16: D = A B + D with A 16 x 32, B 32 x 16, BF16
// operands, FP32 accumulation).  Operand layout (one wave, lane l,
// g = l / 16): A[i][k] with i = l % 16, k = 8 g + e; B[k][j] with
// j = l % 16, same k; D[i][j] with j = l % 16, i = 4 g + r.  The weights
// are BF16 values already; each FP32 activation is split exactly into three
// BF16 parts (hi = its top 8 significant bits, mid = the next 8 of the
// remainder, lo = the rest, which fits BF16 exactly since 24 = 3 x 8), so
// every product is exact and only the FP32 accumulation rounds: FP32
// arithmetic on the matrix cores.
//
// Per 16-node row of the tile's halo-1 region (four rows per wave):
//   first layer  D1[c][node] = sum_s W1[c][s] F[s][node] over K slots
//     s = 12 dy + 4 dx + ci of the 3 x 3 window (27 of 64 slots carry
//     weights), with the features F read from LDS already split, four BF16
//     per node (two MFMAs per part, six in all);
//   H = max(D1, 0) on interior nodes, 0 elsewhere -- the lane holds
//     channels 4g .. 4g+3 of its node, which is exactly the B operand the
//     second layer needs, so H never leaves registers;
//   second layer Z[tap][node] = sum_c W2[c][tap] H[c][node] (K slots
//     8 g + e: hi / mid of channel 4 g + e % 4, then lo of channel 4 g + e
//     and zeros: two MFMAs), written to LDS;
// and after a barrier the output at a node is y = sum_k Z[k][node + o_k].
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct Parts {  // an FP32 value as three BF16 parts, in the upper halves of FP32 words
  uint32_t hi, mid, lo;
};

__device__ __forceinline__ Parts split3(float v) {
  Parts p;
  p.hi = __float_as_uint(v) & 0xffff0000u;
  const float r1 = v - __uint_as_float(p.hi);
  p.mid = __float_as_uint(r1) & 0xffff0000u;
  p.lo = __float_as_uint(r1 - __uint_as_float(p.mid));
  return p;
}

// Eight BF16-valued FP32 numbers as a BF16 vector (exact).
__device__ __forceinline__ bf16x8 pack8(const float (&v)[8]) {
  uint32_t p[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    p[k] = (__float_as_uint(v[2 * k]) >> 16) | (__float_as_uint(v[2 * k + 1]) & 0xffff0000u);
  return __builtin_bit_cast(bf16x8, p);
}

__device__ __forceinline__ uint32_t pair16(uint32_t lo_word, uint32_t hi_word) {
  return (lo_word >> 16) | (hi_word & 0xffff0000u);
}

constexpr int ZS = 12;            // Z row stride in floats (taps 0..8, 16-byte rows)

template <typename C>
struct InferLds {
  float z[NT * ZS];               // Z[node][tap] on the halo-1 region
  C x[2][R3 * R3];                // x on the halo-3 region, two tiles in flight
  float a[R3 * R3];               // coefficient on the halo-3 region
  uint64_t fb[3 * FPL];           // features: part, node; four BF16 each (channels 0-2, then 0)
};

// The lane's operands that do not change from tile to tile.  First-layer K
// slot s (two MFMAs, s in [0, 64)) holds channel s % 4 of feature node
// (dy, dx) = (s / 12, (s % 12) / 4) of the 3 x 3 window (channel 3 and
// s >= 36 are zero weights): with the features stored as four BF16 per
// node, a lane's eight slots of the first MFMA are two whole nodes and
// those of the second one node (lanes 0-15) or nothing.
struct LaneConst {
  bf16x8 w1a, w1b, w2a, w2b;  // A operands: first layer (two MFMAs); second layer (two)
};

__device__ __forceinline__ LaneConst lane_const(const float* __restrict__ w) {
  const int lane = threadIdx.x & 63;
  const int ii = lane & 15, g = lane >> 4;
  float va1[8], vb1[8], va[8], vb[8];
  LaneConst k;
  auto w1 = [&](int s) {  // W1[c = ii][ci][tap] at K slot s
    const int dy = s / 12, dx = (s % 12) / 4, ci = s % 4;
    return s < 36 && ci < 3 ? w[ii * 27 + ci * 9 + 3 * dy + dx] : 0.f;
  };
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    va1[e] = w1(8 * g + e);
    vb1[e] = w1(32 + 8 * g + e);
    const float w2 = ii < 9 ? w[NW1 + (4 * g + (e & 3)) * 9 + ii] : 0.f;  // W2[c][tap = ii]
    va[e] = w2;
    vb[e] = e < 4 ? w2 : 0.f;
  }
  k.w1a = pack8(va1);
  k.w1b = pack8(vb1);
  k.w2a = pack8(va);
  k.w2b = pack8(vb);
  return k;
}

// Global inputs of one tile held in registers: x and a on the halo-3
// region, r on the halo-2 region, at most two values each per lane.  They
// are loaded while the previous tile runs its contractions.
template <typename T, bool ZERO, bool VAR>
struct TileInputs {
  using C = typename Acc<T>::C;
  C x[2], r[2];
  double a[2];  // converted when staged, so the load is not waited for here

  // Offsets are 32-bit: the launcher checks that every array of the call
  // holds fewer than 2^31 elements.
  __device__ __forceinline__ void load(const T* __restrict__ xi, int xp, const T* __restrict__ rr, int rp,
                                       const double* __restrict__ aa, int ap, int nm, int J0, int I0) {
    // Every lane loads from a clamped (in-bounds) position and then keeps or
    // drops the value, so the loads carry no branches.
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int q = threadIdx.x + k * NT;
      {
        const int J = J0 - 3 + q / R3, I = I0 - 3 + q % R3;
        const bool in = (k == 0 || q < R3 * R3) && unsigned(J) < unsigned(nm) && unsigned(I) < unsigned(nm);
        const int o = min(max(J, 0), nm - 1) * xp + min(max(I, 0), nm - 1);
        if constexpr (!ZERO) {
          const C v = C(ldv(xi + o));
          x[k] = in ? v : C(0);
        } else {
          x[k] = C(0);
        }
        if constexpr (VAR) {
          const double v = aa[min(max(J, 0), nm - 1) * ap + min(max(I, 0), nm - 1)];
          a[k] = in ? v : 1.0;
        } else {
          a[k] = 1.0;
        }
      }
      {
        const int J = J0 - 2 + q / R2, I = I0 - 2 + q % R2;
        const bool in = (k == 0 || q < R2 * R2) && unsigned(J - 1) < unsigned(nm - 2) &&
                        unsigned(I - 1) < unsigned(nm - 2);
        const C v = C(ldv(rr + (min(max(J, 1), nm - 2) * rp + min(max(I, 1), nm - 2))));
        r[k] = in ? v : C(0);
      }
    }
  }
};

__device__ __forceinline__ float frcp(float v) { return __builtin_amdgcn_rcpf(v); }

// Features at feature node q of the tile (halo-2 region), split and stored.
// The residual part is formed in the cycle precision C; the coefficient
// factors (face harmonic means, their sum and the two ratios) in FP32 with
// the hardware reciprocal -- all of it is rounded to FP32 for the network.
template <typename C, bool VAR>
__device__ __forceinline__ void put_features(InferLds<C>& L, const C* X, int q, bool interior, C rv,
                                             C hl2) {
  float f0 = 0.f, f1 = 0.f, f2 = 0.f;
  if (interior) {
    const int jj = q / R2, ii = q % R2;
    const int c3 = (jj + 1) * R3 + (ii + 1);
    const C xc = X[c3];
    const C dw = xc - X[c3 - 1], de = xc - X[c3 + 1], ds = xc - X[c3 - R3], dn = xc - X[c3 + R3];
    if constexpr (!VAR) {
      f0 = float((hl2 * rv - (((dw + de) + ds) + dn)) * C(0.25));
    } else {
      const float ac = L.a[c3];
      const float aw0 = L.a[c3 - 1], ae0 = L.a[c3 + 1], as0 = L.a[c3 - R3], an0 = L.a[c3 + R3];
      const float aw = 2.f * ac * aw0 * frcp(ac + aw0), ae = 2.f * ac * ae0 * frcp(ac + ae0);
      const float as = 2.f * ac * as0 * frcp(ac + as0), an = 2.f * ac * an0 * frcp(ac + an0);
      const float sa = ((aw + ae) + as) + an;
      const C flux = ((C(aw) * dw + C(ae) * de) + C(as) * ds) + C(an) * dn;
      f0 = float((hl2 * rv - flux) * C(frcp(sa)));
      f1 = f0 * ((ae - aw) * frcp(ae + aw));
      f2 = f0 * ((an - as) * frcp(an + as));
    }
  }
  const Parts p0 = split3(f0), p1 = split3(f1), p2 = split3(f2);
  // one 8-byte store per part: channels 0, 1, 2 and a zero
  auto node = [](uint32_t c0, uint32_t c1, uint32_t c2) {
    return uint64_t(pair16(c0, c1)) | (uint64_t(c2 >> 16) << 32);
  };
  L.fb[q] = node(p0.hi, p1.hi, p2.hi);
  L.fb[FPL + q] = node(p0.mid, p1.mid, p2.mid);
  L.fb[2 * FPL + q] = node(p0.lo, p1.lo, p2.lo);
}

// Both layers for row jj of the halo-1 region (row J of the lattice); Z to LDS.
template <typename C>
__device__ __forceinline__ void row_contract(InferLds<C>& L, const LaneConst& k, int jj, bool row_in,
                                             bool col_in) {
  const int lane = threadIdx.x & 63;
  const int ii = lane & 15, g = lane >> 4;
  // the lane's window nodes (see lane_const): first MFMA two nodes, second
  // MFMA node (2, 2) for lanes 0-15 (read by all lanes, kept by those)
  const int na = g == 0 ? 0 : g == 1 ? 2 : g == 2 ? R2 + 1 : 2 * R2;
  const int nb = g == 0 ? 1 : g == 1 ? R2 : g == 2 ? R2 + 2 : 2 * R2 + 1;
  const uint64_t* fb = L.fb + jj * R2 + ii;
  f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int part = 0; part < 3; ++part) {
    const uint64_t* fp = fb + part * FPL;
    const uint64_t b1[2] = {fp[na], fp[nb]};
    const uint64_t c = fp[2 * R2 + 2];
    const uint64_t b2[2] = {g == 0 ? c : uint64_t(0), uint64_t(0)};
    d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(k.w1a, __builtin_bit_cast(bf16x8, b1), d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(k.w1b, __builtin_bit_cast(bf16x8, b2), d, 0, 0, 0);
  }
  const bool in = row_in && col_in;
  Parts h[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) h[r] = split3((in & (d[r] > 0.f)) ? d[r] : 0.f);  // no short circuit: a select
  const uint32_t ba[4] = {pair16(h[0].hi, h[1].hi), pair16(h[2].hi, h[3].hi), pair16(h[0].mid, h[1].mid),
                          pair16(h[2].mid, h[3].mid)};
  const uint32_t bb[4] = {pair16(h[0].lo, h[1].lo), pair16(h[2].lo, h[3].lo), 0u, 0u};
  f32x4 z = {0.f, 0.f, 0.f, 0.f};
  z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(k.w2a, __builtin_bit_cast(bf16x8, ba), z, 0, 0, 0);
  z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(k.w2b, __builtin_bit_cast(bf16x8, bb), z, 0, 0, 0);
  if (g < 3) *reinterpret_cast<f32x4*>(L.z + (jj * R1 + ii) * ZS + 4 * g) = z;  // taps 4g .. 4g+3
}

// The three stages of one tile (owned block at (J0, I0)): features from
// x and a in LDS (r of the lane's two halo-2 slots in registers), both
// contractions into Z, and the output sum at owned node (oj, oi).
template <typename C, bool VAR>
__device__ __forceinline__ void tile_features(InferLds<C>& L, const C* X, int nm, int J0, int I0,
                                              const C (&rv)[2], C hl2) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int q = threadIdx.x + k * NT;
    if (q < R2 * R2) {
      const int J = J0 - 2 + q / R2, I = I0 - 2 + q % R2;
      put_features<C, VAR>(L, X, q, J >= 1 && J <= nm - 2 && I >= 1 && I <= nm - 2, rv[k], hl2);
    }
  }
}

template <typename C>
__device__ __forceinline__ void tile_contract(InferLds<C>& L, const LaneConst& kc, int nm, int J0, int I0) {
  const int wave = threadIdx.x >> 6, I = I0 - 1 + (threadIdx.x & 15);
  const bool col_in = I >= 1 && I <= nm - 2;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int jj = wave * 4 + rr, J = J0 - 1 + jj;
    row_contract<C>(L, kc, jj, J >= 1 && J <= nm - 2, col_in);
  }
}

template <typename C>
__device__ __forceinline__ float tile_y(const InferLds<C>& L, int oj, int oi) {
  float y = 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k) y += L.z[((oj + k / 3) * R1 + (oi + k % 3)) * ZS + k];
  return y;
}

template <typename T, bool ZERO, bool ACCUM, bool VAR>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_learned_iter(
    const T* __restrict__ xi, int64_t xp, T* __restrict__ xo, const T* __restrict__ r, int64_t rp,
    const double* __restrict__ a, int64_t ap, double* __restrict__ u, int64_t up, int nm,
    typename Acc<T>::C hl2, const float* __restrict__ w, const int* __restrict__ done) {
  using C = typename Acc<T>::C;
  if (*done) return;
  __shared__ InferLds<C> L;
  const int tiles_x = (nm - 2 + TO - 1) / TO, tiles = tiles_x * tiles_x;
  const int t = threadIdx.x;
  const LaneConst kc = lane_const(w);
  const int xp32 = int(xp), rp32 = int(rp), ap32 = int(ap);
  TileInputs<T, ZERO, VAR> in;
  int tile = blockIdx.x, buf = 0;
  if (tile < tiles)
    in.load(xi, xp32, r, rp32, a, ap32, nm, 1 + (tile / tiles_x) * TO, 1 + (tile % tiles_x) * TO);
  // Barriers per tile: after staging x and a, after the features, after Z.
  // x is double-buffered, so the next tile may be staged while this one's
  // outputs still read x; a, the features and Z are rewritten only after a
  // barrier that follows their last reads.
  for (; tile < tiles; tile += gridDim.x, buf ^= 1) {
    const int J0 = 1 + (tile / tiles_x) * TO, I0 = 1 + (tile % tiles_x) * TO;
    C* X = L.x[buf];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int q = t + k * NT;
      if (q < R3 * R3) {
        X[q] = in.x[k];
        if constexpr (VAR) L.a[q] = float(in.a[k]);
      }
    }
    __syncthreads();
    tile_features<C, VAR>(L, X, nm, J0, I0, in.r, hl2);
    __syncthreads();
    const int next = tile + gridDim.x;
    if (next < tiles)
      in.load(xi, xp32, r, rp32, a, ap32, nm, 1 + (next / tiles_x) * TO, 1 + (next % tiles_x) * TO);
    tile_contract<C>(L, kc, nm, J0, I0);
    __syncthreads();
    if (t < NOWN) {
      const int oj = t / TO, oi = t % TO;
      const int J = J0 + oj, I = I0 + oi;
      if (J <= nm - 2 && I <= nm - 2) {
        const C v = X[(oj + 3) * R3 + (oi + 3)] + C(tile_y(L, oj, oi));
        if constexpr (ACCUM) {
          u[J * int(up) + I] += double(v);
        } else {
          stv(xo + (J * xp32 + I), v);
        }
      }
    }
  }
}

// All `it` learned relaxations of a lattice with at most TO interior nodes
// per side (one tile) in one workgroup, the iterates ping-ponging in LDS.
// x_0 is read from e with stride l (the whole grid) or from the compact
// array (l = 1, chained hand-over; e may then alias xprev), or is 0 (ZERO).
// Writes x_{it-1} to xprev and x_it to xcur on the whole lattice.
template <typename T, bool ZERO, bool VAR>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_learned_small(
    const T* e, int64_t ep, int l, const T* __restrict__ r, int64_t rp,
    const double* __restrict__ a, int64_t ap, T* xprev, T* xcur, int64_t cp, int nm, int it,
    typename Acc<T>::C hl2, const float* __restrict__ w, const int* __restrict__ done) {
  using C = typename Acc<T>::C;
  if (*done) return;
  __shared__ InferLds<C> L;
  const int t = threadIdx.x;
  const LaneConst kc = lane_const(w);
  // the tile's halo-3 region starts at lattice (-2, -2)
  C rv[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int q = t + k * NT;
    if (q < R3 * R3) {
      const int J = q / R3 - 2, I = q % R3 - 2;
      const bool in = J >= 0 && J < nm && I >= 0 && I < nm;
      C xv = C(0);
      if (!ZERO && in) xv = C(ldv(e + int64_t(J) * l * ep + int64_t(I) * l));
      L.x[0][q] = xv;
      L.x[1][q] = xv;
      if constexpr (VAR) L.a[q] = in ? float(a[int64_t(J) * ap + I]) : 1.f;
    }
    rv[k] = C(0);
    if (q < R2 * R2) {
      const int J = q / R2 - 1, I = q % R2 - 1;
      if (J >= 1 && J <= nm - 2 && I >= 1 && I <= nm - 2) rv[k] = C(ldv(r + int64_t(J) * rp + I));
    }
  }
  __syncthreads();
  for (int s = 1; s <= it; ++s) {
    const C* src = L.x[(s - 1) & 1];
    C* dst = L.x[s & 1];
    tile_features<C, VAR>(L, src, nm, 1, 1, rv, hl2);
    __syncthreads();
    tile_contract<C>(L, kc, nm, 1, 1);
    __syncthreads();
    if (t < NOWN) {
      const int oj = t / TO, oi = t % TO;
      if (oj + 1 <= nm - 2 && oi + 1 <= nm - 2) {
        const int q = (oj + 3) * R3 + (oi + 3);
        const C v = src[q] + C(tile_y(L, oj, oi));
        dst[q] = stored<T>(v);  // each iterate rounded to the storage type, as stored by the multi-launch path
      }
    }
    __syncthreads();
  }
  const C* xp_ = L.x[(it - 1) & 1];
  const C* xc_ = L.x[it & 1];
  for (int i = t; i < nm * nm; i += NT) {
    const int J = i / nm, I = i - J * nm;
    const int q = (J + 2) * R3 + (I + 2);
    stv(xprev + int64_t(J) * cp + I, xp_[q]);
    stv(xcur + int64_t(J) * cp + I, xc_[q]);
  }
}

// ---------------------------------------------------------------- training
// Dense FP32 compact arrays of side nm (node (J, I) at J nm + I).

// z = delta - y at interior nodes (y alone when delta is null).
template <bool VAR>
__global__ __launch_bounds__(NT) void k_train_fwd(const float* __restrict__ x,
                                                  const float* __restrict__ r,
                                                  const float* __restrict__ a,
                                                  const float* __restrict__ delta,
                                                  float* __restrict__ z, int nm, float hl2,
                                                  const float* __restrict__ w) {
  __shared__ TileLds<float> L;
  const int J0 = 1 + blockIdx.y * TO, I0 = 1 + blockIdx.x * TO;
  if constexpr (VAR)
    stage_features<float, float, float, float>(L, x, nm, r, nm, a, nm, nm, J0, I0, hl2);
  else
    stage_features<float, float, float, void>(L, x, nm, r, nm, nullptr, 0, nm, J0, I0, hl2);
  float P[HID];
  (void)stage_hidden<float>(L, w, nm, J0, I0, P);
  const int o = threadIdx.x;
  if (o < NOWN) {
    const int J = J0 + o / TO, I = I0 + o % TO;
    if (J <= nm - 2 && I <= nm - 2) {
      const float y = tile_output<float>(L, w, o);
      const int64_t p = int64_t(J) * nm + I;
      z[p] = delta ? delta[p] - y : y;
    }
  }
}

// Gradient partial sums of one sample.  Workgroup b visits tiles b, b + G,
// ...; lane t accumulates elements t, t + 256, t + 512 of the 577-vector
// (576 weight gradients of L = E(z)/E(delta), then E(z)); the row of
// workgroup b goes to part[j * pstride + b].
template <bool VAR>
__global__ __launch_bounds__(NT) void k_train_bwd(const float* __restrict__ x,
                                                  const float* __restrict__ r,
                                                  const float* __restrict__ a,
                                                  const float* __restrict__ z, int nm, float hl2,
                                                  const double* __restrict__ e0,
                                                  const float* __restrict__ w,
                                                  float* __restrict__ part, int64_t pstride) {
  __shared__ TileLds<float> L;
  __shared__ float gs[NT];              // g on the halo-1 region
  __shared__ float zs[R2 * R2];         // z on the halo-2 region
  __shared__ float dp[NOWN * HP];       // dP on owned nodes
  __shared__ float ez[NOWN];            // z (A z) on owned nodes
  const int t = threadIdx.x;
  const int tiles_x = (nm - 2 + TO - 1) / TO;
  const int tiles = tiles_x * tiles_x;
  const float gscale = float(-2.0 / *e0);
  float acc[3] = {0.f, 0.f, 0.f};
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int J0 = 1 + (tile / tiles_x) * TO, I0 = 1 + (tile % tiles_x) * TO;
    if constexpr (VAR)
      stage_features<float, float, float, float>(L, x, nm, r, nm, a, nm, nm, J0, I0, hl2);
    else
      stage_features<float, float, float, void>(L, x, nm, r, nm, nullptr, 0, nm, J0, I0, hl2);
    float P[HID];
    (void)stage_hidden<float>(L, w, nm, J0, I0, P);
    for (int q = t; q < R2 * R2; q += NT) {
      const int J = J0 - 2 + q / R2, I = I0 - 2 + q % R2;
      zs[q] = (J >= 1 && J <= nm - 2 && I >= 1 && I <= nm - 2) ? z[int64_t(J) * nm + I] : 0.f;
    }
    __syncthreads();
    {  // g = -2 (A z) / E(delta) on the halo-1 region, z (A z) on owned nodes
      const int jj = t / R1, ii = t % R1;
      const int J = J0 - 1 + jj, I = I0 - 1 + ii;
      float g = 0.f;
      if (J >= 1 && J <= nm - 2 && I >= 1 && I <= nm - 2) {
        const int c2 = (jj + 1) * R2 + (ii + 1);
        const float zc = zs[c2];
        float az;
        if constexpr (VAR) {
          const int c3 = (jj + 2) * R3 + (ii + 2);
          const float ac = L.a[c3];
          const float aw = hmean(ac, L.a[c3 - 1]), ae = hmean(ac, L.a[c3 + 1]);
          const float as = hmean(ac, L.a[c3 - R3]), an = hmean(ac, L.a[c3 + R3]);
          az = ((aw * (zc - zs[c2 - 1]) + ae * (zc - zs[c2 + 1])) + as * (zc - zs[c2 - R2])) +
               an * (zc - zs[c2 + R2]);
        } else {
          az = (((zc - zs[c2 - 1]) + (zc - zs[c2 + 1])) + (zc - zs[c2 - R2])) + (zc - zs[c2 + R2]);
        }
        g = gscale * az;
        if (jj >= 1 && jj <= TO && ii >= 1 && ii <= TO) ez[(jj - 1) * TO + (ii - 1)] = zc * az;
      } else if (jj >= 1 && jj <= TO && ii >= 1 && ii <= TO) {
        ez[(jj - 1) * TO + (ii - 1)] = 0.f;
      }
      gs[t] = g;
    }
    __syncthreads();
    if (t < NOWN) {  // dP_c(q) = [P_c(q) > 0] sum_k W2[c][k] g(q - o_k) at owned q
      const int oj = t / TO, oi = t % TO;
      const int J = J0 + oj, I = I0 + oi;
      const bool in = J <= nm - 2 && I <= nm - 2;
      float gk[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int dy = k / 3 - 1, dx = k % 3 - 1;
        gk[k] = in ? gs[(oj + 1 - dy) * R1 + (oi + 1 - dx)] : 0.f;
      }
      const float* hq = L.h + ((oj + 1) * R1 + (oi + 1)) * HP;
#pragma unroll
      for (int c = 0; c < HID; ++c) {
        float dh = 0.f;
#pragma unroll
        for (int k = 0; k < 9; ++k) dh = __builtin_fmaf(w[NW1 + c * 9 + k], gk[k], dh);
        dp[t * HP + c] = hq[c] > 0.f ? dh : 0.f;
      }
    }
    __syncthreads();
    // weight gradients over the owned nodes (outside ones carry dP = g = 0)
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int j = t + s * NT;
      if (j < NW1) {
        const int c = j / 27, ci = (j % 27) / 9, k = j % 9;
        const int dy = k / 3 - 1, dx = k % 3 - 1;
        float sum = 0.f;
        for (int o = 0; o < NOWN; ++o) {
          const int oj = o / TO, oi = o % TO;
          const float4 fv = L.f[(oj + 2 + dy) * R2 + (oi + 2 + dx)];
          const float xv = ci == 0 ? fv.x : (ci == 1 ? fv.y : fv.z);
          sum = __builtin_fmaf(dp[o * HP + c], xv, sum);
        }
        acc[s] += sum;
      } else if (j < NW) {
        const int c = (j - NW1) / 9, k = (j - NW1) % 9;
        const int dy = k / 3 - 1, dx = k % 3 - 1;
        float sum = 0.f;
        for (int o = 0; o < NOWN; ++o) {
          const int oj = o / TO, oi = o % TO;
          const float gv = gs[(oj + 1) * R1 + (oi + 1)];
          sum = __builtin_fmaf(gv, L.h[((oj + 1 + dy) * R1 + (oi + 1 + dx)) * HP + c], sum);
        }
        acc[s] += sum;
      } else if (j == NW) {
        float sum = 0.f;
        for (int o = 0; o < NOWN; ++o) sum += ez[o];
        acc[s] += sum;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int j = t + s * NT;
    if (j <= NW) part[int64_t(j) * pstride + blockIdx.x] = acc[s];
  }
}

// Sum of each partial row in a fixed order: out[j] = sum_b part[j][b],
// FP64 accumulation (one workgroup per element j).
__global__ __launch_bounds__(256) void k_train_reduce(const float* __restrict__ part,
                                                      int64_t pstride, int rows,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < rows; b += 256) s += double(part[int64_t(j) * pstride + b]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

// Mean gradient over the batch (the `batch` rows of sums, stride NW + 1,
// added in order), Adam on the FP32 masters (FP32 moments; bias corrections
// and the update in FP64, since 1 - beta^t loses digits in FP32), the BF16
// copy (wbf, nullable)
// and its FP32 expansion w32 for the kernels.  With loss != null,
// loss[step - 1] = mean over the batch of E(z) / E(delta), E(delta) of row b
// at e0s[idx[b]].
__global__ __launch_bounds__(640) void k_train_adam(const double* __restrict__ sums, int batch,
                                                    const double* __restrict__ e0s,
                                                    const int* __restrict__ idx,
                                                    float* __restrict__ theta,
                                                    float* __restrict__ m1, float* __restrict__ m2,
                                                    uint16_t* __restrict__ wbf,
                                                    float* __restrict__ w32, int step, double lr,
                                                    double beta1, double beta2, double eps,
                                                    double* __restrict__ loss) {
  const int j = threadIdx.x;
  if (j < NW) {
    double g = 0.0;
    for (int b = 0; b < batch; ++b) g += sums[b * (NW + 1) + j];
    const float gf = float(g / batch);
    const float mm = float(beta1) * m1[j] + float(1.0 - beta1) * gf;
    const float vv = float(beta2) * m2[j] + float(1.0 - beta2) * (gf * gf);
    m1[j] = mm;
    m2[j] = vv;
    const double mhat = double(mm) / (1.0 - pow(beta1, double(step)));
    const double vhat = double(vv) / (1.0 - pow(beta2, double(step)));
    const float th = float(double(theta[j]) - lr * mhat / (sqrt(vhat) + eps));
    theta[j] = th;
    const uint16_t b16 = to_bf16_bits(th);
    if (wbf) wbf[j] = b16;
    w32[j] = __uint_as_float(uint32_t(b16) << 16);
  } else if (j == NW && loss) {
    double l = 0.0;
    for (int b = 0; b < batch; ++b) l += sums[b * (NW + 1) + NW] / e0s[idx[b]];
    loss[step - 1] = l / batch;
  }
}

// E(v) = sum_p v_p (A v)_p over interior nodes: per-workgroup partials.
template <bool VAR>
__global__ __launch_bounds__(256) void k_energy_part(const float* __restrict__ v,
                                                     const float* __restrict__ a, int nm,
                                                     double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  const int64_t inner = int64_t(nm - 2) * (nm - 2);
  for (int64_t q = blockIdx.x * 256 + threadIdx.x; q < inner; q += int64_t(gridDim.x) * 256) {
    const int J = 1 + int(q / (nm - 2)), I = 1 + int(q % (nm - 2));
    const int64_t p = int64_t(J) * nm + I;
    auto val = [&](int JJ, int II) {
      return (JJ >= 1 && JJ <= nm - 2 && II >= 1 && II <= nm - 2) ? double(v[int64_t(JJ) * nm + II]) : 0.0;
    };
    const double c = v[p];
    double av;
    if constexpr (VAR) {
      const double ac = a[p];
      av = hmean(ac, double(a[p - 1])) * (c - val(J, I - 1)) + hmean(ac, double(a[p + 1])) * (c - val(J, I + 1)) +
           hmean(ac, double(a[p - nm])) * (c - val(J - 1, I)) + hmean(ac, double(a[p + nm])) * (c - val(J + 1, I));
    } else {
      av = (c - val(J, I - 1)) + (c - val(J, I + 1)) + (c - val(J - 1, I)) + (c - val(J + 1, I));
    }
    s += c * av;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_small(const double* __restrict__ part, int count, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < count; ++i) s += part[i];
    *out = s;
  }
}

// FP32 values -> BF16 (RNE) and their FP32 expansion.
__global__ void k_round_weights(const float* __restrict__ src, uint16_t* __restrict__ wbf,
                                float* __restrict__ w32, int count) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) {
    const uint16_t b = to_bf16_bits(src[j]);
    wbf[j] = b;
    w32[j] = __uint_as_float(uint32_t(b) << 16);
  }
}

// Training-sample extraction from a dense FP64 whole grid: the level-l
// lattice, rounded to FP32 (dst side nm, dense).  With sub != null,
// dst = sub[l-lattice] - src[l-lattice] (the error of an iterate).
__global__ void k_lattice_f32(const double* __restrict__ src, int64_t sp, int l,
                              const double* __restrict__ sub, int64_t bp, int nm,
                              float* __restrict__ dst) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x, J = blockIdx.y;
  if (I >= nm) return;
  const double v = src[int64_t(J) * l * sp + int64_t(I) * l];
  dst[int64_t(J) * nm + I] = sub ? float(sub[int64_t(J) * bp + I] - v) : float(v);
}

// v += e over `count` contiguous FP64 values.
__global__ void k_add_dense(double* __restrict__ v, const double* __restrict__ e, int64_t count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) v[i] += e[i];
}

}  // namespace

// ---------------------------------------------------------------- launchers

#define LL_LAUNCH(kernel, grid, block, stream, ...)                                          \
  do {                                                                                      \
    hipEvent_t ev0_, ev1_;                                                                  \
    current_launch_events(&ev0_, &ev1_);                                                    \
    hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, ev0_, ev1_, 0, __VA_ARGS__);     \
    return hipGetLastError();                                                               \
  } while (0)

static dim3 tile_grid(int nm) {
  const int t = (nm - 2 + TO - 1) / TO;
  return dim3(t, t);
}

// Workgroups of NT lanes the device holds at once for kernel k (asked once).
static int resident_blocks(const void* k) {
  static std::mutex mu;
  static std::map<const void*, int> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(k);
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, NT, 0) != hipSuccess || per < 1 || cus < 1) {
    (void)hipGetLastError();
    return 1024;
  }
  return cache[k] = per * cus;
}

template <typename T, bool ZERO, bool ACCUM>
static hipError_t learned_t(int nm, double hl, const void* xi, const Lay& xl, void* xo,
                            const void* r, const Lay& rl, const double* a, const Lay& al,
                            double* u, const Lay& ul, const float* w, const int* done,
                            hipStream_t s) {
  using C = typename Acc<T>::C;
  using S = T;
  const S* x = xi ? static_cast<const S*>(xi) + xl.off : nullptr;
  S* y = xo ? static_cast<S*>(xo) + xl.off : nullptr;
  const S* rr = static_cast<const S*>(r) + rl.off;
  const double* aa = a ? a + al.off : nullptr;
  double* uu = u ? u + ul.off : nullptr;
  const C hl2 = C(hl * hl);
  // 32-bit element offsets inside the kernel
  const int64_t lim = int64_t(1) << 31;
  if ((x && xl.pitch * nm >= lim) || rl.pitch * nm >= lim || (aa && al.pitch * nm >= lim) ||
      (uu && ul.pitch * nm >= lim))
    return hipErrorInvalidValue;
  // one workgroup per tile up to the resident count, then they walk
  const int tx = (nm - 2 + TO - 1) / TO, tiles = tx * tx;
  if (a) {
    auto k = k_learned_iter<S, ZERO, ACCUM, true>;
    const int b = std::min(tiles, resident_blocks(reinterpret_cast<const void*>(k)));
    LL_LAUNCH(k, dim3(b), dim3(NT), s, x, xl.pitch, y, rr, rl.pitch, aa, al.pitch, uu, ul.pitch, nm,
              hl2, w, done);
  }
  auto k = k_learned_iter<S, ZERO, ACCUM, false>;
  const int b = std::min(tiles, resident_blocks(reinterpret_cast<const void*>(k)));
  LL_LAUNCH(k, dim3(b), dim3(NT), s, x, xl.pitch, y, rr, rl.pitch, aa, al.pitch, uu, ul.pitch, nm,
            hl2, w, done);
}

template <typename T>
static hipError_t learned_tm(int nm, double hl, const void* xi, const Lay& xl, void* xo,
                             const void* r, const Lay& rl, const double* a, const Lay& al,
                             double* u, const Lay& ul, const float* w, int mode,
                             const int* done, hipStream_t s) {
  switch (mode & 3) {
    case 0: return learned_t<T, false, false>(nm, hl, xi, xl, xo, r, rl, a, al, u, ul, w, done, s);
    case 1: return learned_t<T, true, false>(nm, hl, xi, xl, xo, r, rl, a, al, u, ul, w, done, s);
    case 2: return learned_t<T, false, true>(nm, hl, xi, xl, xo, r, rl, a, al, u, ul, w, done, s);
    default: return learned_t<T, true, true>(nm, hl, xi, xl, xo, r, rl, a, al, u, ul, w, done, s);
  }
}

hipError_t launch_learned_iter(int prec, int nm, double hl, const void* xi, const Lay& xl,
                               void* xo, const void* r, const Lay& rl, const double* a,
                               const Lay& al, double* u, const Lay& ul, const float* w, int mode,
                               const int* done, hipStream_t s) {
  if (nm < 3) return hipErrorInvalidValue;
  switch (prec) {
    case PREC_F64: return learned_tm<double>(nm, hl, xi, xl, xo, r, rl, a, al, u, ul, w, mode, done, s);
    case PREC_F32: return learned_tm<float>(nm, hl, xi, xl, xo, r, rl, a, al, u, ul, w, mode, done, s);
    default: return learned_tm<bf16s>(nm, hl, xi, xl, xo, r, rl, a, al, u, ul, w, mode, done, s);
  }
}

template <typename T, bool ZERO>
static hipError_t learned_small_t(int nm, int l, int it, double hl, const void* e, const Lay& el,
                                  const void* r, const Lay& rl, const double* a, const Lay& al,
                                  void* xprev, void* xcur, const Lay& cl, const float* w,
                                  const int* done, hipStream_t s) {
  using C = typename Acc<T>::C;
  const T* ee = static_cast<const T*>(e) + el.off;
  const T* rr = static_cast<const T*>(r) + rl.off;
  T* xp = static_cast<T*>(xprev) + cl.off;
  T* xc = static_cast<T*>(xcur) + cl.off;
  const C hl2 = C(hl * hl);
  if (a)
    LL_LAUNCH((k_learned_small<T, ZERO, true>), dim3(1), dim3(NT), s, ee, el.pitch, l, rr, rl.pitch,
              a + al.off, al.pitch, xp, xc, cl.pitch, nm, it, hl2, w, done);
  LL_LAUNCH((k_learned_small<T, ZERO, false>), dim3(1), dim3(NT), s, ee, el.pitch, l, rr, rl.pitch,
            (const double*)nullptr, int64_t(0), xp, xc, cl.pitch, nm, it, hl2, w, done);
}

hipError_t launch_learned_small(int prec, int nm, int l, int it, double hl, bool zero, const void* e,
                                const Lay& el, const void* r, const Lay& rl, const double* a,
                                const Lay& al, void* xprev, void* xcur, const Lay& cl,
                                const float* w, const int* done, hipStream_t s) {
  if (nm < 3 || nm > LEARNED_SMALL_NM || it < 1) return hipErrorInvalidValue;
#define LS_CASE(T)                                                                                 \
  return zero ? learned_small_t<T, true>(nm, l, it, hl, e, el, r, rl, a, al, xprev, xcur, cl, w, done, s) \
              : learned_small_t<T, false>(nm, l, it, hl, e, el, r, rl, a, al, xprev, xcur, cl, w, done, s)
  switch (prec) {
    case PREC_F64: LS_CASE(double);
    case PREC_F32: LS_CASE(float);
    default: LS_CASE(bf16s);
  }
#undef LS_CASE
}

hipError_t launch_train_fwd(int nm, float hl2, const float* x, const float* r, const float* a,
                            const float* delta, float* z, const float* w, hipStream_t s) {
  if (nm < 3) return hipErrorInvalidValue;
  if (a) LL_LAUNCH(k_train_fwd<true>, tile_grid(nm), dim3(NT), s, x, r, a, delta, z, nm, hl2, w);
  LL_LAUNCH(k_train_fwd<false>, tile_grid(nm), dim3(NT), s, x, r, a, delta, z, nm, hl2, w);
}

int train_bwd_rows(int nm) {
  const int t = (nm - 2 + TO - 1) / TO;
  const int tiles = t * t;
  return tiles < TRAIN_MAX_ROWS ? tiles : TRAIN_MAX_ROWS;
}

hipError_t launch_train_bwd(int nm, float hl2, const float* x, const float* r, const float* a,
                            const float* z, const double* e0, const float* w, float* part,
                            int64_t pstride, hipStream_t s) {
  if (nm < 3) return hipErrorInvalidValue;
  const dim3 g(train_bwd_rows(nm));
  if (a) LL_LAUNCH(k_train_bwd<true>, g, dim3(NT), s, x, r, a, z, nm, hl2, e0, w, part, pstride);
  LL_LAUNCH(k_train_bwd<false>, g, dim3(NT), s, x, r, a, z, nm, hl2, e0, w, part, pstride);
}

hipError_t launch_train_reduce(const float* part, int64_t pstride, int rows, double* out,
                               hipStream_t s) {
  LL_LAUNCH(k_train_reduce, dim3(NW + 1), dim3(256), s, part, pstride, rows, out);
}

hipError_t launch_train_adam(const double* sums, int batch, const double* e0s, const int* idx,
                             float* theta, float* m1, float* m2, uint16_t* wbf, float* w32,
                             int step, double lr, double beta1, double beta2, double eps,
                             double* loss, hipStream_t s) {
  LL_LAUNCH(k_train_adam, dim3(1), dim3(640), s, sums, batch, e0s, idx, theta, m1, m2, wbf, w32,
            step, lr, beta1, beta2, eps, loss);
}

hipError_t launch_energy(const float* v, const float* a, int nm, double* part, double* out,
                         hipStream_t s) {
  if (nm < 3) return hipErrorInvalidValue;
  const int64_t inner = int64_t(nm - 2) * (nm - 2);
  int blocks = int((inner + 255) / 256);
  if (blocks > ENERGY_MAX_PARTS) blocks = ENERGY_MAX_PARTS;
  hipError_t e;
  {
    hipEvent_t ev0, ev1;
    current_launch_events(&ev0, &ev1);
    if (a)
      hipExtLaunchKernelGGL(k_energy_part<true>, dim3(blocks), dim3(256), 0, s, ev0, ev1, 0, v, a, nm, part);
    else
      hipExtLaunchKernelGGL(k_energy_part<false>, dim3(blocks), dim3(256), 0, s, ev0, ev1, 0, v, a, nm, part);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sum_small, dim3(1), dim3(64), 0, s, part, blocks, out);
  return hipGetLastError();
}

hipError_t launch_round_weights(const float* src, uint16_t* wbf, float* w32, hipStream_t s) {
  hipLaunchKernelGGL(k_round_weights, dim3((NW + 255) / 256), dim3(256), 0, s, src, wbf, w32, NW);
  return hipGetLastError();
}

hipError_t launch_lattice_f32(const double* src, int64_t sp, int l, const double* sub, int64_t bp,
                              int nm, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_lattice_f32, dim3((nm + 255) / 256, nm), dim3(256), 0, s, src, sp, l, sub,
                     bp, nm, dst);
  return hipGetLastError();
}

hipError_t launch_add_dense(double* v, const double* e, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_add_dense, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, v, e, count);
  return hipGetLastError();
}

}  // namespace homg
