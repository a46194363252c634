// lbm_device.h -- compile-time velocity sets and per-node arithmetic of the
// free-energy LBM step (Simonis et al., arXiv 2212.01617, Sec. 2.2 and
// Algorithm 1), FP32, for the HIP kernels of this library.
//
// Populations of f are kept shifted by their lattice weights, df_i = f_i - w_i,
// so that FP32 (and FP16) storage carries only the deviation from rest.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace frelbm {

// ---------------------------------------------------------------------------
// Velocity sets: rest direction first, then opposite pairs side by side
// (opposite of i is i+1 for odd i, i-1 for even i > 0); cs^2 = 1/3.
// ---------------------------------------------------------------------------
template <int Q> struct VSet;

template <> struct VSet<9> {
  static constexpr int D = 2;
  __host__ __device__ static constexpr int cx(int i) {
    return (i == 1 || i == 5 || i == 7) ? 1 : (i == 2 || i == 6 || i == 8) ? -1 : 0;
  }
  __host__ __device__ static constexpr int cy(int i) {
    return (i == 3 || i == 5 || i == 8) ? 1 : (i == 4 || i == 6 || i == 7) ? -1 : 0;
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr float w(int i) {
    return i == 0 ? 4.0f / 9.0f : (i < 5 ? 1.0f / 9.0f : 1.0f / 36.0f);
  }
  // a_i ~ 3 w_i = w_i / cs^2 for the terms linear in c_i (see exact_lin)
  __host__ __device__ static constexpr float a(int i) {
    return i == 0 ? 0.0f : (i < 5 ? 0x1.555556p-2f : 0x1.555554p-4f);
  }
};

template <> struct VSet<19> {
  static constexpr int D = 3;
  // directions 1..6 are the axes, 7..10 the xy diagonals, 11..14 the xz
  // diagonals, 15..18 the yz diagonals
  __host__ __device__ static constexpr int cx(int i) {
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13)    ? 1
           : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1
                                                                 : 0;
  }
  __host__ __device__ static constexpr int cy(int i) {
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17)   ? 1
           : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18)  ? -1
                                                                 : 0;
  }
  __host__ __device__ static constexpr int cz(int i) {
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18)  ? 1
           : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1
                                                                  : 0;
  }
  __host__ __device__ static constexpr float w(int i) {
    return i == 0 ? 1.0f / 3.0f : (i < 7 ? 1.0f / 18.0f : 1.0f / 36.0f);
  }
  __host__ __device__ static constexpr float a(int i) {
    return i == 0 ? 0.0f : (i < 7 ? 0x1.555554p-3f : 0x1.555556p-4f);
  }
};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Exact first moments in FP32.  The momentum of the equilibria (eqs. feq,
// geq) and of the forcing term (eq. Fi) comes from their parts linear in c_i,
// with coefficients 3 w_i = w_i / cs^2.  Rounded to FP32, the weights give
// sum_i 3 w_i c_ia c_ib = (1 + 7.5e-9) delta_ab (D2Q9; 1.5e-8 for D3Q19), and
// a collision then adds that fraction of the momentum to every cell, in the
// same direction, at every step; over tens of thousands of steps this drift,
// not the random rounding, dominates the difference from exact arithmetic.
// The coefficients a_i are FP32 values chosen so that the identity holds
// exactly for the stored values: for the axis and diagonal directions,
// 2 a_axis + 4 a_diag = 1 (D2Q9) and 2 a_axis + 8 a_diag = 1 (D3Q19), with one
// of them the rounded 3 w_i and the other solved for (both exact in FP32).
// (The check sums in double, which holds these sums of FP32 values exactly.)
template <class V> constexpr bool exact_lin() {
  double s[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int i = 0; i < (V::D == 3 ? 19 : 9); ++i) {
    const int c[3] = {V::cx(i), V::cy(i), V::cz(i)};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) s[a][b] += (double)V::a(i) * (double)(c[a] * c[b]);
  }
  for (int a = 0; a < V::D; ++a)
    for (int b = 0; b < V::D; ++b)
      if (s[a][b] != (a == b ? 1.0 : 0.0)) return false;
  return true;
}
static_assert(exact_lin<VSet<9>>() && exact_lin<VSet<19>>(), "linear coefficients must give exact second moments");

// ---------------------------------------------------------------------------
// Geometry of one lattice in device memory.  The storage grid is the fluid
// domain plus one ghost layer at both ends of every wall axis.  Rows are
// padded to a pitch px (a multiple of 64) so that every 64-cell block of the
// population layout is one aligned row segment: cell index c = x + px*(y +
// ey*z); cells with x >= ex are padding and never touched by the method.
// ---------------------------------------------------------------------------
enum : uint8_t { CELL_FLUID = 0, CELL_SOLID = 1, CELL_ROLLER0 = 2, CELL_GHOST = 8, CELL_PAD = 9 };

// Bit 31 of a cell's neighbour word: the cell itself is not fluid.  Bit i
// (1 <= i < q) of a fluid cell's word: the neighbour along c_i is not fluid
// (bounce-back link); of a solid cell's word: the neighbour along c_i is
// fluid (a source of the cell's stencil fill).
constexpr uint32_t NB_SELF_SOLID = 0x80000000u;

struct Geom {
  int ex, ey, ez;   // storage grid
  int px;           // row pitch (multiple of 64)
  int per[3];       // 1 if the axis is periodic
  int off[3];       // ghost offset (1 on wall axes)
  long long ncell;  // px*ey*ez
};

struct Phys {
  float k1, k2;       // kappa1, kappa2
  float a2q;          // alpha^2 / 4
  float om_f, om_g;   // 1/tau_f, 1/tau_g
  float guo;          // 1 - 1/(2 tau_f)
  float gam3;         // Gamma / cs^2 = 3 Gamma
  float wall_u[3][2][3];
  int n_rollers;
  float rc[4][3];
  float rom[4];
  int rax[4];
  // ternary lattices: kappa3, 1/tau_h, Gamma_psi / cs^2
  float k3, om_h, gam3h;
};

// The three potentials of the ternary free energy (the Remark after the
// mobility relation in Sec. 2.2 adds a coupled Cahn-Hilliard equation per
// further component; the free energy is that of the cited ternary model):
// concentrations C1 = (rho + phi - psi)/2, C2 = (rho - phi - psi)/2, C3 = psi,
// mu_m = kappa_m C_m (1 - C_m)(1 - 2 C_m) - alpha^2 kappa_m lap C_m, and
// mu_rho = (mu_1 + mu_2)/2, mu_phi = (mu_1 - mu_2)/2, mu_psi = mu_3 - mu_rho.
__device__ __forceinline__ void chem_pot3(const Phys &P, float drho, float phi, float psi, float lr, float lp,
                                          float lq, float &mu_rho, float &mu_phi, float &mu_psi) {
  const float a2 = 4.0f * P.a2q;  // alpha^2
  const float c1 = 0.5f * (1.0f + drho + phi - psi), c2 = 0.5f * (1.0f + drho - phi - psi), c3 = psi;
  const float l1 = 0.5f * (lr + lp - lq), l2 = 0.5f * (lr - lp - lq), l3 = lq;
  const float m1 = P.k1 * (c1 * (1.0f - c1) * (1.0f - 2.0f * c1) - a2 * l1);
  const float m2 = P.k2 * (c2 * (1.0f - c2) * (1.0f - 2.0f * c2) - a2 * l2);
  const float m3 = P.k3 * (c3 * (1.0f - c3) * (1.0f - 2.0f * c3) - a2 * l3);
  mu_rho = 0.5f * (m1 + m2);
  mu_phi = 0.5f * (m1 - m2);
  mu_psi = m3 - mu_rho;
}

// Bulk free-energy density of the ternary functional.
__device__ __forceinline__ float psi_bulk3(const Phys &P, float rho, float phi, float psi) {
  const float c1 = 0.5f * (rho + phi - psi), c2 = 0.5f * (rho - phi - psi), c3 = psi;
  return 0.5f * (P.k1 * c1 * c1 * (1.0f - c1) * (1.0f - c1) + P.k2 * c2 * c2 * (1.0f - c2) * (1.0f - c2) +
                 P.k3 * c3 * c3 * (1.0f - c3) * (1.0f - c3));
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Neighbour of a fluid cell: every wall axis has a ghost layer, so only the
// periodic wrap is needed.
template <class V>
__device__ __forceinline__ int nb_fluid(const Geom &G, int x, int y, int z, int i) {
  int xn = wrap(x + V::cx(i), G.ex);
  int yn = wrap(y + V::cy(i), G.ey);
  int zn = V::D == 3 ? wrap(z + V::cz(i), G.ez) : z;
  return xn + G.px * (yn + G.ey * zn);
}

// ---------------------------------------------------------------------------
// Population storage: blocks of 64 consecutive cells, each block holding all
// directions of one population contiguously ([block][direction][64]), so a
// wavefront streams one contiguous 256-byte (FP32) segment per direction.
// S = 0: FP32 for f and g.  S = 1: f and g_1.. as half (round to nearest
// even), g_0 as float in a plane of its own; the half g array keeps the same
// q-direction block shape as f (its plane 0 unused) so both share offsets.
// ---------------------------------------------------------------------------
// Byte offset of population i of cell c in an array of `planes` directions
// of elements of ES bytes.  Offsets are 32-bit (every population array is
// kept under 4 GiB), so the compiler can address with a scalar base plus a
// 32-bit vector offset.
template <int ES>
__device__ __forceinline__ uint32_t blk_offset(int planes, int i, long long c) {
  const uint32_t cc = (uint32_t)c;
  return (((cc >> 6) * (uint32_t)planes + (uint32_t)i) * 64u + (cc & 63u)) * (uint32_t)ES;
}
// Population loads of the moments passes are non-temporal: they read every
// population once and should not displace the coupling fields, which the
// potential re-reads next, from the caches (measured: ordinary loads there
// cost 10% of the FP16 step).  The FP32 collide uses ordinary loads (the
// ldfc/ldgc accessors): a tile's x-shifted reads at odd parity share cache
// lines with the neighbouring tile, which then still finds them cached
// (measured: 2% less FP32 step time).  For the FP16 collide, and for the
// f-only collide of the consistent initialisation, ordinary loads measured
// 2% and 5% slower, so those stay non-temporal.
template <class T, bool NT = true>
__device__ __forceinline__ T ld_at(const T *base, uint32_t off) {
  if constexpr (sizeof(T) == 2) {
    const unsigned short *p = (const unsigned short *)((const char *)base + off);
    const unsigned short u = NT ? __builtin_nontemporal_load(p) : *p;
    return __builtin_bit_cast(T, u);
  } else {
    const T *p = (const T *)((const char *)base + off);
    return NT ? __builtin_nontemporal_load(p) : *p;
  }
}
template <class T>
__device__ __forceinline__ void st_at(T *base, uint32_t off, T v) {
  *(T *)((char *)base + off) = v;
}

// Stochastic rounding to half (FP16 storage with fp16_rounding = 1).  Each
// cell draws a seed per step, a hash of the cell index and the step counter
// (a 32-bit integer finalizer: two multiply-xorshift rounds), and every value
// it stores takes the next number of a xorshift32 stream (Marsaglia, 2003)
// from that seed.  The rounding of one value is unbiased for any stream whose
// numbers are uniform; the hash keeps cells and steps apart.
__device__ __forceinline__ uint32_t sr_seed(long long c, uint32_t step) {
  uint32_t h = (uint32_t)c * 0x9E3779B1u ^ step * 0x85EBCA77u;
  h ^= h >> 16;
  h *= 0x7FEB352Du;
  h ^= h >> 15;
  h *= 0x846CA68Bu;
  h ^= h >> 16;
  return h | 1u;  // xorshift32 needs a nonzero state
}

__device__ __forceinline__ uint32_t sr_next(uint32_t x) {
  x ^= x << 13;
  x ^= x >> 17;
  x ^= x << 5;
  return x;
}

// v rounded to one of the two halves next to it, the one farther from zero
// with probability equal to v's distance from the nearer-to-zero one over
// their spacing, for r uniform in [0, 2^32): unbiased, so a rounding error
// that round-to-nearest would repeat in every cell and at every step (a
// nearly uniform flow) averages out instead.  Where halves are normal
// (|v| >= 2^-14) their grid keeps the top 10 of FP32's 23 mantissa bits:
// adding r's low 13 bits under them and clearing those bits rounds the
// magnitude up exactly when the carry reaches the kept bits, with exactly
// the right probability.  Below 2^-14 the halves are the multiples of 2^-24,
// which is the normal grid of [2^-14, 2^-13): |v| is moved there by adding
// 2^-14, rounded the same way, and moved back (exact).  That one add rounds
// below 2^-37, so there the probability is right to 2^-14 of a step.
// Magnitudes beyond the largest half become inf or nan, as a plain
// conversion would make them inf.
__device__ __forceinline__ float sr_half(float v, uint32_t r) {
  const float a = fabsf(v);
  const float off = a < 0x1p-14f ? 0x1p-14f : 0.0f;
  const float t = __uint_as_float((__float_as_uint(a + off) + (r & 0x1fffu)) & ~0x1fffu) - off;
  return copysignf(t, v);
}

template <int Q, int S> struct Pops;

template <int Q> struct Pops<Q, 0> {
  float *f, *g;
  // g_0 = O(1) is carried as hi + lo: hi in plane 0 of g, lo (the part of
  // g_0 that FP32 rounds away, below 2^-24 |g_0|) scaled by 2^24 in this
  // half-precision plane, one entry per cell.  Rounding g_0 alone to FP32
  // each step moves long runs measurably; the other populations are small.
  __half *g0l;
  // the value a store keeps (identity for FP32)
  __device__ __forceinline__ float round(float v) const { return v; }
  template <bool SR>
  __device__ __forceinline__ float round_at(float v, uint32_t &) const { return v; }
  __device__ __forceinline__ uint32_t step_key() const { return 0u; }
  __device__ __forceinline__ float ldg0lo(long long c) const { return __half2float(g0l[c]) * 0x1p-24f; }
  __device__ __forceinline__ void stg0lo(long long c, float lo) const { g0l[c] = __float2half_rn(lo * 0x1p24f); }
  __device__ __forceinline__ float ldf(int i, long long c) const { return ld_at(f, blk_offset<4>(Q, i, c)); }
  __device__ __forceinline__ float ldg(int i, long long c) const { return ld_at(g, blk_offset<4>(Q, i, c)); }
  __device__ __forceinline__ float ldfc(int i, long long c) const { return ld_at<float, false>(f, blk_offset<4>(Q, i, c)); }
  __device__ __forceinline__ float ldgc(int i, long long c) const { return ld_at<float, false>(g, blk_offset<4>(Q, i, c)); }
  __device__ __forceinline__ void stf(int i, long long c, float v) const { st_at(f, blk_offset<4>(Q, i, c), v); }
  __device__ __forceinline__ void stg(int i, long long c, float v) const { st_at(g, blk_offset<4>(Q, i, c), v); }
};

template <int Q> struct Pops<Q, 1> {
  __half *f, *g;  // g: q planes like f, plane 0 unused
  float *g0;      // g_0
  // step counter of stochastic rounding (null: round to nearest even)
  uint32_t *ctr = nullptr;
  // the value a half store keeps (g_0 is stored in FP32 and not rounded)
  __device__ __forceinline__ float round(float v) const { return __half2float(__float2half_rn(v)); }
  // the same, rounded stochastically with SR from the cell's stream rs (a
  // separate instantiation, so the round-to-nearest kernels keep their
  // register budget)
  template <bool SR>
  __device__ __forceinline__ float round_at(float v, uint32_t &rs) const {
    if constexpr (SR) {
      rs = sr_next(rs);
      return sr_half(v, rs);
    } else {
      return round(v);
    }
  }
  __device__ __forceinline__ uint32_t step_key() const { return ctr ? ctr[0] : 0u; }
  __device__ __forceinline__ float ldf(int i, long long c) const { return __half2float(ld_at(f, blk_offset<2>(Q, i, c))); }
  __device__ __forceinline__ float ldg(int i, long long c) const {
    return i == 0 ? ld_at(g0, (uint32_t)c * 4u) : __half2float(ld_at(g, blk_offset<2>(Q, i, c)));
  }
  __device__ __forceinline__ float ldfc(int i, long long c) const { return ldf(i, c); }
  __device__ __forceinline__ float ldgc(int i, long long c) const { return ldg(i, c); }
  __device__ __forceinline__ void stf(int i, long long c, float v) const { st_at(f, blk_offset<2>(Q, i, c), __float2half_rn(v)); }
  __device__ __forceinline__ void stg(int i, long long c, float v) const {
    if (i == 0) st_at(g0, (uint32_t)c * 4u, v); else st_at(g, blk_offset<2>(Q, i, c), __float2half_rn(v));
  }
};

// ---------------------------------------------------------------------------
// Per-node formulas
// ---------------------------------------------------------------------------

// Bulk chemical-potential polynomial of eqs. (mu_rho, mu_phi):
// s (s-1) (s-2) with s = 1 + a, written as a (a-1) (a+1) for accuracy near
// the bulk values a = 0, +-1.
__device__ __forceinline__ float cubic_shifted(float a) { return a * (a - 1.0f) * (a + 1.0f); }

// mu_rho, mu_phi of eqs. (mu_rho, mu_phi) from drho = rho - 1, phi and the
// Laplacians of rho and phi.
__device__ __forceinline__ void chem_pot(const Phys &P, float drho, float phi, float lap_rho,
                                         float lap_phi, float &mu_rho, float &mu_phi) {
  float ps = cubic_shifted(drho + phi);  // rho + phi = 1 + (drho + phi)
  float pt = cubic_shifted(drho - phi);  // rho - phi = 1 + (drho - phi)
  float bs = 0.125f * P.k1 * ps, bt = 0.125f * P.k2 * pt;
  float ksum = P.k1 + P.k2, kdif = P.k2 - P.k1;
  mu_rho = bs + bt + P.a2q * (kdif * lap_phi - ksum * lap_rho);
  mu_phi = bs - bt + P.a2q * (kdif * lap_rho - ksum * lap_phi);
}

// Bulk free-energy density of eq. (functional) without gradient terms.
__device__ __forceinline__ float psi_bulk(const Phys &P, float rho, float phi) {
  float s = rho + phi, t = rho - phi;
  return 0.03125f * (P.k1 * s * s * (s - 2.0f) * (s - 2.0f) + P.k2 * t * t * (t - 2.0f) * (t - 2.0f));
}

// Velocity of the solid body owning cell (xs, ys, zs) at the midpoint of the
// link from fluid cell (x, y, z) along direction i (halfway bounce-back).
template <class V>
__device__ __forceinline__ void body_velocity(const Geom &G, const Phys &P, uint8_t code, int x,
                                              int y, int z, int xs, int ys, int zs, int i,
                                              float uw[3]) {
  // Phys is read with compile-time indices only (selects instead of a
  // run-time array index), so a copy of it can live in registers.
  uw[0] = uw[1] = uw[2] = 0.0f;
  if (code == CELL_GHOST) {
    const int sc[3] = {xs, ys, zs};
    const int ext[3] = {G.ex, G.ey, G.ez};
    int n = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (G.per[a]) continue;
      int side = sc[a] == 0 ? 0 : (sc[a] == ext[a] - 1 ? 1 : -1);
      if (side < 0) continue;
#pragma unroll
      for (int k = 0; k < 3; ++k) uw[k] += side ? P.wall_u[a][1][k] : P.wall_u[a][0][k];
      ++n;
    }
    if (n > 1) {
      float inv = 1.0f / (float)n;
      uw[0] *= inv; uw[1] *= inv; uw[2] *= inv;
    }
    return;
  }
  const int r = (int)code - CELL_ROLLER0;
  if (r < 0 || r >= P.n_rollers) return;
  float rc0 = 0.0f, rc1 = 0.0f, rc2 = 0.0f, om = 0.0f;
  int ax = 2;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k == r) { rc0 = P.rc[k][0]; rc1 = P.rc[k][1]; rc2 = P.rc[k][2]; om = P.rom[k]; ax = P.rax[k]; }
  float d0 = (float)(x - G.off[0]) + 0.5f * V::cx(i) - rc0;
  float d1 = (float)(y - G.off[1]) + 0.5f * V::cy(i) - rc1;
  float d2 = (float)(z - G.off[2]) + 0.5f * V::cz(i) - rc2;
  if (ax == 0) { uw[1] = -om * d2; uw[2] = om * d1; }
  else if (ax == 1) { uw[0] = om * d2; uw[2] = -om * d0; }
  else { uw[0] = -om * d1; uw[1] = om * d0; }
}

}  // namespace frelbm
