// kernels.hip -- HIP kernels (gfx950) of the free-energy LBM step.
//
// One time step (Algorithm 1 of Simonis et al., arXiv 2212.01617, then
// streaming, Sec. 2.3) is a short sequence of launches over the storage grid:
//   k_moments   rho - 1, phi at fluid cells             (eqs. densMoment, ordeMoment)
//   k_fill_m    rho, phi at solid cells next to fluid   (fluid-neighbour mean)
//   k_potential mu_rho, mu_phi and Pi = rho mu_rho + phi mu_phi   (eqs. mu_rho, mu_phi)
//   k_fill_c    Pi (and rho, phi) at solid cells next to fluid
//   k_collide   force (eq. F), velocity (eq. veloMoment), BGK collision of f
//               with Guo forcing (eqs. bgk, feq, Fi) and of g (eqs. LBEg,
//               geq), streaming with moving bounce-back, in place.
// With FP32 storage the moments at t+1 are instead a by-product of k_collide
// (partial sums on chip) completed by k_combine, so a step is k_fill_m,
// k_potential, k_fill_c, k_collide, k_combine and k_moments runs only after
// the populations are set from outside (initialisation, restores).
//
// Streaming is in place with the AA access pattern: at even time steps a
// cell reads and writes only its own slots (writing direction i into slot
// opp(i)); at odd steps it reads from and writes to its neighbours' slots.
// Each slot is read and written by the same thread within a step, so the
// update is race-free without a second population buffer.
//
// The coupling fields a fluid cell needs from its neighbours are packed into
// one float4 per cell, C = (rho - 1, phi, Pi, mu_rho), with mu_phi in a
// plane of its own; a 32-bit word per cell flags its non-fluid neighbours.
#include "lbm_device.h"
#include "kernels.h"

namespace frelbm {

constexpr int BX = 64, BY = 4;

__device__ __forceinline__ bool cell_of_thread(const Geom &G, int &x, int &y, int &z, long long &c) {
  x = blockIdx.x * BX + threadIdx.x;
  y = blockIdx.y * BY + threadIdx.y;
  z = blockIdx.z;
  if (x >= G.ex || y >= G.ey) return false;
  c = (long long)x + (long long)G.px * ((long long)y + (long long)G.ey * z);
  return true;
}

// XCD-aware tile order for a 1D grid of nb blocks.  Workgroups are handed to
// the 8 XCDs round-robin (block b runs on XCD b % 8) and each XCD has its own
// L2.  With the plain order, the tiles left and right of a tile run on other
// XCDs, and the partial cache lines that an x-shifted access (odd-parity
// streaming, the stencils) reads across the tile edge are fetched from HBM
// once per XCD.  Here consecutive runs of gx tiles (one grid row in x) go
// to one XCD, while the 8 XCDs still work on neighbouring rows at any time.
constexpr int NXCD = 8;
__device__ __forceinline__ uint32_t udiv(uint32_t n, const UDiv &u) { return (__umulhi(n, u.m) + n) >> u.s; }

// Tile of block b: (tile column bx, row of tiles r counted over all planes).
__device__ __forceinline__ void tile_of_block(const TileMap &T, uint32_t b, uint32_t &bx, uint32_t &r) {
  const uint32_t gx = (uint32_t)T.gx;
  uint32_t t = b;
  if (T.xcd && b < (uint32_t)T.full) {
    const uint32_t k = b % NXCD, j = b / NXCD, jq = udiv(j, T.dgx);
    t = (jq * NXCD + k) * gx + (j - jq * gx);
  }
  r = udiv(t, T.dgx);
  bx = t - r * gx;
}

// Cell of this thread in a 1D grid of 64 x blockDim.y tiles (x fastest,
// then y, then z).  A wave is one 64-cell row of its tile, so y and z are
// the same in every lane; saying so lets the row and plane arithmetic run
// on the scalar unit.
__device__ __forceinline__ bool cell_of_tile(const Geom &G, const TileMap &T, int &x, int &y, int &z,
                                             long long &c) {
  const int rows = (int)blockDim.y;
  uint32_t bx, r;
  tile_of_block(T, blockIdx.x, bx, r);
  const uint32_t rq = udiv(r, T.dgy);
  x = (int)bx * BX + threadIdx.x;
  y = __builtin_amdgcn_readfirstlane((int)(r - rq * (uint32_t)T.gy) * rows + (int)threadIdx.y);
  z = (int)rq;
  if (x >= G.ex || y >= G.ey) return false;
  c = (long long)x + (long long)G.px * ((long long)y + (long long)G.ey * z);
  return true;
}

// Neighbour addressing of one cell: the wrapped x, row and plane offsets for
// steps -1, 0, +1 along each axis; neighbour i is at ox[cx+1] + oy[cy+1] +
// oz[cz+1].  Fluid cells never sit on the storage boundary of a wall axis
// (the ghost layer is there), so only periodic axes wrap.
struct Nbr {
  int ox[3], oy[3], oz[3];
  __device__ __forceinline__ Nbr(const Geom &G, int x, int y, int z) {
    ox[0] = wrap(x - 1, G.ex); ox[1] = x; ox[2] = wrap(x + 1, G.ex);
    oy[0] = G.px * wrap(y - 1, G.ey); oy[1] = G.px * y; oy[2] = G.px * wrap(y + 1, G.ey);
    const int pl = G.px * G.ey;
    oz[0] = pl * wrap(z - 1, G.ez); oz[1] = pl * z; oz[2] = pl * wrap(z + 1, G.ez);
  }
  template <class V> __device__ __forceinline__ int at(int i) const {
    return ox[V::cx(i) + 1] + oy[V::cy(i) + 1] + oz[V::cz(i) + 1];
  }
  // the cell x - c_i
  template <class V> __device__ __forceinline__ int back(int i) const {
    return ox[1 - V::cx(i)] + oy[1 - V::cy(i)] + oz[1 - V::cz(i)];
  }
};

// Load the q populations of fluid cell c at time parity `odd` (AA pattern).
// CACHED selects ordinary rather than non-temporal loads (the collide).
template <int Q, int S, bool CACHED = false>
__device__ __forceinline__ void load_pops(const Pops<Q, S> &P, const Nbr &N, long long c, int odd,
                                          float *df, float *g) {
  using V = VSet<Q>;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    // f_i(x) = f_i*(x - c_i) after an odd step, written by x - c_i into its slot opp(i)
    const long long s = (!odd || i == 0) ? c : (long long)N.template back<V>(i);
    const int sl = !odd ? i : opp(i);
    df[i] = CACHED ? P.ldfc(sl, s) : P.ldf(sl, s);
    g[i] = CACHED ? P.ldgc(sl, s) : P.ldg(sl, s);
  }
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Stages of one step, per cell (or per solid boundary cell for the fills).
// The single-lattice kernels and the batched persistent kernels below both
// call these, so a lattice advanced alone or inside a batch takes exactly
// the same arithmetic.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Moments at t+1 as a by-product of collide (FP32 storage).
//
// rho(y, t+1) = sum_i f_i(y, t+1), where f_i(y, t+1) is f*_i(y - c_i) for a
// fluid source y - c_i and cell y's own bounce-back value otherwise (phi
// likewise with g).  The sum is split by the plane of the source: group UP
// (c_z = +1, sources one plane below), S0 (c_z = 0) and DN (c_z = -1),
// combined as (UP + S0) + DN, each group summed in ascending direction order
// in two passes: first the "available" sources -- fluid and inside the
// destination's tile footprint, the 64 x COLLIDE_ROWS columns of the collide
// tile grid that contains it -- then the others.  k_collide forms the first
// pass on chip from the post-collision values of its tile and stores it per
// group; k_combine adds the second pass (tile-edge sources and bounce-backs)
// from the population arrays and, for sources across a tile's x edge, from
// the compact copy XE that k_collide leaves, and stores M; k_moments
// performs both passes from the population arrays.  The additions are the same in every case, so M does
// not depend on which path computed it.  FP16 storage keeps the plain moment
// pass, which reads half the bytes and costs less than the partial planes.
// ---------------------------------------------------------------------------
template <int S> struct ByProduct { static constexpr bool on = S == 0; };

__device__ __forceinline__ bool in_footprint(const Geom &G, int x, int y, int cx, int cy) {
  const int sx = x - cx, sy = y - cy;
  const int xlo = x & ~(BX - 1), ylo = (y / COLLIDE_ROWS) * COLLIDE_ROWS;
  return sx >= xlo && sx < min(xlo + BX, G.ex) && sy >= ylo && sy < min(ylo + COLLIDE_ROWS, G.ey);
}

// Populations that leave a 64-cell row segment sideways.  XE holds, for each
// segment, the post-collision (f, g) of the directions with c_x = -1 at the
// segment's first column (side 0) and of those with c_x = +1 at its last
// storage column (side 1; ex - 1 for a short last segment).  It is laid out
// [z][side][e][segment column bx][y], e counting a side's directions in
// ascending order, so that the rows of one tile read and write consecutive
// entries.  k_collide writes them for every fluid cell on those columns and
// k_combine reads them in place of the population arrays, where each value
// would cost a 128-byte line of its own.
template <class V> struct XEdge {
  static constexpr int NE = V::D == 3 ? 5 : 3;
  // rank of direction i among the directions with the same c_x != 0, in
  // ascending order (D3Q19: 1 7 9 11 13 and 2 8 10 12 14; D2Q9: 1 5 7 and 2 6 8)
  __host__ __device__ static constexpr int slot(int i) {
    return i < 3 ? 0 : (V::D == 3 ? (i - 5) / 2 : (i - 3) / 2);
  }
  // direction of entry e of a side (the inverse of slot)
  __device__ static int dir(int side, int e) { return e == 0 ? 2 - side : 2 * e + (V::D == 3 ? 6 : 4) - side; }
  // entry e of `side` for the segment holding cell (x, y, z)
  __device__ static uint32_t index(const Geom &G, int x, int y, int z, int side, int e) {
    return ((((uint32_t)z * (uint32_t)(G.px >> 6) + (uint32_t)(x >> 6)) * (uint32_t)G.ey + (uint32_t)y) * 2u +
            (uint32_t)side) * NE + (uint32_t)e;
  }
  // entry of direction i (c_x != 0) leaving cell (x, y, z)
  __device__ static uint32_t index(const Geom &G, int x, int y, int z, int i) {
    return index(G, x, y, z, V::cx(i) > 0 ? 1 : 0, slot(i));
  }
};

// Population i of fluid cell c at parity `odd` (AA pattern), as load_pops.
template <int Q, int S>
__device__ __forceinline__ void pop_at(const Pops<Q, S> &P, const Nbr &N, long long c, int odd, int i,
                                       float &f, float &g) {
  using V = VSet<Q>;
  if (!odd || i == 0) {
    f = P.ldf(i, c);
    g = P.ldg(i, c);
  } else {
    const long long s = N.template back<V>(i);
    f = P.ldf(opp(i), s);
    g = P.ldg(opp(i), s);
  }
}

// Whether source y - c_i of fluid cell (x, y) (neighbour word `bits`) is
// summed in the first pass.
template <class V>
__device__ __forceinline__ bool available(const Geom &G, int x, int y, uint32_t bits, int i) {
  if (i == 0) return true;
  return in_footprint(G, x, y, V::cx(i), V::cy(i)) && !((bits >> opp(i)) & 1u);
}

template <int Q>
__device__ __forceinline__ float2 group_total(float2 up, float2 s0, float2 dn) {
  if (VSet<Q>::D == 2) return s0;
  return make_float2((up.x + s0.x) + dn.x, (up.y + s0.y) + dn.y);
}

// Direction sets as bit masks (bit i for direction i).
template <class V> struct DirBits {
  static constexpr int Q = V::D == 3 ? 19 : 9;
  static constexpr uint32_t with(int ax, int sgn) {
    uint32_t m = 0;
    for (int i = 1; i < Q; ++i)
      if ((ax == 0 ? V::cx(i) : ax == 1 ? V::cy(i) : V::cz(i)) == sgn) m |= 1u << i;
    return m;
  }
  static constexpr uint32_t parity(int r) {
    uint32_t m = 0;
    for (int i = 1; i < Q; ++i)
      if ((i & 1) == r) m |= 1u << i;
    return m;
  }
  static constexpr uint32_t XP = with(0, 1), XM = with(0, -1), YP = with(1, 1), YM = with(1, -1);
  static constexpr uint32_t ODD = parity(1), EVEN = parity(0);
  // bit i: the source x - c_i of a fluid cell with neighbour word `bits` is
  // not fluid (bit opp(i) of the word; opp pairs 2k-1 with 2k)
  __device__ static uint32_t solid_sources(uint32_t bits) { return ((bits >> 1) & ODD) | ((bits << 1) & EVEN); }
};

// Neighbour word of cell c.  A 64-cell row segment flagged all-fluid (every
// cell fluid, every neighbour fluid) gives 0 without reading nbm: each wave
// of the single-lattice cell kernels covers exactly one segment, so the flag
// is one scalar load per wave in place of 256 bytes of neighbour words.
template <int Q, int S>
__device__ __forceinline__ uint32_t nb_word(const LatView<Q, S> &L, long long c) {
  if (L.segf) {
    const uint32_t sg = __builtin_amdgcn_readfirstlane((uint32_t)(c >> 6));
    if (L.segf[sg]) return 0u;
  }
  return L.nbm[c];
}

// Second pass for fluid cell c: adds the unavailable sources of each group,
// in ascending direction order, to the first-pass sums grp[cz + 1].  All
// needed loads are issued before the sums.  With XE given (FP32), fluid
// sources across the x edge of the footprint are read from it (the same
// values) through the same load as the population arrays.
template <int Q, int S>
__device__ __forceinline__ void second_pass(const LatView<Q, S> &L, const Nbr &N, long long c, int odd, int x,
                                            int y, int z, uint32_t bits, float2 grp[3], const float2 *XE) {
  using V = VSet<Q>;
  using B = DirBits<V>;
  const int xlo = x & ~(BX - 1), ylo = (y / COLLIDE_ROWS) * COLLIDE_ROWS;
  const uint32_t solid = B::solid_sources(bits);
  // sources across each footprint edge (the complement of in_footprint)
  const uint32_t xe = (x == xlo ? B::XP : 0u) | (x == min(xlo + BX, L.G.ex) - 1 ? B::XM : 0u);
  const uint32_t ye = (y == ylo ? B::YP : 0u) | (y == min(ylo + COLLIDE_ROWS, L.G.ey) - 1 ? B::YM : 0u);
  const uint32_t un = solid | xe | ye;           // unavailable sources
  const uint32_t side = XE ? (xe & ~solid) : 0u;  // of those, read from XE
  float vf[Q], vg[Q];
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    vf[i] = vg[i] = 0.0f;
    if (!((un >> i) & 1u)) continue;
    if constexpr (S == 0) {
      const long long s = !odd ? c : (long long)N.template back<V>(i);
      const int slot = !odd ? i : opp(i);
      const float *pf = L.P.f + blk_offset<4>(Q, slot, s) / 4;
      const float *pg = L.P.g + blk_offset<4>(Q, slot, s) / 4;
      if (V::cx(i) != 0 && ((side >> i) & 1u)) {
        const int sx = wrap(x - V::cx(i), L.G.ex), sy = wrap(y - V::cy(i), L.G.ey);
        const int sz = V::D == 3 ? wrap(z - V::cz(i), L.G.ez) : 0;
        pf = &XE[XEdge<V>::index(L.G, sx, sy, sz, i)].x;
        pg = pf + 1;
      }
      vf[i] = __builtin_nontemporal_load(pf);
      vg[i] = __builtin_nontemporal_load(pg);
    } else {
      pop_at<Q, S>(L.P, N, c, odd, i, vf[i], vg[i]);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if (V::cz(i) != k - 1 || !((un >> i) & 1u)) continue;
      grp[k].x += vf[i];
      grp[k].y += vg[i];
    }
}

// M from the populations alone (state parity ODD).
template <int Q, int S, int ODD>
__device__ __forceinline__ void stage_moments(const LatView<Q, S> &L, int x, int y, int z) {
  using V = VSet<Q>;
  const long long c = (long long)x + (long long)L.G.px * ((long long)y + (long long)L.G.ey * z);
  const uint32_t bits = nb_word<Q, S>(L, c);
  if (bits & NB_SELF_SOLID) return;
  const Nbr N(L.G, x, y, z);
  float df[Q], g[Q];
  load_pops<Q, S>(L.P, N, c, ODD, df, g);
  if (!ByProduct<S>::on) {
    float drho = 0.0f, phi = 0.0f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      drho += df[i];
      phi += g[i];
    }
    L.M[c] = make_float2(drho, phi);
    return;
  }
  float2 grp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) grp[k] = make_float2(0.0f, 0.0f);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (!available<V>(L.G, x, y, bits, i)) continue;
    grp[V::cz(i) + 1].x += df[i];
    grp[V::cz(i) + 1].y += g[i];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (V::cz(i) != k - 1 || available<V>(L.G, x, y, bits, i)) continue;
      grp[k].x += df[i];
      grp[k].y += g[i];
    }
  L.M[c] = group_total<Q>(grp[2], grp[1], grp[0]);
}

// Second pass after collide; the state at t+1 has parity PAR.
template <int Q, int S, int PAR>
__device__ __forceinline__ void stage_combine(const LatView<Q, S> &L, int x, int y, int z) {
  const long long c = (long long)x + (long long)L.G.px * ((long long)y + (long long)L.G.ey * z);
  const uint32_t bits = nb_word<Q, S>(L, c);
  if (bits & NB_SELF_SOLID) return;
  const Nbr N(L.G, x, y, z);
  float2 grp[3];
  grp[1] = L.P0[c];
  if (VSet<Q>::D == 3) {
    grp[0] = L.PD[c];
    grp[2] = L.PU[c];
  } else {
    grp[0] = grp[2] = make_float2(0.0f, 0.0f);
  }
  second_pass<Q, S>(L, N, c, PAR, x, y, z, bits, grp, L.XE);
  L.M[c] = group_total<Q>(grp[2], grp[1], grp[0]);
}

// Weighted mean over the fluid neighbours of solid cell s (coordinates x, y,
// z) of the NC leading floats of a field with stride ST floats per cell.  Bit
// i of `fluid_bits` (the solid cell's neighbour word) is set when the
// neighbour along c_i is fluid; all loads are issued before the sums, which
// run in direction order.
template <int Q, int NC, int ST>
__device__ __forceinline__ void fluid_mean(const float *__restrict__ X, uint32_t fluid_bits, const Geom &G,
                                           int x, int y, int z, float *out) {
  using V = VSet<Q>;
  float v[Q][NC];
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (!((fluid_bits >> i) & 1u)) continue;
    const int xn = wrap(x + V::cx(i), G.ex), yn = wrap(y + V::cy(i), G.ey);
    const int zn = V::D == 3 ? wrap(z + V::cz(i), G.ez) : z;
    const long long n2 = (long long)xn + (long long)G.px * ((long long)yn + (long long)G.ey * zn);
#pragma unroll
    for (int k = 0; k < NC; ++k) v[i][k] = X[ST * n2 + k];
  }
  float num[NC], den = 0.0f;
#pragma unroll
  for (int k = 0; k < NC; ++k) num[k] = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (!((fluid_bits >> i) & 1u)) continue;
    const float w = V::w(i);
#pragma unroll
    for (int k = 0; k < NC; ++k) num[k] += w * v[i][k];
    den += w;
  }
  const float inv = den > 0.0f ? 1.0f / den : 0.0f;
#pragma unroll
  for (int k = 0; k < NC; ++k) out[k] = num[k] * inv;
}

__device__ __forceinline__ void cell_coords(const Geom &G, int s, int &x, int &y, int &z) {
  x = s % G.px;
  int r = s / G.px;
  y = r % G.ey;
  z = r / G.ey;
}

// Solid cells next to fluid take the lattice-weighted mean of their fluid
// neighbours: rho, phi into M ...
template <int Q, int S>
__device__ __forceinline__ void stage_fill_m(const LatView<Q, S> &L, int s) {
  int x, y, z;
  cell_coords(L.G, s, x, y, z);
  float v[2];
  fluid_mean<Q, 2, 2>((const float *)L.M, L.nbm[s], L.G, x, y, z, v);
  L.M[s] = make_float2(v[0], v[1]);
}

// ... and Pi into C (with the filled rho, phi copied from M).
template <int Q, int S>
__device__ __forceinline__ void stage_fill_c(const LatView<Q, S> &L, int s) {
  int x, y, z;
  cell_coords(L.G, s, x, y, z);
  float pi;
  fluid_mean<Q, 1, 4>((const float *)L.C + 2, L.nbm[s], L.G, x, y, z, &pi);
  const float2 m = L.M[s];
  L.C[s] = make_float4(m.x, m.y, pi, 0.0f);
}

// Laplacians of rho and phi at a cell with moments m0; fetch(i) gives the
// moments of the neighbour along c_i.
template <int Q, class Fetch>
__device__ __forceinline__ void laplacians(Fetch fetch, float2 m0, float &lr, float &lp) {
  using V = VSet<Q>;
  float ar = 0.0f, ap = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const float2 m = fetch(i);
    ar += V::w(i) * (m.x - m0.x);
    ap += V::w(i) * (m.y - m0.y);
  }
  lr = 6.0f * ar;  // 2 / cs^2
  lp = 6.0f * ap;
}

// Pi and mu_phi of fluid cell c into C = (rho - 1, phi, Pi, mu_phi); mu_rho
// is recovered where needed as (Pi - phi mu_phi) / rho (coupling_mu_rho).
template <int Q, int S>
__device__ __forceinline__ void store_potential(const LatView<Q, S> &L, long long c, float2 m0, float lr,
                                                float lp) {
  float mr, mp;
  chem_pot(L.ph, m0.x, m0.y, lr, lp, mr, mp);
  L.C[c] = make_float4(m0.x, m0.y, (1.0f + m0.x) * mr + m0.y * mp, mp);
}

// mu_rho of a cell from its coupling values C = (rho - 1, phi, Pi, mu_phi).
__device__ __forceinline__ float coupling_mu_rho(float4 c) { return (c.z - c.y * c.w) / (1.0f + c.x); }

template <int Q, int S>
__device__ __forceinline__ void stage_potential(const LatView<Q, S> &L, int x, int y, int z) {
  using V = VSet<Q>;
  const long long c = (long long)x + (long long)L.G.px * ((long long)y + (long long)L.G.ey * z);
  if (L.nbm[c] & NB_SELF_SOLID) return;
  const Nbr N(L.G, x, y, z);
  const float2 m0 = L.M[c];
  float lr, lp;
  laplacians<Q>([&](int i) { return L.M[N.template at<V>(i)]; }, m0, lr, lp);
  store_potential<Q, S>(L, c, m0, lr, lp);
}

// Force of eq. (F) in product-rule form:
//   -rho grad mu_rho - phi grad mu_phi
//     = mu_rho grad rho + mu_phi grad phi - grad(rho mu_rho + phi mu_phi),
// gradients by the lattice stencil (1/cs^2) sum_i w_i c_i X(x + c_i).
template <int Q>
__device__ __forceinline__ void force(const float4 *__restrict__ C, const Nbr &N, float mu_rho,
                                      float mu_phi, float F[3]) {
  using V = VSet<Q>;
  float gr[3] = {0, 0, 0}, gp[3] = {0, 0, 0}, gq[3] = {0, 0, 0};
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    float4 m = C[N.template at<V>(i)];
    float w = 3.0f * V::w(i);
    if (V::cx(i)) { gr[0] += V::cx(i) * w * m.x; gp[0] += V::cx(i) * w * m.y; gq[0] += V::cx(i) * w * m.z; }
    if (V::cy(i)) { gr[1] += V::cy(i) * w * m.x; gp[1] += V::cy(i) * w * m.y; gq[1] += V::cy(i) * w * m.z; }
    if (V::cz(i)) { gr[2] += V::cz(i) * w * m.x; gp[2] += V::cz(i) * w * m.y; gq[2] += V::cz(i) * w * m.z; }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) F[a] = mu_rho * gr[a] + mu_phi * gp[a] - gq[a];
}

// f_i^eq - w_i = w_i (rho - 1) + a_i (c_i . m) + w_i q_i (q_i: the
// second-order part) rounded once to FP32: the three parts are summed in FP64.
// Summed in FP32, each partial sum rounds, and in a region where rho, m and
// u vary by less than an ulp every cell rounds the same way at every step:
// the equilibrium's momentum then differs from m by the same amount in
// every cell, and the flow drifts.
__device__ __forceinline__ float feq_shifted(float wi, float ai, double drho, float cm, float wq) {
  return (float)__builtin_fma((double)ai, (double)cm, __builtin_fma((double)wi, drho, (double)wq));
}

// Collision of one fluid cell and streaming of its populations (AA pattern
// of parity ODD): every population goes to the slot it streams to.  If
// `post` is given, the stored value of each moving population i > 0 also goes
// to post[i - 1][tid] (f) and post[Q - 1 + i - 1][tid] (g); the rest
// populations are returned in rest_out.  For a link into a solid cell that
// slot is never read; bounce_back() then moves the population to the slot the
// cell reads it from next step.
//
// The equilibria (eqs. feq, geq) and the Guo term (eq. Fi) are split into
// their parts of zeroth, first and second order in c_i.  The first-order part
// of f^eq is formed from the momentum m = j + F/2 itself, a_i (c_i . m), not
// from rho times u = m / rho: a rounded 1/rho takes the same value over wide
// regions where rho varies by less than an ulp, and rho u would then differ
// from m by the same fraction in every cell of such a region, at every step.
// With the coefficients a_i (exact_lin) the momentum of f^eq is m and that of
// the Guo term (1 - 1/(2 tau_f)) F, to the rounding of the individual terms.
//
// FP32 storage carries g_0 = O(1) as hi + lo (lo in a half-precision plane,
// scaled by 2^24): the increment of g_0 is formed from the moving populations
// alone, tau_g^-1 sum_{i>0} (g_i - g_i^eq), which equals (g_0^eq - g_0) / tau_g
// since g_0^eq complements the others to phi, and added to hi + lo with the
// rounding error of the sum kept (TwoSum, Knuth).
template <int Q, int S, int ODD, int NT, bool SR = false>
__device__ __forceinline__ void collide_cell(const Pops<Q, S> &P, const Nbr &N, long long c,
                                             const float4 *__restrict__ C,
                                             const Phys &ph, float (*post)[NT], int tid, float &rho_out,
                                             float &phi_out, float2 &rest_out, uint32_t &rs) {
  using V = VSet<Q>;
  constexpr bool X = S == 0;  // g_0 as hi + lo
  const float4 cc = C[c];
  const float mu_phi = cc.w, mu_rho = coupling_mu_rho(cc);
  float F[3];
  force<Q>(C, N, mu_rho, mu_phi, F);
  // FP16 storage loads g only after f is collided and stored (fewer live
  // registers); with FP32 storage and the moment sums the split costs
  // registers instead, so f and g are loaded together.
  constexpr bool SPLIT = S == 1;
  float df[Q], g[Q];
  if constexpr (SPLIT) {
#pragma unroll
    for (int i = 0; i < Q; ++i) df[i] = (!ODD || i == 0) ? P.ldfc(i, c) : P.ldfc(opp(i), N.template back<V>(i));
  } else {
    load_pops<Q, S, true>(P, N, c, ODD, df, g);
  }
  float drho = 0.0f, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += df[i];
    j[0] += V::cx(i) * df[i];
    j[1] += V::cy(i) * df[i];
    j[2] += V::cz(i) * df[i];
  }
  const float rho = 1.0f + drho;
  const float inv_rho = 1.0f / rho;
  const float m[3] = {j[0] + 0.5f * F[0], j[1] + 0.5f * F[1], j[2] + 0.5f * F[2]};  // eq. veloMoment: rho u
  // u = m / rho enters the terms of second order; they are written with m
  // and 1/rho so that u itself is not kept (registers)
  const float mmr = (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) * inv_rho;  // rho |u|^2
  const float uF = (m[0] * F[0] + m[1] * F[1] + m[2] * F[2]) * inv_rho;   // u . F
  // rho times the second-order part of the equilibria over w_i, from
  // cm = c_i . m and cu = c_i . u; the same expression in both loops, so f and g
  // see the same value
  auto rquad = [&](float cm, float cu) { return 4.5f * cm * cu - 1.5f * mmr; };
  float phi = 0.0f, gm = 0.0f;  // gm: sum of the moving g_i (FP32: g_0 as hi + lo)
  if constexpr (!SPLIT) {
    if constexpr (X) {
      // phi = g_0 + sum of the moving g_i, the latter also used for g_0 below
#pragma unroll
      for (int i = 1; i < Q; ++i) gm += g[i];
      phi = g[0] + gm;
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) phi += g[i];
    }
  }
  float geq_rest = 0.0f;
  // post-collision g_i of direction i > 0, stored to the slot it streams to
  auto collide_g = [&](int i) {
    const float cm = V::cx(i) * m[0] + V::cy(i) * m[1] + V::cz(i) * m[2];
    const float cu = cm * inv_rho;
    const float geq = V::w(i) * ph.gam3 * mu_phi + phi * (V::a(i) * cu + V::w(i) * (rquad(cm, cu) * inv_rho));
    geq_rest += geq;
    const float gs = P.template round_at<SR>(g[i] + ph.om_g * (geq - g[i]), rs);
    if (post) post[Q - 1 + i - 1][tid] = gs;
    // streamed: slot (x, opp(i)) after an even step, (x + c_i, i) after an odd one
    if (!ODD) P.stg(opp(i), c, gs);
    else P.stg(i, N.template at<V>(i), gs);
  };
  const double drho_d = (double)drho;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float cF = V::cx(i) * F[0] + V::cy(i) * F[1] + V::cz(i) * F[2];
    const float cm = V::cx(i) * m[0] + V::cy(i) * m[1] + V::cz(i) * m[2];
    const float cu = cm * inv_rho;
    const float wi = V::w(i), ai = V::a(i);
    const float dfeq = feq_shifted(wi, ai, drho_d, cm, wi * rquad(cm, cu));     // f_i^eq - w_i
    const float src = ph.guo * (ai * cF - 3.0f * wi * uF + 3.0f * ai * cu * cF);  // Guo term
    const float fs = P.template round_at<SR>(df[i] + ph.om_f * (dfeq - df[i]) + src, rs);
    if (i == 0) {
      P.stf(0, c, fs);
      rest_out.x = fs;
      continue;
    }
    if (post) post[i - 1][tid] = fs;
    if (!ODD) P.stf(opp(i), c, fs);
    else P.stf(i, N.template at<V>(i), fs);
    if constexpr (!SPLIT) collide_g(i);
  }
  if constexpr (SPLIT) {
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = (!ODD || i == 0) ? P.ldgc(i, c) : P.ldgc(opp(i), N.template back<V>(i));
#pragma unroll
    for (int i = 0; i < Q; ++i) phi += g[i];
#pragma unroll
    for (int i = 1; i < Q; ++i) collide_g(i);
  }
  float g0s;
  if constexpr (X) {
    const float t = ph.om_g * (gm - geq_rest) + P.ldg0lo(c);
    g0s = g[0] + t;
    const float tb = g0s - g[0];
    P.stg0lo(c, (g[0] - (g0s - tb)) + (t - tb));
  } else {
    g0s = g[0] + ph.om_g * ((phi - geq_rest) - g[0]);  // g_0 is stored in FP32
  }
  P.stg(0, c, g0s);
  rest_out.y = g0s;
  rho_out = rho;
  phi_out = phi;
}

// Moving halfway bounce-back on the links of cell c into solid cells:
//   f_opp(i)(x, t+1) = f*_i(x) - 2 w_i rho (c_i . u_w) / cs^2   (same for g with phi)
// f*_i is read back from the slot collide_cell() wrote it to and the result
// goes to the slot the cell reads direction opp(i) from next step: (x + c_i,
// i) after an even step, (x, opp(i)) after an odd one.  Only cells next to
// a solid take this path; keeping it after the branch-free main loop (rather
// than a branch per direction inside it) holds the register count down.
template <int Q, int S, int ODD, bool WITH_G = true, bool SR = false>
__device__ __forceinline__ void bounce_back(const Pops<Q, S> &P, const Nbr &N, long long c, uint32_t bits,
                                         const uint8_t *__restrict__ mask, const Geom &G, const Phys &ph,
                                         int x, int y, int z, float rho, float phi, uint32_t &rs) {
  using V = VSet<Q>;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (!((bits >> i) & 1u)) continue;
    const long long n = N.template at<V>(i);
    const int sp = ODD ? i : opp(i);
    const long long sc = ODD ? n : c;
    const float fs = P.ldfc(sp, sc), gs = WITH_G ? P.ldgc(sp, sc) : 0.0f;
    const int xs = wrap(x + V::cx(i), G.ex), ys = wrap(y + V::cy(i), G.ey);
    const int zs = V::D == 3 ? wrap(z + V::cz(i), G.ez) : z;
    float uw[3];
    body_velocity<V>(G, ph, mask[n], x, y, z, xs, ys, zs, i, uw);
    const float k = 6.0f * V::w(i) * (V::cx(i) * uw[0] + V::cy(i) * uw[1] + V::cz(i) * uw[2]);
    const float fb = P.template round_at<SR>(fs - k * rho, rs);
    const float gb = P.template round_at<SR>(gs - k * phi, rs);
    const int bp = ODD ? opp(i) : i;
    const long long bc = ODD ? c : n;
    P.stf(bp, bc, fb);
    if (WITH_G) P.stg(bp, bc, gb);
  }
}

// Collide and stream a cell.  With the by-product (FP32), every thread of
// the 64 x COLLIDE_ROWS block must call this (it holds a barrier); `active`
// marks threads on a storage cell.  After the barrier each thread forms the
// first pass of the moment groups of its column: S0 for this plane, UP for
// the plane above and DN for the plane below (all their sources lie in this
// plane), from the tile's post-collision values.
template <int Q, int S, int ODD, bool SR = false>
__device__ __forceinline__ void stage_collide(const LatView<Q, S> &L, int x, int y, int z, bool active) {
  using V = VSet<Q>;
  constexpr int NT = BX * COLLIDE_ROWS;
  const long long c = (long long)x + (long long)L.G.px * ((long long)y + (long long)L.G.ey * z);
  if (!ByProduct<S>::on) {
    if (!active) return;
    const uint32_t bits = nb_word<Q, S>(L, c);
    if (bits & NB_SELF_SOLID) return;
    const Nbr N(L.G, x, y, z);
    float rho, phi;
    float2 rest;
    uint32_t rs = SR ? sr_seed(c, L.P.step_key()) : 0u;
    collide_cell<Q, S, ODD, NT, SR>(L.P, N, c, L.C, L.ph, nullptr, 0, rho, phi, rest, rs);
    if (bits != 0u) bounce_back<Q, S, ODD, true, SR>(L.P, N, c, bits, L.mask, L.G, L.ph, x, y, z, rho, phi, rs);
    return;
  }
  __shared__ float post[2 * (Q - 1)][NT];
  __shared__ unsigned char live[NT];
  const int tid = threadIdx.y * BX + threadIdx.x;
  bool fluid = false;
  float2 rest = make_float2(0.0f, 0.0f);
  if (active) {
    const uint32_t bits = nb_word<Q, S>(L, c);
    fluid = !(bits & NB_SELF_SOLID);
    if (fluid) {
      const Nbr N(L.G, x, y, z);
      float rho, phi;
      uint32_t rs = 0u;
      collide_cell<Q, S, ODD, NT>(L.P, N, c, L.C, L.ph, post, tid, rho, phi, rest, rs);
      if (bits != 0u) bounce_back<Q, S, ODD>(L.P, N, c, bits, L.mask, L.G, L.ph, x, y, z, rho, phi, rs);
    }
  }
  live[tid] = fluid ? 1 : 0;
  __syncthreads();
  // XE entries of this row: lane e < NE stores entry e of side 0 (first
  // column), lane NE + e entry e of side 1 (last column), if that cell is fluid
  if (threadIdx.x < 2 * XEdge<V>::NE) {
    const int side = threadIdx.x >= XEdge<V>::NE ? 1 : 0, e = threadIdx.x - side * XEdge<V>::NE;
    const int xlo = x & ~(BX - 1), xs = side ? min(xlo + BX, L.G.ex) - 1 : xlo;
    const int st = threadIdx.y * BX + (xs - xlo);
    if (live[st]) {
      const int i = XEdge<V>::dir(side, e);
      L.XE[XEdge<V>::index(L.G, xs, y, z, side, e)] = make_float2(post[i - 1][st], post[Q - 1 + i - 1][st]);
    }
  }
  if (!active) return;
  float2 grp[3];
  grp[0] = grp[2] = make_float2(0.0f, 0.0f);
  // direction 0 first, added to zero as in the other paths (a solid cell's
  // sums are never read)
  grp[1] = make_float2(0.0f + rest.x, 0.0f + rest.y);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (!in_footprint(L.G, x, y, V::cx(i), V::cy(i))) continue;
    const int st = tid - V::cx(i) - BX * V::cy(i);
    if (!live[st]) continue;
    grp[V::cz(i) + 1].x += post[i - 1][st];
    grp[V::cz(i) + 1].y += post[Q - 1 + i - 1][st];
  }
  L.P0[c] = grp[1];
  if (V::D == 3) {
    const long long pl = (long long)L.G.px * L.G.ey;
    int zu = z + 1, zd = z - 1;
    if (zu == L.G.ez) zu = L.G.per[2] ? 0 : -1;
    if (zd < 0) zd = L.G.per[2] ? L.G.ez - 1 : -1;
    if (zu >= 0) L.PU[c + (zu - z) * pl] = grp[2];
    if (zd >= 0) L.PD[c + (zd - z) * pl] = grp[0];
  }
}

// ---------------------------------------------------------------------------
// Kernels over one lattice: one thread per storage cell (64 x 4 blocks), one
// thread per solid boundary cell for the fills.
// ---------------------------------------------------------------------------
// Stage ids; the first three double as indices of the launch shapes (the
// moments pass, k_moments or k_combine, shares shape 0).
enum Stage {
  ST_MOMENTS = SHAPE_MOMENTS, ST_POTENTIAL = SHAPE_POTENTIAL, ST_COLLIDE = SHAPE_COLLIDE, ST_COMBINE = 3,
  ST_PRE_MOMENTS = 4, ST_PRE_COLLIDE = 5  // consistent initialisation
};

// ---------------------------------------------------------------------------
// Consistent initialisation (Sec. 2.3, after Mei et al. 2006): pre-iterations
// of f in which the velocity of the equilibrium and of the Guo term is held
// at the prescribed u0 and phi at phi0 (both in AUX = (u0, phi0)), while
// rho = sum f evolves; g is not stepped.  The potential and force stages of
// the step are reused on M = (rho - 1, phi0).
// ---------------------------------------------------------------------------
template <int Q, int S, int ODD>
__device__ __forceinline__ void stage_pre_moments(const LatView<Q, S> &L, int x, int y, int z) {
  using V = VSet<Q>;
  const long long c = (long long)x + (long long)L.G.px * ((long long)y + (long long)L.G.ey * z);
  if (L.nbm[c] & NB_SELF_SOLID) return;
  const Nbr N(L.G, x, y, z);
  float drho = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) drho += (!ODD || i == 0) ? L.P.ldf(i, c) : L.P.ldf(opp(i), N.template back<V>(i));
  L.M[c] = make_float2(drho, L.AUX[c].w);
}

template <int Q, int S, int ODD>
__device__ __forceinline__ void stage_pre_collide(const LatView<Q, S> &L, int x, int y, int z) {
  using V = VSet<Q>;
  const long long c = (long long)x + (long long)L.G.px * ((long long)y + (long long)L.G.ey * z);
  const uint32_t bits = nb_word<Q, S>(L, c);
  if (bits & NB_SELF_SOLID) return;
  const Nbr N(L.G, x, y, z);
  const float4 cc = L.C[c];
  const float mu_phi = cc.w, mu_rho = coupling_mu_rho(cc);
  float F[3];
  force<Q>(L.C, N, mu_rho, mu_phi, F);
  float df[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) df[i] = (!ODD || i == 0) ? L.P.ldf(i, c) : L.P.ldf(opp(i), N.template back<V>(i));
  float drho = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) drho += df[i];
  const float rho = 1.0f + drho;
  const float4 a = L.AUX[c];
  const float u[3] = {a.x, a.y, a.z};
  const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const float uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float cu = V::cx(i) * u[0] + V::cy(i) * u[1] + V::cz(i) * u[2];
    const float cF = V::cx(i) * F[0] + V::cy(i) * F[1] + V::cz(i) * F[2];
    const float wi = V::w(i);
    const float poly = 3.0f * cu + 4.5f * cu * cu - 1.5f * uu;
    const float dfeq = wi * (drho + rho * poly);
    const float src = L.ph.guo * wi * (3.0f * (cF - uF) + 9.0f * cu * cF);
    const float fs = L.P.round(df[i] + L.ph.om_f * (dfeq - df[i]) + src);
    if (!ODD) L.P.stf(opp(i), c, fs);
    else L.P.stf(i, N.template at<V>(i), fs);
  }
  uint32_t rs = 0u;
  if (bits != 0u) bounce_back<Q, S, ODD, false>(L.P, N, c, bits, L.mask, L.G, L.ph, x, y, z, rho, 0.0f, rs);
}

// Per-cell stages other than collide (ODD: parity of the state they read).
template <int Q, int S, int STAGE, int ODD>
__device__ __forceinline__ void run_stage(const LatView<Q, S> &L, int x, int y, int z) {
  if constexpr (STAGE == ST_MOMENTS) stage_moments<Q, S, ODD>(L, x, y, z);
  else if constexpr (STAGE == ST_COMBINE) stage_combine<Q, S, ODD>(L, x, y, z);
  else if constexpr (STAGE == ST_PRE_MOMENTS) stage_pre_moments<Q, S, ODD>(L, x, y, z);
  else if constexpr (STAGE == ST_PRE_COLLIDE) stage_pre_collide<Q, S, ODD>(L, x, y, z);
  else stage_potential<Q, S>(L, x, y, z);
}

// The collide keeps the compiler's register choice (3 waves per SIMD for
// D3Q19): capped at 128 VGPRs (4 waves) it spills 52-56 bytes per lane in FP16
// storage and was measured 16% slower (186 against 160 us at 256x128x128).
template <int Q, int S, int STAGE, int ODD, bool SR = false>
__global__ __launch_bounds__(BX *MAX_ROWS) void k_cells(LatView<Q, S> L) {
  int x, y, z;
  long long c;
  const bool in = cell_of_tile(L.G, L.tm, x, y, z, c);
  if (STAGE == ST_COLLIDE) {
    stage_collide<Q, S, ODD, SR>(L, x, y, z, in);
    return;
  }
  if constexpr (S == 1 && STAGE == ST_MOMENTS) {
    // a step's moments pass runs before its collide, after the previous
    // collide: the counter the collide reads advances once per step
    if (L.tick && L.P.ctr && blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) L.P.ctr[0] += 1u;
  }
  if (in) run_stage<Q, S, STAGE, ODD>(L, x, y, z);
}

template <int Q, int S, int PI>
__global__ __launch_bounds__(256) void k_fill(LatView<Q, S> L) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L.n_fill) return;
  if (PI) stage_fill_c<Q, S>(L, L.fill[k]);
  else stage_fill_m<Q, S>(L, L.fill[k]);
}

// Potential of a single lattice with the moments staged through LDS: a block
// owns a 64 x blockDim.y column of cells over `tz` consecutive planes and
// keeps three planes of M (with a one-cell halo in x and y) in a ring, so
// each M value is read from memory about once per block instead of once per
// neighbour.  Same arithmetic as stage_potential.
constexpr int RING_W = BX + 2;
using PotRing = float2[3][MAX_ROWS + 2][RING_W];

// The potential of planes [z0, z1) of the 64 x blockDim.y column (bx, by);
// every thread of the block takes part (barriers), and the ring is free
// again on return.
template <int Q, int S>
__device__ __forceinline__ void potential_column(const LatView<Q, S> &L, PotRing &ring, int bx, int by, int z0,
                                                 int z1) {
  using V = VSet<Q>;
  constexpr int HW = RING_W;
  const Geom &G = L.G;
  const int rows = (int)blockDim.y;
  const int xlo = bx * BX, ylo = by * rows;
  const int w = min(BX, G.ex - xlo), h = min(rows, G.ey - ylo);  // cells of the tile on the lattice
  const int tid = threadIdx.y * BX + threadIdx.x, nth = BX * rows;
  const int hcells = (rows + 2) * HW;
  // plane zs (wrapped on a periodic axis, skipped outside a wall axis) into
  // ring slot `slot`; halo columns and rows beyond the tile's cells + 1 are
  // never read
  auto load_plane = [&](int zs, int slot) {
    int zz = zs;
    if (zz < 0 || zz >= G.ez) zz = G.per[2] ? wrap(zz, G.ez) : -1;
    for (int k = tid; k < hcells; k += nth) {
      const int hy = k / HW, hx = k - hy * HW;
      float2 v = make_float2(0.0f, 0.0f);
      if (zz >= 0 && hx <= w + 1 && hy <= h + 1) {
        int xg = xlo - 1 + hx, yg = ylo - 1 + hy;
        bool ok = true;
        if (xg < 0 || xg >= G.ex) { if (G.per[0]) xg = wrap(xg, G.ex); else ok = false; }
        if (yg < 0 || yg >= G.ey) { if (G.per[1]) yg = wrap(yg, G.ey); else ok = false; }
        if (ok) v = L.M[(long long)xg + (long long)G.px * ((long long)yg + (long long)G.ey * zz)];
      }
      ring[slot][hy][hx] = v;
    }
  };
  if (V::D == 3) load_plane(z0 - 1, 0);
  load_plane(z0, 1);
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int z = z0; z < z1; ++z) {
    const int sd = (z - z0) % 3, sc = (z - z0 + 1) % 3, su = (z - z0 + 2) % 3;
    if (V::D == 3) load_plane(z + 1, su);
    __syncthreads();
    if (tx < w && ty < h) {
      const long long c = (long long)(xlo + tx) + (long long)G.px * ((long long)(ylo + ty) + (long long)G.ey * z);
      if (!(nb_word<Q, S>(L, c) & NB_SELF_SOLID)) {
        const float2 m0 = ring[sc][ty + 1][tx + 1];
        float lr, lp;
        laplacians<Q>([&](int i) {
          const int sl = V::cz(i) < 0 ? sd : (V::cz(i) > 0 ? su : sc);
          return ring[sl][ty + 1 + V::cy(i)][tx + 1 + V::cx(i)];
        }, m0, lr, lp);
        store_potential<Q, S>(L, c, m0, lr, lp);
      }
    }
    __syncthreads();
  }
}

template <int Q, int S>
__global__ __launch_bounds__(BX *MAX_ROWS) void k_potential_zm(LatView<Q, S> L, int tz) {
  __shared__ PotRing ring;
  uint32_t ubx, ur;
  tile_of_block(L.tm, blockIdx.x, ubx, ur);
  const uint32_t uch = udiv(ur, L.tm.dgy);
  const int by = (int)(ur - uch * (uint32_t)L.tm.gy), z0 = (int)uch * tz;
  potential_column<Q, S>(L, ring, (int)ubx, by, z0, min(z0 + tz, L.G.ez));
}

// ---------------------------------------------------------------------------
// Batched persistent kernels: a fixed grid walks a device-side work list of
// (slot, block-x, block-y, z) items (or (slot, cell) fill items) for the
// lattices of one (velocity set, storage) class.  The list and its length
// live in device memory, so a captured graph stays valid while lattices join
// and leave the batch.
// ---------------------------------------------------------------------------
template <int Q, int S>
__device__ __forceinline__ LatView<Q, S> view_of(char *base, const Inst &I) {
  LatView<Q, S> L;
  L.P = pops_of<Q, S>(base + I.f, base + I.g, (float *)(base + I.g0));
  L.nbm = (const uint32_t *)(base + I.nbm); L.mask = (const uint8_t *)(base + I.mask);
  L.segf = (const uint8_t *)(base + I.segf);  // a work item is a 64-wide tile: one segment per wave
  L.M = (float2 *)(base + I.M); L.C = (float4 *)(base + I.C);
  L.P0 = (float2 *)(base + I.P0); L.PU = (float2 *)(base + I.PU); L.PD = (float2 *)(base + I.PD);
  L.XE = (float2 *)(base + I.XE);
  L.AUX = nullptr;
  L.G = I.G; L.ph = I.ph; L.fill = (const int *)(base + I.fill); L.n_fill = I.n_fill;
  L.tick = 0;
  return L;
}

template <int Q, int S, int STAGE, int ODD>
__global__ __launch_bounds__(BX *MAX_ROWS) void k_batch_cells(char *base, const Inst *__restrict__ inst, const int4 *__restrict__ work,
                                                        const int *__restrict__ range) {
  const int start = range[0], n = range[1];
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int4 it = work[start + w];
    const LatView<Q, S> L = view_of<Q, S>(base, inst[it.x]);
    const int x = it.y * BX + threadIdx.x, y = it.z * (int)blockDim.y + threadIdx.y, z = it.w;
    const bool in = x < L.G.ex && y < L.G.ey;
    if (STAGE == ST_COLLIDE) {
      stage_collide<Q, S, ODD>(L, x, y, z, in);
      if (ByProduct<S>::on) __syncthreads();  // the tile buffer is reused by the next item
    } else if (in) {
      run_stage<Q, S, STAGE, ODD>(L, x, y, z);
    }
  }
}

// The batch potential: z-marching columns (slot, block-x, block-y, first
// plane) of range[2] planes each, as k_potential_zm marches them.
template <int Q, int S>
__global__ __launch_bounds__(BX *MAX_ROWS) void k_batch_potential(char *base, const Inst *__restrict__ inst,
                                                               const int4 *__restrict__ cols,
                                                               const int *__restrict__ range) {
  __shared__ PotRing ring;
  const int start = range[0], n = range[1], tz = range[2];
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int4 it = cols[start + w];
    const LatView<Q, S> L = view_of<Q, S>(base, inst[it.x]);
    potential_column<Q, S>(L, ring, it.y, it.z, it.w, min(it.w + tz, L.G.ez));
  }
}

template <int Q, int S, int PI>
__global__ __launch_bounds__(256) void k_batch_fill(char *base, const Inst *__restrict__ inst, const int2 *__restrict__ work,
                                                    const int *__restrict__ range) {
  const int start = range[0], n = range[1];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int2 it = work[start + k];
    const LatView<Q, S> L = view_of<Q, S>(base, inst[it.x]);
    if (PI) stage_fill_c<Q, S>(L, it.y);
    else stage_fill_m<Q, S>(L, it.y);
  }
}

// Initialisation at equilibrium (Sec. 2.3).  M holds (rho0 - 1, phi0) with
// solid cells filled; U0 holds u0.  Writes the parity-0 layout.
template <int Q, int S>
__global__ __launch_bounds__(BX *BY) void k_init(Pops<Q, S> P, const uint32_t *__restrict__ nbm,
                                                 const float2 *__restrict__ M,
                                                 const float4 *__restrict__ U0, Geom G, Phys ph) {
  using V = VSet<Q>;
  int x, y, z;
  long long c;
  if (!cell_of_thread(G, x, y, z, c)) return;
  if (nbm[c] & NB_SELF_SOLID) return;
  const Nbr N(G, x, y, z);
  float2 m0 = M[c];
  float lr, lp, mr, mp;
  laplacians<Q>([&](int i) { return M[N.template at<V>(i)]; }, m0, lr, lp);
  chem_pot(ph, m0.x, m0.y, lr, lp, mr, mp);
  float4 u4 = U0[c];
  float u[3] = {u4.x, u4.y, u4.z};
  float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  float drho = m0.x, rho = 1.0f + drho, phi = m0.y;
  float rest = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    float cu = V::cx(i) * u[0] + V::cy(i) * u[1] + V::cz(i) * u[2];
    float poly = 3.0f * cu + 4.5f * cu * cu - 1.5f * uu;
    P.stf(i, c, V::w(i) * (drho + rho * poly));
    if (i > 0) {
      float geq = V::w(i) * (ph.gam3 * mp + phi * poly);
      rest += geq;
      P.stg(i, c, geq);
    }
  }
  P.stg(0, c, phi - rest);
}

// g at its equilibrium g^eq(phi0, mu_phi, u0) (eq. geq; g_0 by complement),
// parity-0 slots, with AUX = (u0, phi0) and C (mu_phi in C.w) current.
template <int Q, int S>
__global__ __launch_bounds__(BX *BY) void k_reinit_g(Pops<Q, S> P, const uint32_t *__restrict__ nbm,
                                                     const float4 *__restrict__ C,
                                                     const float4 *__restrict__ AUX, Geom G, Phys ph) {
  using V = VSet<Q>;
  int x, y, z;
  long long c;
  if (!cell_of_thread(G, x, y, z, c)) return;
  if (nbm[c] & NB_SELF_SOLID) return;
  const float4 a = AUX[c];
  const float u[3] = {a.x, a.y, a.z};
  const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const float phi = a.w, mp = C[c].w;
  float rest = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const float cu = V::cx(i) * u[0] + V::cy(i) * u[1] + V::cz(i) * u[2];
    const float poly = 3.0f * cu + 4.5f * cu * cu - 1.5f * uu;
    const float geq = V::w(i) * (ph.gam3 * mp + phi * poly);
    rest += geq;
    P.stg(i, c, geq);
  }
  P.stg(0, c, phi - rest);
  if constexpr (S == 0) P.stg0lo(c, 0.0f);
}

// Observables (u with F/2, bulk pressure) at the current time; M and C must
// be current.  OUT[c] = (ux, uy, uz, P).
template <int Q, int S>
__global__ __launch_bounds__(BX *BY) void k_observe(Pops<Q, S> P, const uint32_t *__restrict__ nbm,
                                                    const float4 *__restrict__ C,
                                                    float4 *__restrict__ OUT, Geom G, Phys ph, int odd) {
  using V = VSet<Q>;
  int x, y, z;
  long long c;
  if (!cell_of_thread(G, x, y, z, c)) return;
  if (nbm[c] & NB_SELF_SOLID) {
    OUT[c] = make_float4(0, 0, 0, 0);
    return;
  }
  const Nbr N(G, x, y, z);
  float df[Q], g[Q];
  load_pops<Q, S>(P, N, c, odd, df, g);
  float j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    j[0] += V::cx(i) * df[i];
    j[1] += V::cy(i) * df[i];
    j[2] += V::cz(i) * df[i];
  }
  const float4 m0 = C[c];
  float F[3];
  force<Q>(C, N, coupling_mu_rho(m0), m0.w, F);
  const float rho = 1.0f + m0.x;
  const float inv = 1.0f / rho;
  // P = cs^2 rho + rho mu_rho + phi mu_phi - psi_b, with Pi = rho mu_rho + phi mu_phi
  const float pres = rho / 3.0f + m0.z - psi_bulk(ph, rho, m0.y);
  OUT[c] = make_float4((j[0] + 0.5f * F[0]) * inv, (j[1] + 0.5f * F[1]) * inv,
                       (j[2] + 0.5f * F[2]) * inv, pres);
}

// Unshifted populations of the storage cells [c0, c0 + n), as [2q + 1][n]
// floats: f_i + w_i, g_i, then the low part of g_0 (FP32 storage; zero with
// FP16 storage).  Solid cells read 0.
template <int Q, int S>
__global__ __launch_bounds__(256) void k_read_pops(Pops<Q, S> P, const uint32_t *__restrict__ nbm,
                                                   float *__restrict__ out, Geom G, int odd, long long c0,
                                                   int n) {
  using V = VSet<Q>;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const long long c = c0 + t;
  if (nbm[c] & NB_SELF_SOLID) {
    for (int i = 0; i <= 2 * Q; ++i) out[(long long)i * n + t] = 0.0f;
    return;
  }
  int x, y, z;
  x = (int)(c % G.px);
  const long long r = c / G.px;
  y = (int)(r % G.ey);
  z = (int)(r / G.ey);
  const Nbr N(G, x, y, z);
  float df[Q], g[Q];
  load_pops<Q, S>(P, N, c, odd, df, g);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    out[(long long)i * n + t] = df[i] + V::w(i);
    out[(long long)(Q + i) * n + t] = g[i];
  }
  float lo = 0.0f;
  if constexpr (S == 0) lo = P.ldg0lo(c);
  out[(long long)2 * Q * n + t] = lo;
}

// Global sums over fluid cells: compensated FP32 per thread, FP64 across the
// block; one partial per block (summed on the host in FP64).
// part[b*8 + k]: k = 0 sum(rho-1), 1 sum phi, 2 sum |phi|, 3..5 sum rho u,
// 6 non-finite count, 7 fluid count.
__device__ __forceinline__ void kahan(float &s, float &comp, float v) {
  float y = v - comp;
  float t = s + y;
  comp = (t - s) - y;
  s = t;
}

__global__ __launch_bounds__(256) void k_reduce(const float4 *__restrict__ C, const float4 *__restrict__ OUT,
                                                const uint32_t *__restrict__ nbm, long long ncell,
                                                double *__restrict__ part) {
  float s[6] = {0, 0, 0, 0, 0, 0}, e[6] = {0, 0, 0, 0, 0, 0};
  unsigned bad = 0, nfl = 0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
       c += (long long)gridDim.x * blockDim.x) {
    if (nbm[c] & NB_SELF_SOLID) continue;
    float4 m = C[c];
    float4 o = OUT[c];
    float rho = 1.0f + m.x;
    float v[6] = {m.x, m.y, fabsf(m.y), rho * o.x, rho * o.y, rho * o.z};
    bool fin = isfinite(m.x) && isfinite(m.y) && isfinite(o.x) && isfinite(o.y) && isfinite(o.z);
    bad += fin ? 0u : 1u;
    ++nfl;
    if (fin)
#pragma unroll
      for (int k = 0; k < 6; ++k) kahan(s[k], e[k], v[k]);
  }
  __shared__ double red[8][256];
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = (double)s[k] - (double)e[k];
  red[6][threadIdx.x] = (double)bad;
  red[7][threadIdx.x] = (double)nfl;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 8; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 8; ++k) part[blockIdx.x * 8 + k] = red[k][0];
}

// Sums the nb block partials of k_reduce, for each of the 8 quantities in
// block order (the order fre_reduce sums them on the host), into total[8].
__global__ __launch_bounds__(64) void k_reduce_final(const double *__restrict__ part, int nb,
                                                     double *__restrict__ total) {
  const int k = threadIdx.x;
  if (k >= 8) return;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) acc += part[b * 8 + k];
  total[k] = acc;
}

// ---------------------------------------------------------------------------
// Ternary lattices (Sec. 2.2, Remark after the mobility relation): a third
// order parameter psi with its own population h, FP32 storage, one thread
// per cell in each pass.  A step is k3_moments, k3_fill (M), k3_potential,
// k3_fill (Pi), k3_collide; the arithmetic follows the binary stages, with
// the potentials of chem_pot3 and the force
//   mu_rho grad rho + mu_phi grad phi + mu_psi grad psi - grad Pi,
//   Pi = rho mu_rho + phi mu_phi + psi mu_psi,
// the product-rule form of -rho grad mu_rho - phi grad mu_phi - psi grad mu_psi.
// h_0 and g_0 are carried as hi + lo like g_0 of the binary FP32 state.
// ---------------------------------------------------------------------------
template <int Q> struct T3View {
  float *f, *g, *h;
  __half *g0l, *h0l;
  const uint32_t *nbm;
  const uint8_t *mask;
  float4 *M4;   // (rho - 1, phi, psi, 0)
  float4 *C4;   // (rho - 1, phi, psi, Pi)
  float2 *CM;   // (mu_phi, mu_psi)
  float4 *AUX;  // u0 at init; (u, P) after observe
  Geom G;
  Phys ph;
  const int *fill;
  int n_fill;
  TileMap tm;  // block order of k3_moments and k3_collide (64 x 4 tiles)
  // NT: non-temporal load, for passes that read each population once and
  // nothing else of the cell again
  template <bool NT = false>
  __device__ float ld(const float *a, int i, long long c) const { return ld_at<float, NT>(a, blk_offset<4>(Q, i, c)); }
  __device__ void st(float *a, int i, long long c, float v) const { st_at(a, blk_offset<4>(Q, i, c), v); }
};

// population i of fluid cell c at parity `odd` (AA pattern, as load_pops)
template <int Q, bool NT = false>
__device__ __forceinline__ float ld3(const T3View<Q> &T, const float *a, const Nbr &N, long long c, int odd, int i) {
  using V = VSet<Q>;
  return (!odd || i == 0) ? T.template ld<NT>(a, i, c) : T.template ld<NT>(a, opp(i), N.template back<V>(i));
}

template <int Q>
__global__ __launch_bounds__(BX *BY) void k3_moments(T3View<Q> T, int odd) {
  int x, y, z;
  long long c;
  if (!cell_of_tile(T.G, T.tm, x, y, z, c)) return;
  if (T.nbm[c] & NB_SELF_SOLID) return;
  const Nbr N(T.G, x, y, z);
  float dr = 0.0f, ph = 0.0f, ps = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    dr += ld3<Q, true>(T, T.f, N, c, odd, i);
    ph += ld3<Q, true>(T, T.g, N, c, odd, i);
    ps += ld3<Q, true>(T, T.h, N, c, odd, i);
  }
  T.M4[c] = make_float4(dr, ph, ps, 0.0f);
}

// solid cells next to fluid: (rho - 1, phi, psi) into M4 (PI = 0), or Pi into
// C4 with (rho - 1, phi, psi) copied from M4 (PI = 1); the lattice-weighted
// mean over fluid neighbours (reading R5)
template <int Q, int PI>
__global__ __launch_bounds__(256) void k3_fill(T3View<Q> T) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T.n_fill) return;
  const int s = T.fill[k];
  int x, y, z;
  cell_coords(T.G, s, x, y, z);
  if (PI) {
    float pi;
    fluid_mean<Q, 1, 4>((const float *)T.C4 + 3, T.nbm[s], T.G, x, y, z, &pi);
    const float4 m = T.M4[s];
    T.C4[s] = make_float4(m.x, m.y, m.z, pi);
  } else {
    float v[3];
    fluid_mean<Q, 3, 4>((const float *)T.M4, T.nbm[s], T.G, x, y, z, v);
    T.M4[s] = make_float4(v[0], v[1], v[2], 0.0f);
  }
}

template <int Q>
__device__ __forceinline__ void t3_potential_at(const T3View<Q> &T, const Nbr &N, long long c) {
  using V = VSet<Q>;
  const float4 m0 = T.M4[c];
  float ar = 0.0f, ap = 0.0f, aq = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const float4 m = T.M4[N.template at<V>(i)];
    ar += V::w(i) * (m.x - m0.x);
    ap += V::w(i) * (m.y - m0.y);
    aq += V::w(i) * (m.z - m0.z);
  }
  float mr, mp, mq;
  chem_pot3(T.ph, m0.x, m0.y, m0.z, 6.0f * ar, 6.0f * ap, 6.0f * aq, mr, mp, mq);
  T.C4[c] = make_float4(m0.x, m0.y, m0.z, (1.0f + m0.x) * mr + m0.y * mp + m0.z * mq);
  T.CM[c] = make_float2(mp, mq);
}

template <int Q>
__global__ __launch_bounds__(BX *BY) void k3_potential(T3View<Q> T) {
  int x, y, z;
  long long c;
  if (!cell_of_thread(T.G, x, y, z, c)) return;
  if (T.nbm[c] & NB_SELF_SOLID) return;
  t3_potential_at<Q>(T, Nbr(T.G, x, y, z), c);
}

// force and mu_rho of a fluid cell from C4, CM
template <int Q>
__device__ __forceinline__ void t3_force(const T3View<Q> &T, const Nbr &N, long long c, float F[3], float &mu_phi,
                                         float &mu_psi) {
  using V = VSet<Q>;
  const float4 cc = T.C4[c];
  const float2 cm = T.CM[c];
  mu_phi = cm.x;
  mu_psi = cm.y;
  const float mu_rho = (cc.w - cc.y * cm.x - cc.z * cm.y) / (1.0f + cc.x);
  float gr[3] = {0, 0, 0}, gp[3] = {0, 0, 0}, gq[3] = {0, 0, 0}, gw[3] = {0, 0, 0};
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const float4 m = T.C4[N.template at<V>(i)];
    const float w = 3.0f * V::w(i);
    const int cv[3] = {V::cx(i), V::cy(i), V::cz(i)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (!cv[a]) continue;
      gr[a] += cv[a] * w * m.x;
      gp[a] += cv[a] * w * m.y;
      gq[a] += cv[a] * w * m.z;
      gw[a] += cv[a] * w * m.w;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) F[a] = mu_rho * gr[a] + mu_phi * gp[a] + mu_psi * gq[a] - gw[a];
}

// collision of one Cahn-Hilliard population (g or h) of a fluid cell with
// order parameter value X, potential mu and 3 Gamma = gam3, relaxing at om;
// rest population as hi + lo; streamed in place (AA parity ODD)
template <int Q, int ODD>
__device__ __forceinline__ float t3_collide_ch(const T3View<Q> &T, float *a, __half *lo, const Nbr &N, long long c,
                                               const float m[3], float inv_rho, float mmr, float mu, float gam3,
                                               float om) {
  using V = VSet<Q>;
  float v[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) v[i] = ld3<Q>(T, a, N, c, ODD, i);
  float gm = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) gm += v[i];
  const float X = v[0] + gm;
  float rest = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const float cmi = V::cx(i) * m[0] + V::cy(i) * m[1] + V::cz(i) * m[2];
    const float cu = cmi * inv_rho;
    const float eq = V::w(i) * gam3 * mu + X * (V::a(i) * cu + V::w(i) * ((4.5f * cmi * cu - 1.5f * mmr) * inv_rho));
    rest += eq;
    const float s = v[i] + om * (eq - v[i]);
    if (!ODD) T.st(a, opp(i), c, s);
    else T.st(a, i, N.template at<V>(i), s);
  }
  const float t = om * (gm - rest) + __half2float(lo[c]) * 0x1p-24f;
  const float r0 = v[0] + t;
  const float tb = r0 - v[0];
  lo[c] = __float2half_rn(((v[0] - (r0 - tb)) + (t - tb)) * 0x1p24f);
  T.st(a, 0, c, r0);
  return X;
}

template <int Q, int ODD>
__global__ __launch_bounds__(BX *BY) void k3_collide(T3View<Q> T) {
  using V = VSet<Q>;
  int x, y, z;
  long long c;
  if (!cell_of_tile(T.G, T.tm, x, y, z, c)) return;
  const uint32_t bits = T.nbm[c];
  if (bits & NB_SELF_SOLID) return;
  const Nbr N(T.G, x, y, z);
  float F[3], mu_phi, mu_psi;
  t3_force<Q>(T, N, c, F, mu_phi, mu_psi);
  // f: BGK with the Guo term, first moments exact as in collide_cell
  float df[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) df[i] = ld3<Q>(T, T.f, N, c, ODD, i);
  float drho = 0.0f, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += df[i];
    j[0] += V::cx(i) * df[i];
    j[1] += V::cy(i) * df[i];
    j[2] += V::cz(i) * df[i];
  }
  const float rho = 1.0f + drho, inv_rho = 1.0f / rho;
  const float m[3] = {j[0] + 0.5f * F[0], j[1] + 0.5f * F[1], j[2] + 0.5f * F[2]};
  const float mmr = (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) * inv_rho;
  const float uF = (m[0] * F[0] + m[1] * F[1] + m[2] * F[2]) * inv_rho;
  const double drho_d = (double)drho;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float cF = V::cx(i) * F[0] + V::cy(i) * F[1] + V::cz(i) * F[2];
    const float cm = V::cx(i) * m[0] + V::cy(i) * m[1] + V::cz(i) * m[2];
    const float cu = cm * inv_rho;
    const float wi = V::w(i), ai = V::a(i);
    const float dfeq = feq_shifted(wi, ai, drho_d, cm, wi * (4.5f * cm * cu - 1.5f * mmr));
    const float src = T.ph.guo * (ai * cF - 3.0f * wi * uF + 3.0f * ai * cu * cF);
    const float fs = df[i] + T.ph.om_f * (dfeq - df[i]) + src;
    if (!ODD || i == 0) T.st(T.f, i == 0 ? 0 : opp(i), c, fs);
    else T.st(T.f, i, N.template at<V>(i), fs);
  }
  const float phi = t3_collide_ch<Q, ODD>(T, T.g, T.g0l, N, c, m, inv_rho, mmr, mu_phi, T.ph.gam3, T.ph.om_g);
  const float psi = t3_collide_ch<Q, ODD>(T, T.h, T.h0l, N, c, m, inv_rho, mmr, mu_psi, T.ph.gam3h, T.ph.om_h);
  if (!bits) return;
  // moving halfway bounce-back, as bounce_back() for each population
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (!((bits >> i) & 1u)) continue;
    const long long n = N.template at<V>(i);
    const int sp = ODD ? i : opp(i);
    const long long sc = ODD ? n : c;
    const int xs = wrap(x + V::cx(i), T.G.ex), ys = wrap(y + V::cy(i), T.G.ey);
    const int zs = V::D == 3 ? wrap(z + V::cz(i), T.G.ez) : z;
    float uw[3];
    body_velocity<V>(T.G, T.ph, T.mask[n], x, y, z, xs, ys, zs, i, uw);
    const float k = 6.0f * V::w(i) * (V::cx(i) * uw[0] + V::cy(i) * uw[1] + V::cz(i) * uw[2]);
    const int bp = ODD ? opp(i) : i;
    const long long bc = ODD ? c : n;
    T.st(T.f, bp, bc, T.ld(T.f, sp, sc) - k * rho);
    T.st(T.g, bp, bc, T.ld(T.g, sp, sc) - k * phi);
    T.st(T.h, bp, bc, T.ld(T.h, sp, sc) - k * psi);
  }
}

// equilibrium initialisation from M4 (filled) and u0 in AUX
template <int Q>
__global__ __launch_bounds__(BX *BY) void k3_init(T3View<Q> T) {
  using V = VSet<Q>;
  int x, y, z;
  long long c;
  if (!cell_of_thread(T.G, x, y, z, c)) return;
  if (T.nbm[c] & NB_SELF_SOLID) return;
  const Nbr N(T.G, x, y, z);
  t3_potential_at<Q>(T, N, c);
  const float4 m0 = T.M4[c];
  const float2 mu = T.CM[c];
  const float4 u4 = T.AUX[c];
  const float u[3] = {u4.x, u4.y, u4.z};
  const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const float rho = 1.0f + m0.x;
  float rg = 0.0f, rh = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float cu = V::cx(i) * u[0] + V::cy(i) * u[1] + V::cz(i) * u[2];
    const float poly = 3.0f * cu + 4.5f * cu * cu - 1.5f * uu;
    T.st(T.f, i, c, V::w(i) * (m0.x + rho * poly));
    if (i > 0) {
      const float ge = V::w(i) * (T.ph.gam3 * mu.x + m0.y * poly);
      const float he = V::w(i) * (T.ph.gam3h * mu.y + m0.z * poly);
      rg += ge;
      rh += he;
      T.st(T.g, i, c, ge);
      T.st(T.h, i, c, he);
    }
  }
  T.st(T.g, 0, c, m0.y - rg);
  T.st(T.h, 0, c, m0.z - rh);
}

// observables (u with F/2, bulk pressure) into AUX; C4, CM current
template <int Q>
__global__ __launch_bounds__(BX *BY) void k3_observe(T3View<Q> T, int odd) {
  using V = VSet<Q>;
  int x, y, z;
  long long c;
  if (!cell_of_thread(T.G, x, y, z, c)) return;
  if (T.nbm[c] & NB_SELF_SOLID) {
    T.AUX[c] = make_float4(0, 0, 0, 0);
    return;
  }
  const Nbr N(T.G, x, y, z);
  float F[3], mp, mq;
  t3_force<Q>(T, N, c, F, mp, mq);
  float j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float v = ld3<Q>(T, T.f, N, c, odd, i);
    j[0] += V::cx(i) * v;
    j[1] += V::cy(i) * v;
    j[2] += V::cz(i) * v;
  }
  const float4 cc = T.C4[c];
  const float rho = 1.0f + cc.x, inv = 1.0f / rho;
  const float pres = rho / 3.0f + cc.w - psi_bulk3(T.ph, rho, cc.y, cc.z);
  T.AUX[c] = make_float4((j[0] + 0.5f * F[0]) * inv, (j[1] + 0.5f * F[1]) * inv, (j[2] + 0.5f * F[2]) * inv, pres);
}

// populations of the storage cells [c0, c0 + n) as [3q + 2][n] floats: f_i +
// w_i, g_i, h_i, then the low parts of g_0 and h_0; solid cells read 0
template <int Q>
__global__ __launch_bounds__(256) void k3_read_pops(T3View<Q> T, int odd, float *__restrict__ out, long long c0,
                                                    int n) {
  using V = VSet<Q>;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const long long c = c0 + t;
  if (T.nbm[c] & NB_SELF_SOLID) {
    for (int i = 0; i < 3 * Q + 2; ++i) out[(long long)i * n + t] = 0.0f;
    return;
  }
  const int x = (int)(c % T.G.px);
  const long long r = c / T.G.px;
  const Nbr N(T.G, x, (int)(r % T.G.ey), (int)(r / T.G.ey));
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    out[(long long)i * n + t] = ld3<Q>(T, T.f, N, c, odd, i) + V::w(i);
    out[(long long)(Q + i) * n + t] = ld3<Q>(T, T.g, N, c, odd, i);
    out[(long long)(2 * Q + i) * n + t] = ld3<Q>(T, T.h, N, c, odd, i);
  }
  out[(long long)3 * Q * n + t] = __half2float(T.g0l[c]) * 0x1p-24f;
  out[(long long)(3 * Q + 1) * n + t] = __half2float(T.h0l[c]) * 0x1p-24f;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static dim3 cell_grid(const Geom &G) { return dim3((G.ex + BX - 1) / BX, (G.ey + BY - 1) / BY, G.ez); }
static dim3 cell_block() { return dim3(BX, BY, 1); }
static dim3 tile_grid(const Geom &G, int rows) {
  return dim3((unsigned)(((G.ex + BX - 1) / BX) * ((G.ey + rows - 1) / rows) * G.ez));
}
static int fill_blocks(int n) { return (n + 255) / 256; }

template <int Q, int S>
static LatView<Q, S> view_of_args(const LaunchArgs &a) {
  LatView<Q, S> L;
  L.P = make_pops<Q, S>(a);
  L.nbm = a.nbm; L.segf = a.segf; L.mask = a.mask; L.M = a.M; L.C = a.C;
  L.P0 = a.P0; L.PU = a.PU; L.PD = a.PD; L.XE = a.XE; L.AUX = a.AUX;
  L.G = a.G; L.ph = a.ph; L.fill = a.fill_list; L.n_fill = a.n_fill;
  L.tick = 0;
  return L;
}

// Launch of a cell stage with its shape (the moments pass -- k_moments or
// k_combine -- uses shape 0; with the by-product the collide tile always has
// COLLIDE_ROWS rows and only its block order varies).
template <int Q, int S, int STAGE>
static void cells_launch(const LaunchArgs &a, int odd, int tick = 0) {
  LatView<Q, S> L = view_of_args<Q, S>(a);
  L.tick = tick;
  const Shape sh = a.shape[STAGE <= ST_COLLIDE ? STAGE : SHAPE_MOMENTS];
  const int rows = (STAGE == ST_COLLIDE && ByProduct<S>::on) ? COLLIDE_ROWS : sh.rows;
  const dim3 grid = tile_grid(a.G, rows), block(BX, rows, 1);
  L.tm = TileMap(a.G.ex, a.G.ey, rows, (int)grid.x, sh.xcd);
  if constexpr (S == 1 && STAGE == ST_COLLIDE) {
    if (a.ctr) {  // stochastic rounding
      if (odd) k_cells<Q, S, STAGE, 1, true><<<grid, block, 0, a.stream>>>(L);
      else k_cells<Q, S, STAGE, 0, true><<<grid, block, 0, a.stream>>>(L);
      return;
    }
  }
  if (odd) k_cells<Q, S, STAGE, 1><<<grid, block, 0, a.stream>>>(L);
  else k_cells<Q, S, STAGE, 0><<<grid, block, 0, a.stream>>>(L);
}

template <int Q, int S, int PI>
static void fill_launch(const LaunchArgs &a) {
  if (a.n_fill) k_fill<Q, S, PI><<<fill_blocks(a.n_fill), 256, 0, a.stream>>>(view_of_args<Q, S>(a));
}

template <int Q, int S>
static void moments_launch(const LaunchArgs &a, int odd, int tick = 0) { cells_launch<Q, S, ST_MOMENTS>(a, odd, tick); }

// The z-marching potential: planes per block chosen so that the grid has
// about 2048 blocks (8 per CU).
template <int Q, int S>
static void potential_launch(const LaunchArgs &a) {
  LatView<Q, S> L = view_of_args<Q, S>(a);
  const Shape sh = a.shape[SHAPE_POTENTIAL];
  const int tiles = ((a.G.ex + BX - 1) / BX) * ((a.G.ey + sh.rows - 1) / sh.rows);
  int nch = (2048 + tiles - 1) / tiles;
  nch = nch < 1 ? 1 : (nch > a.G.ez ? a.G.ez : nch);
  const int tz = (a.G.ez + nch - 1) / nch;
  nch = (a.G.ez + tz - 1) / tz;
  L.tm = TileMap(a.G.ex, a.G.ey, sh.rows, tiles * nch, sh.xcd);
  k_potential_zm<Q, S><<<dim3((unsigned)(tiles * nch)), dim3(BX, sh.rows, 1), 0, a.stream>>>(L, tz);
}

// Coupling fields of the current state: solid fills of rho, phi, then
// mu_rho, mu_phi, Pi, then the solid fill of Pi.
template <int Q, int S>
static void couple_seq(const LaunchArgs &a, hipEvent_t *ev, int &k) {
  auto mark = [&]() { if (ev) (void)hipEventRecord(ev[k++], a.stream); };
  fill_launch<Q, S, 0>(a);
  mark();
  potential_launch<Q, S>(a);
  mark();
  fill_launch<Q, S, 1>(a);
  mark();
}

// One step from state parity `odd`.  Plain: moments, coupling fields,
// collide + stream.  By-product (M valid at entry): coupling fields, collide
// + stream with the first moment pass, second moment pass (M valid again).
// ev (if not null) receives an event before the first launch and after each.
template <int Q, int S>
static void step_seq(const LaunchArgs &a, int odd, hipEvent_t *ev) {
  int k = 0;
  if (ev) (void)hipEventRecord(ev[k++], a.stream);
  if (!ByProduct<S>::on) {
    moments_launch<Q, S>(a, odd, 1);  // the step's moments advance the rounding counter
    if (ev) (void)hipEventRecord(ev[k++], a.stream);
  }
  couple_seq<Q, S>(a, ev, k);
  cells_launch<Q, S, ST_COLLIDE>(a, odd);
  if (ev) (void)hipEventRecord(ev[k++], a.stream);
  if (ByProduct<S>::on) {
    cells_launch<Q, S, ST_COMBINE>(a, odd ^ 1);
    if (ev) (void)hipEventRecord(ev[k++], a.stream);
  }
}

template <int Q, int S> static void step_impl(const LaunchArgs &a, int odd) { step_seq<Q, S>(a, odd, nullptr); }
template <int Q, int S> static void step_events_impl(const LaunchArgs &a, int odd, hipEvent_t *ev) { step_seq<Q, S>(a, odd, ev); }


template <int Q, int S>
static void observe_impl(const LaunchArgs &a, int odd) {
  int k = 0;
  if (!ByProduct<S>::on) moments_launch<Q, S>(a, odd);  // by-product: M is valid
  couple_seq<Q, S>(a, nullptr, k);
  k_observe<Q, S><<<cell_grid(a.G), cell_block(), 0, a.stream>>>(make_pops<Q, S>(a), a.nbm, a.C, a.AUX, a.G, a.ph, odd);
}

template <int Q, int S>
static void init_impl(const LaunchArgs &a) {
  Pops<Q, S> P = make_pops<Q, S>(a);
  fill_launch<Q, S, 0>(a);
  k_init<Q, S><<<cell_grid(a.G), cell_block(), 0, a.stream>>>(P, a.nbm, a.M, a.AUX, a.G, a.ph);
  moments_launch<Q, S>(a, 0);  // M of the populations just set
}

template <int Q, int S>
static void consistent_init_impl(const LaunchArgs &a, long long n) {
  int k = 0;
  for (long long it = 0; it < n; ++it) {
    const int odd = (int)(it & 1);
    cells_launch<Q, S, ST_PRE_MOMENTS>(a, odd);
    couple_seq<Q, S>(a, nullptr, k);
    cells_launch<Q, S, ST_PRE_COLLIDE>(a, odd);
  }
  // mu_phi of the new rho with phi0, then g^eq(phi0, mu_phi, u0) and M
  cells_launch<Q, S, ST_PRE_MOMENTS>(a, 0);
  couple_seq<Q, S>(a, nullptr, k);
  k_reinit_g<Q, S><<<cell_grid(a.G), cell_block(), 0, a.stream>>>(make_pops<Q, S>(a), a.nbm, a.C, a.AUX, a.G, a.ph);
  moments_launch<Q, S>(a, 0);
}

template <int Q, int S>
static void read_pops_impl(const LaunchArgs &a, int odd, float *out, long long c0, int n) {
  k_read_pops<Q, S><<<(n + 255) / 256, 256, 0, a.stream>>>(make_pops<Q, S>(a), a.nbm, out, a.G, odd, c0, n);
}

#define FRE_DISPATCH(fn, ...)                                   \
  do {                                                          \
    if (a.q == 9 && a.storage == 0) fn<9, 0>(__VA_ARGS__);      \
    else if (a.q == 9) fn<9, 1>(__VA_ARGS__);                   \
    else if (a.storage == 0) fn<19, 0>(__VA_ARGS__);            \
    else fn<19, 1>(__VA_ARGS__);                                \
  } while (0)

void launch_step(const LaunchArgs &a, int odd) { FRE_DISPATCH(step_impl, a, odd); }
void launch_step_events(const LaunchArgs &a, int odd, hipEvent_t *ev) { FRE_DISPATCH(step_events_impl, a, odd, ev); }
int step_kernel_count() { return 5; }
template <int Q, int S> static void slots_impl(int *slot) {
  static const int plain[5] = {0, 1, 2, 3, 4}, bp[5] = {1, 2, 3, 4, 5};
  for (int k = 0; k < 5; ++k) slot[k] = ByProduct<S>::on ? bp[k] : plain[k];
}
int step_kernel_slots(const LaunchArgs &a, int *slot) {
  FRE_DISPATCH(slots_impl, slot);
  return 6;
}
const char *step_kernel_name(int k) {
  static const char *names[6] = {"k_moments", "k_fill_m", "k_potential", "k_fill_c", "k_collide", "k_combine"};
  return (k >= 0 && k < 6) ? names[k] : nullptr;
}
void launch_moments(const LaunchArgs &a, int odd) { FRE_DISPATCH(moments_launch, a, odd); }
void launch_consistent_init(const LaunchArgs &a, long long n) { FRE_DISPATCH(consistent_init_impl, a, n); }
bool uses_by_product(const LaunchArgs &a) { return a.storage == 0; }
void launch_observe(const LaunchArgs &a, int odd) { FRE_DISPATCH(observe_impl, a, odd); }
void launch_init(const LaunchArgs &a) { FRE_DISPATCH(init_impl, a); }
void launch_read_pops(const LaunchArgs &a, int odd, float *out, long long c0, int n) {
  FRE_DISPATCH(read_pops_impl, a, odd, out, c0, n);
}

// One batched step of one class: the same five stages over every lattice of
// the class listed in the work lists (ranges: cells [start, n], fills
// [start, n]).
template <int Q, int S>
static void batch_step_impl(const BatchArgs &b, int cls, int odd) {
  const int *rc = b.range + BATCH_RANGE * cls, *rf = rc + 2, *rp = rc + 4;
  const dim3 bl(BX, b.rows, 1);
  if (!ByProduct<S>::on) {
    if (odd) k_batch_cells<Q, S, ST_MOMENTS, 1><<<b.grid_cells, bl, 0, b.stream>>>(b.base, b.inst, b.work, rc);
    else k_batch_cells<Q, S, ST_MOMENTS, 0><<<b.grid_cells, bl, 0, b.stream>>>(b.base, b.inst, b.work, rc);
  }
  k_batch_fill<Q, S, 0><<<b.grid_fill, 256, 0, b.stream>>>(b.base, b.inst, b.fill, rf);
  k_batch_potential<Q, S><<<b.grid_cols, bl, 0, b.stream>>>(b.base, b.inst, b.cols, rp);
  k_batch_fill<Q, S, 1><<<b.grid_fill, 256, 0, b.stream>>>(b.base, b.inst, b.fill, rf);
  if (odd) k_batch_cells<Q, S, ST_COLLIDE, 1><<<b.grid_cells, bl, 0, b.stream>>>(b.base, b.inst, b.work, rc);
  else k_batch_cells<Q, S, ST_COLLIDE, 0><<<b.grid_cells, bl, 0, b.stream>>>(b.base, b.inst, b.work, rc);
  if (ByProduct<S>::on) {
    if (odd) k_batch_cells<Q, S, ST_COMBINE, 0><<<b.grid_cells, bl, 0, b.stream>>>(b.base, b.inst, b.work, rc);
    else k_batch_cells<Q, S, ST_COMBINE, 1><<<b.grid_cells, bl, 0, b.stream>>>(b.base, b.inst, b.work, rc);
  }
}

void launch_batch_step(const BatchArgs &b, int cls, int odd) {
  switch (cls) {
    case 0: batch_step_impl<9, 0>(b, cls, odd); break;
    case 1: batch_step_impl<9, 1>(b, cls, odd); break;
    case 2: batch_step_impl<19, 0>(b, cls, odd); break;
    default: batch_step_impl<19, 1>(b, cls, odd); break;
  }
}

void launch_reduce(const LaunchArgs &a, double *part) {
  k_reduce<<<reduce_blocks(), 256, 0, a.stream>>>(a.C, a.AUX, a.nbm, a.G.ncell, part);
}
void launch_reduce_total(const LaunchArgs &a, double *part, double *total) {
  launch_reduce(a, part);
  k_reduce_final<<<1, 64, 0, a.stream>>>(part, reduce_blocks(), total);
}

// ---------------------------------------------------------------------------
// ternary host launchers
// ---------------------------------------------------------------------------
template <int Q>
static T3View<Q> t3_view(const LaunchArgs &a) {
  T3View<Q> T;
  T.f = (float *)a.f; T.g = (float *)a.g; T.h = (float *)a.h;
  T.g0l = (__half *)a.g0; T.h0l = a.h0l;
  T.nbm = a.nbm; T.mask = a.mask;
  T.M4 = (float4 *)a.M; T.C4 = a.C; T.CM = a.CM; T.AUX = a.AUX;
  T.G = a.G; T.ph = a.ph; T.fill = a.fill_list; T.n_fill = a.n_fill;
  return T;
}

// the population passes over 64 x BY tiles in the XCD-aware block order
// of the binary cell kernels (a tile's x neighbours on the same XCD, so the
// cache lines that odd-parity streaming shares across a tile edge are
// fetched once)
template <int Q>
static dim3 t3_tiles(const LaunchArgs &a, T3View<Q> &T) {
  const dim3 grid = tile_grid(a.G, BY);
  T.tm = TileMap(a.G.ex, a.G.ey, BY, (int)grid.x, 1);
  return grid;
}

template <int Q>
static void t3_couple(const LaunchArgs &a, int odd) {
  T3View<Q> T = t3_view<Q>(a);
  const dim3 tiles = t3_tiles<Q>(a, T);
  k3_moments<Q><<<tiles, cell_block(), 0, a.stream>>>(T, odd);
  if (a.n_fill) k3_fill<Q, 0><<<fill_blocks(a.n_fill), 256, 0, a.stream>>>(T);
  k3_potential<Q><<<cell_grid(a.G), cell_block(), 0, a.stream>>>(T);
  if (a.n_fill) k3_fill<Q, 1><<<fill_blocks(a.n_fill), 256, 0, a.stream>>>(T);
}

template <int Q>
static void t3_step(const LaunchArgs &a, int odd) {
  t3_couple<Q>(a, odd);
  T3View<Q> T = t3_view<Q>(a);
  const dim3 tiles = t3_tiles<Q>(a, T);
  if (odd) k3_collide<Q, 1><<<tiles, cell_block(), 0, a.stream>>>(T);
  else k3_collide<Q, 0><<<tiles, cell_block(), 0, a.stream>>>(T);
}

void launch_step3(const LaunchArgs &a, int odd) {
  if (a.q == 9) t3_step<9>(a, odd);
  else t3_step<19>(a, odd);
}

void launch_observe3(const LaunchArgs &a, int odd) {
  if (a.q == 9) {
    t3_couple<9>(a, odd);
    k3_observe<9><<<cell_grid(a.G), cell_block(), 0, a.stream>>>(t3_view<9>(a), odd);
  } else {
    t3_couple<19>(a, odd);
    k3_observe<19><<<cell_grid(a.G), cell_block(), 0, a.stream>>>(t3_view<19>(a), odd);
  }
}

template <int Q>
static void t3_init(const LaunchArgs &a) {
  const T3View<Q> T = t3_view<Q>(a);
  if (a.n_fill) k3_fill<Q, 0><<<fill_blocks(a.n_fill), 256, 0, a.stream>>>(T);
  k3_init<Q><<<cell_grid(a.G), cell_block(), 0, a.stream>>>(T);
}

void launch_init3(const LaunchArgs &a) {
  if (a.q == 9) t3_init<9>(a);
  else t3_init<19>(a);
}

void launch_read_pops3(const LaunchArgs &a, int odd, float *out, long long c0, int n) {
  if (a.q == 9) k3_read_pops<9><<<(n + 255) / 256, 256, 0, a.stream>>>(t3_view<9>(a), odd, out, c0, n);
  else k3_read_pops<19><<<(n + 255) / 256, 256, 0, a.stream>>>(t3_view<19>(a), odd, out, c0, n);
}

}  // namespace frelbm
