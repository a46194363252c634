// kernels.h -- launch interface between the host library and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "lbm_device.h"

namespace frelbm {

// Launch shape of one cell kernel: rows of 64 cells per block (1, 2, 4 or
// 8) and whether blocks are placed in XCD-aware order.  The shape changes
// only which thread does which cell, never the arithmetic.
struct Shape {
  int rows;
  int xcd;
};
enum { SHAPE_MOMENTS = 0, SHAPE_POTENTIAL = 1, SHAPE_COLLIDE = 2, N_SHAPES = 3 };
constexpr int MAX_ROWS = 8;
// Rows of the collide tiles (64 x COLLIDE_ROWS cells) with FP32 storage: the
// tile is also the footprint over which collide sums next-step moments on
// chip, so it is fixed (another footprint would group the sums differently).
constexpr int COLLIDE_ROWS = 4;
inline bool shape_ok(const Shape &s) {
  return (s.rows == 1 || s.rows == 2 || s.rows == 4 || s.rows == 8) && (s.xcd == 0 || s.xcd == 1);
}

// Everything one launch sequence needs; all pointers are device pointers
// carved from the caller's buffer.
struct LaunchArgs {
  int q;        // 9 or 19
  int storage;  // 0 FP32, 1 FP16
  Geom G;
  Phys ph;
  void *f, *g;  // population blocks (float or half)
  float *g0;    // FP16 storage: g_0 plane; FP32 storage: the half plane of g_0's low part
  uint8_t *mask;
  uint32_t *nbm;  // per cell: non-fluid neighbour bits, NB_SELF_SOLID
  uint8_t *segf;  // per 64-cell row segment: 1 when every cell is fluid with fluid neighbours only
  uint32_t *ctr;  // FP16 storage with stochastic rounding: the step counter (else null)
  float2 *M;    // (rho - 1, phi)
  float4 *C;    // (rho - 1, phi, Pi = rho mu_rho + phi mu_phi, mu_phi)
  float2 *P0, *PU, *PD;  // FP32: first-pass moment sums by source plane (same, below, above)
  float2 *XE;   // FP32: post-collision (f, g) leaving each 64-cell row segment sideways
  float4 *AUX;  // u0 at init; (ux, uy, uz, P) after observe
  int *fill_list;
  int n_fill;
  Shape shape[N_SHAPES];
  hipStream_t stream;
  // ternary lattices (FP32): M holds (rho - 1, phi, psi, 0) as float4 and C
  // (rho - 1, phi, psi, Pi); h is the third population with the half plane
  // of h_0's low part, CM holds (mu_phi, mu_psi)
  int ternary;
  void *h;
  __half *h0l;
  float2 *CM;
};

template <int Q, int S> inline Pops<Q, S> make_pops(const LaunchArgs &a);
template <> inline Pops<9, 0> make_pops<9, 0>(const LaunchArgs &a) { return Pops<9, 0>{(float *)a.f, (float *)a.g, (__half *)a.g0}; }
template <> inline Pops<19, 0> make_pops<19, 0>(const LaunchArgs &a) { return Pops<19, 0>{(float *)a.f, (float *)a.g, (__half *)a.g0}; }
template <> inline Pops<9, 1> make_pops<9, 1>(const LaunchArgs &a) { return Pops<9, 1>{(__half *)a.f, (__half *)a.g, a.g0, a.ctr}; }
template <> inline Pops<19, 1> make_pops<19, 1>(const LaunchArgs &a) { return Pops<19, 1>{(__half *)a.f, (__half *)a.g, a.g0, a.ctr}; }

// Device view of one lattice for the kernels of one (velocity set, storage)
// class.
// n / d for 0 <= n < 2^31 and a divisor d >= 1 fixed at launch, as a
// multiply-high and a shift (Granlund and Montgomery, 1994): with
// s = ceil(log2 d) and m = floor(2^32 (2^s - d) / d) + 1, n / d equals
// (mulhi(n, m) + n) >> s.  The tile decode divides block indices, which are
// the same across a wave, so it runs on the scalar unit instead of as a
// per-lane reciprocal sequence.
struct UDiv {
  uint32_t d = 1, m = 1, s = 0;
  UDiv() = default;
  explicit UDiv(uint32_t dv) : d(dv) {
    while ((1ull << s) < dv) ++s;
    m = (uint32_t)(((1ull << 32) * ((1ull << s) - dv)) / dv + 1u);
  }
};

// Order of the 64 x rows tiles in a 1D grid of `blocks` blocks: gx tiles per
// row of tiles, gy rows of tiles per plane; with xcd set, the first `full`
// blocks follow the XCD-aware order (whole rounds of 8 rows of tiles).
struct TileMap {
  int gx = 1, gy = 1, xcd = 0, full = 0;
  UDiv dgx, dgy;
  TileMap() = default;
  TileMap(int ex, int ey, int rows, int blocks, int xcd_order)
      : gx((ex + 63) / 64), gy((ey + rows - 1) / rows), xcd(xcd_order),
        full(xcd_order ? blocks / (8 * gx) * (8 * gx) : 0), dgx((uint32_t)gx), dgy((uint32_t)gy) {}
};

template <int Q, int S> struct LatView {
  Pops<Q, S> P;
  const uint32_t *nbm;
  const uint8_t *segf;  // all-fluid segment flags, or null (then nbm is always read)
  const uint8_t *mask;
  float2 *M;
  float4 *C;
  float2 *P0, *PU, *PD;
  float2 *XE;
  const float4 *AUX;  // (u0, phi0) during the consistent initialisation
  Geom G;
  Phys ph;
  const int *fill;
  int n_fill;
  TileMap tm;  // block order of the single-lattice tile kernels
  int tick;    // the moments pass of a step advances the rounding step counter
};

// One slot of a batch, as stored in device memory.  Arrays are given as
// byte offsets from the batch's base pointer (a kernel argument), so the
// kernels address them as global memory, as they do kernel-argument pointers.
struct Inst {
  Geom G;
  Phys ph;
  long long f, g, g0, mask, nbm, segf, M, C, P0, PU, PD, XE, fill;
  int n_fill;
};

template <int Q, int S>
__host__ __device__ inline Pops<Q, S> pops_of(void *f, void *g, float *g0);
template <> __host__ __device__ inline Pops<9, 0> pops_of<9, 0>(void *f, void *g, float *g0) { return Pops<9, 0>{(float *)f, (float *)g, (__half *)g0}; }
template <> __host__ __device__ inline Pops<19, 0> pops_of<19, 0>(void *f, void *g, float *g0) { return Pops<19, 0>{(float *)f, (float *)g, (__half *)g0}; }
template <> __host__ __device__ inline Pops<9, 1> pops_of<9, 1>(void *f, void *g, float *g0) { return Pops<9, 1>{(__half *)f, (__half *)g, g0}; }
template <> __host__ __device__ inline Pops<19, 1> pops_of<19, 1>(void *f, void *g, float *g0) { return Pops<19, 1>{(__half *)f, (__half *)g, g0}; }

// Device tables of a batch.  range[BATCH_RANGE*cls + 0..1]: start and
// length of the class's cell work items; + 2..3: the same for fill items;
// + 4..5: the same for potential columns, + 6: planes per column.
constexpr int BATCH_RANGE = 8;
struct BatchArgs {
  char *base;  // origin of the Inst offsets
  const Inst *inst;
  const int4 *work;
  const int4 *cols;  // potential columns (slot, block-x, block-y, first plane)
  const int2 *fill;
  const int *range;
  int grid_cells, grid_fill;
  int grid_cols;  // potential columns: 8 blocks per CU (the LDS ring fits 10)
  int rows;  // rows of 64 cells per work item (and per block)
  hipStream_t stream;
};

// Batch classes: the (velocity set, storage) pairs.
constexpr int N_BATCH_CLASSES = 4;
inline int batch_class(int q, int storage) { return (q == 19 ? 2 : 0) + storage; }

void launch_batch_step(const BatchArgs &b, int cls, int odd);
void launch_step(const LaunchArgs &a, int odd);
// A step launches 5 kernels; ev receives an event before the first and after
// each.  The kernels are named by slot: step_kernel_name(0..5) = k_moments,
// k_fill_m, k_potential, k_fill_c, k_collide, k_combine; step_kernel_slots
// gives, for the lattice's class, the slot of each of its 5 launches.
void launch_step_events(const LaunchArgs &a, int odd, hipEvent_t *ev);
int step_kernel_count();
int step_kernel_slots(const LaunchArgs &a, int *slot);
const char *step_kernel_name(int k);
void launch_moments(const LaunchArgs &a, int odd);
bool uses_by_product(const LaunchArgs &a);
void launch_observe(const LaunchArgs &a, int odd);
void launch_init(const LaunchArgs &a);
// n (even) pre-iterations of f with u held at AUX.xyz and phi at AUX.w, then
// g reset to its equilibrium and M recomputed (consistent initialisation).
void launch_consistent_init(const LaunchArgs &a, long long n);
// Populations of the storage cells [c0, c0 + n) as [2q + 1][n] floats.
void launch_read_pops(const LaunchArgs &a, int odd, float *out, long long c0, int n);
// Ternary lattices: one step, the observables (into AUX; C, CM current), the
// equilibrium initialisation (M filled from host fields, AUX = u0) and the
// populations of storage cells [c0, c0 + n) as [3q + 2][n] floats.
void launch_step3(const LaunchArgs &a, int odd);
void launch_observe3(const LaunchArgs &a, int odd);
void launch_init3(const LaunchArgs &a);
void launch_read_pops3(const LaunchArgs &a, int odd, float *out, long long c0, int n);
// blocks (partials of 8 doubles) of the global reduction
constexpr int REDUCE_BLOCKS = 1024;
inline int reduce_blocks() { return REDUCE_BLOCKS; }
void launch_reduce(const LaunchArgs &a, double *part);
// launch_reduce, then the sum of the reduce_blocks() partials in block order
// into total[8] on the device.
void launch_reduce_total(const LaunchArgs &a, double *part, double *total);

}  // namespace frelbm
