// api.hip -- host side of the C ABI declared in include/frelbm.h.
//
// A lattice lives entirely in the caller's device buffer: population blocks
// (64 cells by direction), the cell mask and neighbour words, the moments
// (rho - 1, phi), the coupling values (rho - 1, phi, Pi, mu_phi), the FP32
// path's partial moment sums, an auxiliary float4 field, the list of solid
// cells next to fluid, and the reduction partials.  Steps are enqueued on the caller's stream; on a
// non-default stream runs of 16 steps, and pairs of steps (even + odd AA
// parity), are captured once into HIP graphs and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/frelbm.h"
#include "kernels.h"

using namespace frelbm;

namespace {

thread_local std::string g_err;

fre_status fail(fre_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
fre_status fail(fre_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(FRE_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Plan {
  int q;
  int ext[3];
  int per[3];
  int off[3];
  int px;          // row pitch: ext[0] rounded up to a multiple of 64
  long long ncell;  // px * ext[1] * ext[2]
  size_t o_f, o_g, o_g0, o_h, o_h0, o_ctr, o_mask, o_nbm, o_segf, o_M, o_C, o_CM, o_P0, o_PU, o_PD, o_XE, o_AUX, o_fill, o_part, total;
};

fre_status validate(const fre_params *p) {
  if (!p) return fail(FRE_EINVAL, "params is NULL");
  if (p->kind != FRE_D2Q9 && p->kind != FRE_D3Q19) return fail(FRE_EINVAL, "kind %d not D2Q9/D3Q19", p->kind);
  if (p->storage != FRE_FP32 && p->storage != FRE_FP16) return fail(FRE_EINVAL, "storage %d", p->storage);
  if (p->ternary != 0 && p->ternary != 1) return fail(FRE_EINVAL, "ternary must be 0 or 1 (got %d)", p->ternary);
  if (p->fp16_rounding != 0 && p->fp16_rounding != 1)
    return fail(FRE_EINVAL, "fp16_rounding must be 0 or 1 (got %d)", p->fp16_rounding);
  if (p->fp16_rounding && (p->storage != FRE_FP16 || p->ternary))
    return fail(FRE_EINVAL, "stochastic rounding (fp16_rounding = 1) needs FP16 storage of a binary lattice");
  if (p->ternary) {
    if (p->storage != FRE_FP32) return fail(FRE_EINVAL, "ternary lattices need FP32 storage");
    if (!(p->kappa3 > 0) || !std::isfinite(p->kappa3)) return fail(FRE_EINVAL, "kappa3 must be > 0");
    if (!(p->tau_h > 0.5) || !std::isfinite(p->tau_h)) return fail(FRE_EINVAL, "tau_h must exceed 1/2");
    if (!(p->M3 >= 0.0) || !std::isfinite(p->M3)) return fail(FRE_EINVAL, "mobility M3 must be >= 0");
  }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(FRE_EINVAL, "sizes must be >= 1");
  for (int a = 0; a < 3; ++a)
    if (p->bc[a] != FRE_PERIODIC && p->bc[a] != FRE_WALL) return fail(FRE_EINVAL, "bc[%d]=%d", a, p->bc[a]);
  if (p->kind == FRE_D2Q9 && (p->nz != 1 || p->bc[2] != FRE_PERIODIC))
    return fail(FRE_EINVAL, "D2Q9 needs nz = 1 and a periodic z axis");
  {
    // population arrays are addressed with 32-bit byte offsets
    const int q = p->kind == FRE_D2Q9 ? 9 : 19;
    const double px = std::ceil((p->nx + (p->bc[0] == FRE_WALL ? 2.0 : 0.0)) / 64.0) * 64.0;
    const double cells = px * (p->ny + (p->bc[1] == FRE_WALL ? 2.0 : 0.0)) * (p->nz + (p->bc[2] == FRE_WALL ? 2.0 : 0.0));
    const double bytes = cells * q * (p->storage == FRE_FP32 ? 4.0 : 2.0);
    if (bytes >= 4294967296.0 || cells >= 1073741824.0)
      return fail(FRE_EINVAL, "lattice too large: a population array would exceed 4 GiB (%.0f cells)", cells);
  }
  if (!(p->tau_f > 0.5) || !(p->tau_g > 0.5)) return fail(FRE_EINVAL, "tau_f, tau_g must exceed 1/2");
  if (!(p->M > 0.0) || !std::isfinite(p->M)) return fail(FRE_EINVAL, "mobility M must be > 0");
  if (p->use_paper_form) {
    if (!(p->kappa1 > 0) || !(p->kappa2 > 0) || !(p->alpha > 0))
      return fail(FRE_EINVAL, "kappa1, kappa2, alpha must be > 0");
  } else if (!(p->A > 0) || !(p->kappa > 0)) {
    return fail(FRE_EINVAL, "A and kappa must be > 0");
  }
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 2; ++s) {
      const double *u = p->wall_u[a][s];
      double m = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      if (!(m <= 0.1)) return fail(FRE_EINVAL, "wall speed %g exceeds 0.1 (Mach guard)", m);
    }
  if (p->n_rollers < 0 || p->n_rollers > 4) return fail(FRE_EINVAL, "n_rollers must be 0..4");
  for (int k = 0; k < p->n_rollers; ++k) {
    const fre_roller &r = p->rollers[k];
    if (r.axis < 0 || r.axis > 2) return fail(FRE_EINVAL, "roller %d axis", k);
    if (!std::isfinite(r.omega) || !(std::fabs(r.omega) * r.radius <= 0.1))
      return fail(FRE_EINVAL, "roller %d tip speed exceeds 0.1 (Mach guard)", k);
  }
  return FRE_OK;
}

Plan make_plan(const fre_params *p) {
  Plan P{};
  P.q = p->kind == FRE_D2Q9 ? 9 : 19;
  int n[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a) {
    P.per[a] = p->bc[a] == FRE_PERIODIC;
    P.off[a] = P.per[a] ? 0 : 1;
    P.ext[a] = n[a] + 2 * P.off[a];
  }
  P.px = (int)align_up((size_t)P.ext[0], 64);
  P.ncell = (long long)P.px * P.ext[1] * P.ext[2];  // a multiple of 64
  size_t es = p->storage == FRE_FP32 ? 4 : 2;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, kAlign); return at; };
  P.o_f = take((size_t)P.q * P.ncell * es);
  if (p->storage == FRE_FP32) {
    P.o_g = take((size_t)P.q * P.ncell * 4);
    // the low part of g_0, in half precision, scaled by 2^24
    P.o_g0 = take((size_t)P.ncell * 2);
  } else {
    // plane 0 of the half array is unused (g_0 lives in an FP32 plane), so
    // f and g share every block offset
    P.o_g = take((size_t)P.q * P.ncell * 2);
    P.o_g0 = take((size_t)P.ncell * 4);
  }
  const bool t3 = p->ternary != 0;
  if (t3) {
    // the third population and the low part of its rest population, inside
    // the population range (checkpoints carry them)
    P.o_h = take((size_t)P.q * P.ncell * 4);
    P.o_h0 = take((size_t)P.ncell * 2);
  }
  // the step counter of stochastic rounding, inside the population range
  // (checkpoints carry it)
  P.o_ctr = p->fp16_rounding ? take(256) : 0;
  P.o_mask = take((size_t)P.ncell);
  P.o_nbm = take((size_t)P.ncell * 4);
  P.o_segf = take((size_t)P.ncell / 64);
  P.o_M = take((size_t)P.ncell * (t3 ? 16 : 8));
  P.o_C = take((size_t)P.ncell * 16);
  P.o_CM = t3 ? take((size_t)P.ncell * 8) : 0;
  // FP32: first-pass moment sums of the collide (same plane; below and above
  // in 3D); the ternary step has no by-product moments
  const bool bp = p->storage == FRE_FP32 && !t3;
  P.o_P0 = bp ? take((size_t)P.ncell * 8) : 0;
  P.o_PU = bp && P.q == 19 ? take((size_t)P.ncell * 8) : 0;
  P.o_PD = bp && P.q == 19 ? take((size_t)P.ncell * 8) : 0;
  // FP32: per 64-cell row segment, the post-collision (f, g) of the
  // populations that leave it through its first and last column
  P.o_XE = bp ? take((size_t)(P.ncell / 64) * 2 * (P.q == 19 ? 5 : 3) * 8) : 0;
  P.o_AUX = take((size_t)P.ncell * 16);
  P.o_fill = take((size_t)P.ncell * 4);
  P.o_part = take((size_t)reduce_blocks() * 8 * sizeof(double));
  P.total = o;
  return P;
}

Phys make_phys(const fre_params *p) {
  Phys ph{};
  double k1, k2, al;
  if (p->use_paper_form) {
    k1 = p->kappa1; k2 = p->kappa2; al = p->alpha;
  } else {
    k1 = k2 = 4.0 * p->A;
    al = std::sqrt(p->kappa / (2.0 * p->A));
  }
  ph.k1 = (float)k1;
  ph.k2 = (float)k2;
  ph.a2q = (float)(al * al / 4.0);
  ph.om_f = (float)(1.0 / p->tau_f);
  ph.om_g = (float)(1.0 / p->tau_g);
  ph.guo = (float)(1.0 - 0.5 / p->tau_f);
  ph.gam3 = (float)(3.0 * p->M / (p->tau_g - 0.5));
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 2; ++s)
      for (int b = 0; b < 3; ++b) ph.wall_u[a][s][b] = (float)p->wall_u[a][s][b];
  if (p->ternary) {
    ph.k3 = (float)p->kappa3;
    ph.om_h = (float)(1.0 / p->tau_h);
    ph.gam3h = (float)(3.0 * p->M3 / (p->tau_h - 0.5));
  }
  ph.n_rollers = p->n_rollers;
  for (int k = 0; k < p->n_rollers; ++k) {
    for (int a = 0; a < 3; ++a) ph.rc[k][a] = (float)p->rollers[k].center[a];
    ph.rom[k] = (float)p->rollers[k].omega;
    ph.rax[k] = p->rollers[k].axis;
  }
  return ph;
}

}  // namespace

struct fre_lattice {
  fre_params p;
  Plan plan;
  LaunchArgs a;
  uint8_t *base;
  long long n_user;
  int64_t t;
  int state;  // 0 ok, 1 failed
  std::vector<int> fill_host;
  hipGraphExec_t graph;  // two steps starting at even parity
  bool graph_ok;
  hipGraphExec_t graph_run;  // kGraphRun steps starting at even parity
  bool graph_run_ok;
  fre_batch *batch;      // non-null while the lattice is a batch member
  int dev;               // device current at init
};

struct fre_batch {
  uint8_t *base;
  size_t bytes;
  hipStream_t stream;
  int max_slots, cap_work, cap_fill;
  Inst *d_inst;
  int4 *d_work;
  int4 *d_cols;  // potential columns
  int2 *d_fill;
  int *d_range;  // [N_BATCH_CLASSES][BATCH_RANGE]: see BatchArgs
  std::vector<fre_lattice *> slot;
  std::vector<Inst> h_inst;
  std::vector<int4> h_work, h_cols;
  std::vector<int2> h_fill;
  std::vector<int> h_range;
  int parity;         // common AA parity of the members
  unsigned classes;   // bit c: class c has members
  int rows;           // rows of 64 cells per work item
  int blocks_per_cu;  // persistent grid of the cell kernels
  int ncu;
  hipGraphExec_t graph;      // two steps starting at even parity
  bool graph_ok;
  hipGraphExec_t graph_run;  // kGraphRun steps starting at even parity
  bool graph_run_ok;
  int grid_cells, grid_fill;
};

namespace {

// Launches of the captured graph may still be queued on the stream, and the
// executable holds their kernel arguments: destroying it before they have
// run lets them read whatever reuses that memory (for example the arguments
// of the next graph, with new parameters), so the stream is drained first.
// Steps per graph launch of a lattice's long runs (even).
constexpr int kGraphRun = 16;

void reset_graph(fre_lattice *L) {
  if (L->graph_ok || L->graph_run_ok) (void)hipStreamSynchronize(L->a.stream);
  if (L->graph_ok) (void)hipGraphExecDestroy(L->graph);
  if (L->graph_run_ok) (void)hipGraphExecDestroy(L->graph_run);
  L->graph_ok = L->graph_run_ok = false;
}

// A batch member's state is advanced on the batch's stream: wait for it
// before touching the lattice on its own stream.
fre_status sync_batch(fre_lattice *L) {
  if (L && L->batch) HIP_TRY(hipStreamSynchronize(L->batch->stream));
  return FRE_OK;
}

long long ext_index(const Plan &P, int x, int y, int z) {
  return (long long)(x + P.off[0]) + (long long)P.px * ((long long)(y + P.off[1]) + (long long)P.ext[1] * (z + P.off[2]));
}

fre_status build_mask(fre_lattice *L, const uint8_t *user_mask, std::vector<uint8_t> &mask,
                      std::vector<uint32_t> &nbm, std::vector<uint8_t> &segf) {
  const Plan &P = L->plan;
  const fre_params &p = L->p;
  mask.assign((size_t)P.ncell, CELL_GHOST);
  for (long long c = 0; c < P.ncell; ++c)
    if (c % P.px >= P.ext[0]) mask[c] = CELL_PAD;
  for (int z = 0; z < p.nz; ++z)
    for (int y = 0; y < p.ny; ++y)
      for (int x = 0; x < p.nx; ++x) {
        long long u = x + (long long)p.nx * (y + (long long)p.ny * z);
        uint8_t code = user_mask ? user_mask[u] : 0;
        if (code > 1 && code >= 2 + p.n_rollers)
          return fail(FRE_EINVAL, "mask code %d at cell %lld: no such roller", code, u);
        mask[ext_index(P, x, y, z)] = code;
      }
  // solid cells with at least one fluid neighbour get stencil fills
  auto dir = [&](int i, int a) {
    if (P.q == 9) return a == 0 ? VSet<9>::cx(i) : a == 1 ? VSet<9>::cy(i) : VSet<9>::cz(i);
    return a == 0 ? VSet<19>::cx(i) : a == 1 ? VSet<19>::cy(i) : VSet<19>::cz(i);
  };
  L->fill_host.clear();
  nbm.assign((size_t)P.ncell, NB_SELF_SOLID);
  for (int z = 0; z < P.ext[2]; ++z)
    for (int y = 0; y < P.ext[1]; ++y)
      for (int x = 0; x < P.ext[0]; ++x) {
        long long s = x + (long long)P.px * (y + (long long)P.ext[1] * z);
        if (mask[s] == CELL_FLUID) {
          uint32_t bits = 0;
          for (int i = 1; i < P.q; ++i) {
            int v[3] = {x + dir(i, 0), y + dir(i, 1), z + dir(i, 2)};
            for (int a = 0; a < 3; ++a) v[a] = (v[a] % P.ext[a] + P.ext[a]) % P.ext[a];
            long long n = v[0] + (long long)P.px * (v[1] + (long long)P.ext[1] * v[2]);
            if (mask[n] != CELL_FLUID) bits |= 1u << i;
          }
          nbm[s] = bits;
          continue;
        }
        uint32_t fluid = 0;
        for (int i = 1; i < P.q; ++i) {
          int v[3] = {x + dir(i, 0), y + dir(i, 1), z + dir(i, 2)};
          bool ok = true;
          for (int a = 0; a < 3; ++a) {
            if (P.per[a]) v[a] = (v[a] % P.ext[a] + P.ext[a]) % P.ext[a];
            else if (v[a] < 0 || v[a] >= P.ext[a]) ok = false;
          }
          if (!ok) continue;
          long long n = v[0] + (long long)P.px * (v[1] + (long long)P.ext[1] * v[2]);
          if (mask[n] == CELL_FLUID) fluid |= 1u << i;
        }
        nbm[s] = NB_SELF_SOLID | fluid;
        if (fluid) L->fill_host.push_back((int)s);
      }
  // 64-cell row segments whose cells are all fluid with fluid neighbours only
  segf.assign((size_t)(P.ncell / 64), 0);
  for (size_t k = 0; k < segf.size(); ++k) {
    bool all = true;
    for (size_t j = 0; j < 64 && all; ++j) all = nbm[64 * k + j] == 0u;
    segf[k] = all ? 1 : 0;
  }
  return FRE_OK;
}

void bind_args(fre_lattice *L) {
  const Plan &P = L->plan;
  LaunchArgs &a = L->a;
  a.q = P.q;
  a.storage = L->p.storage;
  a.G.ex = P.ext[0]; a.G.ey = P.ext[1]; a.G.ez = P.ext[2];
  for (int k = 0; k < 3; ++k) { a.G.per[k] = P.per[k]; a.G.off[k] = P.off[k]; }
  a.G.px = P.px;
  a.G.ncell = P.ncell;
  a.ph = make_phys(&L->p);
  a.f = L->base + P.o_f;
  a.g = L->base + P.o_g;
  a.g0 = (float *)(L->base + P.o_g0);  // FP16: the g_0 plane; FP32: the half plane of g_0's low part
  a.mask = L->base + P.o_mask;
  a.nbm = (uint32_t *)(L->base + P.o_nbm);
  a.segf = L->base + P.o_segf;
  a.ctr = P.o_ctr ? (uint32_t *)(L->base + P.o_ctr) : nullptr;
  a.M = (float2 *)(L->base + P.o_M);
  a.C = (float4 *)(L->base + P.o_C);
  a.P0 = P.o_P0 ? (float2 *)(L->base + P.o_P0) : nullptr;
  a.PU = P.o_PU ? (float2 *)(L->base + P.o_PU) : nullptr;
  a.PD = P.o_PD ? (float2 *)(L->base + P.o_PD) : nullptr;
  a.XE = P.o_XE ? (float2 *)(L->base + P.o_XE) : nullptr;
  a.AUX = (float4 *)(L->base + P.o_AUX);
  a.ternary = L->p.ternary;
  a.h = P.o_h ? L->base + P.o_h : nullptr;
  a.h0l = P.o_h0 ? (__half *)(L->base + P.o_h0) : nullptr;
  a.CM = P.o_CM ? (float2 *)(L->base + P.o_CM) : nullptr;
  a.fill_list = (int *)(L->base + P.o_fill);
  a.n_fill = (int)L->fill_host.size();
}

size_t pops_bytes(const Plan &P, int storage) { return P.o_mask - P.o_f; }

// one step of either kind of lattice
void launch_lattice_step(const LaunchArgs &a, int odd) {
  if (a.ternary) launch_step3(a, odd);
  else launch_step(a, odd);
}

fre_status observe(fre_lattice *L) {
  if (L->a.ternary) launch_observe3(L->a, (int)(L->t & 1));
  else launch_observe(L->a, (int)(L->t & 1));
  HIP_TRY(hipGetLastError());
  return FRE_OK;
}

}  // namespace

extern "C" {

const char *fre_last_error(void) { return g_err.c_str(); }

fre_status fre_footprint(const fre_params *p, size_t *device_bytes) {
  fre_status s = validate(p);
  if (s != FRE_OK) return s;
  if (!device_bytes) return fail(FRE_EINVAL, "device_bytes is NULL");
  *device_bytes = make_plan(p).total;
  return FRE_OK;
}

}  // extern "C"

namespace {

// fre_lattice_init and fre_lattice_init3: psi0 is NULL for a binary lattice
fre_status lattice_init(const fre_params *p, void *device_buf, size_t bytes, void *hip_stream,
                        const double *phi0, const double *psi0, const double *rho0, const double *u0,
                        const uint8_t *solid_mask, fre_lattice **out) {
  if (!out) return fail(FRE_EINVAL, "out is NULL");
  *out = nullptr;
  fre_status s = validate(p);
  if (s != FRE_OK) return s;
  const bool t3 = p->ternary != 0;
  if (t3 && !psi0) return fail(FRE_EINVAL, "a ternary lattice needs psi0 (use fre_lattice_init3)");
  if (!t3 && psi0) return fail(FRE_EINVAL, "psi0 given for a binary lattice (set ternary = 1)");
  if (!phi0) return fail(FRE_EINVAL, "phi0 is NULL");
  if (!device_buf) return fail(FRE_EINVAL, "device_buf is NULL");
  if ((uintptr_t)device_buf % kAlign) return fail(FRE_EINVAL, "device_buf must be 256-byte aligned");
  Plan P = make_plan(p);
  if (bytes < P.total) return fail(FRE_ENOMEM, "buffer of %zu bytes < footprint %zu", bytes, P.total);
  long long N = (long long)p->nx * p->ny * p->nz;
  for (long long u = 0; u < N; ++u) {
    if (!std::isfinite(phi0[u]) || (psi0 && !std::isfinite(psi0[u])) ||
        (rho0 && !(std::isfinite(rho0[u]) && rho0[u] > 0)) ||
        (u0 && !(std::isfinite(u0[u]) && std::isfinite(u0[N + u]) && std::isfinite(u0[2 * N + u]))))
      return fail(FRE_EINVAL, "non-finite or non-positive initial value at cell %lld", u);
  }
  fre_lattice *L = new fre_lattice();
  L->p = *p;
  L->plan = P;
  L->base = (uint8_t *)device_buf;
  L->n_user = N;
  L->t = 0;
  L->state = 0;
  L->graph_ok = L->graph_run_ok = false;
  if (hipGetDevice(&L->dev) != hipSuccess) { delete L; return fail(FRE_EDEVICE, "hipGetDevice failed"); }
  std::vector<uint8_t> mask;
  std::vector<uint32_t> nbm;
  std::vector<uint8_t> segf;
  s = build_mask(L, solid_mask, mask, nbm, segf);
  if (s != FRE_OK) { delete L; return s; }
  bind_args(L);
  for (int k = 0; k < N_SHAPES; ++k) L->a.shape[k] = Shape{4, 1};
  L->a.stream = (hipStream_t)hip_stream;
  // initial fields in storage layout
  // M: (rho - 1, phi), or (rho - 1, phi, psi, 0) on a ternary lattice
  const int mw = t3 ? 4 : 2;
  std::vector<float> M((size_t)P.ncell * mw, 0.0f), U((size_t)P.ncell * 4, 0.0f);
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        long long u = x + (long long)p->nx * (y + (long long)p->ny * z);
        long long e = ext_index(P, x, y, z);
        if (mask[e] != CELL_FLUID) continue;
        M[mw * e] = rho0 ? (float)(rho0[u] - 1.0) : 0.0f;
        M[mw * e + 1] = (float)phi0[u];
        if (t3) M[mw * e + 2] = (float)psi0[u];
        if (u0)
          for (int k = 0; k < 3; ++k) U[4 * e + k] = (float)u0[(long long)k * N + u];
      }
  hipStream_t st = L->a.stream;
  auto cleanup = [&](fre_status r) { if (r != FRE_OK) delete L; return r; };
#define INIT_TRY(expr)                                                             \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return cleanup(fail(FRE_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_))); \
  } while (0)
  INIT_TRY(hipMemsetAsync(L->base + P.o_f, 0, pops_bytes(P, p->storage), st));
  INIT_TRY(hipMemcpyAsync(L->a.mask, mask.data(), mask.size(), hipMemcpyHostToDevice, st));
  INIT_TRY(hipMemcpyAsync(L->a.M, M.data(), M.size() * 4, hipMemcpyHostToDevice, st));
  INIT_TRY(hipMemcpyAsync(L->a.AUX, U.data(), U.size() * 4, hipMemcpyHostToDevice, st));
  if (!L->fill_host.empty())
    INIT_TRY(hipMemcpyAsync(L->a.fill_list, L->fill_host.data(), L->fill_host.size() * 4, hipMemcpyHostToDevice, st));
  INIT_TRY(hipMemcpyAsync(L->a.nbm, nbm.data(), nbm.size() * 4, hipMemcpyHostToDevice, st));
  INIT_TRY(hipMemcpyAsync(L->a.segf, segf.data(), segf.size(), hipMemcpyHostToDevice, st));
  INIT_TRY(hipMemsetAsync(L->a.C, 0, (size_t)P.ncell * 16, st));
  if (t3) {
    INIT_TRY(hipMemsetAsync(L->a.CM, 0, (size_t)P.ncell * 8, st));
    launch_init3(L->a);
  } else {
    launch_init(L->a);
  }
  INIT_TRY(hipGetLastError());
  INIT_TRY(hipStreamSynchronize(st));
#undef INIT_TRY
  *out = L;
  return FRE_OK;
}

}  // namespace

extern "C" {

fre_status fre_lattice_init(const fre_params *p, void *device_buf, size_t bytes, void *hip_stream,
                            const double *phi0, const double *rho0, const double *u0,
                            const uint8_t *solid_mask, fre_lattice **out) {
  if (p && p->ternary) {
    if (out) *out = nullptr;
    return fail(FRE_EINVAL, "ternary lattices are created with fre_lattice_init3");
  }
  return lattice_init(p, device_buf, bytes, hip_stream, phi0, nullptr, rho0, u0, solid_mask, out);
}

fre_status fre_lattice_init3(const fre_params *p, void *device_buf, size_t bytes, void *hip_stream,
                             const double *phi0, const double *psi0, const double *rho0, const double *u0,
                             const uint8_t *solid_mask, fre_lattice **out) {
  if (p && !p->ternary) {
    if (out) *out = nullptr;
    return fail(FRE_EINVAL, "fre_lattice_init3 needs ternary = 1");
  }
  if (!psi0) {
    if (out) *out = nullptr;
    return fail(FRE_EINVAL, "psi0 is NULL");
  }
  return lattice_init(p, device_buf, bytes, hip_stream, phi0, psi0, rho0, u0, solid_mask, out);
}

fre_status fre_consistent_init(fre_lattice *L, const double *phi0, const double *u0, int64_t n) {
  if (!L) return fail(FRE_EINVAL, "lattice is NULL");
  if (!phi0) return fail(FRE_EINVAL, "phi0 is NULL");
  if (n < 0 || (n & 1)) return fail(FRE_EINVAL, "the number of pre-iterations must be even and >= 0 (got %lld)",
                                    (long long)n);
  if (L->state) return fail(FRE_ESTATE, "lattice is in the failed state");
  if (L->batch) return fail(FRE_ESTATE, "lattice is a batch member: remove it first");
  if (L->t != 0) return fail(FRE_ESTATE, "consistent initialisation is only possible before the first step");
  if (L->p.ternary) return fail(FRE_EINVAL, "consistent initialisation is not available for ternary lattices");
  const fre_params *p = &L->p;
  const Plan &P = L->plan;
  const long long N = L->n_user;
  for (long long u = 0; u < N; ++u)
    if (!std::isfinite(phi0[u]) ||
        (u0 && !(std::isfinite(u0[u]) && std::isfinite(u0[N + u]) && std::isfinite(u0[2 * N + u]))))
      return fail(FRE_EINVAL, "non-finite value at cell %lld", u);
  // AUX = (u0, phi0) in storage layout
  std::vector<float> U((size_t)P.ncell * 4, 0.0f);
  for (int z = 0; z < p->nz; ++z)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        const long long u = x + (long long)p->nx * (y + (long long)p->ny * z);
        const long long e = ext_index(P, x, y, z);
        if (u0)
          for (int k = 0; k < 3; ++k) U[4 * e + k] = (float)u0[(long long)k * N + u];
        U[4 * e + 3] = (float)phi0[u];
      }
  hipStream_t st = L->a.stream;
  HIP_TRY(hipMemcpyAsync(L->a.AUX, U.data(), U.size() * 4, hipMemcpyHostToDevice, st));
  launch_consistent_init(L->a, (long long)n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return FRE_OK;
}

fre_status fre_set_params(fre_lattice *L, const fre_params *p) {
  if (!L) return fail(FRE_EINVAL, "lattice is NULL");
  fre_status s = validate(p);
  if (s != FRE_OK) return s;
  if (L->batch) return fail(FRE_ESTATE, "lattice is a batch member: remove it before changing parameters");
  const fre_params &o = L->p;
  if (p->kind != o.kind || p->nx != o.nx || p->ny != o.ny || p->nz != o.nz || p->storage != o.storage ||
      p->bc[0] != o.bc[0] || p->bc[1] != o.bc[1] || p->bc[2] != o.bc[2] || p->n_rollers != o.n_rollers ||
      p->ternary != o.ternary || p->fp16_rounding != o.fp16_rounding)
    return fail(FRE_EINVAL, "shape, storage, bc, roller count, the ternary flag and fp16_rounding cannot change");
  L->p = *p;
  L->a.ph = make_phys(p);
  reset_graph(L);
  return FRE_OK;
}

fre_status fre_step(fre_lattice *L, int64_t n) {
  if (!L) return fail(FRE_EINVAL, "lattice is NULL");
  if (n < 0) return fail(FRE_EINVAL, "negative step count");
  if (L->state) return fail(FRE_ESTATE, "lattice is in the failed state");
  if (L->batch) return fail(FRE_ESTATE, "lattice is a batch member: step the batch");
  hipStream_t st = L->a.stream;
  auto one = [&]() -> fre_status {
    launch_lattice_step(L->a, (int)(L->t & 1));
    HIP_TRY(hipGetLastError());
    L->t += 1;
    return FRE_OK;
  };
  if (st == nullptr || n < 4) {
    for (int64_t k = 0; k < n; ++k) {
      fre_status s = one();
      if (s != FRE_OK) return s;
    }
    return FRE_OK;
  }
  if (L->t & 1) {
    fre_status s = one();
    if (s != FRE_OK) return s;
    --n;
  }
  // a graph of `pairs` even + odd step pairs
  auto capture = [&](int pairs, hipGraphExec_t *out) -> fre_status {
    hipGraph_t g;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < pairs; ++k) {
      launch_lattice_step(L->a, 0);
      launch_lattice_step(L->a, 1);
    }
    hipError_t e = hipStreamEndCapture(st, &g);
    if (e != hipSuccess) return fail(FRE_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(FRE_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    return FRE_OK;
  };
  // runs of kGraphRun steps (each graph launch leaves the GPU idle for a few
  // microseconds, so longer graphs leave it idle less often), then pairs
  if (n >= kGraphRun) {
    if (!L->graph_run_ok) {
      fre_status s = capture(kGraphRun / 2, &L->graph_run);
      if (s != FRE_OK) return s;
      L->graph_run_ok = true;
    }
    for (; n >= kGraphRun; n -= kGraphRun) {
      HIP_TRY(hipGraphLaunch(L->graph_run, st));
      L->t += kGraphRun;
    }
  }
  if (n >= 2) {
    if (!L->graph_ok) {
      fre_status s = capture(1, &L->graph);
      if (s != FRE_OK) return s;
      L->graph_ok = true;
    }
    for (; n >= 2; n -= 2) {
      HIP_TRY(hipGraphLaunch(L->graph, st));
      L->t += 2;
    }
  }
  if (n) return one();
  return FRE_OK;
}

fre_status fre_read_moments(fre_lattice *L, uint32_t field_mask, double *host_out, size_t n_doubles) {
  if (!L || !host_out) return fail(FRE_EINVAL, "NULL argument");
  if (fre_status bs = sync_batch(L)) return bs;
  const bool t3 = L->p.ternary != 0;
  const int nfield = t3 ? 8 : 6;
  if (field_mask == 0 || (field_mask & ~((1u << nfield) - 1u)))
    return fail(FRE_EINVAL, "bad field mask 0x%x%s", field_mask,
                (!t3 && (field_mask & (FRE_F_PSI | FRE_F_MU_PSI))) ? " (psi fields need a ternary lattice)" : "");
  size_t need = 0;
  const long long N = L->n_user;
  for (int b = 0; b < nfield; ++b)
    if (field_mask & (1u << b)) need += (b == 2 ? 3 : 1) * (size_t)N;
  if (n_doubles < need) return fail(FRE_EINVAL, "output holds %zu doubles, need %zu", n_doubles, need);
  const Plan &P = L->plan;
  fre_status s = observe(L);
  if (s != FRE_OK) return s;
  std::vector<float> Cv((size_t)P.ncell * 4), AUX((size_t)P.ncell * 4), CM(t3 ? (size_t)P.ncell * 2 : 0);
  std::vector<uint8_t> mask((size_t)P.ncell);
  hipStream_t st = L->a.stream;
  HIP_TRY(hipMemcpyAsync(Cv.data(), L->a.C, Cv.size() * 4, hipMemcpyDeviceToHost, st));
  if (t3) HIP_TRY(hipMemcpyAsync(CM.data(), L->a.CM, CM.size() * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(AUX.data(), L->a.AUX, AUX.size() * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(mask.data(), L->a.mask, mask.size(), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const fre_params &p = L->p;
  double *o = host_out;
  for (int b = 0; b < nfield; ++b) {
    if (!(field_mask & (1u << b))) continue;
    int ncomp = b == 2 ? 3 : 1;
    for (int k = 0; k < ncomp; ++k) {
      for (int z = 0; z < p.nz; ++z)
        for (int y = 0; y < p.ny; ++y)
          for (int x = 0; x < p.nx; ++x) {
            long long u = x + (long long)p.nx * (y + (long long)p.ny * z);
            long long e = ext_index(P, x, y, z);
            double v = 0.0;
            if (mask[e] == CELL_FLUID && t3) {
              // C = (rho - 1, phi, psi, Pi), CM = (mu_phi, mu_psi):
              // mu_rho = (Pi - phi mu_phi - psi mu_psi) / rho
              const double rho = 1.0 + (double)Cv[4 * e];
              switch (b) {
                case 0: v = rho; break;
                case 1: v = Cv[4 * e + 1]; break;
                case 2: v = AUX[4 * e + k]; break;
                case 3: v = ((double)Cv[4 * e + 3] - (double)Cv[4 * e + 1] * CM[2 * e] -
                             (double)Cv[4 * e + 2] * CM[2 * e + 1]) / rho; break;
                case 4: v = CM[2 * e]; break;
                case 5: v = AUX[4 * e + 3]; break;
                case 6: v = Cv[4 * e + 2]; break;
                default: v = CM[2 * e + 1]; break;
              }
            } else if (mask[e] == CELL_FLUID) {
              switch (b) {
                case 0: v = 1.0 + (double)Cv[4 * e]; break;
                case 1: v = Cv[4 * e + 1]; break;
                case 2: v = AUX[4 * e + k]; break;
                // C = (rho - 1, phi, Pi, mu_phi): mu_rho = (Pi - phi mu_phi) / rho
                case 3: v = ((double)Cv[4 * e + 2] - (double)Cv[4 * e + 1] * Cv[4 * e + 3]) / (1.0 + Cv[4 * e]); break;
                case 4: v = Cv[4 * e + 3]; break;
                default: v = AUX[4 * e + 3]; break;
              }
            }
            o[u] = v;
          }
      o += N;
    }
  }
  return FRE_OK;
}

fre_status fre_read_populations(fre_lattice *L, double *f_out, double *g_out, size_t n_doubles_each) {
  if (!L || !f_out || !g_out) return fail(FRE_EINVAL, "NULL argument");
  if (L->p.ternary) return fail(FRE_EINVAL, "ternary lattices are read with fre_read_populations3");
  if (fre_status bs = sync_batch(L)) return bs;
  const Plan &P = L->plan;
  const long long N = L->n_user;
  if (n_doubles_each < (size_t)P.q * N) return fail(FRE_EINVAL, "outputs need q*N doubles each");
  // staged in chunks through the lattice's AUX field (4 floats per cell, no
  // other state lives there between calls): 2q + 1 planes per chunk -- f_i +
  // w_i, g_i, and the low part of g_0 (zero with FP16 storage)
  const int planes = 2 * P.q + 1;
  const long long chunk = std::max(1LL, 4 * P.ncell / planes);
  float *stage = (float *)L->a.AUX;
  std::vector<float> h((size_t)planes * (size_t)std::min(chunk, P.ncell));
  const fre_params &p = L->p;
  const int odd = (int)(L->t & 1);
  for (long long c0 = 0; c0 < P.ncell; c0 += chunk) {
    const int n = (int)std::min(chunk, P.ncell - c0);
    launch_read_pops(L->a, odd, stage, c0, n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h.data(), stage, (size_t)planes * n * sizeof(float), hipMemcpyDeviceToHost, L->a.stream));
    HIP_TRY(hipStreamSynchronize(L->a.stream));
    for (long long c = c0; c < c0 + n; ++c) {
      const int x = (int)(c % P.px) - P.off[0];
      const long long r = c / P.px;
      const int y = (int)(r % P.ext[1]) - P.off[1], z = (int)(r / P.ext[1]) - P.off[2];
      if (x < 0 || x >= p.nx || y < 0 || y >= p.ny || z < 0 || z >= p.nz) continue;
      const long long u = x + (long long)p.nx * (y + (long long)p.ny * z);
      const size_t t = (size_t)(c - c0);
      for (int i = 0; i < P.q; ++i) {
        f_out[(long long)i * N + u] = h[(size_t)i * n + t];
        g_out[(long long)i * N + u] = (double)h[(size_t)(P.q + i) * n + t] +
                                      (i == 0 ? (double)h[(size_t)2 * P.q * n + t] : 0.0);
      }
    }
  }
  return FRE_OK;
}

fre_status fre_read_populations3(fre_lattice *L, double *f_out, double *g_out, double *h_out,
                                 size_t n_doubles_each) {
  if (!L || !f_out || !g_out || !h_out) return fail(FRE_EINVAL, "NULL argument");
  if (!L->p.ternary) return fail(FRE_EINVAL, "fre_read_populations3 needs a ternary lattice");
  const Plan &P = L->plan;
  const long long N = L->n_user;
  if (n_doubles_each < (size_t)P.q * N) return fail(FRE_EINVAL, "outputs need q*N doubles each");
  // staged in chunks through AUX as fre_read_populations: 3q + 2 planes --
  // f_i + w_i, g_i, h_i, and the low parts of g_0 and h_0
  const int planes = 3 * P.q + 2;
  const long long chunk = std::max(1LL, 4 * P.ncell / planes);
  float *stage = (float *)L->a.AUX;
  std::vector<float> hb((size_t)planes * (size_t)std::min(chunk, P.ncell));
  const fre_params &p = L->p;
  const int odd = (int)(L->t & 1);
  for (long long c0 = 0; c0 < P.ncell; c0 += chunk) {
    const int n = (int)std::min(chunk, P.ncell - c0);
    launch_read_pops3(L->a, odd, stage, c0, n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(hb.data(), stage, (size_t)planes * n * sizeof(float), hipMemcpyDeviceToHost, L->a.stream));
    HIP_TRY(hipStreamSynchronize(L->a.stream));
    for (long long c = c0; c < c0 + n; ++c) {
      const int x = (int)(c % P.px) - P.off[0];
      const long long r = c / P.px;
      const int y = (int)(r % P.ext[1]) - P.off[1], z = (int)(r / P.ext[1]) - P.off[2];
      if (x < 0 || x >= p.nx || y < 0 || y >= p.ny || z < 0 || z >= p.nz) continue;
      const long long u = x + (long long)p.nx * (y + (long long)p.ny * z);
      const size_t t = (size_t)(c - c0);
      for (int i = 0; i < P.q; ++i) {
        f_out[(long long)i * N + u] = hb[(size_t)i * n + t];
        g_out[(long long)i * N + u] = (double)hb[(size_t)(P.q + i) * n + t] +
                                      (i == 0 ? (double)hb[(size_t)3 * P.q * n + t] : 0.0);
        h_out[(long long)i * N + u] = (double)hb[(size_t)(2 * P.q + i) * n + t] +
                                      (i == 0 ? (double)hb[(size_t)(3 * P.q + 1) * n + t] : 0.0);
      }
    }
  }
  return FRE_OK;
}

fre_status fre_reduce(fre_lattice *L, double out[8]) {
  if (!L || !out) return fail(FRE_EINVAL, "NULL argument");
  if (fre_status bs = sync_batch(L)) return bs;
  fre_status s = observe(L);
  if (s != FRE_OK) return s;
  double *part = (double *)(L->base + L->plan.o_part);
  launch_reduce(L->a, part);
  HIP_TRY(hipGetLastError());
  std::vector<double> h((size_t)reduce_blocks() * 8);
  HIP_TRY(hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, L->a.stream));
  HIP_TRY(hipStreamSynchronize(L->a.stream));
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = 0; b < reduce_blocks(); ++b)
    for (int k = 0; k < 8; ++k) acc[k] += h[(size_t)b * 8 + k];
  out[0] = acc[7] + acc[0];  // sum rho = n_fluid + sum (rho - 1)
  for (int k = 1; k < 8; ++k) out[k] = acc[k];
  if (acc[6] > 0) {
    L->state = 1;
    return fail(FRE_ENUMERIC, "%.0f fluid cells hold non-finite values at step %lld", acc[6], (long long)L->t);
  }
  return FRE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free reduction.  Its block partials and totals live in this
// file-scope device array (one copy per GPU, held until the process ends)
// instead of the lattice buffer.  Host code uses the array through the
// address hipGetSymbolAddress gives on each device, never through its name.
// ---------------------------------------------------------------------------
constexpr int kScratchDoubles = REDUCE_BLOCKS * 8 + 8;  // partials, then 8 totals
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on device `dev`, which must be current;
// looked up once per device.
fre_status scratch_of_device(int dev, double **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) return fail(FRE_EDEVICE, "device %d out of range", dev);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FRE_EDEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = (double *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return FRE_OK;
}
}  // namespace

extern "C" {

fre_status fre_reduce_noalloc(fre_lattice *L, double out[8]) {
  if (!L || !out) return fail(FRE_EINVAL, "NULL argument");
  if (fre_status bs = sync_batch(L)) return bs;
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != L->dev) HIP_TRY(hipSetDevice(L->dev));
  auto finish = [&](fre_status st) {
    if (cur != L->dev) (void)hipSetDevice(cur);
    return st;
  };
  double *ptr = nullptr;
  fre_status s = scratch_of_device(L->dev, &ptr);
  if (s != FRE_OK) return finish(s);
  s = observe(L);
  if (s != FRE_OK) return finish(s);
  // every block writes all 8 of its partials, so nothing needs clearing
  launch_reduce_total(L->a, ptr, ptr + (size_t)REDUCE_BLOCKS * 8);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, ptr + (size_t)REDUCE_BLOCKS * 8, 8 * sizeof(double), hipMemcpyDeviceToHost, L->a.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->a.stream);
  if (e != hipSuccess) return finish(fail(FRE_EDEVICE, "reduction failed: %s", hipGetErrorString(e)));
  out[0] = out[7] + out[0];  // sum rho = n_fluid + sum (rho - 1)
  if (out[6] > 0) {
    L->state = 1;
    return finish(fail(FRE_ENUMERIC, "%.0f fluid cells hold non-finite values at step %lld", out[6], (long long)L->t));
  }
  return finish(FRE_OK);
}

fre_status fre_info(const fre_lattice *L, int64_t *step, int32_t *state) {
  if (!L) return fail(FRE_EINVAL, "lattice is NULL");
  if (step) *step = L->t;
  if (state) *state = L->state;
  return FRE_OK;
}

namespace {
struct CkptHeader {
  char magic[8];
  int32_t version, kind, nx, ny, nz, storage;
  int64_t step;
  uint64_t pops_bytes;
  fre_params params;
};
}  // namespace

fre_status fre_state_bytes(const fre_lattice *L, size_t *bytes) {
  if (!L || !bytes) return fail(FRE_EINVAL, "NULL argument");
  *bytes = sizeof(CkptHeader) + pops_bytes(L->plan, L->p.storage);
  return FRE_OK;
}

fre_status fre_save(fre_lattice *L, void *host, size_t bytes) {
  if (fre_status bs = sync_batch(L)) return bs;
  size_t need;
  fre_status s = fre_state_bytes(L, &need);
  if (s != FRE_OK) return s;
  if (!host || bytes < need) return fail(FRE_EINVAL, "checkpoint buffer needs %zu bytes", need);
  CkptHeader h{};
  memcpy(h.magic, "FRELBM01", 8);
  h.version = 1;
  h.kind = L->p.kind; h.nx = L->p.nx; h.ny = L->p.ny; h.nz = L->p.nz; h.storage = L->p.storage;
  h.step = L->t;
  h.pops_bytes = pops_bytes(L->plan, L->p.storage);
  h.params = L->p;
  memcpy(host, &h, sizeof h);
  HIP_TRY(hipMemcpyAsync((uint8_t *)host + sizeof h, L->base + L->plan.o_f, h.pops_bytes, hipMemcpyDeviceToHost, L->a.stream));
  HIP_TRY(hipStreamSynchronize(L->a.stream));
  return FRE_OK;
}

fre_status fre_load(fre_lattice *L, const void *host, size_t bytes) {
  if (!L || !host || bytes < sizeof(CkptHeader)) return fail(FRE_EINVAL, "bad checkpoint buffer");
  if (L->batch) return fail(FRE_ESTATE, "lattice is a batch member: remove it before loading");
  CkptHeader h;
  memcpy(&h, host, sizeof h);
  if (memcmp(h.magic, "FRELBM01", 8) != 0 || h.version != 1) return fail(FRE_EINVAL, "not a checkpoint");
  if (h.kind != L->p.kind || h.nx != L->p.nx || h.ny != L->p.ny || h.nz != L->p.nz || h.storage != L->p.storage ||
      h.pops_bytes != pops_bytes(L->plan, L->p.storage) || bytes < sizeof h + h.pops_bytes)
    return fail(FRE_EINVAL, "checkpoint shape/storage does not match this lattice");
  fre_status s = fre_set_params(L, &h.params);
  if (s != FRE_OK) return s;
  HIP_TRY(hipMemcpyAsync(L->base + L->plan.o_f, (const uint8_t *)host + sizeof h, h.pops_bytes, hipMemcpyHostToDevice, L->a.stream));
  L->t = h.step;
  if (!L->p.ternary) launch_moments(L->a, (int)(L->t & 1));  // M of the restored populations
                                                            // (the ternary step makes its own)
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(L->a.stream));
  L->state = 0;
  return FRE_OK;
}

}  // extern "C"

namespace {

// Mean duration (ms) of each kernel of the step over n individually launched
// steps, from HIP events recorded on the lattice's stream around every launch.
fre_status time_kernels(fre_lattice *L, int64_t n, double *kernel_ms) {
  const int K = step_kernel_count();
  int slot[8];
  const int nslot = step_kernel_slots(L->a, slot);
  std::vector<hipEvent_t> ev((size_t)(K + 1) * n);
  for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
  for (int k = 0; k < nslot; ++k) kernel_ms[k] = -1.0;  // slots this class does not launch
  for (int k = 0; k < K; ++k) kernel_ms[slot[k]] = 0.0;
  fre_status st = FRE_OK;
  for (int64_t s = 0; s < n; ++s) {
    launch_step_events(L->a, (int)(L->t & 1), &ev[(size_t)s * (K + 1)]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { st = fail(FRE_EDEVICE, "launch failed: %s", hipGetErrorString(e)); break; }
    L->t += 1;
  }
  if (st == FRE_OK) {
    hipError_t e = hipStreamSynchronize(L->a.stream);
    if (e != hipSuccess) st = fail(FRE_EDEVICE, "sync failed: %s", hipGetErrorString(e));
  }
  if (st == FRE_OK)
    for (int64_t s = 0; s < n; ++s)
      for (int k = 0; k < K; ++k) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev[(size_t)s * (K + 1) + k], ev[(size_t)s * (K + 1) + k + 1]);
        kernel_ms[slot[k]] += ms / (double)n;
      }
  for (auto &e : ev) (void)hipEventDestroy(e);
  return st;
}

// Population state of a lattice kept on the host while the tuners step it.
struct HostState {
  std::vector<uint8_t> pops;
  int64_t t = 0;
};

fre_status snapshot(fre_lattice *L, HostState &h) {
  const size_t nb = pops_bytes(L->plan, L->p.storage);
  h.pops.resize(nb);
  h.t = L->t;
  HIP_TRY(hipMemcpyAsync(h.pops.data(), L->base + L->plan.o_f, nb, hipMemcpyDeviceToHost, L->a.stream));
  HIP_TRY(hipStreamSynchronize(L->a.stream));
  return FRE_OK;
}

fre_status restore(fre_lattice *L, const HostState &h) {
  HIP_TRY(hipMemcpyAsync(L->base + L->plan.o_f, h.pops.data(), h.pops.size(), hipMemcpyHostToDevice, L->a.stream));
  L->t = h.t;
  launch_moments(L->a, (int)(L->t & 1));  // M of the restored populations
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(L->a.stream));
  return FRE_OK;
}

// Kernel slot timed for each launch shape: the moments pass (k_moments, or
// k_combine with the by-product), k_potential, k_collide.
int stage_slot(const fre_lattice *L, int shape) {
  if (shape == SHAPE_MOMENTS) return uses_by_product(L->a) ? 5 : 0;
  return shape == SHAPE_POTENTIAL ? 2 : 4;
}
const Shape kCandidates[] = {{1, 0}, {2, 0}, {4, 0}, {8, 0}, {1, 1}, {2, 1}, {4, 1}, {8, 1}};

}  // namespace

extern "C" {

fre_status fre_profile_step(fre_lattice *L, int64_t n, double *kernel_ms, int32_t max_kernels,
                            int32_t *n_kernels) {
  if (!L || !kernel_ms || !n_kernels) return fail(FRE_EINVAL, "NULL argument");
  if (n < 1) return fail(FRE_EINVAL, "n must be >= 1");
  if (L->state) return fail(FRE_ESTATE, "lattice is in the failed state");
  int slot[8];
  const int K = step_kernel_slots(L->a, slot);
  if (L->p.ternary) return fail(FRE_EINVAL, "per-kernel profiling is not available for ternary lattices");
  if (max_kernels < K) return fail(FRE_EINVAL, "kernel_ms needs %d entries", K);
  if (L->batch) return fail(FRE_ESTATE, "lattice is a batch member: profile it alone");
  fre_status st = time_kernels(L, n, kernel_ms);
  *n_kernels = K;
  return st;
}

fre_status fre_set_launch_shape(fre_lattice *L, const int32_t cfg[6]) {
  if (!L || !cfg) return fail(FRE_EINVAL, "NULL argument");
  if (L->p.ternary) return fail(FRE_EINVAL, "ternary lattices have one launch shape");
  Shape sh[N_SHAPES];
  for (int k = 0; k < N_SHAPES; ++k) {
    sh[k] = Shape{cfg[2 * k], cfg[2 * k + 1]};
    if (!shape_ok(sh[k])) return fail(FRE_EINVAL, "bad launch shape (%d rows, xcd %d)", sh[k].rows, sh[k].xcd);
    if (k == SHAPE_COLLIDE && uses_by_product(L->a) && sh[k].rows != COLLIDE_ROWS)
      return fail(FRE_EINVAL, "with FP32 storage the collide tile has %d rows", COLLIDE_ROWS);
  }
  if (fre_status bs = sync_batch(L)) return bs;
  HIP_TRY(hipStreamSynchronize(L->a.stream));
  for (int k = 0; k < N_SHAPES; ++k) L->a.shape[k] = sh[k];
  reset_graph(L);
  return FRE_OK;
}

fre_status fre_get_launch_shape(const fre_lattice *L, int32_t cfg[6]) {
  if (!L || !cfg) return fail(FRE_EINVAL, "NULL argument");
  for (int k = 0; k < N_SHAPES; ++k) {
    cfg[2 * k] = L->a.shape[k].rows;
    cfg[2 * k + 1] = L->a.shape[k].xcd;
  }
  return FRE_OK;
}

fre_status fre_autotune(fre_lattice *L, int64_t n, int32_t cfg_out[6], double stage_ms[3]) {
  if (!L) return fail(FRE_EINVAL, "lattice is NULL");
  if (n < 2 || n > 10000) return fail(FRE_EINVAL, "n must be in [2, 10000]");
  if (L->p.ternary) return fail(FRE_EINVAL, "ternary lattices have one launch shape");
  if (L->state) return fail(FRE_ESTATE, "lattice is in the failed state");
  if (L->batch) return fail(FRE_ESTATE, "lattice is a batch member: tune the batch");
  n += n & 1;  // both parities equally
  HostState h;
  fre_status s = snapshot(L, h);
  if (s != FRE_OK) return s;
  const Shape saved[N_SHAPES] = {L->a.shape[0], L->a.shape[1], L->a.shape[2]};
  double best[N_SHAPES] = {1e300, 1e300, 1e300};
  Shape pick[N_SHAPES] = {saved[0], saved[1], saved[2]};
  double ms[16];
  for (const Shape &c : kCandidates) {
    for (int k = 0; k < N_SHAPES; ++k) L->a.shape[k] = c;
    s = time_kernels(L, 2, ms);  // warm-up
    if (s == FRE_OK) s = time_kernels(L, n, ms);
    if (s != FRE_OK) break;
    for (int k = 0; k < N_SHAPES; ++k) {
      // the by-product collide runs COLLIDE_ROWS rows whatever the shape says
      if (k == SHAPE_COLLIDE && uses_by_product(L->a) && c.rows != COLLIDE_ROWS) continue;
      const double t = ms[stage_slot(L, k)];
      if (t < best[k]) { best[k] = t; pick[k] = c; }
    }
  }
  fre_status r = restore(L, h);
  for (int k = 0; k < N_SHAPES; ++k) L->a.shape[k] = s == FRE_OK ? pick[k] : saved[k];
  reset_graph(L);
  if (s != FRE_OK) return s;
  if (r != FRE_OK) return r;
  if (cfg_out) fre_get_launch_shape(L, cfg_out);
  if (stage_ms)
    for (int k = 0; k < N_SHAPES; ++k) stage_ms[k] = best[k];
  return FRE_OK;
}

const char *fre_kernel_name(int32_t k) { return step_kernel_name(k); }

void fre_lattice_destroy(fre_lattice *L) {
  if (!L) return;
  if (L->batch) {
    fre_batch *B = L->batch;
    for (size_t k = 0; k < B->slot.size(); ++k)
      if (B->slot[k] == L) fre_batch_remove(B, (int32_t)k);
  }
  reset_graph(L);
  delete L;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
namespace {

struct BatchPlan {
  size_t o_inst, o_work, o_cols, o_fill, o_range, total;
};

BatchPlan batch_plan(int max_slots, int64_t max_work, int64_t max_fill) {
  BatchPlan P{};
  size_t o = 0;
  auto take = [&](size_t b) { size_t at = o; o = align_up(o + b, kAlign); return at; };
  P.o_inst = take((size_t)max_slots * sizeof(Inst));
  P.o_work = take((size_t)max_work * sizeof(int4));
  P.o_cols = take((size_t)max_work * sizeof(int4));  // a column holds at least one tile
  P.o_fill = take((size_t)max_fill * sizeof(int2));
  P.o_range = take(BATCH_RANGE * N_BATCH_CLASSES * sizeof(int));
  P.total = o;
  return P;
}

int64_t work_items(const Geom &G, int rows) {
  return (int64_t)((G.ex + 63) / 64) * ((G.ey + rows - 1) / rows) * G.ez;
}

// Work items are tiles of 64 x COLLIDE_ROWS cells.
void lattice_needs(const fre_lattice *L, int64_t *n_work, int64_t *n_fill) {
  *n_work = work_items(L->a.G, COLLIDE_ROWS);
  *n_fill = (int64_t)L->fill_host.size();
}

long long rel(const void *p, const void *base) { return (long long)((uintptr_t)p - (uintptr_t)base); }

Inst inst_of(const fre_lattice *L, const void *base) {
  Inst I{};
  I.G = L->a.G;
  I.ph = L->a.ph;
  I.f = rel(L->a.f, base);
  I.g = rel(L->a.g, base);
  I.g0 = L->a.g0 ? rel(L->a.g0, base) : 0;
  I.mask = rel(L->a.mask, base);
  I.nbm = rel(L->a.nbm, base);
  I.segf = rel(L->a.segf, base);
  I.M = rel(L->a.M, base);
  I.C = rel(L->a.C, base);
  I.P0 = L->a.P0 ? rel(L->a.P0, base) : 0;
  I.PU = L->a.PU ? rel(L->a.PU, base) : 0;
  I.PD = L->a.PD ? rel(L->a.PD, base) : 0;
  I.XE = L->a.XE ? rel(L->a.XE, base) : 0;
  I.fill = rel(L->a.fill_list, base);
  I.n_fill = L->a.n_fill;
  return I;
}

// As reset_graph: the batch's queued graph launches finish first.
void batch_reset_graph(fre_batch *B) {
  if (B->graph_ok || B->graph_run_ok) (void)hipStreamSynchronize(B->stream);
  if (B->graph_ok) (void)hipGraphExecDestroy(B->graph);
  if (B->graph_run_ok) (void)hipGraphExecDestroy(B->graph_run);
  B->graph_ok = B->graph_run_ok = false;
}

// Work-list order for the XCDs.  The persistent cell kernels walk a class's
// list grid-stride over a grid that is a multiple of 8 blocks, so item w
// runs on XCD w % 8 (workgroups go to the XCDs round-robin, each with its own
// L2).  Rows of tiles (one member, plane and tile row: the tiles along x)
// are dealt to the 8 XCDs in turn, and the list takes the XCDs' items in
// turn, so that a tile's x neighbours run on its own XCD and the cache lines
// that an x-shifted access shares across a tile edge are fetched once.
// Members of different widths can leave the XCDs' shares unequal; once
// some run out, the remaining items keep their order but not their XCD.
constexpr int NXCD_HOST = 8;

void xcd_interleave(std::vector<int4> (&rows)[NXCD_HOST], std::vector<int4> &out) {
  size_t most = 0;
  for (const auto &q : rows) most = std::max(most, q.size());
  for (size_t j = 0; j < most; ++j)
    for (const auto &q : rows)
      if (j < q.size()) out.push_back(q[j]);
}

// Rebuild and upload the instance table and the work lists, grouped by
// class; the ranges tell each class's persistent kernels what to walk.
fre_status batch_rebuild(fre_batch *B) {
  HIP_TRY(hipStreamSynchronize(B->stream));
  B->h_inst.assign(B->slot.size(), Inst{});
  B->h_work.clear();
  B->h_cols.clear();
  B->h_fill.clear();
  B->h_range.assign(BATCH_RANGE * N_BATCH_CLASSES, 0);
  unsigned classes = 0;
  for (int cls = 0; cls < N_BATCH_CLASSES; ++cls) {
    int *rg = &B->h_range[BATCH_RANGE * cls];
    rg[0] = (int)B->h_work.size();
    rg[2] = (int)B->h_fill.size();
    rg[4] = (int)B->h_cols.size();
    std::vector<int4> rows_of_xcd[NXCD_HOST], cols_of_xcd[NXCD_HOST];
    int nrows = 0, ncolrows = 0;
    // planes per potential column: about 8 columns per CU over the class,
    // as the single-lattice potential's grid, at most 16 planes
    int64_t column_planes = 0;
    for (fre_lattice *L : B->slot)
      if (L && batch_class(L->a.q, L->a.storage) == cls)
        column_planes += (int64_t)((L->a.G.ex + 63) / 64) * ((L->a.G.ey + B->rows - 1) / B->rows) * L->a.G.ez;
    const int64_t target = 8 * (int64_t)B->ncu;
    const int tz = (int)std::max<int64_t>(1, std::min<int64_t>(16, (column_planes + target - 1) / target));
    rg[6] = tz;
    for (size_t k = 0; k < B->slot.size(); ++k) {
      fre_lattice *L = B->slot[k];
      if (!L || batch_class(L->a.q, L->a.storage) != cls) continue;
      classes |= 1u << cls;
      B->h_inst[k] = inst_of(L, B->base);
      const Geom &G = L->a.G;
      const int gx = (G.ex + 63) / 64, gy = (G.ey + B->rows - 1) / B->rows;
      for (int z = 0; z < G.ez; ++z)
        for (int by = 0; by < gy; ++by) {
          auto &q = rows_of_xcd[nrows++ % NXCD_HOST];
          for (int bx = 0; bx < gx; ++bx) q.push_back(make_int4((int)k, bx, by, z));
        }
      for (int z = 0; z < G.ez; z += tz)
        for (int by = 0; by < gy; ++by) {
          auto &q = cols_of_xcd[ncolrows++ % NXCD_HOST];
          for (int bx = 0; bx < gx; ++bx) q.push_back(make_int4((int)k, bx, by, z));
        }
      for (int s : L->fill_host) B->h_fill.push_back(make_int2((int)k, s));
    }
    xcd_interleave(rows_of_xcd, B->h_work);
    xcd_interleave(cols_of_xcd, B->h_cols);
    rg[1] = (int)B->h_work.size() - rg[0];
    rg[3] = (int)B->h_fill.size() - rg[2];
    rg[5] = (int)B->h_cols.size() - rg[4];
  }
  if ((int64_t)B->h_work.size() > B->cap_work || (int64_t)B->h_fill.size() > B->cap_fill)
    return fail(FRE_ENOMEM, "batch work lists exceed their capacity (%zu/%d cells, %zu/%d fills)",
                B->h_work.size(), B->cap_work, B->h_fill.size(), B->cap_fill);
  if (!B->h_inst.empty())
    HIP_TRY(hipMemcpyAsync(B->d_inst, B->h_inst.data(), B->h_inst.size() * sizeof(Inst), hipMemcpyHostToDevice, B->stream));
  if (!B->h_work.empty())
    HIP_TRY(hipMemcpyAsync(B->d_work, B->h_work.data(), B->h_work.size() * sizeof(int4), hipMemcpyHostToDevice, B->stream));
  if (!B->h_cols.empty())
    HIP_TRY(hipMemcpyAsync(B->d_cols, B->h_cols.data(), B->h_cols.size() * sizeof(int4), hipMemcpyHostToDevice, B->stream));
  if (!B->h_fill.empty())
    HIP_TRY(hipMemcpyAsync(B->d_fill, B->h_fill.data(), B->h_fill.size() * sizeof(int2), hipMemcpyHostToDevice, B->stream));
  HIP_TRY(hipMemcpyAsync(B->d_range, B->h_range.data(), BATCH_RANGE * N_BATCH_CLASSES * sizeof(int), hipMemcpyHostToDevice, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  if (classes != B->classes) batch_reset_graph(B);  // the graph launches one sequence per class
  B->classes = classes;
  return FRE_OK;
}

BatchArgs batch_args(const fre_batch *B) {
  BatchArgs b;
  b.base = (char *)B->base;
  b.inst = B->d_inst;
  b.work = B->d_work;
  b.cols = B->d_cols;
  b.fill = B->d_fill;
  b.range = B->d_range;
  b.grid_cells = B->grid_cells;
  b.grid_fill = B->grid_fill;
  b.grid_cols = 8 * B->ncu;
  b.rows = B->rows;
  b.stream = B->stream;
  return b;
}

void batch_launch_step(const fre_batch *B, int odd) {
  const BatchArgs b = batch_args(B);
  for (int cls = 0; cls < N_BATCH_CLASSES; ++cls)
    if (B->classes & (1u << cls)) launch_batch_step(b, cls, odd);
}

}  // namespace

fre_status fre_batch_footprint(int32_t max_slots, int64_t max_work, int64_t max_fill, size_t *bytes) {
  if (max_slots < 1 || max_work < 1 || max_fill < 0 || !bytes) return fail(FRE_EINVAL, "bad batch capacities");
  if (max_work > INT32_MAX || max_fill > INT32_MAX) return fail(FRE_EINVAL, "batch capacities exceed 2^31");
  *bytes = batch_plan(max_slots, max_work, max_fill).total;
  return FRE_OK;
}

fre_status fre_lattice_batch_needs(const fre_lattice *L, int64_t *n_work, int64_t *n_fill) {
  if (!L || !n_work || !n_fill) return fail(FRE_EINVAL, "NULL argument");
  lattice_needs(L, n_work, n_fill);
  return FRE_OK;
}

fre_status fre_batch_create(void *device_buf, size_t bytes, void *hip_stream, int32_t max_slots,
                            int64_t max_work, int64_t max_fill, fre_batch **out) {
  if (!out) return fail(FRE_EINVAL, "out is NULL");
  *out = nullptr;
  size_t need;
  fre_status s = fre_batch_footprint(max_slots, max_work, max_fill, &need);
  if (s != FRE_OK) return s;
  if (!device_buf || (uintptr_t)device_buf % kAlign) return fail(FRE_EINVAL, "device_buf must be 256-byte aligned");
  if (bytes < need) return fail(FRE_ENOMEM, "batch buffer of %zu bytes < %zu", bytes, need);
  const BatchPlan P = batch_plan(max_slots, max_work, max_fill);
  fre_batch *B = new fre_batch();
  B->base = (uint8_t *)device_buf;
  B->bytes = bytes;
  B->stream = (hipStream_t)hip_stream;
  B->max_slots = max_slots;
  B->cap_work = (int)max_work;
  B->cap_fill = (int)max_fill;
  B->d_inst = (Inst *)(B->base + P.o_inst);
  B->d_work = (int4 *)(B->base + P.o_work);
  B->d_cols = (int4 *)(B->base + P.o_cols);
  B->d_fill = (int2 *)(B->base + P.o_fill);
  B->d_range = (int *)(B->base + P.o_range);
  B->slot.assign(max_slots, nullptr);
  B->parity = 0;
  B->classes = 0;
  B->graph_ok = B->graph_run_ok = false;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  B->ncu = ncu;
  B->rows = COLLIDE_ROWS;
  B->blocks_per_cu = 8;
  B->grid_cells = ncu * B->blocks_per_cu;
  B->grid_fill = ncu * 2;
  s = batch_rebuild(B);
  if (s != FRE_OK) { delete B; return s; }
  *out = B;
  return FRE_OK;
}

fre_status fre_batch_add(fre_batch *B, fre_lattice *L, int32_t *slot) {
  if (!B || !L || !slot) return fail(FRE_EINVAL, "NULL argument");
  if (L->batch) return fail(FRE_EINVAL, "lattice is already a batch member");
  if (L->p.ternary) return fail(FRE_EINVAL, "ternary lattices are stepped on their own");
  if (L->p.fp16_rounding) return fail(FRE_EINVAL, "lattices with stochastic rounding are stepped on their own");
  if (L->state) return fail(FRE_ESTATE, "lattice is in the failed state");
  int free_slot = -1, members = 0;
  for (int k = 0; k < B->max_slots; ++k) {
    if (B->slot[k]) ++members;
    else if (free_slot < 0) free_slot = k;
  }
  if (free_slot < 0) return fail(FRE_ENOMEM, "batch is full (%d slots)", B->max_slots);
  // all members share the AA parity; a lattice one step out of phase takes
  // one step on its own first (the same arithmetic as inside the batch)
  if (members == 0) {
    B->parity = (int)(L->t & 1);
    batch_reset_graph(B);
  } else if ((int)(L->t & 1) != B->parity) {
    fre_status s = fre_step(L, 1);
    if (s != FRE_OK) return s;
  }
  HIP_TRY(hipStreamSynchronize(L->a.stream));
  B->slot[free_slot] = L;
  L->batch = B;
  fre_status s = batch_rebuild(B);
  if (s != FRE_OK) {
    B->slot[free_slot] = nullptr;
    L->batch = nullptr;
    (void)batch_rebuild(B);
    return s;
  }
  *slot = free_slot;
  return FRE_OK;
}

fre_status fre_batch_remove(fre_batch *B, int32_t slot) {
  if (!B || slot < 0 || slot >= B->max_slots || !B->slot[slot]) return fail(FRE_EINVAL, "no lattice in that slot");
  fre_lattice *L = B->slot[slot];
  HIP_TRY(hipStreamSynchronize(B->stream));
  B->slot[slot] = nullptr;
  L->batch = nullptr;
  return batch_rebuild(B);
}

fre_status fre_batch_step(fre_batch *B, int64_t n) {
  if (!B) return fail(FRE_EINVAL, "batch is NULL");
  if (n < 0) return fail(FRE_EINVAL, "negative step count");
  if (!B->classes || n == 0) return FRE_OK;
  for (fre_lattice *L : B->slot)
    if (L && L->state) return fail(FRE_ESTATE, "a member lattice is in the failed state");
  hipStream_t st = B->stream;
  int64_t done = 0;
  auto one = [&]() -> fre_status {
    batch_launch_step(B, B->parity);
    HIP_TRY(hipGetLastError());
    B->parity ^= 1;
    ++done;
    return FRE_OK;
  };
  fre_status s = FRE_OK;
  if (st == nullptr || n < 4) {
    for (int64_t k = 0; k < n && s == FRE_OK; ++k) s = one();
  } else {
    if (B->parity) { s = one(); --n; }
    // a graph of `pairs` even + odd step pairs
    auto capture = [&](int pairs, hipGraphExec_t *out) -> fre_status {
      hipGraph_t g;
      HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < pairs; ++k) {
        batch_launch_step(B, 0);
        batch_launch_step(B, 1);
      }
      hipError_t e = hipStreamEndCapture(st, &g);
      if (e != hipSuccess) return fail(FRE_EDEVICE, "batch graph capture failed: %s", hipGetErrorString(e));
      e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(FRE_EDEVICE, "batch graph instantiate failed: %s", hipGetErrorString(e));
      return FRE_OK;
    };
    // runs of kGraphRun steps, then pairs, as for a single lattice
    auto replay = [&](hipGraphExec_t *gx, bool *ok, int steps) {
      if (s == FRE_OK && n >= steps && !*ok) {
        s = capture(steps / 2, gx);
        *ok = s == FRE_OK;
      }
      for (; s == FRE_OK && n >= steps; n -= steps) {
        hipError_t e = hipGraphLaunch(*gx, st);
        if (e != hipSuccess) s = fail(FRE_EDEVICE, "batch graph launch failed: %s", hipGetErrorString(e));
        else done += steps;
      }
    };
    replay(&B->graph_run, &B->graph_run_ok, kGraphRun);
    replay(&B->graph, &B->graph_ok, 2);
    if (s == FRE_OK && n) s = one();
  }
  for (fre_lattice *L : B->slot)
    if (L) L->t += done;
  return s;
}

fre_status fre_batch_set_launch_shape(fre_batch *B, int32_t blocks_per_cu) {
  if (!B) return fail(FRE_EINVAL, "batch is NULL");
  if (blocks_per_cu < 1 || blocks_per_cu > 32)
    return fail(FRE_EINVAL, "bad batch launch shape (%d blocks per CU)", blocks_per_cu);
  HIP_TRY(hipStreamSynchronize(B->stream));
  B->blocks_per_cu = blocks_per_cu;
  B->grid_cells = B->ncu * blocks_per_cu;
  batch_reset_graph(B);
  return FRE_OK;
}

fre_status fre_batch_get_launch_shape(const fre_batch *B, int32_t *blocks_per_cu) {
  if (!B || !blocks_per_cu) return fail(FRE_EINVAL, "NULL argument");
  *blocks_per_cu = B->blocks_per_cu;
  return FRE_OK;
}

fre_status fre_batch_autotune(fre_batch *B, int64_t n, int32_t *blocks_per_cu, double *ms_per_step) {
  if (!B) return fail(FRE_EINVAL, "batch is NULL");
  if (n < 2 || n > 10000) return fail(FRE_EINVAL, "n must be in [2, 10000]");
  if (!B->classes) return fail(FRE_ESTATE, "batch has no members to tune on");
  for (fre_lattice *L : B->slot)
    if (L && L->state) return fail(FRE_ESTATE, "a member lattice is in the failed state");
  n += n & 1;
  HIP_TRY(hipStreamSynchronize(B->stream));
  std::vector<HostState> hs(B->slot.size());
  for (size_t k = 0; k < B->slot.size(); ++k)
    if (B->slot[k]) {
      fre_status s = snapshot(B->slot[k], hs[k]);
      if (s != FRE_OK) return s;
    }
  const int parity0 = B->parity, bpc0 = B->blocks_per_cu;
  static const int kBpc[] = {2, 4, 8, 16};
  double best = 1e300;
  int best_bpc = bpc0;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  fre_status s = FRE_OK;
  for (int bpc : kBpc) {
    if ((s = fre_batch_set_launch_shape(B, bpc)) != FRE_OK) break;
    int par = B->parity;
    for (int w = 0; w < 2; ++w, par ^= 1) batch_launch_step(B, par);
    (void)hipEventRecord(e0, B->stream);
    for (int64_t k = 0; k < n; ++k, par ^= 1) batch_launch_step(B, par);
    (void)hipEventRecord(e1, B->stream);
    hipError_t e = hipStreamSynchronize(B->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) { s = fail(FRE_EDEVICE, "batch tuning step failed: %s", hipGetErrorString(e)); break; }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms / n < best) { best = ms / n; best_bpc = bpc; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (size_t k = 0; k < B->slot.size(); ++k)
    if (B->slot[k]) {
      fre_status r = restore(B->slot[k], hs[k]);
      if (r != FRE_OK && s == FRE_OK) s = r;
    }
  B->parity = parity0;
  fre_status r = fre_batch_set_launch_shape(B, s == FRE_OK ? best_bpc : bpc0);
  if (s != FRE_OK) return s;
  if (r != FRE_OK) return r;
  if (blocks_per_cu) *blocks_per_cu = B->blocks_per_cu;
  if (ms_per_step) *ms_per_step = best;
  return FRE_OK;
}

fre_status fre_batch_info(const fre_batch *B, int32_t *members, int32_t *parity) {
  if (!B) return fail(FRE_EINVAL, "batch is NULL");
  int m = 0;
  for (fre_lattice *L : B->slot) m += L != nullptr;
  if (members) *members = m;
  if (parity) *parity = B->parity;
  return FRE_OK;
}

void fre_batch_destroy(fre_batch *B) {
  if (!B) return;
  (void)hipStreamSynchronize(B->stream);
  for (fre_lattice *L : B->slot)
    if (L) L->batch = nullptr;
  batch_reset_graph(B);
  delete B;
}

}  // extern "C"
