// kernels.h -- launch interface between the host library and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "lbm_device.h"

namespace frelbm {

// Everything one launch sequence needs; all pointers are device pointers
// carved from the caller's buffer.
struct LaunchArgs {
  int q;        // 9 or 19
  int storage;  // 0 FP32, 1 FP16
  Geom G;
  Phys ph;
  void *f, *g;  // population blocks (float or half)
  float *g0;    // FP16 storage only: g_0 plane
  uint8_t *mask;
  uint32_t *nbm;  // per cell: non-fluid neighbour bits, NB_SELF_SOLID
  float2 *M;    // (rho - 1, phi)
  float4 *C;    // (rho - 1, phi, Pi = rho mu_rho + phi mu_phi, mu_rho)
  float *MUP;   // mu_phi
  float4 *AUX;  // u0 at init; (ux, uy, uz, P) after observe
  int *fill_list;
  int n_fill;
  hipStream_t stream;
};

template <int Q, int S> inline Pops<Q, S> make_pops(const LaunchArgs &a);
template <> inline Pops<9, 0> make_pops<9, 0>(const LaunchArgs &a) { return Pops<9, 0>{(float *)a.f, (float *)a.g}; }
template <> inline Pops<19, 0> make_pops<19, 0>(const LaunchArgs &a) { return Pops<19, 0>{(float *)a.f, (float *)a.g}; }
template <> inline Pops<9, 1> make_pops<9, 1>(const LaunchArgs &a) { return Pops<9, 1>{(__half *)a.f, (__half *)a.g, a.g0}; }
template <> inline Pops<19, 1> make_pops<19, 1>(const LaunchArgs &a) { return Pops<19, 1>{(__half *)a.f, (__half *)a.g, a.g0}; }

void launch_step(const LaunchArgs &a, int odd);
void launch_step_events(const LaunchArgs &a, int odd, hipEvent_t *ev);
int step_kernel_count();
const char *step_kernel_name(int k);
void launch_observe(const LaunchArgs &a, int odd);
void launch_init(const LaunchArgs &a);
void launch_read_pops(const LaunchArgs &a, int odd, float *out);
int reduce_blocks();
void launch_reduce(const LaunchArgs &a, double *part);

}  // namespace frelbm
