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
  void *f, *g;  // population planes (float or half)
  float *g0;    // FP16 storage only: g_0 plane
  uint8_t *mask;
  float2 *M;    // (rho - 1, phi)
  float2 *MU;   // (mu_rho, mu_phi)
  float *PI;    // rho mu_rho + phi mu_phi
  float4 *AUX;  // u0 at init; (ux, uy, uz, P) after observe
  int *fill_list;
  int n_fill;
  hipStream_t stream;
};

template <int S> inline Pops<S> make_pops(const LaunchArgs &a);
template <> inline Pops<0> make_pops<0>(const LaunchArgs &a) {
  Pops<0> p;
  p.f = (float *)a.f;
  p.g = (float *)a.g;
  p.np = a.G.np;
  return p;
}
template <> inline Pops<1> make_pops<1>(const LaunchArgs &a) {
  Pops<1> p;
  p.f = (__half *)a.f;
  p.g = (__half *)a.g;
  p.g0 = a.g0;
  p.np = a.G.np;
  return p;
}

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
