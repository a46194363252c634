// Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
// library's host code (test infrastructure): parameter validation, the
// buffer plan, the batch plan, argument checks and error reporting, through
// the C ABI, with no device present.  Every call here must fail or succeed
// before any device work; an invalid access or undefined operation aborts.
#include <cstdio>
#include <cstring>

#include "../../include/frelbm.h"

static int bad = 0;

#define EXPECT(cond)                                                      \
  do {                                                                    \
    if (!(cond)) {                                                        \
      std::fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond, fre_last_error()); \
      bad = 1;                                                            \
    }                                                                     \
  } while (0)

static fre_params base(int kind, int nx, int ny, int nz) {
  fre_params p;
  std::memset(&p, 0, sizeof p);
  p.kind = kind;
  p.nx = nx; p.ny = ny; p.nz = nz;
  p.A = 0.04; p.kappa = 0.09;
  p.tau_f = 1.0; p.tau_g = 1.0; p.M = 0.1;
  return p;
}

int main() {
  size_t b = 0, b16 = 0, b3 = 0;
  // valid shapes, both velocity sets, both storages, ragged rows, walls
  const int shapes[][4] = {{0, 1, 1, 1}, {0, 65, 3, 1}, {0, 400, 200, 1}, {1, 1, 1, 1}, {1, 130, 9, 7},
                           {1, 256, 128, 128}, {1, 63, 1, 2}};
  for (const auto &s : shapes)
    for (int st = 0; st < 2; ++st)
      for (int wall = 0; wall < 2; ++wall) {
        fre_params p = base(s[0], s[1], s[2], s[3]);
        p.storage = st;
        p.bc[1] = wall;
        if (s[0] == 1) p.bc[2] = wall;
        EXPECT(fre_footprint(&p, &b) == FRE_OK && b > 0);
      }
  fre_params p = base(1, 64, 32, 32);
  EXPECT(fre_footprint(&p, &b) == FRE_OK);
  p.storage = FRE_FP16;
  EXPECT(fre_footprint(&p, &b16) == FRE_OK && b16 < b);
  p = base(1, 64, 32, 32);
  p.ternary = 1; p.kappa3 = 0.1; p.M3 = 0.05; p.tau_h = 1.0;
  EXPECT(fre_footprint(&p, &b3) == FRE_OK && b3 > b);
  // refusals
  fre_params q;
  q = base(2, 8, 8, 1); EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(0, 8, 8, 2); EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 0, 8, 8); EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 8, -3, 8); EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 1 << 20, 1 << 20, 1 << 20); EXPECT(fre_footprint(&q, &b) != FRE_OK);
  q = base(1, 256, 256, 863); EXPECT(fre_footprint(&q, &b) != FRE_OK);
  q = base(1, 8, 8, 8); q.tau_f = 0.5; EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 8, 8, 8); q.M = -1.0; EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 8, 8, 8); q.storage = 9; EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 8, 8, 8); q.bc[0] = 3; EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 8, 8, 8); q.n_rollers = 5; EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 8, 8, 8); q.n_rollers = 1; q.rollers[0].axis = 4; EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 8, 8, 8); q.wall_u[0][0][0] = 1.0; EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 8, 8, 8); q.A = 0.0 / 0.0; EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 8, 8, 8); q.ternary = 2; EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 8, 8, 8); q.ternary = 1; q.kappa3 = 0.1; q.tau_h = 0.4; EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  q = base(1, 8, 8, 8); q.ternary = 1; q.kappa3 = 0.1; q.tau_h = 1.0; q.storage = FRE_FP16;
  EXPECT(fre_footprint(&q, &b) == FRE_EINVAL);
  EXPECT(fre_footprint(nullptr, &b) == FRE_EINVAL);
  EXPECT(fre_footprint(&p, nullptr) == FRE_EINVAL);
  // entry points refuse NULL handles and buffers before any device work
  fre_lattice *L = reinterpret_cast<fre_lattice *>(1);
  fre_params ok = base(1, 8, 8, 8);
  double phi[512] = {0};
  EXPECT(fre_lattice_init(&ok, nullptr, 1 << 20, nullptr, phi, nullptr, nullptr, nullptr, &L) == FRE_EINVAL);
  EXPECT(L == nullptr);
  EXPECT(fre_lattice_init(&ok, reinterpret_cast<void *>(0x1001), 1 << 20, nullptr, phi, nullptr, nullptr, nullptr,
                          &L) == FRE_EINVAL);
  EXPECT(fre_lattice_init(&ok, reinterpret_cast<void *>(0x1000), 16, nullptr, phi, nullptr, nullptr, nullptr, &L) ==
         FRE_ENOMEM);
  EXPECT(fre_lattice_init(&p, reinterpret_cast<void *>(0x1000), 16, nullptr, phi, nullptr, nullptr, nullptr, &L) ==
         FRE_EINVAL);
  EXPECT(fre_lattice_init3(&ok, reinterpret_cast<void *>(0x1000), 16, nullptr, phi, phi, nullptr, nullptr, nullptr,
                           &L) == FRE_EINVAL);
  EXPECT(fre_lattice_init3(&p, reinterpret_cast<void *>(0x1000), 16, nullptr, phi, nullptr, nullptr, nullptr,
                           nullptr, &L) == FRE_EINVAL);
  EXPECT(fre_step(nullptr, 1) == FRE_EINVAL);
  EXPECT(fre_read_moments(nullptr, FRE_F_PHI, phi, 512) == FRE_EINVAL);
  EXPECT(fre_read_populations(nullptr, phi, phi, 512) == FRE_EINVAL);
  EXPECT(fre_read_populations3(nullptr, phi, phi, phi, 512) == FRE_EINVAL);
  double out[8];
  EXPECT(fre_reduce(nullptr, out) == FRE_EINVAL);
  EXPECT(fre_reduce_noalloc(nullptr, out) == FRE_EINVAL);
  int64_t t;
  int32_t st;
  EXPECT(fre_info(nullptr, &t, &st) == FRE_EINVAL);
  EXPECT(fre_state_bytes(nullptr, &b) == FRE_EINVAL);
  EXPECT(fre_load(nullptr, phi, sizeof phi) == FRE_EINVAL);
  int32_t cfg[6];
  EXPECT(fre_get_launch_shape(nullptr, cfg) == FRE_EINVAL);
  EXPECT(fre_set_launch_shape(nullptr, cfg) == FRE_EINVAL);
  EXPECT(fre_autotune(nullptr, 4, cfg, nullptr) == FRE_EINVAL);
  EXPECT(fre_consistent_init(nullptr, phi, nullptr, 2) == FRE_EINVAL);
  fre_lattice_destroy(nullptr);
  // batch plan
  EXPECT(fre_batch_footprint(4, 1000, 100, &b) == FRE_OK && b > 0);
  EXPECT(fre_batch_footprint(0, 1000, 100, &b) == FRE_EINVAL);
  EXPECT(fre_batch_footprint(4, -1, 100, &b) == FRE_EINVAL);
  fre_batch *B = reinterpret_cast<fre_batch *>(1);
  EXPECT(fre_batch_create(nullptr, 1 << 20, nullptr, 4, 1000, 100, &B) == FRE_EINVAL);
  EXPECT(fre_batch_step(nullptr, 1) == FRE_EINVAL);
  EXPECT(fre_batch_remove(nullptr, 0) == FRE_EINVAL);
  fre_batch_destroy(nullptr);
  // kernel names: every slot named, NULL beyond the last and below 0
  int named = 0;
  for (int k = -2; k < 40; ++k) {
    const char *n = fre_kernel_name(k);
    if (n) {
      EXPECT(k >= 0 && std::strlen(n) > 0);
      ++named;
    }
  }
  EXPECT(named >= 6);
  EXPECT(std::strlen(fre_last_error()) > 0);
  std::printf(bad ? "FAILED\n" : "OK\n");
  return bad;
}
