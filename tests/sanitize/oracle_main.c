/* Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle (test infrastructure).  The oracle source is compiled into this
 * translation unit so that its internal types are visible.  Runs binary and
 * ternary lattices with walls, moving walls, a solid box and a roller,
 * consistent initialisation, observation, population read/write and the
 * stencil probe, on lattices small enough to finish in seconds; any invalid
 * access or undefined operation aborts the process. */
#include "../../oracle/frelbm_oracle.c"

#include <stdio.h>

static void fields(long n, double *phi, double *psi, double *rho, double *u) {
  for (long k = 0; k < n; ++k) {
    phi[k] = (k % 7 < 3) ? 0.9 : -0.9;
    if (psi) psi[k] = 0.1 * (double)(k % 5) / 5.0;
    rho[k] = 1.0 + 0.001 * (double)(k % 3);
    u[k] = 0.002 * (double)(k % 4);
    u[n + k] = -0.001 * (double)(k % 2);
    u[2 * n + k] = 0.0;
  }
}

static int run(int kind, int nx, int ny, int nz, int with_mask, int ternary) {
  or_params p;
  memset(&p, 0, sizeof p);
  p.kind = kind;
  p.nx = nx; p.ny = ny; p.nz = nz;
  p.bc[1] = 1;
  if (kind == 1) p.bc[2] = 1;
  p.wall_u[1][0][0] = -0.01;
  p.wall_u[1][1][0] = 0.01;
  p.kappa1 = 0.16; p.kappa2 = 0.12; p.alpha = 1.0;
  p.tau_f = 0.8; p.tau_g = 1.1; p.M = 0.1;
  long n = (long)nx * ny * nz;
  double *phi = calloc(n, sizeof(double)), *psi = calloc(n, sizeof(double));
  double *rho = calloc(n, sizeof(double)), *u = calloc(3 * n, sizeof(double));
  uint8_t *mask = calloc(n, 1);
  fields(n, phi, psi, rho, u);
  if (kind == 0) for (long k = 0; k < n; ++k) u[2 * n + k] = 0.0;
  if (with_mask) {
    mask[nx / 2 + (long)nx * (ny / 2)] = 1;
    p.n_rollers = 1;
    p.roller_center[0][0] = 1.5; p.roller_center[0][1] = 1.5;
    p.roller_omega[0] = 0.01;
    p.roller_axis[0] = 2;
    mask[1 + (long)nx * 1] = 2;
    mask[2 + (long)nx * 1] = 2;
  }
  or_state *s = ternary ? or3_create(&p, 0.2, 0.07, 0.9, mask, phi, psi, rho, u)
                        : or_create(&p, mask, phi, rho, u);
  if (!s) { fprintf(stderr, "create failed\n"); return 1; }
  const int q = kind == 0 ? 9 : 19;
  double *obs = calloc((size_t)11 * n, sizeof(double));
  double *f = calloc((size_t)q * n, sizeof(double)), *g = calloc((size_t)q * n, sizeof(double));
  double *h = calloc((size_t)q * n, sizeof(double));
  if (ternary) {
    or3_step(s, 7);
    or3_observe(s, obs);
    or3_get_populations(s, f, g, h);
  } else {
    if (or_consistent_init(s, phi, u, 4) != 0) { fprintf(stderr, "consistent init failed\n"); return 1; }
    or_step(s, 7);
    or_observe(s, obs);
    or_get_populations(s, f, g);
    or_set_populations(s, f, g);
    or_step(s, 1);
    double *lap = calloc(n, sizeof(double)), *grad = calloc(3 * n, sizeof(double));
    or_stencils(s, phi, lap, grad);
    free(lap); free(grad);
  }
  double acc = 0.0;
  for (long k = 0; k < n; ++k) acc += obs[n + k];
  printf("kind=%d %dx%dx%d mask=%d ternary=%d t=%ld sum_phi=%.6f\n", kind, nx, ny, nz, with_mask, ternary,
         or_time(s), acc);
  or_destroy(s);
  free(phi); free(psi); free(rho); free(u); free(mask); free(obs); free(f); free(g); free(h);
  return 0;
}

int main(void) {
  int bad = 0;
  bad |= run(0, 7, 6, 1, 0, 0);
  bad |= run(0, 9, 8, 1, 1, 0);
  bad |= run(1, 5, 6, 4, 0, 0);
  bad |= run(1, 1, 1, 1, 0, 0);
  bad |= run(0, 8, 7, 1, 1, 1);
  bad |= run(1, 5, 4, 3, 0, 1);
  /* invalid geometry is refused, not read out of bounds */
  or_params z;
  memset(&z, 0, sizeof z);
  z.kind = 0; z.nx = 4; z.ny = 4; z.nz = 2;
  if (or_create_geometry(&z, NULL) != NULL) { fprintf(stderr, "bad geometry accepted\n"); bad = 1; }
  printf(bad ? "FAILED\n" : "OK\n");
  return bad;
}
