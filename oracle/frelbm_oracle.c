/*
 * frelbm_oracle.c -- plain FP64 CPU oracle of the free-energy lattice Boltzmann
 * (FRE LBM) time step for a binary mixture: a Navier-Stokes population f (BGK
 * collision with Guo forcing) and a Cahn-Hilliard population g (BGK collision
 * towards the chemical-potential equilibrium), coupled by the thermodynamic
 * force F = -rho grad(mu_rho) - phi grad(mu_phi).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU library.
 *
 * Written for clarity, not speed: IEEE FP64, no FMA contraction
 * (-ffp-contract=off), two population buffers with push streaming, AoS layout
 * f[cell*q + i], OpenMP only over independent per-cell loops.
 *
 * Paper: Simonis, Nguyen, Avis, Doerfler, Krause, "Binary mixture flow with
 * free energy lattice Boltzmann methods" (arXiv 2212.01617).
 *   Sec. 2.2, eq. (LBE) + (bgk)           f_i(x+c_i,t+1) = f_i - (f_i-f_i^eq)/tau + S_i
 *   Sec. 2.2, eq. (feq)                   second-order equilibrium of f
 *   Sec. 2.2, eq. (Fi)                    Guo forcing term S_i
 *   Sec. 2.2, eqs. (densMoment, veloMoment)  rho = sum f, rho u = sum c f + F/2
 *   Sec. 2.2, eq. (F)                     F = -rho grad mu_rho - phi grad mu_phi
 *   Sec. 2.2, eqs. (mu_rho, mu_phi)       chemical potentials of the functional
 *   Sec. 2.2, eq. (ordeMoment), (LBEg), (geq)  g population and its equilibrium
 *   Sec. 2.2, mobility relation           M = Gamma (tau_g - 1/2)
 *   Sec. 2.3                              collide/stream split, equilibrium init
 *   Algorithm 1                           order of the per-node computation
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - Laplacian and gradient: isotropic lattice-weighted stencils over the
 *     same neighbour set as the velocity set,
 *       lap X(x)  = (2/cs^2) sum_{i!=0} w_i [X(x+c_i) - X(x)]
 *       grad X(x) = (1/cs^2) sum_i w_i c_i X(x+c_i).
 *   - Force discretisation: eq. (F) is applied through the product-rule
 *     identity -rho grad mu_rho - phi grad mu_phi
 *         = mu_rho grad rho + mu_phi grad phi - grad(rho mu_rho + phi mu_phi),
 *     every gradient taken with the stencil above.  Both sides are equal in
 *     the continuum; the left side discretised directly with central
 *     differences feeds the undamped odd-even (Nyquist) velocity mode of BGK
 *     and grows without bound at strong interfaces (e.g. A = 0.04,
 *     kappa = 0.09, tau = 1), the right side does not.
 *   - Solid cells (walls, rollers, obstacles) take, for the stencils, the
 *     lattice-weighted mean of their fluid neighbours; this applies to every
 *     field a stencil reads there: rho, phi and Pi = rho mu_rho + phi mu_phi.
 *   - Velocity boundaries: halfway bounce-back with the moving-wall term,
 *       f_ib(x,t+1) = f_i*(x) - 2 w_i rho(x) (c_i.u_w)/cs^2,
 *       g_ib(x,t+1) = g_i*(x) - 2 w_i phi(x) (c_i.u_w)/cs^2,
 *     u_w being the body velocity at the link midpoint x + c_i/2.
 *   - A WALL axis is closed by one layer of solid ghost cells at each end
 *     (the wall sits halfway between the last fluid node and the ghost).
 *     A ghost cell lying in the ghost layers of several axes moves with the
 *     mean of those walls' velocities.
 *   - Initialisation: f = f^eq(rho0,u0), g = g^eq(phi0, mu_phi(rho0,phi0), u0).
 *   - Three components (Sec. 2.2, Remark after the mobility relation): the
 *     free energy of the cited ternary model, see the or3_ functions at the
 *     end of this file.
 *   - Consistent initialisation (Sec. 2.3 cites Mei, Luo, Lallemand and
 *     d'Humieres 2006, without details): pre-iterations of the f population
 *     in which the velocity of the equilibrium and of the forcing term is
 *     held at the prescribed u0 and phi at phi0, while rho evolves and the
 *     non-equilibrium part of f develops; g is not stepped.  Afterwards g is
 *     reset to g^eq(phi0, mu_phi(rho, phi0), u0) with the new rho.  The time
 *     counter stays at 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXQ 19

/* ---------------------------------------------------------------------- */
/* Velocity sets (project ordering: rest first, then opposite pairs adjacent,
 * so that the opposite of i is i+1 for odd i and i-1 for even i > 0).      */
/* ---------------------------------------------------------------------- */
static const int OR_C9[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
static const double OR_W9[9] = {
    4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static const int OR_C19[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double OR_W19[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

#define CS2 (1.0 / 3.0)

static int or_q(int kind) { return kind == 0 ? 9 : 19; }
static const int (*or_c(int kind))[3] { return kind == 0 ? OR_C9 : OR_C19; }
static const double *or_w(int kind) { return kind == 0 ? OR_W9 : OR_W19; }
static int or_opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

/* Copy the velocity set out (for the lattice-table tests). */
int or_tables(int kind, int *q, int *c_out, double *w_out) {
  if (kind != 0 && kind != 1) return -1;
  int n = or_q(kind);
  const int(*c)[3] = or_c(kind);
  const double *w = or_w(kind);
  *q = n;
  for (int i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) c_out[3 * i + a] = c[i][a];
    w_out[i] = w[i];
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Per-node formulas                                                       */
/* ---------------------------------------------------------------------- */

/* Sec. 2.2, eq. (feq): f_i^eq = w_i rho [1 + c.u/cs^2
 *                                + u_a u_b (c_a c_b - cs^2 delta_ab)/(2 cs^4)] */
void or_feq(int kind, double rho, const double u[3], double *out) {
  int q = or_q(kind);
  const int(*c)[3] = or_c(kind);
  const double *w = or_w(kind);
  for (int i = 0; i < q; ++i) {
    double cu = c[i][0] * u[0] + c[i][1] * u[1] + c[i][2] * u[2];
    double quad = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double d = (a == b) ? 1.0 : 0.0;
        quad += u[a] * u[b] * (c[i][a] * c[i][b] - CS2 * d);
      }
    out[i] = w[i] * rho * (1.0 + cu / CS2 + quad / (2.0 * CS2 * CS2));
  }
}

/* Sec. 2.2, eq. (Fi), Guo forcing:
 * S_i = (1 - 1/(2 tau)) w_i [ (c_i - u)/cs^2 + (c_i.u) c_i / cs^4 ] . F   */
void or_guo(int kind, double tau, const double u[3], const double F[3],
            double *out) {
  int q = or_q(kind);
  const int(*c)[3] = or_c(kind);
  const double *w = or_w(kind);
  for (int i = 0; i < q; ++i) {
    double cu = c[i][0] * u[0] + c[i][1] * u[1] + c[i][2] * u[2];
    double s = 0.0;
    for (int a = 0; a < 3; ++a)
      s += ((c[i][a] - u[a]) / CS2 + cu * c[i][a] / (CS2 * CS2)) * F[a];
    out[i] = (1.0 - 1.0 / (2.0 * tau)) * w[i] * s;
  }
}

/* Sec. 2.2, eq. (geq): for i != 0
 *   g_i^eq = w_i [ Gamma mu_phi/cs^2 + phi c.u/cs^2
 *                  + phi u_a u_b (c_a c_b - cs^2 delta_ab)/(2 cs^4) ]
 * and g_0^eq = phi - sum_{i!=0} g_i^eq.                                    */
void or_geq(int kind, double phi, double mu_phi, double Gamma,
            const double u[3], double *out) {
  int q = or_q(kind);
  const int(*c)[3] = or_c(kind);
  const double *w = or_w(kind);
  double rest = 0.0;
  for (int i = 1; i < q; ++i) {
    double cu = c[i][0] * u[0] + c[i][1] * u[1] + c[i][2] * u[2];
    double quad = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double d = (a == b) ? 1.0 : 0.0;
        quad += u[a] * u[b] * (c[i][a] * c[i][b] - CS2 * d);
      }
    out[i] = w[i] * (Gamma * mu_phi / CS2 + phi * cu / CS2 +
                     phi * quad / (2.0 * CS2 * CS2));
    rest += out[i];
  }
  out[0] = phi - rest;
}

/* Sec. 2.2, eqs. (mu_rho) and (mu_phi).  out[0] = mu_rho, out[1] = mu_phi. */
void or_mu(double kappa1, double kappa2, double alpha, double rho, double phi,
           double lap_rho, double lap_phi, double *out) {
  double s = rho + phi, t = rho - phi;
  double ps = s * (s - 2.0) * (s - 1.0);
  double pt = t * (t - 2.0) * (t - 1.0);
  double a2 = alpha * alpha;
  out[0] = kappa1 / 8.0 * ps + kappa2 / 8.0 * pt +
           a2 / 4.0 * ((kappa1 + kappa2) * (-lap_rho) + (kappa2 - kappa1) * lap_phi);
  out[1] = kappa1 / 8.0 * ps - kappa2 / 8.0 * pt +
           a2 / 4.0 * ((kappa1 + kappa2) * (-lap_phi) + (kappa2 - kappa1) * lap_rho);
}

/* Bulk part of the free-energy density of eq. (functional) (gradient terms
 * dropped): psi_b = kappa1/32 s^2 (s-2)^2 + kappa2/32 t^2 (t-2)^2.         */
static double or_psi_bulk(double kappa1, double kappa2, double rho,
                          double phi) {
  double s = rho + phi, t = rho - phi;
  return kappa1 / 32.0 * s * s * (s - 2.0) * (s - 2.0) +
         kappa2 / 32.0 * t * t * (t - 2.0) * (t - 2.0);
}

/* ---------------------------------------------------------------------- */
/* Lattice state                                                           */
/* ---------------------------------------------------------------------- */

typedef struct {
  int32_t kind;           /* 0 = D2Q9, 1 = D3Q19 */
  int32_t nx, ny, nz;     /* fluid domain (nz = 1 for D2Q9) */
  int32_t bc[3];          /* 0 periodic, 1 wall at both ends of the axis */
  double wall_u[3][2][3]; /* [axis][low, high][component] */
  int32_t n_rollers;      /* cells with mask code 2+k move with roller k */
  double roller_center[4][3];
  double roller_omega[4];
  int32_t roller_axis[4];
  double kappa1, kappa2, alpha; /* free-energy parameters, eq. (functional) */
  double tau_f, tau_g, M;       /* relaxation times and mobility */
} or_params;

enum { OR_FLUID = 0, OR_STATIC = 1, OR_ROLLER0 = 2, OR_GHOST = 8 };

typedef struct {
  or_params p;
  int q;
  int ext[3];  /* extended grid (fluid domain + ghost layers on wall axes) */
  int off[3];  /* ghost offset per axis */
  long ncell;  /* cells of the extended grid */
  uint8_t *kind;
  double *f, *g, *fn, *gn;       /* populations, [cell*q + i] */
  double *rho, *phi, *jx, *jy, *jz;
  double *lr, *lp;               /* laplacians */
  double *mur, *mup;             /* chemical potentials */
  double *pi;                    /* rho mu_rho + phi mu_phi */
  double *Fx, *Fy, *Fz, *ux, *uy, *uz;
  long t;
  /* ternary extension (or3_*): third order parameter psi and its population
   * h; NULL / 0 for a binary lattice */
  int ternary;
  double kappa3, M3, tau_h;
  double *h, *hn, *psi, *lq, *muq;
} or_state;

static long or_idx(const or_state *s, int x, int y, int z) {
  return (long)x + (long)s->ext[0] * ((long)y + (long)s->ext[1] * (long)z);
}

static void or_xyz(const or_state *s, long cell, int *x, int *y, int *z) {
  *x = (int)(cell % s->ext[0]);
  long r = cell / s->ext[0];
  *y = (int)(r % s->ext[1]);
  *z = (int)(r / s->ext[1]);
}

/* Neighbour of `cell` along direction i: periodic axes wrap, wall axes end at
 * the ghost layer (returns -1 beyond it). */
static long or_nb(const or_state *s, long cell, int i) {
  int x[3];
  or_xyz(s, cell, &x[0], &x[1], &x[2]);
  const int(*c)[3] = or_c(s->p.kind);
  for (int a = 0; a < 3; ++a) {
    int v = x[a] + c[i][a];
    if (s->p.bc[a] == 0) {
      v = ((v % s->ext[a]) + s->ext[a]) % s->ext[a];
    } else if (v < 0 || v >= s->ext[a]) {
      return -1;
    }
    x[a] = v;
  }
  return or_idx(s, x[0], x[1], x[2]);
}

/* Velocity of the solid body that owns solid cell `sc`, evaluated at the
 * midpoint of the link from fluid cell `fc` along direction i. */
static void or_body_velocity(const or_state *s, long fc, long sc, int i,
                             double uw[3]) {
  uw[0] = uw[1] = uw[2] = 0.0;
  int k = s->kind[sc];
  if (k == OR_STATIC) return;
  if (k == OR_GHOST) {
    int x[3], n = 0;
    or_xyz(s, sc, &x[0], &x[1], &x[2]);
    for (int a = 0; a < 3; ++a) {
      if (s->p.bc[a] != 1) continue;
      int side = -1;
      if (x[a] == 0) side = 0;
      if (x[a] == s->ext[a] - 1) side = 1;
      if (side < 0) continue;
      for (int b = 0; b < 3; ++b) uw[b] += s->p.wall_u[a][side][b];
      ++n;
    }
    if (n > 1)
      for (int b = 0; b < 3; ++b) uw[b] /= n;
    return;
  }
  int r = k - OR_ROLLER0;
  if (r < 0 || r >= s->p.n_rollers) return;
  int x[3];
  or_xyz(s, fc, &x[0], &x[1], &x[2]);
  const int(*c)[3] = or_c(s->p.kind);
  double pt[3], d[3];
  for (int a = 0; a < 3; ++a) {
    pt[a] = (double)(x[a] - s->off[a]) + 0.5 * c[i][a];
    d[a] = pt[a] - s->p.roller_center[r][a];
  }
  double om = s->p.roller_omega[r];
  switch (s->p.roller_axis[r]) {
    case 0: uw[1] = -om * d[2]; uw[2] = om * d[1]; break;
    case 1: uw[0] = om * d[2]; uw[2] = -om * d[0]; break;
    default: uw[0] = -om * d[1]; uw[1] = om * d[0]; break;
  }
}

/* Solid cells take the lattice-weighted mean of their fluid neighbours. */
static void or_fill_solid(const or_state *s, double *X) {
  const double *w = or_w(s->p.kind);
#pragma omp parallel for schedule(static)
  for (long sc = 0; sc < s->ncell; ++sc) {
    if (s->kind[sc] == OR_FLUID) continue;
    double num = 0.0, den = 0.0;
    for (int i = 1; i < s->q; ++i) {
      long n = or_nb(s, sc, i);
      if (n < 0 || s->kind[n] != OR_FLUID) continue;
      num += w[i] * X[n];
      den += w[i];
    }
    X[sc] = den > 0.0 ? num / den : 0.0;
  }
}

static double or_lap_at(const or_state *s, const double *X, long cell) {
  const double *w = or_w(s->p.kind);
  double acc = 0.0;
  for (int i = 1; i < s->q; ++i) {
    long n = or_nb(s, cell, i);
    acc += w[i] * (X[n] - X[cell]);
  }
  return 2.0 / CS2 * acc;
}

static void or_grad_at(const or_state *s, const double *X, long cell,
                       double g[3]) {
  const double *w = or_w(s->p.kind);
  const int(*c)[3] = or_c(s->p.kind);
  g[0] = g[1] = g[2] = 0.0;
  for (int i = 0; i < s->q; ++i) {
    long n = or_nb(s, cell, i);
    for (int a = 0; a < 3; ++a) g[a] += w[i] * c[i][a] * X[n];
  }
  for (int a = 0; a < 3; ++a) g[a] /= CS2;
}

/* Moments at fluid cells (eqs. densMoment, ordeMoment, first moment). */
static void or_moments(or_state *s) {
  const int(*c)[3] = or_c(s->p.kind);
#pragma omp parallel for schedule(static)
  for (long x = 0; x < s->ncell; ++x) {
    if (s->kind[x] != OR_FLUID) {
      s->rho[x] = s->phi[x] = s->jx[x] = s->jy[x] = s->jz[x] = 0.0;
      continue;
    }
    double r = 0.0, p = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < s->q; ++i) {
      double fi = s->f[x * s->q + i];
      r += fi;
      p += s->g[x * s->q + i];
      for (int a = 0; a < 3; ++a) j[a] += c[i][a] * fi;
    }
    s->rho[x] = r;
    s->phi[x] = p;
    s->jx[x] = j[0];
    s->jy[x] = j[1];
    s->jz[x] = j[2];
  }
}

/* Chemical potentials from the current rho, phi; also Pi = rho mu_rho +
 * phi mu_phi.  Fills solid cells of rho, phi and Pi as a side effect. */
static void or_potentials(or_state *s) {
  or_fill_solid(s, s->rho);
  or_fill_solid(s, s->phi);
#pragma omp parallel for schedule(static)
  for (long x = 0; x < s->ncell; ++x) {
    if (s->kind[x] != OR_FLUID) continue;
    s->lr[x] = or_lap_at(s, s->rho, x);
    s->lp[x] = or_lap_at(s, s->phi, x);
    double mu[2];
    or_mu(s->p.kappa1, s->p.kappa2, s->p.alpha, s->rho[x], s->phi[x],
          s->lr[x], s->lp[x], mu);
    s->mur[x] = mu[0];
    s->mup[x] = mu[1];
    s->pi[x] = s->rho[x] * mu[0] + s->phi[x] * mu[1];
  }
  or_fill_solid(s, s->pi);
}

/* Force (eq. F, product-rule form) and velocity (eq. veloMoment) at fluid
 * cells. */
static void or_force_velocity(or_state *s) {
#pragma omp parallel for schedule(static)
  for (long x = 0; x < s->ncell; ++x) {
    if (s->kind[x] != OR_FLUID) {
      s->Fx[x] = s->Fy[x] = s->Fz[x] = 0.0;
      s->ux[x] = s->uy[x] = s->uz[x] = 0.0;
      continue;
    }
    double gr[3], gp[3], gpi[3];
    or_grad_at(s, s->rho, x, gr);
    or_grad_at(s, s->phi, x, gp);
    or_grad_at(s, s->pi, x, gpi);
    double F[3];
    for (int a = 0; a < 3; ++a)
      F[a] = s->mur[x] * gr[a] + s->mup[x] * gp[a] - gpi[a];
    s->Fx[x] = F[0];
    s->Fy[x] = F[1];
    s->Fz[x] = F[2];
    s->ux[x] = (s->jx[x] + 0.5 * F[0]) / s->rho[x];
    s->uy[x] = (s->jy[x] + 0.5 * F[1]) / s->rho[x];
    s->uz[x] = (s->jz[x] + 0.5 * F[2]) / s->rho[x];
  }
}

/* ---------------------------------------------------------------------- */
/* Public API                                                              */
/* ---------------------------------------------------------------------- */

static void *or_zalloc(size_t n) { return calloc(n ? n : 1, 1); }

void or_destroy(or_state *s) {
  if (!s) return;
  free(s->h); free(s->hn); free(s->psi); free(s->lq); free(s->muq);
  free(s->kind); free(s->f); free(s->g); free(s->fn); free(s->gn);
  free(s->rho); free(s->phi); free(s->jx); free(s->jy); free(s->jz);
  free(s->lr); free(s->lp); free(s->mur); free(s->mup); free(s->pi);
  free(s->Fx); free(s->Fy); free(s->Fz); free(s->ux); free(s->uy); free(s->uz);
  free(s);
}

/* Geometry only: builds the extended grid and the cell kinds from the
 * fluid-domain mask (0 fluid, 1 static solid, 2+k roller k). */
or_state *or_create_geometry(const or_params *p, const uint8_t *mask) {
  if (p->kind != 0 && p->kind != 1) return NULL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
  if (p->kind == 0 && (p->nz != 1 || p->bc[2] != 0)) return NULL;
  or_state *s = (or_state *)or_zalloc(sizeof(or_state));
  s->p = *p;
  s->q = or_q(p->kind);
  int n[3] = {p->nx, p->ny, p->nz};
  s->ncell = 1;
  for (int a = 0; a < 3; ++a) {
    s->off[a] = p->bc[a] == 1 ? 1 : 0;
    s->ext[a] = n[a] + 2 * s->off[a];
    s->ncell *= s->ext[a];
  }
  size_t nc = (size_t)s->ncell, d = sizeof(double);
  s->kind = (uint8_t *)or_zalloc(nc);
  s->f = (double *)or_zalloc(nc * s->q * d);
  s->g = (double *)or_zalloc(nc * s->q * d);
  s->fn = (double *)or_zalloc(nc * s->q * d);
  s->gn = (double *)or_zalloc(nc * s->q * d);
  double **fields[] = {&s->rho, &s->phi, &s->jx, &s->jy, &s->jz, &s->lr,
                       &s->lp, &s->mur, &s->mup, &s->pi, &s->Fx, &s->Fy, &s->Fz,
                       &s->ux, &s->uy, &s->uz};
  for (size_t k = 0; k < sizeof(fields) / sizeof(fields[0]); ++k)
    *fields[k] = (double *)or_zalloc(nc * d);
  for (long cell = 0; cell < s->ncell; ++cell) {
    int x[3];
    or_xyz(s, cell, &x[0], &x[1], &x[2]);
    int ghost = 0;
    for (int a = 0; a < 3; ++a)
      if (s->off[a] && (x[a] == 0 || x[a] == s->ext[a] - 1)) ghost = 1;
    if (ghost) {
      s->kind[cell] = OR_GHOST;
      continue;
    }
    long u = (long)(x[0] - s->off[0]) +
             (long)p->nx * ((long)(x[1] - s->off[1]) +
                            (long)p->ny * (long)(x[2] - s->off[2]));
    s->kind[cell] = mask ? mask[u] : OR_FLUID;
  }
  return s;
}

static long or_user_to_ext(const or_state *s, long u) {
  int x = (int)(u % s->p.nx);
  long r = u / s->p.nx;
  int y = (int)(r % s->p.ny);
  int z = (int)(r / s->p.ny);
  return or_idx(s, x + s->off[0], y + s->off[1], z + s->off[2]);
}

static double or_gamma(const or_state *s) {
  return s->p.M / (s->p.tau_g - 0.5);
}

/* Initialisation (Sec. 2.3): populations at their equilibria.
 * phi0, rho0 (may be NULL -> 1), u0 (may be NULL -> 0; layout [3][N]) are
 * given on the fluid domain, x fastest. */
or_state *or_create(const or_params *p, const uint8_t *mask,
                    const double *phi0, const double *rho0, const double *u0) {
  or_state *s = or_create_geometry(p, mask);
  if (!s) return NULL;
  long N = (long)p->nx * p->ny * p->nz;
  double *ux0 = (double *)or_zalloc(s->ncell * sizeof(double));
  double *uy0 = (double *)or_zalloc(s->ncell * sizeof(double));
  double *uz0 = (double *)or_zalloc(s->ncell * sizeof(double));
  for (long u = 0; u < N; ++u) {
    long e = or_user_to_ext(s, u);
    if (s->kind[e] != OR_FLUID) continue;
    s->phi[e] = phi0[u];
    s->rho[e] = rho0 ? rho0[u] : 1.0;
    if (u0) {
      ux0[e] = u0[u];
      uy0[e] = u0[N + u];
      uz0[e] = u0[2 * N + u];
    }
  }
  or_potentials(s);
  double G = or_gamma(s);
  for (long e = 0; e < s->ncell; ++e) {
    if (s->kind[e] != OR_FLUID) continue;
    double uu[3] = {ux0[e], uy0[e], uz0[e]};
    or_feq(p->kind, s->rho[e], uu, &s->f[e * s->q]);
    or_geq(p->kind, s->phi[e], s->mup[e], G, uu, &s->g[e * s->q]);
  }
  free(ux0); free(uy0); free(uz0);
  s->t = 0;
  return s;
}

/* One time step: Algorithm 1 at every fluid node, then streaming (push into
 * the second buffer) with moving bounce-back on links into solid cells. */
static void or_step1(or_state *s) {
  int q = s->q, kind = s->p.kind;
  const int(*c)[3] = or_c(kind);
  const double *w = or_w(kind);
  double G = or_gamma(s);
  double tf = s->p.tau_f, tg = s->p.tau_g;
  or_moments(s);
  or_potentials(s);
  or_force_velocity(s);
  /* collide + stream; every target slot is written exactly once */
#pragma omp parallel for schedule(static)
  for (long x = 0; x < s->ncell; ++x) {
    if (s->kind[x] != OR_FLUID) continue;
    double u[3] = {s->ux[x], s->uy[x], s->uz[x]};
    double F[3] = {s->Fx[x], s->Fy[x], s->Fz[x]};
    double feq[OR_MAXQ], geq[OR_MAXQ], S[OR_MAXQ];
    or_feq(kind, s->rho[x], u, feq);
    or_guo(kind, tf, u, F, S);
    or_geq(kind, s->phi[x], s->mup[x], G, u, geq);
    for (int i = 0; i < q; ++i) {
      double fs = s->f[x * q + i] - (s->f[x * q + i] - feq[i]) / tf + S[i];
      double gs = s->g[x * q + i] - (s->g[x * q + i] - geq[i]) / tg;
      long y = or_nb(s, x, i);
      if (y >= 0 && s->kind[y] == OR_FLUID) {
        s->fn[y * q + i] = fs;
        s->gn[y * q + i] = gs;
      } else {
        double uw[3];
        or_body_velocity(s, x, y, i, uw);
        double cu = c[i][0] * uw[0] + c[i][1] * uw[1] + c[i][2] * uw[2];
        int ib = or_opp(i);
        s->fn[x * q + ib] = fs - 2.0 * w[i] * s->rho[x] * cu / CS2;
        s->gn[x * q + ib] = gs - 2.0 * w[i] * s->phi[x] * cu / CS2;
      }
    }
  }
  double *t1 = s->f; s->f = s->fn; s->fn = t1;
  double *t2 = s->g; s->g = s->gn; s->gn = t2;
  s->t += 1;
}

void or_step(or_state *s, long n) {
  for (long k = 0; k < n; ++k) or_step1(s);
}

/* Consistent initialisation after Mei et al. (2006), as cited in Sec. 2.3:
 * n pre-iterations of f with the velocity held at u0 (layout [3][N], NULL =
 * 0) and phi held at phi0 (N values), both on the fluid domain; rho = sum f
 * evolves.  Each pre-iteration takes the step's own moments, potentials and
 * force (eqs. densMoment, mu_rho, mu_phi, F) on (rho, phi0), then collides f
 * towards f^eq(rho, u0) with the Guo term S(u0, F) and streams it with the
 * moving bounce-back (eqs. bgk, feq, Fi; Sec. 2.3).  g is left alone during
 * the iterations and is then set to g^eq(phi0, mu_phi(rho, phi0), u0)
 * (eq. geq).  Returns -1 if called after the first step. */
int or_consistent_init(or_state *s, const double *phi0, const double *u0, long n) {
  if (s->t != 0) return -1;
  int q = s->q, kind = s->p.kind;
  const int(*c)[3] = or_c(kind);
  const double *w = or_w(kind);
  double tf = s->p.tau_f;
  long N = (long)s->p.nx * s->p.ny * s->p.nz;
  double *ph0 = (double *)or_zalloc(s->ncell * sizeof(double));
  double *U[3];
  for (int a = 0; a < 3; ++a) U[a] = (double *)or_zalloc(s->ncell * sizeof(double));
  for (long u = 0; u < N; ++u) {
    long e = or_user_to_ext(s, u);
    ph0[e] = phi0[u];
    if (u0)
      for (int a = 0; a < 3; ++a) U[a][e] = u0[(long)a * N + u];
  }
  for (long k = 0; k < n; ++k) {
    or_moments(s);
    for (long x = 0; x < s->ncell; ++x)
      if (s->kind[x] == OR_FLUID) s->phi[x] = ph0[x];
    or_potentials(s);
    or_force_velocity(s);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < s->ncell; ++x) {
      if (s->kind[x] != OR_FLUID) continue;
      double u[3] = {U[0][x], U[1][x], U[2][x]};
      double F[3] = {s->Fx[x], s->Fy[x], s->Fz[x]};
      double feq[OR_MAXQ], S[OR_MAXQ];
      or_feq(kind, s->rho[x], u, feq);
      or_guo(kind, tf, u, F, S);
      for (int i = 0; i < q; ++i) {
        double fs = s->f[x * q + i] - (s->f[x * q + i] - feq[i]) / tf + S[i];
        long y = or_nb(s, x, i);
        if (y >= 0 && s->kind[y] == OR_FLUID) {
          s->fn[y * q + i] = fs;
        } else {
          double uw[3];
          or_body_velocity(s, x, y, i, uw);
          double cu = c[i][0] * uw[0] + c[i][1] * uw[1] + c[i][2] * uw[2];
          s->fn[x * q + or_opp(i)] = fs - 2.0 * w[i] * s->rho[x] * cu / CS2;
        }
      }
    }
    double *t1 = s->f; s->f = s->fn; s->fn = t1;
  }
  or_moments(s);
  for (long x = 0; x < s->ncell; ++x)
    if (s->kind[x] == OR_FLUID) s->phi[x] = ph0[x];
  or_potentials(s);
  double G = or_gamma(s);
  for (long x = 0; x < s->ncell; ++x) {
    if (s->kind[x] != OR_FLUID) continue;
    double u[3] = {U[0][x], U[1][x], U[2][x]};
    or_geq(kind, ph0[x], s->mup[x], G, u, &s->g[x * q]);
  }
  free(ph0);
  for (int a = 0; a < 3; ++a) free(U[a]);
  return 0;
}

long or_time(const or_state *s) { return s->t; }

/* Observables at the current time on the fluid domain (x fastest).
 * out has 9*N entries: rho, phi, ux, uy, uz, mu_rho, mu_phi, P, solid flag.
 * u includes the F/2 correction (eq. veloMoment).  P is the bulk pressure
 * cs^2 rho + rho mu_rho + phi mu_phi - psi_b (valid away from interfaces).
 * Solid cells report zeros and flag 1. */
void or_observe(or_state *s, double *out) {
  or_moments(s);
  or_potentials(s);
  or_force_velocity(s);
  long N = (long)s->p.nx * s->p.ny * s->p.nz;
  for (long u = 0; u < N; ++u) {
    long e = or_user_to_ext(s, u);
    double *o[9];
    for (int k = 0; k < 9; ++k) o[k] = out + (long)k * N + u;
    if (s->kind[e] != OR_FLUID) {
      for (int k = 0; k < 8; ++k) *o[k] = 0.0;
      *o[8] = 1.0;
      continue;
    }
    double r = s->rho[e], ph = s->phi[e];
    *o[0] = r;
    *o[1] = ph;
    *o[2] = s->ux[e];
    *o[3] = s->uy[e];
    *o[4] = s->uz[e];
    *o[5] = s->mur[e];
    *o[6] = s->mup[e];
    *o[7] = CS2 * r + r * s->mur[e] + ph * s->mup[e] -
            or_psi_bulk(s->p.kappa1, s->p.kappa2, r, ph);
    *o[8] = 0.0;
  }
}

/* Populations on the fluid domain, layout [q][N]; solid cells give zeros. */
void or_get_populations(const or_state *s, double *f_out, double *g_out) {
  long N = (long)s->p.nx * s->p.ny * s->p.nz;
  for (long u = 0; u < N; ++u) {
    long e = or_user_to_ext(s, u);
    for (int i = 0; i < s->q; ++i) {
      int fl = s->kind[e] == OR_FLUID;
      f_out[(long)i * N + u] = fl ? s->f[e * s->q + i] : 0.0;
      g_out[(long)i * N + u] = fl ? s->g[e * s->q + i] : 0.0;
    }
  }
}

/* Overwrite the populations (layout [q][N]) at fluid cells. */
void or_set_populations(or_state *s, const double *f_in, const double *g_in) {
  long N = (long)s->p.nx * s->p.ny * s->p.nz;
  for (long u = 0; u < N; ++u) {
    long e = or_user_to_ext(s, u);
    if (s->kind[e] != OR_FLUID) continue;
    for (int i = 0; i < s->q; ++i) {
      s->f[e * s->q + i] = f_in[(long)i * N + u];
      s->g[e * s->q + i] = g_in[(long)i * N + u];
    }
  }
}

/* The stencil operators applied to a field X given on the fluid domain:
 * solid cells are filled by the fluid-neighbour mean, then the Laplacian
 * (lap_out, N) and gradient (grad_out, [3][N]) are taken at fluid cells. */
void or_stencils(or_state *s, const double *X, double *lap_out,
                 double *grad_out) {
  long N = (long)s->p.nx * s->p.ny * s->p.nz;
  double *tmp = (double *)or_zalloc(s->ncell * sizeof(double));
  for (long u = 0; u < N; ++u) {
    long e = or_user_to_ext(s, u);
    if (s->kind[e] == OR_FLUID) tmp[e] = X[u];
  }
  or_fill_solid(s, tmp);
  for (long u = 0; u < N; ++u) {
    long e = or_user_to_ext(s, u);
    if (s->kind[e] != OR_FLUID) {
      lap_out[u] = 0.0;
      for (int a = 0; a < 3; ++a) grad_out[(long)a * N + u] = 0.0;
      continue;
    }
    lap_out[u] = or_lap_at(s, tmp, e);
    double gr[3];
    or_grad_at(s, tmp, e, gr);
    for (int a = 0; a < 3; ++a) grad_out[(long)a * N + u] = gr[a];
  }
  free(tmp);
}

/* ====================================================================== */
/* Ternary extension (Sec. 2.2, Remark after the mobility relation): one   */
/* more Cahn-Hilliard equation, for a third order parameter psi, and one   */
/* more population h.  The free energy is that of the ternary model the    */
/* Remark cites (Semprebon, Krueger and Kusumaatmaja 2016), written with   */
/* the concentrations C1 = (rho + phi - psi)/2, C2 = (rho - phi - psi)/2,  */
/* C3 = psi:                                                               */
/*   Psi = int sum_m [ kappa_m/2 C_m^2 (1 - C_m)^2                         */
/*                     + alpha^2 kappa_m/2 |grad C_m|^2 ] dV,              */
/* which for C3 = 0 is eq. (functional) term by term.  The potentials are  */
/* the functional derivatives, through the chain rule from                 */
/*   mu_m = kappa_m C_m (1 - C_m)(1 - 2 C_m) - alpha^2 kappa_m lap C_m:    */
/*   mu_rho = (mu_1 + mu_2)/2, mu_phi = (mu_1 - mu_2)/2,                   */
/*   mu_psi = mu_3 - (mu_1 + mu_2)/2;                                      */
/* the force generalises eq. (F) to -rho grad mu_rho - phi grad mu_phi     */
/* - psi grad mu_psi (the divergence of the chemical pressure of this      */
/* functional), taken in the same product-rule form as the binary step;    */
/* h has the equilibrium of eq. (geq) with (psi, mu_psi, Gamma_psi),       */
/* Gamma_psi = M_psi / (tau_h - 1/2), and the walls treat it as g.         */
/* ====================================================================== */

/* The three potentials at a node from rho, phi, psi and their Laplacians.
 * out[0] = mu_rho, out[1] = mu_phi, out[2] = mu_psi. */
void or3_mu(double kappa1, double kappa2, double kappa3, double alpha, double rho,
            double phi, double psi, double lap_rho, double lap_phi, double lap_psi,
            double *out) {
  double C[3] = {0.5 * (rho + phi - psi), 0.5 * (rho - phi - psi), psi};
  double L[3] = {0.5 * (lap_rho + lap_phi - lap_psi),
                 0.5 * (lap_rho - lap_phi - lap_psi), lap_psi};
  double k[3] = {kappa1, kappa2, kappa3};
  double m[3];
  for (int a = 0; a < 3; ++a)
    m[a] = k[a] * C[a] * (1.0 - C[a]) * (1.0 - 2.0 * C[a]) -
           alpha * alpha * k[a] * L[a];
  out[0] = 0.5 * (m[0] + m[1]);
  out[1] = 0.5 * (m[0] - m[1]);
  out[2] = m[2] - 0.5 * (m[0] + m[1]);
}

/* Bulk free-energy density of the ternary functional. */
double or3_psi_bulk(double kappa1, double kappa2, double kappa3, double rho,
                    double phi, double psi) {
  double C[3] = {0.5 * (rho + phi - psi), 0.5 * (rho - phi - psi), psi};
  double k[3] = {kappa1, kappa2, kappa3};
  double e = 0.0;
  for (int a = 0; a < 3; ++a)
    e += 0.5 * k[a] * C[a] * C[a] * (1.0 - C[a]) * (1.0 - C[a]);
  return e;
}

static double or3_gamma(const or_state *s) { return s->M3 / (s->tau_h - 0.5); }

static void or3_moments(or_state *s) {
  const int(*c)[3] = or_c(s->p.kind);
  int q = s->q;
#pragma omp parallel for schedule(static)
  for (long x = 0; x < s->ncell; ++x) {
    if (s->kind[x] != OR_FLUID) {
      s->rho[x] = s->phi[x] = s->psi[x] = s->jx[x] = s->jy[x] = s->jz[x] = 0.0;
      continue;
    }
    double r = 0.0, p = 0.0, z = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < q; ++i) {
      double fi = s->f[x * q + i];
      r += fi;
      p += s->g[x * q + i];
      z += s->h[x * q + i];
      for (int a = 0; a < 3; ++a) j[a] += c[i][a] * fi;
    }
    s->rho[x] = r;
    s->phi[x] = p;
    s->psi[x] = z;
    s->jx[x] = j[0];
    s->jy[x] = j[1];
    s->jz[x] = j[2];
  }
}

/* The three potentials and Pi = rho mu_rho + phi mu_phi + psi mu_psi at fluid
 * cells; solid cells filled for rho, phi, psi and Pi (reading R5). */
static void or3_potentials(or_state *s) {
  or_fill_solid(s, s->rho);
  or_fill_solid(s, s->phi);
  or_fill_solid(s, s->psi);
#pragma omp parallel for schedule(static)
  for (long x = 0; x < s->ncell; ++x) {
    if (s->kind[x] != OR_FLUID) continue;
    s->lr[x] = or_lap_at(s, s->rho, x);
    s->lp[x] = or_lap_at(s, s->phi, x);
    s->lq[x] = or_lap_at(s, s->psi, x);
    double mu[3];
    or3_mu(s->p.kappa1, s->p.kappa2, s->kappa3, s->p.alpha, s->rho[x], s->phi[x],
           s->psi[x], s->lr[x], s->lp[x], s->lq[x], mu);
    s->mur[x] = mu[0];
    s->mup[x] = mu[1];
    s->muq[x] = mu[2];
    s->pi[x] = s->rho[x] * mu[0] + s->phi[x] * mu[1] + s->psi[x] * mu[2];
  }
  or_fill_solid(s, s->pi);
}

/* F = mu_rho grad rho + mu_phi grad phi + mu_psi grad psi - grad Pi (equal in
 * the continuum to -rho grad mu_rho - phi grad mu_phi - psi grad mu_psi) and
 * u = (j + F/2)/rho at fluid cells. */
static void or3_force_velocity(or_state *s) {
#pragma omp parallel for schedule(static)
  for (long x = 0; x < s->ncell; ++x) {
    if (s->kind[x] != OR_FLUID) {
      s->Fx[x] = s->Fy[x] = s->Fz[x] = 0.0;
      s->ux[x] = s->uy[x] = s->uz[x] = 0.0;
      continue;
    }
    double gr[3], gp[3], gq[3], gpi[3];
    or_grad_at(s, s->rho, x, gr);
    or_grad_at(s, s->phi, x, gp);
    or_grad_at(s, s->psi, x, gq);
    or_grad_at(s, s->pi, x, gpi);
    double F[3];
    for (int a = 0; a < 3; ++a)
      F[a] = s->mur[x] * gr[a] + s->mup[x] * gp[a] + s->muq[x] * gq[a] - gpi[a];
    s->Fx[x] = F[0];
    s->Fy[x] = F[1];
    s->Fz[x] = F[2];
    s->ux[x] = (s->jx[x] + 0.5 * F[0]) / s->rho[x];
    s->uy[x] = (s->jy[x] + 0.5 * F[1]) / s->rho[x];
    s->uz[x] = (s->jz[x] + 0.5 * F[2]) / s->rho[x];
  }
}

/* A ternary lattice: the binary parameters (kappa1, kappa2, alpha, tau_f,
 * tau_g, M for phi) plus kappa3, the mobility M3 and relaxation time tau_h
 * of psi.  Initialisation at equilibrium as in Sec. 2.3:
 * f = f^eq(rho0, u0), g = g^eq(phi0, mu_phi, u0), h = g^eq(psi0, mu_psi, u0)
 * with the potentials of the initial fields.  psi0 on the fluid domain. */
or_state *or3_create(const or_params *p, double kappa3, double M3, double tau_h,
                     const uint8_t *mask, const double *phi0, const double *psi0,
                     const double *rho0, const double *u0) {
  or_state *s = or_create_geometry(p, mask);
  if (!s) return NULL;
  s->ternary = 1;
  s->kappa3 = kappa3;
  s->M3 = M3;
  s->tau_h = tau_h;
  size_t nc = (size_t)s->ncell, d = sizeof(double);
  s->h = (double *)or_zalloc(nc * s->q * d);
  s->hn = (double *)or_zalloc(nc * s->q * d);
  s->psi = (double *)or_zalloc(nc * d);
  s->lq = (double *)or_zalloc(nc * d);
  s->muq = (double *)or_zalloc(nc * d);
  long N = (long)p->nx * p->ny * p->nz;
  double *U[3];
  for (int a = 0; a < 3; ++a) U[a] = (double *)or_zalloc(nc * d);
  for (long u = 0; u < N; ++u) {
    long e = or_user_to_ext(s, u);
    if (s->kind[e] != OR_FLUID) continue;
    s->phi[e] = phi0[u];
    s->psi[e] = psi0[u];
    s->rho[e] = rho0 ? rho0[u] : 1.0;
    if (u0)
      for (int a = 0; a < 3; ++a) U[a][e] = u0[(long)a * N + u];
  }
  or3_potentials(s);
  double G = or_gamma(s), G3 = or3_gamma(s);
  for (long e = 0; e < s->ncell; ++e) {
    if (s->kind[e] != OR_FLUID) continue;
    double uu[3] = {U[0][e], U[1][e], U[2][e]};
    or_feq(p->kind, s->rho[e], uu, &s->f[e * s->q]);
    or_geq(p->kind, s->phi[e], s->mup[e], G, uu, &s->g[e * s->q]);
    or_geq(p->kind, s->psi[e], s->muq[e], G3, uu, &s->h[e * s->q]);
  }
  for (int a = 0; a < 3; ++a) free(U[a]);
  s->t = 0;
  return s;
}

/* One ternary time step: the binary step with the third order parameter. */
static void or3_step1(or_state *s) {
  int q = s->q, kind = s->p.kind;
  const int(*c)[3] = or_c(kind);
  const double *w = or_w(kind);
  double G = or_gamma(s), G3 = or3_gamma(s);
  double tf = s->p.tau_f, tg = s->p.tau_g, th = s->tau_h;
  or3_moments(s);
  or3_potentials(s);
  or3_force_velocity(s);
#pragma omp parallel for schedule(static)
  for (long x = 0; x < s->ncell; ++x) {
    if (s->kind[x] != OR_FLUID) continue;
    double u[3] = {s->ux[x], s->uy[x], s->uz[x]};
    double F[3] = {s->Fx[x], s->Fy[x], s->Fz[x]};
    double feq[OR_MAXQ], geq[OR_MAXQ], heq[OR_MAXQ], S[OR_MAXQ];
    or_feq(kind, s->rho[x], u, feq);
    or_guo(kind, tf, u, F, S);
    or_geq(kind, s->phi[x], s->mup[x], G, u, geq);
    or_geq(kind, s->psi[x], s->muq[x], G3, u, heq);
    for (int i = 0; i < q; ++i) {
      double fs = s->f[x * q + i] - (s->f[x * q + i] - feq[i]) / tf + S[i];
      double gs = s->g[x * q + i] - (s->g[x * q + i] - geq[i]) / tg;
      double hs = s->h[x * q + i] - (s->h[x * q + i] - heq[i]) / th;
      long y = or_nb(s, x, i);
      if (y >= 0 && s->kind[y] == OR_FLUID) {
        s->fn[y * q + i] = fs;
        s->gn[y * q + i] = gs;
        s->hn[y * q + i] = hs;
      } else {
        double uw[3];
        or_body_velocity(s, x, y, i, uw);
        double cu = c[i][0] * uw[0] + c[i][1] * uw[1] + c[i][2] * uw[2];
        int ib = or_opp(i);
        s->fn[x * q + ib] = fs - 2.0 * w[i] * s->rho[x] * cu / CS2;
        s->gn[x * q + ib] = gs - 2.0 * w[i] * s->phi[x] * cu / CS2;
        s->hn[x * q + ib] = hs - 2.0 * w[i] * s->psi[x] * cu / CS2;
      }
    }
  }
  double *t1 = s->f; s->f = s->fn; s->fn = t1;
  double *t2 = s->g; s->g = s->gn; s->gn = t2;
  double *t3 = s->h; s->h = s->hn; s->hn = t3;
  s->t += 1;
}

void or3_step(or_state *s, long n) {
  for (long k = 0; k < n; ++k) or3_step1(s);
}

/* Ternary observables on the fluid domain: out has 11*N entries: rho, phi,
 * psi, ux, uy, uz, mu_rho, mu_phi, mu_psi, P, solid flag, with P = cs^2 rho
 * + Pi - psi_b. */
void or3_observe(or_state *s, double *out) {
  or3_moments(s);
  or3_potentials(s);
  or3_force_velocity(s);
  long N = (long)s->p.nx * s->p.ny * s->p.nz;
  for (long u = 0; u < N; ++u) {
    long e = or_user_to_ext(s, u);
    double *o[11];
    for (int k = 0; k < 11; ++k) o[k] = out + (long)k * N + u;
    if (s->kind[e] != OR_FLUID) {
      for (int k = 0; k < 10; ++k) *o[k] = 0.0;
      *o[10] = 1.0;
      continue;
    }
    double r = s->rho[e], ph = s->phi[e], ps = s->psi[e];
    *o[0] = r;
    *o[1] = ph;
    *o[2] = ps;
    *o[3] = s->ux[e];
    *o[4] = s->uy[e];
    *o[5] = s->uz[e];
    *o[6] = s->mur[e];
    *o[7] = s->mup[e];
    *o[8] = s->muq[e];
    *o[9] = CS2 * r + r * s->mur[e] + ph * s->mup[e] + ps * s->muq[e] -
            or3_psi_bulk(s->p.kappa1, s->p.kappa2, s->kappa3, r, ph, ps);
    *o[10] = 0.0;
  }
}

/* Ternary populations on the fluid domain, layout [q][N] each. */
void or3_get_populations(const or_state *s, double *f_out, double *g_out,
                         double *h_out) {
  or_get_populations(s, f_out, g_out);
  long N = (long)s->p.nx * s->p.ny * s->p.nz;
  for (long u = 0; u < N; ++u) {
    long e = or_user_to_ext(s, u);
    for (int i = 0; i < s->q; ++i)
      h_out[(long)i * N + u] = s->kind[e] == OR_FLUID ? s->h[e * s->q + i] : 0.0;
  }
}

/* Replace the ternary populations of the fluid cells (layout [q][N] each,
 * as or3_get_populations); solid cells keep theirs.  The state of a ternary
 * lattice between steps is exactly these post-stream populations, so a
 * lattice given another's populations continues that run. */
void or3_set_populations(or_state *s, const double *f_in, const double *g_in,
                         const double *h_in) {
  or_set_populations(s, f_in, g_in);
  long N = (long)s->p.nx * s->p.ny * s->p.nz;
  for (long u = 0; u < N; ++u) {
    long e = or_user_to_ext(s, u);
    if (s->kind[e] != OR_FLUID) continue;
    for (int i = 0; i < s->q; ++i) s->h[e * s->q + i] = h_in[(long)i * N + u];
  }
}
