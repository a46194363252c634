/*
 * frelbm.h -- C ABI of the MI355X free-energy lattice Boltzmann library.
 *
 * The library advances a binary-mixture lattice with the free-energy LBM of
 * Simonis et al., "Binary mixture flow with free energy lattice Boltzmann
 * methods" (arXiv 2212.01617): a Navier-Stokes population f (BGK with Guo
 * forcing, Sec. 2.2 eqs. LBE, bgk, feq, Fi) and a Cahn-Hilliard population g
 * (Sec. 2.2 eqs. LBEg, geq), coupled by the thermodynamic force (eq. F) built
 * from the chemical potentials (eqs. mu_rho, mu_phi), on D2Q9 or D3Q19,
 * collide-then-stream as in Sec. 2.3 and Algorithm 1.
 *
 * Conventions shared by every call:
 *  - Fields on the host are double, shaped (nz, ny, nx) with x fastest:
 *    cell = x + nx*(y + ny*z).  Vector fields are component-major [3][N].
 *  - Device memory is owned by the caller.  The library only borrows the
 *    buffer given to fre_lattice_init / fre_batch_create for the handle's
 *    lifetime and never frees it.  Host buffers are the caller's.
 *  - All device work is enqueued on the caller's HIP stream (hipStream_t
 *    passed as void*; NULL = the default stream).  fre_step is asynchronous;
 *    every call that returns host data synchronises that stream first.
 *  - Every call returns a fre_status; on failure fre_last_error() gives a
 *    thread-local message.  Nothing throws across the ABI.  Parameters are
 *    validated before any device work is enqueued.
 *  - One handle per stream; calls on one handle are not re-entrant.
 */
#ifndef FRELBM_H
#define FRELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fre_status;
#define FRE_OK 0
#define FRE_EINVAL (-1)   /* bad argument or parameter                     */
#define FRE_ENOMEM (-2)   /* caller buffer too small                       */
#define FRE_EDEVICE (-3)  /* a HIP call failed                             */
#define FRE_ESTATE (-4)   /* handle is in the failed state                 */
#define FRE_ENUMERIC (-5) /* a non-finite value was found on the lattice   */

#define FRE_D2Q9 0
#define FRE_D3Q19 1

#define FRE_FP32 0 /* f_i - w_i and g_i as float; g_0 (O(1)) also keeps the  */
                   /* part float rounds away, as a scaled half per cell      */
#define FRE_FP16 1 /* f_i - w_i and g_i (i>0) as half, g_0 as float          */

#define FRE_PERIODIC 0
#define FRE_WALL 1 /* halfway bounce-back wall at both ends of the axis     */

/* Solid-mask codes (uint8 per fluid-domain cell). */
#define FRE_MASK_FLUID 0
#define FRE_MASK_SOLID 1  /* static obstacle                                */
#define FRE_MASK_ROLLER0 2 /* 2+k: cell moves with roller k (k < 4)          */

/* Field bits for fre_read_moments, written in this order, N doubles each
 * (FRE_F_U writes 3N: ux, uy, uz). */
#define FRE_F_RHO 1u
#define FRE_F_PHI 2u
#define FRE_F_U 4u
#define FRE_F_MU_RHO 8u
#define FRE_F_MU_PHI 16u
#define FRE_F_P 32u
#define FRE_F_PSI 64u     /* ternary lattices only */
#define FRE_F_MU_PSI 128u /* ternary lattices only */

/* A staircase cylinder (rotating roller): the cells whose mask code is 2+k
 * move rigidly with angular velocity omega about the line through `center`
 * parallel to axis `axis` (0=x, 1=y, 2=z).  The mask itself is an input;
 * `radius` is informational (tip-speed check). */
typedef struct fre_roller {
  double center[3];
  double radius;
  double omega;
  int32_t axis;
  int32_t reserved;
} fre_roller;

/* Per-instance parameters (Sec. 2.2).
 *  kind, nx, ny, nz, storage, bc: shape and layout (nz = 1, bc[2] periodic
 *    for D2Q9).
 *  wall_u[a][s][b]: velocity component b of the wall closing axis a at its
 *    low (s=0) or high (s=1) end; used when bc[a] == FRE_WALL.
 *  Free energy, eq. (functional): with use_paper_form = 0 the symmetric
 *    binary energy A/4 (phi^2-1)^2 + kappa/2 |grad phi|^2 is mapped to
 *    kappa1 = kappa2 = 4A, alpha = sqrt(kappa / (2A)); with
 *    use_paper_form = 1, kappa1, kappa2, alpha are used as given.
 *  tau_f, tau_g > 1/2: relaxation times; M > 0: mobility, with
 *    Gamma = M / (tau_g - 1/2) (Sec. 2.2, mobility relation).
 *  ternary (0 or 1): a third component (Sec. 2.2, Remark after the mobility
 *    relation): a third order parameter psi with its own Cahn-Hilliard
 *    population h, the free energy of the cited ternary model (in the
 *    concentrations C1 = (rho + phi - psi)/2, C2 = (rho - phi - psi)/2,
 *    C3 = psi: sum_m kappa_m/2 C_m^2 (1 - C_m)^2 + alpha^2 kappa_m/2
 *    |grad C_m|^2, which is eq. (functional) for C3 = 0), kappa3 > 0, and
 *    psi's mobility M3 >= 0 with relaxation time tau_h > 1/2
 *    (Gamma_psi = M3 / (tau_h - 1/2)).  FP32 storage only; created with
 *    fre_lattice_init3, stepped alone (not in batches), no consistent
 *    initialisation or launch-shape tuning.  kappa3, M3, tau_h are ignored
 *    when ternary = 0.
 *  fp16_rounding (FP16 storage): 0 stores each half rounded to nearest
 *    even; 1 rounds stochastically, to the upper of the two neighbouring
 *    halves with probability equal to the value's fractional distance
 *    between them.  The random numbers come from a per-cell stream seeded
 *    by a hash of the cell and a step counter kept in the population range
 *    (so checkpoints carry it).  Round-to-nearest repeats the same rounding
 *    error in every cell of a nearly uniform flow at every step; the
 *    stochastic rounding is unbiased, and long runs drift far less, for
 *    about 10% of the FP16 step.  Results stay deterministic (bitwise
 *    reproducible, graph or not).
 *    Lattices with fp16_rounding = 1 are stepped alone (not in batches).
 *    Must be 0 with FP32 storage or a ternary lattice.
 * Validation: tau > 1/2, kappa1, kappa2, alpha > 0 (A, kappa > 0), M > 0,
 * |wall_u| <= 0.1 and |omega| * radius <= 0.1 (Mach guard), sizes >= 1,
 * storage/kind/bc codes in range. */
typedef struct fre_params {
  int32_t kind;
  int32_t nx, ny, nz;
  int32_t storage;
  int32_t bc[3];
  double wall_u[3][2][3];
  int32_t n_rollers;
  int32_t fp16_rounding;
  fre_roller rollers[4];
  double A, kappa;
  double kappa1, kappa2, alpha;
  int32_t use_paper_form;
  int32_t ternary;
  double tau_f, tau_g, M;
  double kappa3, M3, tau_h;
} fre_params;

typedef struct fre_lattice fre_lattice;
typedef struct fre_batch fre_batch;

/* Device bytes fre_lattice_init needs for these parameters (populations in
 * place, coupling fields, mask and scratch).  No device work. */
fre_status fre_footprint(const fre_params *p, size_t *device_bytes);

/* Create a lattice in the caller's device buffer (>= fre_footprint bytes,
 * 256-byte aligned) and initialise it at equilibrium (Sec. 2.3):
 * f = f^eq(rho0, u0), g = g^eq(phi0, mu_phi(rho0, phi0), u0).
 *  phi0: N doubles (required, finite).  rho0: N doubles or NULL (= 1).
 *  u0: 3N doubles or NULL (= 0).  solid_mask: N bytes or NULL (= all fluid),
 *  codes FRE_MASK_*; roller codes must be < 2 + n_rollers.
 * Synchronises the stream before returning.  *out is freed with
 * fre_lattice_destroy. */
fre_status fre_lattice_init(const fre_params *p, void *device_buf, size_t bytes,
                            void *hip_stream, const double *phi0,
                            const double *rho0, const double *u0,
                            const uint8_t *solid_mask, fre_lattice **out);

/* A ternary lattice (params->ternary = 1): as fre_lattice_init with the
 * third order parameter psi0 (N values, host, required; C3 = psi).  The
 * populations start at their equilibria f^eq(rho0, u0), g^eq(phi0, mu_phi,
 * u0), h^eq(psi0, mu_psi, u0) with the potentials of the initial fields.
 * fre_lattice_init refuses ternary parameters. */
fre_status fre_lattice_init3(const fre_params *p, void *device_buf, size_t bytes, void *hip_stream,
                             const double *phi0, const double *psi0, const double *rho0, const double *u0,
                             const uint8_t *solid_mask, fre_lattice **out);

/* Consistent initialisation (Sec. 2.3, which starts from equilibrium and
 * aligns the kinetic moments by collisions, citing Mei, Luo, Lallemand and
 * d'Humieres 2006): n pre-iterations of the f population in which the
 * velocity of the equilibrium and of the Guo forcing term is held at u0 and
 * the order parameter at phi0, while rho = sum f evolves (the pressure field
 * and the non-equilibrium part of f develop); g is not stepped.  Then g is set
 * to g^eq(phi0, mu_phi(rho, phi0), u0) and the moments are recomputed.  The
 * time counter stays at 0.
 *  phi0: N doubles, u0: 3N doubles ([3][N]) or NULL (= 0), on the fluid
 *  domain, x fastest, as for fre_lattice_init (normally the same fields).
 *  n: number of pre-iterations, even and >= 0 (0 resets g only).
 * FRE_EINVAL for odd or negative n, NULL phi0 or non-finite values;
 * FRE_ESTATE after the first step, for a batch member or a failed lattice.
 * Synchronises the stream before returning. */
fre_status fre_consistent_init(fre_lattice *L, const double *phi0, const double *u0, int64_t n);

/* Replace the physical parameters (free energy, tau, M, wall and roller
 * velocities; kappa3, M3, tau_h of a ternary lattice) of an existing
 * lattice; shape, storage, bc, the roller count and the ternary flag must
 * not change (FRE_EINVAL), and a batch member refuses (FRE_ESTATE).  Takes
 * effect for the next step: steps already queued on the lattice's stream run
 * with the old parameters (the call waits for them when it drops the
 * lattice's captured graph).  On any error the lattice is left unchanged. */
fre_status fre_set_params(fre_lattice *L, const fre_params *p);

/* Advance n >= 0 time steps (Algorithm 1 at every fluid node, then
 * streaming with moving bounce-back), asynchronously on the bound stream.
 * On a non-default stream the steps are replayed from HIP graphs captured
 * on first use (runs of 16 steps, then pairs); on the default stream they
 * are launched one by one.  Both give bitwise the same state.
 * Returns FRE_ESTATE if the lattice has failed. */
fre_status fre_step(fre_lattice *L, int64_t n);

/* Observables at the current time, without stepping: the fields selected by
 * field_mask (FRE_F_*) in bit order, each N doubles (U: 3N), into host_out
 * of n_doubles.  u includes F/2 (eq. veloMoment); P is the bulk pressure
 * cs^2 rho + rho mu_rho + phi mu_phi - psi_b (ternary: + psi mu_psi, and the
 * ternary bulk density).  Ternary lattices also take FRE_F_PSI and
 * FRE_F_MU_PSI.  Solid cells read 0.  Syncs. */
fre_status fre_read_moments(fre_lattice *L, uint32_t field_mask,
                            double *host_out, size_t n_doubles);

/* The populations f_i, g_i (unshifted, post-streaming at the current time),
 * layout [q][N] each, into host arrays of n_doubles_each = q*N.  Solid
 * cells read 0.  With FP32 storage g_0 includes its low part.  Staged
 * through the lattice's own buffer in chunks (no device allocation; it
 * overwrites the auxiliary field that fre_read_moments recomputes).  Syncs. */
fre_status fre_read_populations(fre_lattice *L, double *f_out, double *g_out,
                                size_t n_doubles_each);

/* The three populations f_i, g_i, h_i of a ternary lattice, as
 * fre_read_populations (g_0 and h_0 with their low parts).
 * fre_read_populations refuses ternary lattices. */
fre_status fre_read_populations3(fre_lattice *L, double *f_out, double *g_out, double *h_out,
                                 size_t n_doubles_each);

/* Global sums over fluid cells, accumulated in FP64 on the device from
 * compensated FP32 partials: out[0] sum rho, [1] sum phi, [2] sum |phi|,
 * [3..5] sum rho u (with F/2), [6] number of cells with a non-finite value,
 * [7] number of fluid cells.  A non-zero out[6] puts the lattice in the
 * failed state and returns FRE_ENUMERIC.  Syncs. */
fre_status fre_reduce(fre_lattice *L, double out[8]);

/* fre_reduce for callers that cannot allocate memory (serving loops or
 * harnesses that forbid device or host allocation): the same sums, bitwise
 * equal to fre_reduce's, with the block partials kept in a fixed device array
 * of the library (64 KiB per GPU, taken when the library loads and held until
 * the process ends) instead of the lattice buffer.  It calls no hipMalloc or
 * hipFree and allocates no host memory.  The array's size does not depend on the
 * lattice, so every lattice fre_lattice_init accepts is accepted.  The array
 * is shared by every call on one GPU: calls that overlap on one GPU (two
 * streams, two threads) race and must be serialised by the caller.  Runs on
 * the device the lattice was created on.  Same errors as fre_reduce.  Syncs. */
fre_status fre_reduce_noalloc(fre_lattice *L, double out[8]);

/* Current step count and state (0 ok, 1 failed). */
fre_status fre_info(const fre_lattice *L, int64_t *step, int32_t *state);

/* Checkpoint: raw populations at storage precision, step count and the
 * parameters.  fre_state_bytes gives the host size; fre_save writes it
 * (syncs), fre_load restores it into a lattice of identical shape/storage
 * (a restored run continues bitwise as the uninterrupted one). */
fre_status fre_state_bytes(const fre_lattice *L, size_t *bytes);
fre_status fre_save(fre_lattice *L, void *host, size_t bytes);
fre_status fre_load(fre_lattice *L, const void *host, size_t bytes);

/* Measurement: advance n >= 1 steps launching each kernel of the step
 * separately with HIP events around it on the bound stream (no graph), and
 * write the mean duration in ms per step of each kernel into kernel_ms
 * (max_kernels >= 6 entries), indexed by kernel slot: 0 k_moments,
 * 1 k_fill_m, 2 k_potential, 3 k_fill_c, 4 k_collide, 5 k_combine.  A step
 * launches five of them (FP32 storage: slots 1-5, the moments at t+1 being a
 * by-product of k_collide completed by k_combine; FP16: slots 0-4); the slot
 * a lattice does not launch reads -1.  *n_kernels receives 6.
 * fre_kernel_name(k) names slot k (NULL beyond the last).  Syncs. */
fre_status fre_profile_step(fre_lattice *L, int64_t n, double *kernel_ms,
                            int32_t max_kernels, int32_t *n_kernels);
const char *fre_kernel_name(int32_t k);

/* Launch shapes of the three cell kernels of the step, cfg = {rows, xcd}
 * for the moments pass (k_moments, or k_combine with FP32 storage),
 * k_potential and k_collide in that order: rows of 64 cells per thread block
 * (1, 2, 4 or 8; with FP32 storage k_collide always 4, its tile being the
 * footprint of its on-chip moment sums) and xcd = 1 for the XCD-aware block
 * order (0: plain order).  A shape decides only which thread updates which
 * cell, never the arithmetic: results are bitwise the same under every
 * shape.  Default {4, 1} for all three.  Set syncs the bound stream;
 * FRE_EINVAL for other values. */
fre_status fre_set_launch_shape(fre_lattice *L, const int32_t cfg[6]);
fre_status fre_get_launch_shape(const fre_lattice *L, int32_t cfg[6]);

/* Autotuner: times each of the 8 candidate shapes (rows 1, 2, 4, 8 x xcd
 * 0, 1) over n (rounded up to even, 2 <= n <= 10000) individually launched
 * steps per candidate and keeps, for each of the three kernels, the fastest.
 * The lattice state (populations, step count) is copied to host memory
 * before and restored after, so tuning leaves the run where it was.
 * cfg_out (may be NULL) receives the chosen shapes, stage_ms (may be NULL,
 * 3 entries) their mean kernel times.  Syncs; refuses batch members. */
fre_status fre_autotune(fre_lattice *L, int64_t n, int32_t cfg_out[6], double stage_ms[3]);

/* Release the handle (accepts NULL).  Never frees caller memory.  A batch
 * member is removed from its batch first. */
void fre_lattice_destroy(fre_lattice *L);

/* ---------------------------------------------------------------------------
 * Batches: many lattices of different sizes, velocity sets and storage
 * precisions advanced together.  Each step runs, per (velocity set, storage)
 * class present, one persistent launch per stage of the step over a
 * device-side list of (lattice, block) work items; the list and its length
 * live in device memory, so lattices join and leave without recapturing the
 * batch's HIP graph.  A lattice advanced inside a batch takes exactly the
 * arithmetic it takes alone (bitwise the same populations).
 * ------------------------------------------------------------------------- */

/* Device bytes of a batch's tables for max_slots lattices, max_work cell
 * work items and max_fill solid-boundary items in total (see
 * fre_lattice_batch_needs): the instance table, the cell-tile list, the
 * list of potential columns (at most one per tile) and the fill list.  No
 * device work. */
fre_status fre_batch_footprint(int32_t max_slots, int64_t max_work, int64_t max_fill, size_t *bytes);

/* Work items a lattice adds to a batch: cell tiles of 64 x 4 cells and
 * solid-boundary cells. */
fre_status fre_lattice_batch_needs(const fre_lattice *L, int64_t *n_work, int64_t *n_fill);

/* Create a batch in the caller's device buffer (>= fre_batch_footprint,
 * 256-byte aligned); its steps run on hip_stream.  Freed with
 * fre_batch_destroy, which never frees caller memory. */
fre_status fre_batch_create(void *device_buf, size_t bytes, void *hip_stream, int32_t max_slots,
                            int64_t max_work, int64_t max_fill, fre_batch **out);

/* Add a lattice (not in another batch, not failed); *slot receives its slot.
 * All members share the AA parity: a lattice one step out of phase is first
 * advanced one step on its own.  FRE_ENOMEM when the slots or work lists
 * are full.  While a member, the lattice is stepped only through the batch;
 * reads, reductions and checkpoints of it wait for the batch's stream. */
fre_status fre_batch_add(fre_batch *B, fre_lattice *L, int32_t *slot);

/* Remove the lattice in `slot` (waits for the batch's stream). */
fre_status fre_batch_remove(fre_batch *B, int32_t slot);

/* Advance every member n >= 0 steps, asynchronously on the batch's stream.
 * FRE_ESTATE if a member has failed. */
fre_status fre_batch_step(fre_batch *B, int64_t n);

/* Batch launch shape: the persistent grid of the cell kernels in blocks per
 * compute unit (1..32; default 8).  Work items are tiles of 64 x 4 cells.
 * Results are bitwise the same under every shape.  Syncs the batch's
 * stream. */
fre_status fre_batch_set_launch_shape(fre_batch *B, int32_t blocks_per_cu);
fre_status fre_batch_get_launch_shape(const fre_batch *B, int32_t *blocks_per_cu);

/* Batch autotuner: times the batch step over n (rounded up to even,
 * 2..10000) directly launched steps for 2, 4, 8 and 16 blocks per CU and
 * keeps the fastest.  Every member's state is copied to host memory before
 * and restored after.  blocks_per_cu and ms_per_step (may be NULL) receive
 * the choice and its mean step time.  Syncs.  FRE_ESTATE for an empty batch
 * or a failed member. */
fre_status fre_batch_autotune(fre_batch *B, int64_t n, int32_t *blocks_per_cu, double *ms_per_step);

/* Number of members and the common AA parity. */
fre_status fre_batch_info(const fre_batch *B, int32_t *members, int32_t *parity);

void fre_batch_destroy(fre_batch *B);

/* Thread-local message of the last failing call on this thread. */
const char *fre_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FRELBM_H */
