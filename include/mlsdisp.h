/*
 * mlsdisp.h -- C ABI of the MI355X (gfx950) multilevel summation library for
 * periodic r^-6 dispersion.
 *
 * Method: Tameling, Springer, Bientinesi, Ismail, "Multilevel Summation for
 * Dispersion: A Linear-Time Algorithm for r^-6 Potentials", J. Chem. Phys.
 * 2014 (arXiv 1308.4005).  One call to mls_evaluate runs the algorithm of
 * Sec. II.B on the GPU: linked-cell binning (Sec. III.D), the local pair sum
 * with g_0 (eq:g_0, eq:evaluation with k = 0), anterpolation
 * (eq:anterpolation), l-1 restrictions, the cutoff stencils of levels
 * 1..l-1 (eq:g_k), the all-to-all sum on the periodic coarsest grid with its
 * pre-summed kernel (eq:last-grid-periodic-transformed), l-1 prolongations,
 * interpolation (eq:interpolation) and the energy with the self-interaction
 * term removed (eq:interpolation-pot, eq:self-interaction-energy).
 *
 * Problem statement the calls follow (Sec. II.A.1, II.D):
 *   E = -1/2 sum_i sum_{(j,n) != (i,0)} xi_i xi_j |x_i - x_j - n o L|^-6,
 *   xi_i = sqrt(C6_i)  (geometric mixing, eq:xi-general: C6_ij = sqrt(C6_i C6_j)),
 * approximated by MLS with cutoff a, finest spacing h, p-point Hermite basis
 * (p = 4: the cubic of eq:Phi-Hermite; p = 6: the C1 quintic Hermite) and l
 * grid levels.  Forces are F_i = -dE_MLS/dx_i, exact derivatives of the MLS
 * energy.  E is negative (attractive dispersion).
 *
 * Conventions for every call:
 *   - All array arguments are DEVICE pointers (memory of the device current
 *     when the plan was created) unless a comment says "host".
 *   - Positions are (n,3) row-major float64, any real values (wrapped into
 *     the box internally); C6 are (n) float64, >= 0.
 *   - Outputs are overwritten, never accumulated; inputs and outputs are
 *     float64 in both precisions; the precision only changes internal
 *     arithmetic.
 *   - The caller owns every array it passes; the plan owns its workspace
 *     (allocated in mls_plan_create, freed in mls_plan_destroy).
 *   - A plan is not thread safe; distinct plans are independent.  Two
 *     evaluations on one plan must be ordered (same stream, or synchronised).
 *   - Argument errors are reported synchronously by the return code with a
 *     detail string in mls_last_error() (thread local).  Errors in the data
 *     (non-finite positions or C6, negative C6) raise a device flag that
 *     mls_plan_status reads.  No call aborts the process.
 */
#ifndef MLSDISP_H
#define MLSDISP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mls_plan_s* mls_plan_t;
typedef struct mls_batch_s* mls_batch_t;

typedef enum {
  MLS_OK = 0,
  MLS_ERR_INVALID_ARG = -1, /* a parameter or pointer is out of range */
  MLS_ERR_UNSUPPORTED = -2, /* valid request this build does not handle */
  MLS_ERR_HIP = -3,         /* a HIP runtime call failed */
  MLS_ERR_OOM = -4,         /* device allocation failed */
  MLS_ERR_NONFINITE = -5    /* device flag: non-finite or negative input */
} mls_status;

typedef enum { MLS_FP64 = 0, MLS_MIXED = 1 } mls_precision;

/* Mixing rule of the pair coefficients (Sec. II.D). */
typedef enum { MLS_GEOMETRIC = 0, MLS_LORENTZ_BERTHELOT = 1 } mls_mixing;

/* Method parameters (Sec. III.D lists a, h, p, l as the knobs). */
typedef struct {
  double box[3];  /* L_x, L_y, L_z > 0: orthorhombic, periodic in all three
                     dimensions (Sec. II.C), origin at the box corner */
  double cutoff;  /* a > 0: local cutoff (eq:g_0); level k reaches 2^k a */
  double h;       /* target finest spacing > 0; each finest dimension gets
                     n = 2^(l-1) max(1, floor(L/(2^(l-1) h) + 1/2)) points
                     (uniform grids, Sec. III.A; spacing 2^(k-1) L/n on
                     level k) unless grid[] is given */
  int order;      /* p: 4 (cubic Hermite, eq:Phi-Hermite) or 6 (quintic) */
  int levels;     /* l >= 1 grids, or 0: the largest l whose coarsest grid
                     keeps >= p points per dimension */
  int grid[3];    /* explicit finest grid (each divisible by 2^(l-1)), or
                     all 0 to derive it from h */
  int precision;  /* mls_precision: MLS_FP64 computes everything in FP64;
                     MLS_MIXED does pair, grid-transfer and stencil
                     arithmetic in FP32 with FP64 accumulation of energy,
                     forces and grid charges, and keeps the coarsest level
                     and the energy reduction in FP64 */
  int continuity; /* k = 1..4: smoothing function gamma_k, the order-k Taylor
                     polynomial of rho^-6 = (1 + u)^(-1/2) in u = rho^12 - 1
                     for rho < 1 (C^k at rho = 1; the family of Sec. III.B).
                     2 is eq:gamma; 0 means 2 */
  int mixing;     /* mls_mixing: MLS_GEOMETRIC (per-atom C6, mls_evaluate) or
                     MLS_LORENTZ_BERTHELOT (per-atom epsilon and sigma,
                     mls_evaluate_lb; FP64 plans only) */
  double skin;    /* >= 0, below a (0: none).  Linked cells at least (a + skin)/2
                     wide (a + skin where the box is narrow) and every cell
                     search widened by skin/2, so the sorted atoms and cells
                     of one binning stay valid while no atom has moved more
                     than skin/2: mls_md_run then bins again only when an
                     atom has moved that far since the last binning (checked
                     on the device every step) and otherwise re-gathers the
                     new positions through the stored order.  Other entry
                     points bin on every call.  Results do not depend on the
                     skin beyond rounding. */
} mls_params;

/* Resolved plan geometry (host struct filled by mls_plan_get_info). */
typedef struct {
  int levels;              /* l */
  int grid[3];             /* finest grid n_1 */
  int coarsest[3];         /* n_l */
  int cells[3];            /* linked cells per dimension */
  double h_eff[3];         /* finest spacing L_d / n_1,d */
  int64_t taps;            /* stencil offsets of levels 1..l-1 */
  int64_t n_max;           /* largest n mls_evaluate accepts */
  int64_t workspace_bytes; /* device memory the plan holds */
  int precision;
  int order;
  double cell_width[3];    /* linked-cell width L_d / cells_d */
  int continuity;          /* k of gamma_k */
  int mixing;              /* mls_mixing */
  int stencil_path;        /* mls_stencil_path: kernel and arithmetic of the
                              level stencils of levels 1..l-1 */
} mls_plan_info;

/* Level-stencil kernels (mls_plan_info.stencil_path).  R is the stencil's
 * half width in finest-grid points, ceil(2a / h) per dimension at most.
 * FP32 tiles serve MLS_MIXED plans up to R = 12, FP64 tiles FP64 plans up
 * to R = 8; beyond that both precisions run FP64 kernels (a streaming kernel
 * up to R = 12, then one thread per output point over the tap table). */
typedef enum {
  MLS_STENCIL_NONE = 0,        /* l = 1: no level stencils */
  MLS_STENCIL_TILE_F32 = 1,
  MLS_STENCIL_TILE_F64 = 2,
  MLS_STENCIL_STREAM_F64 = 3,
  MLS_STENCIL_TAPS_F64 = 4,
  MLS_STENCIL_TILE_MFMA_F32 = 5  /* mixed, R <= 6: the FP32 tile on v_mfma_f32_16x16x4_f32
                                   (z band x folded mirror images), selected at plan
                                   creation by MLS_STENCIL_MFMA=1 in the environment */
} mls_stencil_path;

/* Build a plan on the current HIP device: resolves grids, levels and linked
 * cells, tabulates the level-1 stencil g_1 (eq:g_k; the same table serves
 * every level k < l scaled by 2^(-6(k-1)), Sec. II.A.4) and the coarsest
 * kernel K_l[delta] = sum_n g_l(|delta o h_l + n o L|) by an Ewald-type r^-6
 * lattice sum (eq:last-grid-periodic-transformed; precomputed once, Sec.
 * II.C), and allocates the workspace for up to n_max atoms.
 * params: host pointer; out: host pointer receiving the plan.
 * Errors: MLS_ERR_INVALID_ARG (bad parameter), MLS_ERR_OOM, MLS_ERR_HIP. */
mls_status mls_plan_create(const mls_params* params, int64_t n_max, mls_plan_t* out);

/* Copy the resolved geometry into *info (host). */
mls_status mls_plan_get_info(mls_plan_t plan, mls_plan_info* info);

/* One MLS energy-and-force evaluation (Sec. II.B), enqueued on `stream`
 * (a hipStream_t; NULL = the null stream).  No host synchronisation and no
 * allocation.
 *   n          0 <= n <= n_max atoms (n = 0 gives E = 0)
 *   pos        device (n,3) float64, row-major
 *   c6         device (n) float64, >= 0
 *   energy     device, 1 float64: E (required)
 *   forces     device (n,3) float64 F = -dE/dx, or NULL
 *   potential  device (n) float64: u_i = e^{0,tot}_i of eq:interpolation,
 *              including the grid self term gamma(0)/a^6 xi_i, or NULL
 *   dE_dc6     device (n) float64: dE/dC6_i = -(u_i - gamma(0) a^-6 xi_i) /
 *              (2 xi_i) (infinite where C6_i = 0), or NULL
 * Errors: MLS_ERR_INVALID_ARG (null plan/pos/c6/energy, n out of range),
 * MLS_ERR_HIP (launch failure). */
mls_status mls_evaluate(mls_plan_t plan, int64_t n, const double* pos, const double* c6,
                        double* energy, double* forces, double* potential, double* dE_dc6,
                        void* stream);

/* Potential energy and forces of the full pair potential eq:disp-pair-pot,
 * V_ij = C^rep_ij r^-12 - C^disp_ij r^-6 (Sec. II.D), for molecular dynamics
 * (Sec. III.A): the dispersion part exactly as mls_evaluate, plus the
 * repulsive part with geometric mixing C^rep_ij = sqrt(C12_i C12_j), summed
 * directly over every periodic image closer than rc (no grid part: the
 * r^-12 term is short-ranged):
 *   E_rep = 1/2 sum_i sum'_{(j,n), r < rc} C^rep_ij r^-12,  F_rep = -grad E_rep.
 * The repulsion is evaluated on the atoms binned by the same evaluation, in
 * the precision of the local part (mixed plans: FP32 pair terms summed in
 * FP64, as the dispersion).  Plan: geometric mixing.
 *   c12     device (n) FP64, finite and >= 0 (else device flag bit 3)
 *   rc      repulsion cutoff, 0 < rc <= a (host)
 *   energy  device, 1 FP64: E_disp + E_rep (overwritten)
 *   forces  device (n,3) FP64, or NULL
 * Same ordering, threading and error behaviour as mls_evaluate. */
mls_status mls_evaluate_md(mls_plan_t plan, int64_t n, const double* pos, const double* c6, const double* c12,
                           double rc, double* energy, double* forces, void* stream);

/* nsteps steps of velocity-Verlet molecular dynamics with the forces of
 * mls_evaluate_md (the paper's MD runs, Sec. III.A, do not name their
 * integrator; velocity Verlet is the standard choice):
 *   v += dt/2 F/m;  x += dt v;  F = F(x);  v += dt/2 F/m.
 * pos and vel (device (n,3) FP64) are advanced in place; positions are not
 * wrapped (the evaluation wraps them internally).  Outputs, all device FP64:
 *   forces  (n,3): forces at the final positions (required when n > 0)
 *   epot    (nsteps+1): potential energy after each force evaluation
 *           (index 0: initial positions)
 *   ekin    (nsteps+1): kinetic energy 1/2 sum_i |v_i|^2 / inv_mass_i at the
 *           same instants
 *   inv_mass device (n) FP64: 1/m_i, finite and > 0 (else device flag bit 3,
 *           as are non-finite velocities)
 *   dt      time step (host, finite); nsteps >= 0 (0: one evaluation)
 * Enqueued on `stream` with no host synchronisation and no allocation
 * (nsteps + 1 evaluations and nsteps + 1 integrator launches).  Errors: as
 * mls_evaluate_md, plus MLS_ERR_INVALID_ARG for null outputs, nsteps < 0 or
 * non-finite dt. */
mls_status mls_md_run(mls_plan_t plan, int64_t n, double* pos, double* vel, const double* c6, const double* c12,
                      double rc, const double* inv_mass, double dt, int nsteps, double* forces, double* epot,
                      double* ekin, void* stream);

/* Multiple time stepping (r-RESPA) with the MLS splitting itself: the fast
 * force is the local part of eq:evaluation (k = 0, the g_0 pair sum) plus the
 * repulsion of mls_evaluate_md; the slow force is the grid part (levels
 * 1..l, eq:anterpolation to eq:interpolation), the smooth remainder, applied
 * every k_slow steps: the split of length scales for multiple-time-step
 * methods that Sec. I credits the method with, here with two time steps
 * (r-RESPA, Tuckerman, Berne and Martyna 1992).  One outer step of
 * k_slow * dt:
 *   v += (k_slow dt / 2) F_slow/m;
 *   k_slow times: v += dt/2 F_fast/m; x += dt v; F_fast(x); v += dt/2 F_fast/m;
 *   F_slow(x); v += (k_slow dt / 2) F_slow/m.
 * k_slow = 1 is velocity Verlet with F_fast + F_slow (mls_md_run up to
 * rounding order).  nsteps counts inner steps and must be a multiple of
 * k_slow.  Outputs (device FP64):
 *   forces  (n,3): F_fast + F_slow at the final positions
 *   epot    (nsteps/k_slow + 1): E_fast + E_slow after each outer step
 *           (index 0: initial positions), where E_fast = -1/2 sum_i xi_i e0_i
 *           + E_rep and E_slow = the rest of the MLS energy
 *   ekin    (nsteps/k_slow + 1): kinetic energy at the same instants
 * Arguments, flags, ordering and errors as mls_md_run, plus
 * MLS_ERR_INVALID_ARG for k_slow < 1 or nsteps not a multiple of k_slow.
 * Every fast and every slow evaluation bins the atoms itself (no neighbour
 * structure is reused across steps). */
mls_status mls_md_run_mts(mls_plan_t plan, int64_t n, double* pos, double* vel, const double* c6,
                          const double* c12, double rc, const double* inv_mass, double dt, int nsteps, int k_slow,
                          double* forces, double* epot, double* ekin, void* stream);

/* Multiple time stepping per MLS level (r-RESPA with three nested time
 * steps), the level-by-level version of mls_md_run_mts's split:
 *   fast = the local part of eq:evaluation (k = 0) plus the repulsion,
 *          every step dt;
 *   mid  = the level-1 grid part, the interpolation (eq:interpolation) of
 *          the level-1 stencil result e^1 alone, every k_mid steps (empty,
 *          zero, for l = 1);
 *   slow = the rest of the grid part: the interpolation of E^1 prolongated
 *          from E^2 without e^1 (levels 2..l; for l = 1 the coarsest level,
 *          which is level 1), with the self-energy term, every k_mid k_slow
 *          steps.
 * Interpolation is linear, so mid + slow is the whole grid part.  One outer
 * step of k_mid k_slow dt:
 *   v += (k_mid k_slow dt/2) F_slow/m;
 *   k_slow times: v += (k_mid dt/2) F_mid/m;
 *                 k_mid times: v += dt/2 F_fast/m; x += dt v; F_fast(x); v += dt/2 F_fast/m;
 *                 F_mid(x); v += (k_mid dt/2) F_mid/m;
 *   F_slow(x); v += (k_mid k_slow dt/2) F_slow/m.
 * k_slow = 1 is mls_md_run_mts with k_slow = k_mid; k_mid = k_slow = 1 is
 * mls_md_run (up to rounding order).  nsteps counts inner steps and must be a
 * multiple of k_mid k_slow.  Outputs (device FP64): forces (n,3) = F_fast +
 * F_mid + F_slow at the final positions; epot and ekin
 * (nsteps / (k_mid k_slow) + 1): E_fast + E_mid + E_slow and the kinetic
 * energy at the outer-step boundaries (index 0: initial positions).
 * Arguments, flags, ordering and errors as mls_md_run_mts, plus
 * MLS_ERR_INVALID_ARG for k_mid < 1, k_slow < 1 or nsteps not a multiple of
 * k_mid k_slow.  Plan: geometric mixing. */
mls_status mls_md_run_mts_levels(mls_plan_t plan, int64_t n, double* pos, double* vel, const double* c6,
                                 const double* c12, double rc, const double* inv_mass, double dt, int nsteps,
                                 int k_mid, int k_slow, double* forces, double* epot, double* ekin, void* stream);

/* One evaluation under Lorentz-Berthelot mixing (Sec. II.D,
 * eq:disp-pair-pot-multilevel-LorentzBerthelot): pair coefficient
 * C_ij = 2 sqrt(eps_i eps_j) ((sigma_i + sigma_j)/2)^6 (eq:xi-lj), so
 * E = -1/2 sum_{i,j,n}' C_ij r^-6 (LJ dispersion sign) and F = -grad E.  The
 * local part uses C_ij directly; the grid part runs the steps of Sec. II.B
 * once per charge vector xi_{i,k} = sigma_i^k sqrt(binom(6,k) 2 eps_i) / 8,
 * k = 0..6, pairing vector k with vector 6 - k (seven instances, as the paper
 * states).  The plan must have mixing = MLS_LORENTZ_BERTHELOT.  In MLS_MIXED
 * precision the pair kernel evaluates C_ij and g_0 in FP32 and the level
 * stencils work in FP32 on the charges minus their mean, as under geometric
 * mixing; anterpolation sums, the coarsest level and interpolation stay FP64.
 *   eps, sigma  device (n) FP64, finite and >= 0 (else a device flag, as C6)
 *   energy      device, 1 FP64 (overwritten); forces device (n,3) or NULL
 * Same ordering, threading and error behaviour as mls_evaluate. */
mls_status mls_evaluate_lb(mls_plan_t plan, int64_t n, const double* pos, const double* eps, const double* sigma,
                           double* energy, double* forces, void* stream);

/* Intermediate results of the last evaluation, for per-stage checks.
 * `what` selects the array, written to device memory `dst` of `capacity`
 * bytes (MLS_ERR_INVALID_ARG if too small), enqueued on `stream`:
 *   MLS_STAGE_PERM        int32 (n): original index of the s-th cell-sorted atom
 *   MLS_STAGE_CELL_START  int32 (cells+1): first sorted atom of each cell
 *   MLS_STAGE_E0          float64 (n), original order: local potential e^0_i
 *   MLS_STAGE_FLOC        float64 (n,3), original order: local forces
 *   MLS_STAGE_Q           float64 grid of level `level`: q^k (charges)
 *   MLS_STAGE_E_LEVEL     float64 grid of level `level`: e^k (evaluation)
 *   MLS_STAGE_E_TOTAL     float64 grid of level `level`: E^k (after prolongation)
 * Grids are x fastest (index (z*ny + y)*nx + x), level 1 = finest. */
enum {
  MLS_STAGE_PERM = 0,
  MLS_STAGE_CELL_START = 1,
  MLS_STAGE_E0 = 2,
  MLS_STAGE_FLOC = 3,
  MLS_STAGE_Q = 4,
  MLS_STAGE_E_LEVEL = 5,
  MLS_STAGE_E_TOTAL = 6
};
mls_status mls_plan_copy_stage(mls_plan_t plan, int what, int level, void* dst, int64_t capacity,
                               void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * evaluation of mls_evaluate for the parameters in *params (host), with the
 * plan's workspace in a 64 MiB device array that the library holds per
 * device until the process ends, instead of memory from mls_plan_create.
 * Calls no hipMalloc, hipFree or other allocating routine, and creates no
 * stream or event: every stage runs in order on `stream`.  Each call waits
 * for `stream` (an earlier call's work on it still reads the array),
 * rebuilds the plan's tables on the host (the coarsest lattice kernel among
 * them, so each call costs a plan creation: suited to small systems),
 * uploads them, clears what must start at zero, and enqueues the
 * evaluation.  Arguments as for mls_evaluate (n atoms, device pos, c6,
 * energy, forces, potential, dE_dc6; outputs overwritten).  All calls on one
 * device share the array: calls that overlap on one device (different
 * streams or threads) race.  The data flags of mls_plan_status are not
 * reported.
 * Errors: MLS_ERR_INVALID_ARG (as mls_evaluate, or Lorentz-Berthelot mixing),
 * MLS_ERR_UNSUPPORTED when the workspace for n atoms and these grids exceeds
 * the 64 MiB array (the message says so), MLS_ERR_HIP. */
mls_status mls_evaluate_noalloc(const mls_params* params, int64_t n, const double* pos, const double* c6,
                                double* energy, double* forces, double* potential, double* dE_dc6,
                                void* stream);

/* Synchronise the plan's last stream and report the device flags set by
 * evaluations since the previous call (bit 0: non-finite position, bit 1:
 * non-finite or negative C6, bit 2: internal consistency check of the
 * anterpolation blocking failed, results invalid, bit 3: non-finite or
 * negative C12, non-finite velocity or non-positive inverse mass in the MD
 * entry points), then clear them.
 * *flags: host.  Returns MLS_ERR_NONFINITE when bit 0, 1 or 3 is set,
 * MLS_ERR_HIP when only bit 2 is, else MLS_OK. */
mls_status mls_plan_status(mls_plan_t plan, int* flags);

/* Per-stage device timing for measurement: with timing enabled, each
 * following evaluation (up to 256) records hipEvents on its own stream
 * between the stages listed below.  mls_plan_read_timing synchronises, writes
 * the summed milliseconds of every stage over the recorded evaluations into
 * ms[MLS_NUM_STAGES] (host) and the evaluation count into *count (host),
 * and starts a new recording window.  Enabling timing creates the events;
 * evaluations themselves never allocate. */
enum {
  MLS_T_BINNING = 0,   /* wrap, cell count, scan, scatter, in-cell order */
  MLS_T_PAIR = 1,      /* local g_0 pair sum */
  MLS_T_ANTERP = 2,    /* anterpolation */
  MLS_T_RESTRICT = 3,  /* all restrictions */
  MLS_T_STENCIL = 4,   /* cutoff stencils of levels 1..l-1 */
  MLS_T_COARSEST = 5,  /* all-to-all on the coarsest grid */
  MLS_T_PROLONG = 6,   /* all prolongations */
  MLS_T_INTERP = 7,    /* interpolation, outputs, energy reduction */
  MLS_NUM_STAGES = 8
};
mls_status mls_plan_set_timing(mls_plan_t plan, int enable);
mls_status mls_plan_read_timing(mls_plan_t plan, double* ms, int* count);

/* Release the plan and its workspace (NULL is accepted). */
mls_status mls_plan_destroy(mls_plan_t plan);

/* ---------------------------------------------------------------------------
 * Batched form: many independent periodic boxes of uneven size, each with its
 * own parameter set (grids, levels and cells are resolved per box exactly as
 * mls_plan_create does; the method is that of Sec. II applied to every box).
 * One evaluation of the batch is a fixed sequence of launches, one per phase
 * of Sec. II.B (binning, local part, anterpolation, each restriction, the
 * level stencils, the coarsest level, each prolongation, interpolation);
 * each launch covers every box with work in that phase by walking a
 * (box, block) work list with a persistent grid.  The sequence is captured
 * into a hipGraph on first use and replayed.
 *
 *   nbox       1 .. 2^20 boxes
 *   per_box    host (nbox) parameter sets; precision, order, continuity and
 *              mixing must agree
 *   n_per_box  host (nbox) atom counts >= 0 (total < 2^31)
 *   autotune   nonzero: the first mls_batch_evaluate times every stage over
 *              a set of persistent grid sizes and stencil tile depths on the
 *              caller's data, keeps the fastest per stage, then captures.
 *              That first call synchronises the device.
 *
 * Layout: atoms of box b are rows off[b] .. off[b+1]-1 of pos (n,3), c6 (n),
 * forces (n,3) and dE_dc6 (n), off being the exclusive prefix sum of
 * n_per_box; energies is device (nbox).  All arrays are device FP64 owned by
 * the caller; forces and dE_dc6 may be NULL.  Outputs are overwritten.
 * Changing any of the five pointers between calls rebuilds the launch tables
 * and the graph, which synchronises the device; calls with the same pointers
 * are enqueue-only.  Errors: as mls_evaluate; mls_batch_create returns
 * MLS_ERR_UNSUPPORTED for a box whose level-stencil window 2a/h exceeds 8
 * grid points.  A batch is not thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct {
  int blocks[MLS_NUM_STAGES]; /* persistent grid of each MLS_T_* stage in blocks; 0 = one block per item */
  int stencil_zc;             /* z extent of a level-stencil tile: 16 or 8 (16 applies to windows <= 6) */
  double tuned_ms;            /* one evaluation with this shape, as timed by the autotuner (0: not timed) */
  double stage_ms[MLS_NUM_STAGES]; /* its MLS_T_* stages (0: not timed) */
} mls_batch_tuning;

mls_status mls_batch_create(int nbox, const mls_params* per_box, const int64_t* n_per_box,
                            int autotune, mls_batch_t* out);
mls_status mls_batch_evaluate(mls_batch_t batch, const double* pos, const double* c6,
                              double* energies, double* forces, double* dE_dc6, void* stream);
/* Batched Lorentz-Berthelot evaluation (Sec. II.D, as mls_evaluate_lb per
 * box): the boxes were created with mixing = MLS_LORENTZ_BERTHELOT (FP64 or
 * mixed precision).  Every chain phase (charges, anterpolation, restrictions,
 * level stencils, coarsest level, prolongations) covers the seven charge
 * vectors of every box in one launch.
 *   eps, sigma  device (n) FP64 in the batch's row layout, finite and >= 0
 *   energies    device (nbox); forces device (n,3) or NULL
 * Changing any of the six pointers rebuilds the launch tables as above.
 * Errors: as mls_batch_evaluate; MLS_ERR_INVALID_ARG on a geometric batch
 * (and mls_batch_evaluate on a Lorentz-Berthelot batch). */
mls_status mls_batch_evaluate_lb(mls_batch_t batch, const double* pos, const double* eps, const double* sigma,
                                 double* energies, double* forces, void* stream);
/* enable (default) or disable graph replay; disabled, every call launches eagerly */
mls_status mls_batch_set_graph(mls_batch_t batch, int enable);
/* current launch shape (after autotuning: the tuned one) / force a shape (cancels a pending autotune) */
mls_status mls_batch_get_tuning(mls_batch_t batch, mls_batch_tuning* tuning);
mls_status mls_batch_set_tuning(mls_batch_t batch, const mls_batch_tuning* tuning);
/* resolved grids, levels and cells of box `box` (as mls_plan_get_info) */
mls_status mls_batch_box_info(mls_batch_t batch, int box, mls_plan_info* info);
/* synchronises; ORs the data flags of every box (MLS_ERR_NONFINITE if any) and clears them */
mls_status mls_batch_status(mls_batch_t batch, int* device_flags);
mls_status mls_batch_destroy(mls_batch_t batch);

/* Static description of a status code. */
const char* mls_status_string(int status);

/* Detail of the last error raised on the calling thread ("" if none). */
const char* mls_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MLSDISP_H */
