/*
 * ehdlb.h — C ABI of the ternary electrohydrodynamic lattice-Boltzmann library (gfx950).
 *
 * One library call advances the coupled system the paper defines in its Methods
 * section: three conservative Allen-Cahn phase fields (droplet, lubricant,
 * ambient; Eqs. 8, 15-19), incompressible flow with capillary and electric
 * forcing (Eqs. 9-12), the Gauss law for the potential (Eq. 13, solved to a
 * tolerance every step as the inner iteration of Eq. 21 does) and leaky-
 * dielectric charge transport (Eq. 14), on a lattice with micropillar walls,
 * energy-based wetting (Eq. 20) and electrodes.  The problem statement follows
 * the Results section (Fig. 1): pillars and substrate grounded, electrodes
 * held at their potential, insulating (Neumann) walls elsewhere.
 *
 * Conventions
 *   - Lattice units.  Phase index 0 = droplet, 1 = lubricant, 2 = ambient.
 *   - Node index n = x + Nx*(y + Ny*z), x fastest; 2D lattices have Nz = 1.
 *   - Every axis wraps in index space; an axis declared non-periodic must have
 *     solid end layers (EHDLB_EINVAL otherwise).
 *   - Host arrays passed in are copied during the call; the caller keeps
 *     ownership.  Device memory is never allocated by the library: the caller
 *     provides one device workspace (ehdlb_workspace_bytes) and a HIP stream
 *     at ehdlb_bind, and keeps both alive until ehdlb_destroy.
 *   - Every call returns an ehdlb_status; nothing throws across the ABI.  The
 *     message of the last error is available from ehdlb_last_error.
 *   - A context is single-threaded: concurrent calls on one context are not
 *     allowed; distinct contexts are independent.
 */
#ifndef EHDLB_H
#define EHDLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EHDLB_MAX_ELECTRODES 4

typedef enum {
  EHDLB_OK = 0,
  EHDLB_EINVAL = -1,      /* invalid parameter, geometry or argument          */
  EHDLB_ESTATE = -2,      /* call out of order (e.g. step before set_phase)   */
  EHDLB_EHIP = -3,        /* HIP runtime error (message in ehdlb_last_error)  */
  EHDLB_ENOMEM = -4,      /* workspace smaller than ehdlb_workspace_bytes     */
  EHDLB_ENONFINITE = -5,  /* non-finite field detected (sticky)               */
  EHDLB_ENOCONV = -6      /* potential solve hit its iteration cap (sticky)   */
} ehdlb_status;

typedef enum { EHDLB_FP64 = 0, EHDLB_FP32_DEV = 1 } ehdlb_precision;

/* Node flags (uint8): fluid, grounded solid (potential 0: pillars and
 * substrate), insulating solid (zero normal flux), electrode k (potential
 * V_k(t)).  Every non-fluid node is a wall for the populations. */
typedef enum {
  EHDLB_FLUID = 0,
  EHDLB_GROUND = 1,
  EHDLB_INSULATOR = 2,
  EHDLB_ELECTRODE0 = 3
} ehdlb_flag;

/* Fields readable with ehdlb_read_field, always returned as float64 on the host.
 * PHI*: phase fields of the current populations (Eq. 19).  UX..UZ: velocity of
 * the last completed step (u = j + F/2, F / rho with unequal densities).  P: cs^2
 * times the zeroth moment of the flow populations' deviation, the pressure at unit
 * density (p / rho with unequal densities).  RHO_E: charge density of the current populations.
 * POT: potential solved in the last completed step.  Q: Ohmic source of the
 * last completed step.  POPS: the current populations in canonical order
 * [family][q][node] with families g (deviation from w), f1, f2, f3, h (the
 * last only when the field is on); size ehdlb_num_populations doubles. */
typedef enum {
  EHDLB_FIELD_PHI1 = 0, EHDLB_FIELD_PHI2 = 1, EHDLB_FIELD_PHI3 = 2,
  EHDLB_FIELD_UX = 3, EHDLB_FIELD_UY = 4, EHDLB_FIELD_UZ = 5,
  EHDLB_FIELD_P = 6, EHDLB_FIELD_RHO_E = 7, EHDLB_FIELD_POT = 8,
  EHDLB_FIELD_Q = 9, EHDLB_FIELD_POPS = 10
} ehdlb_field;

typedef struct ehdlb_ctx ehdlb_ctx;

typedef struct {
  int32_t dim;          /* 2 (D2Q9) or 3 (D3Q19)                                */
  int32_t n[3];         /* Nx, Ny, Nz (Nz = 1 in 2D); each >= 1                 */
  int32_t periodic[3];  /* 1: the axis wraps; 0: its two end layers are solid  */
  int32_t precision;    /* ehdlb_precision                                      */
} ehdlb_lattice;

typedef struct {
  double tau_flow[3];       /* flow relaxation time per phase (> 1/2); nu = (tau - 1/2)/3,
                               mixed linearly in the phase fields                         */
  double mobility;          /* M of Eq. 8 (> 0)                                           */
  double width;             /* W_int of Eqs. 8, 10, 18, 20 (> 0)                          */
  double gamma12, gamma13, gamma23;   /* pair tensions (> 0), Eq. 11; each Upsilon_i nonzero
                                         (negative for a spreading phase, e.g. the
                                         lubricant cloaking the droplet when gamma13 >
                                         gamma12 + gamma23) and Upsilon_T finite            */
  double cos12, cos13, cos23;         /* cos(theta_ij) of Eq. 20, theta_ij measured through
                                         phase i                                          */
  int32_t ehd;              /* 0: no electric field (no potential, no charge family)      */
  int32_t reserved0;
  double eps[3];            /* permittivity per phase (> 0), mixed linearly               */
  double cond[3];           /* conductivity per phase (>= 0), mixed linearly              */
  double charge_diffusion;  /* alpha of Eq. 14 (>= 0)                                     */
  double body_force[3];     /* uniform body force density                                 */
  double electrode_volts[EHDLB_MAX_ELECTRODES];  /* constant V_k unless a schedule is set;
                                                    NaN: switched off and floating (below) */
  double poisson_tol;       /* stop when max|b - A phi| <= tol * max|b| (residual in FP64),
                               or when it reaches the rounding floor of phi stored in the
                               path's precision, 8 eps max_i sum_j |A_ij phi_j|           */
  int32_t poisson_max_iter; /* iteration cap of the potential solve (>= 1)                */
  int32_t poisson_check_every;  /* residual check period in iterations (>= 1)             */
  double s_high;            /* relaxation rate of the raw moments the paper leaves unspecified
                               (Eq. 15 and the Eq. 20 pair give S without its entries): order
                               >= 2 for the phase fields and the charge, >= 3 for the flow,
                               in (0, 2); 0 means the default 1 (those moments then leave
                               the collision at equilibrium)                              */
  double rho[3];            /* density per phase (> 0; 0 means the default 1), mixed
                               linearly (Eq. 9 with rho(Phi)).  All 1: the incompressible
                               flow about the unit density.  Unequal: the velocity-based
                               form (the flow populations carry p / (rho cs^2); the
                               acceleration F / rho with the pressure force
                               -cs^2 p* grad(rho) and the viscous force
                               nu (grad u + grad u^T) . grad(rho)), which ehdlb_adjoint
                               reverses as well                                        */
} ehdlb_params;

typedef struct {
  int64_t step;             /* completed steps                                          */
  double mass[3];           /* sum of Phi_i over fluid nodes                            */
  double centroid[3];       /* Phi_1-weighted mean node coordinate (NaN, undefined,     */
                            /* when mass[0] is 0: no droplet)                           */
  double velocity[3];       /* Phi_1-weighted mean velocity of the last completed step  */
                            /* (0 when that step's Phi_1 sums to 0)                     */
  double total_charge;      /* sum of rho_e over fluid nodes                            */
  double sum_phi_drift;     /* max |Phi_1 + Phi_2 + Phi_3 - 1| over fluid nodes         */
  double poisson_residual;  /* last relative FP64 residual of the potential solve       */
  double poisson_initial_residual; /* its relative residual before iterating (warm start) */
  int32_t poisson_iters;    /* iterations of the last potential solve                   */
  int32_t flags;            /* bit 0: non-finite seen; bit 1: solve hit its cap         */
} ehdlb_obs;

/* Validate lattice and parameters and create a context (no device work).
 * EINVAL: dim not 2/3, sizes < 1, Nz != 1 in 2D, tau <= 1/2, M <= 0, W <= 0,
 * a tension <= 0, a zero Upsilon_i or an infinite Upsilon_T, eps <= 0, cond < 0, alpha < 0, tol <= 0, max_iter < 1,
 * s_high outside (0, 2), a density < 0. */
ehdlb_status ehdlb_create(const ehdlb_lattice* lattice, const ehdlb_params* params,
                          ehdlb_ctx** out);

/* Bytes of device workspace the context needs (populations A/B, fields,
 * solver hierarchy, reduction scratch).  Valid right after create. */
size_t ehdlb_workspace_bytes(const ehdlb_ctx* ctx);

/* Bind a caller-owned device buffer of at least ehdlb_workspace_bytes bytes
 * (256-byte aligned) on the current HIP device, and the HIP stream (a
 * hipStream_t, or NULL for the null stream) all work is enqueued on.
 * ENOMEM if bytes is too small; EINVAL on a misaligned pointer. */
ehdlb_status ehdlb_bind(ehdlb_ctx* ctx, void* device_workspace, size_t bytes, void* hip_stream);

/* Node flags, host array of N uint8 (ehdlb_flag values; 3 + k for electrode k).
 * Builds the wetting links of solid nodes next to fluid and the potential
 * solver's hierarchy on the host, then copies them to the device.
 * EINVAL: unknown flag, electrode index >= EHDLB_MAX_ELECTRODES, fluid on the
 * end layer of a non-periodic axis, a fluid node without a fluid neighbour, or
 * (field on) a fluid region with no grounded or electrode face.
 * Can be called before bind (then only validation and host tables). */
ehdlb_status ehdlb_set_geometry(ehdlb_ctx* ctx, const uint8_t* flags);

/* Initial phase fields, host float64 array [3][N].  Populations are set to
 * equilibrium at rest (u = 0, rho = 1), rho_e = 0 (no bulk free charge), and
 * the step counter to 0.  Needs bind and set_geometry (ESTATE otherwise). */
ehdlb_status ehdlb_set_phase(ehdlb_ctx* ctx, const double* phi);

/* Optional initial charge density, host float64 [N] (after set_phase). */
ehdlb_status ehdlb_set_charge(ehdlb_ctx* ctx, const double* rho_e);

/* Piecewise-constant voltage schedule of electrode k: during step t (0-based)
 * the electrode holds volts[s] with s = floor(t * n_seg / t_total), clamped to
 * n_seg - 1 for t >= t_total.  The array is copied.  A NaN voltage switches
 * the electrode off and leaves it floating for that segment: its faces then
 * carry no flux (insulating, as the walls without electrodes), the reading of
 * the switching protocols of the Results (Fig. 5), where an electrode that is
 * switched off stops acting on the droplet; the adjoint's dL/dV of such a
 * segment is 0.  A region whose only Dirichlet faces float has a singular
 * potential problem (the solve then reports ENOCONV).  EINVAL on k out of
 * range, n_seg < 0, t_total < 1 or an infinite voltage.  n_seg = 0 clears the
 * schedule. */
ehdlb_status ehdlb_set_schedule(ehdlb_ctx* ctx, int32_t electrode, int32_t n_seg,
                                const double* volts, int64_t t_total);

/* Advance n >= 0 steps.  Work is enqueued on the bound stream; the call
 * synchronises only for the potential solve's residual checks. */
ehdlb_status ehdlb_step(ehdlb_ctx* ctx, int64_t n);

/* Copy one field, as float64, to N values at dst (POPS: see above), the droplet
 * and flow fields the paper reports (Results: charge and flow fields, Fig. 2-3).
 * dst_is_device = 0: dst is host memory; the call synchronises the bound stream.
 * dst_is_device = 1: dst is device memory on the bound device (8-byte aligned);
 * the conversion is enqueued on the bound stream and the call returns without
 * waiting (dst is valid once the stream reaches that point).  The caller owns dst. */
ehdlb_status ehdlb_read_field(ehdlb_ctx* ctx, int32_t field, void* dst, int32_t dst_is_device);

/* Number of doubles ehdlb_read_field(EHDLB_FIELD_POPS) writes. */
size_t ehdlb_num_populations(const ehdlb_ctx* ctx);

/* Droplet observables of the current state (FP64 fixed-order reductions).
 * Synchronises.  Returns ENONFINITE / ENOCONV (sticky) after filling *out. */
ehdlb_status ehdlb_observables(ehdlb_ctx* ctx, ehdlb_obs* out);

/* For callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the droplet observables of
 * ehdlb_observables, computed by the same kernels in the same order, enqueued on
 * the bound stream without any host synchronisation or allocation; their
 * per-block partials live in a library-held device array (9 MiB per device,
 * kept until the process ends) instead of the workspace.  dev_out: 12 float64 in
 * device memory (8-byte aligned, caller-owned): mass[3], centroid[3],
 * velocity[3], total charge, max |sum Phi - 1|, count of fluid nodes with a
 * non-finite value (the context's sticky flags are not updated).  EINVAL for a
 * lattice above 2^24 nodes (16,777,216) or a null/misaligned dev_out; ESTATE
 * before set_phase or with another device current than at ehdlb_bind.  Every
 * call on one GPU shares that array: calls that overlap on one GPU (other
 * contexts, other streams or threads) race and must be serialised by the caller. */
ehdlb_status ehdlb_observables_device(ehdlb_ctx* ctx, double* dev_out);

/* Full state (populations, previous-step fields, potential, step counter) as
 * an opaque device blob of ehdlb_state_bytes bytes; save/load copy on the
 * bound stream (device to device). */
size_t ehdlb_state_bytes(const ehdlb_ctx* ctx);
ehdlb_status ehdlb_save_state(ehdlb_ctx* ctx, void* device_dst);
ehdlb_status ehdlb_load_state(ehdlb_ctx* ctx, const void* device_src);

/* Wetting links built by set_geometry (host, no device needed): for each
 * solid node next to fluid, the node index and the direction index n* of
 * the link along which its phase values are extrapolated.  Writes at most
 * cap entries and returns the total count (or a negative status). */
int64_t ehdlb_wetting_links(const ehdlb_ctx* ctx, int64_t* nodes, int32_t* dirs, int64_t cap);

/* Adjoint (reverse mode) of the whole coupled step with respect to a piecewise-
 * constant electrode-voltage schedule, for programmable droplet manipulation
 * (the target application of the Results' electrode-switching protocols).
 * Not in the paper: a training-system pattern (checkpoint and recompute).
 *
 * ehdlb_adjoint_workspace_bytes: device bytes for T steps with a checkpoint
 *   every K steps (ceil(T/K) full states, one final state, K per-step records
 *   of moments/potential/previous fields, the cotangent arrays).
 * ehdlb_forward_checkpointed: runs T steps from the current state (step t0),
 *   saving the checkpoints into the caller's device buffer (256-byte aligned,
 *   at least the size above); afterwards the context is at step t0 + T.
 * ehdlb_adjoint: given dL/d(centroid) and dL/d(velocity) of the final state
 *   (the observables of ehdlb_observables), returns on the host dL/dV for
 *   every segment of electrode k's schedule (n_seg doubles; one value if it
 *   has none).  For each segment, last to first, it reloads the checkpoint,
 *   recomputes K steps storing their records, and runs the adjoint steps
 *   backwards; the potential solve is differentiated as exact (one solve with
 *   the same symmetric matrix per step).  Deterministic; ends at the final
 *   state again.  ESTATE if anything that changes the state or the steps was
 *   called since the checkpointed forward (ehdlb_generation differs: set_geometry,
 *   set_phase, set_charge, set_schedule, set_solver_options, step with n > 0,
 *   load_state, another forward_checkpointed), EINVAL if the field is off.  With
 *   unequal phase densities the record holds the raw second moments of the flow
 *   populations, from which the reverse of the velocity-based form (the
 *   acceleration F/rho with the pressure and viscous density-gradient forces of
 *   the provisional collision) is rebuilt. */
size_t ehdlb_adjoint_workspace_bytes(const ehdlb_ctx* ctx, int64_t T, int32_t K);
ehdlb_status ehdlb_forward_checkpointed(ehdlb_ctx* ctx, int64_t T, int32_t K, void* device_workspace,
                                        size_t bytes);
ehdlb_status ehdlb_adjoint(ehdlb_ctx* ctx, const double dL_dcentroid[3], const double dL_dvelocity[3],
                           int32_t electrode, double* dL_dvolts);

/* Options of the potential solver: conjugate gradients preconditioned by one
 * symmetric multigrid V-cycle (aggregation of 2 cells per axis, Galerkin coarse
 * operators, dense solve on the coarsest level).  Smoothing: the degree-2
 * Chebyshev polynomial of the Jacobi-preconditioned operator D^-1 A on
 * [lo, hi] (0 < lo < hi <= 2; D^-1 A has its spectrum in (0, 2]), applied once
 * before and once after the coarse correction; overcorrect in (0, 4]: scale of
 * the coarse-grid correction.  warm_start (forward solves): 0 = each step's
 * solve starts from the previous step's potential; 1 = from the linear
 * extrapolation 2 phi(t-1) - phi(t-2); 2 = from the Galerkin projection of the
 * step's system onto the potentials of the last five steps (formed in the
 * basis phi(t-1) and its backward differences), the A-norm-optimal start in
 * their span, followed by at least one CG iteration; 3 = the same projection
 * without the minimum (fewest iterations; a solve that keeps the projected
 * start carries its error into the next steps' starts, correlated from step to
 * step, which biases gradients of the trajectory: ~6e-4 against the FP64
 * adjoint on 512x256 FP32 instead of ~1e-4 with 2); 4 (default) = 3 in
 * ehdlb_step and 2 in the forward that a gradient differentiates
 * (ehdlb_forward_checkpointed, and the adjoint's recompute of it), so plain
 * forward runs take the fewest iterations and gradients keep their accuracy
 * (the two forwards agree to the solver tolerance).  The adjoint's solves
 * always start from the projection onto the adjoint potentials of steps
 * t+1..t+6.  The earlier potentials are part of the saved state, so replays
 * from a checkpoint take the same iterates; switching modes in mid-run projects
 * once onto stale potentials (still a valid start).  Defaults lo = 0.5, hi = 2,
 * overcorrect = 2, warm_start = 4.  EINVAL outside the ranges. */
ehdlb_status ehdlb_set_solver_options(ehdlb_ctx* ctx, double lo, double hi, double overcorrect,
                                      int32_t warm_start);

/* Optional timing of the step's three phases with HIP events recorded on the
 * bound stream: [0] moments and wetting ghosts, [1] potential solve (setup,
 * multigrid-preconditioned CG, residual checks), [2] fused collide-stream.
 * set_timing(1) resets the accumulators (it creates events: needs a device);
 * ehdlb_timing synchronises and returns the summed milliseconds per phase and
 * the number of timed steps. */
ehdlb_status ehdlb_set_timing(ehdlb_ctx* ctx, int32_t on);
ehdlb_status ehdlb_timing(ehdlb_ctx* ctx, double* ms3, int64_t* steps);

/* Potential-solve statistics accumulated since the context was created or the last call
 * with reset != 0 (which clears them after reading).  Per kind k (0: solves of the forward
 * steps, 1: adjoint solves of ehdlb_adjoint): counts[2k] solves, counts[2k+1] conjugate-
 * gradient iterations, max_rel0[k] the largest initial relative residual max|b - A x0|/max|b|
 * of the warm start.  counts: int64[4], max_rel0: double[2] (host, either may be NULL). */
ehdlb_status ehdlb_solver_stats(ehdlb_ctx* ctx, int32_t reset, int64_t* counts, double* max_rel0);

/* Host-only workload presets (no context, no device): the droplet / lubricant /
 * ambient configurations of the paper's problem statement (Results, Fig. 1 and
 * its text: micropillars of solid fraction 0.25 infused with lubricant to their
 * tops, a droplet cap on the lubricant, an electrode segment on the opposite
 * wall, grounded pillars and substrate, insulating walls elsewhere; Methods:
 * M = 0.0025, W = 4; Fig. 2 contact angles theta_13 = 100, theta_23 = 5 degrees)
 * at the sizes of the named workloads:
 *   EHDLB_PRESET_C1  2D 128x64, 6-cell lubricant film, droplet R = 20, no field,
 *                    initial phase fields jittered by +-1e-6 (counter-based
 *                    SplitMix64 draws keyed by seed, node and component)
 *   EHDLB_PRESET_C2  2D 512x256, pillars 8/16/12, droplet R = 40, electrode 0.05
 *                    on 64 cells of the top wall 40 lu ahead of the droplet
 *   EHDLB_PRESET_C3  3D 256x128x96, pillars 6x6x10 at pitch 12, droplet R = 30
 *   EHDLB_PRESET_C4  the C2 geometry in the FP32 path (the schedule is the
 *                    caller's: ehdlb_set_schedule)
 *   EHDLB_PRESET_C5  3D 384x192x128, droplet R = 48
 *   EHDLB_PRESET_C1S..C4S reduced variants with the same structure (64x32,
 *                    128x64, 48x32x24, 96x48).
 * Writes the lattice and parameters; flags (N uint8) and phi ([3][N] float64) if
 * the pointers are not NULL (N = nx ny nz of the written lattice: call once with
 * NULL arrays to learn it).  seed keys the jitter of C1 and C1S only.  EINVAL on
 * an unknown id. */
enum {
  EHDLB_PRESET_C1 = 1, EHDLB_PRESET_C2 = 2, EHDLB_PRESET_C3 = 3, EHDLB_PRESET_C4 = 4, EHDLB_PRESET_C5 = 5,
  EHDLB_PRESET_C1S = 11, EHDLB_PRESET_C2S = 12, EHDLB_PRESET_C3S = 13, EHDLB_PRESET_C4S = 14
};
ehdlb_status ehdlb_preset(int32_t preset_id, ehdlb_lattice* lattice, ehdlb_params* params, uint8_t* flags,
                          double* phi, uint64_t seed);

/* Forward generation of the context: a counter bumped by every call that changes
 * the state or what the next steps compute (set_geometry, set_phase, set_charge,
 * set_schedule, set_solver_options, step with n > 0, load_state,
 * forward_checkpointed).  A caller that holds a checkpointed forward (for
 * example an autograd node) records it and checks it before ehdlb_adjoint. */
uint64_t ehdlb_generation(const ehdlb_ctx* ctx);

/* Bandwidth references (measurement only; no context, no method arithmetic): kernels
 * that are timed beside the fused collide-stream step to give its memory traffic two
 * ceilings.  All queue one launch on hip_stream (NULL: the null stream) and return.
 *   kind 0: copy `bytes` from src to dst, 16 bytes per lane (one float4 per thread);
 *           bytes and both addresses multiples of 16.
 *   kind 1: the same copy with 4 bytes per lane (one float per thread).
 *   kind 2: the population access pattern of the fused step without its arithmetic:
 *           nf (1..5) families of q single-precision populations per node of a periodic
 *           dims[0] x dims[1] x dims[2] lattice, stored by population ([nf][q][nodes],
 *           x fastest); each population is loaded once and stored at the node its
 *           lattice velocity points to (q = 9: D2Q9 with dims[2] = 1; q = 19: D3Q19).
 *           src and dst hold at least nf q nodes floats (`bytes` each) and do not overlap.
 *   kind 3: kind 2 with the population loads marked non-temporal.
 * EINVAL for an unknown kind, NULL buffers, sizes or alignments outside the above; EHIP
 * if the launch fails.  dst's contents are unspecified afterwards. */
ehdlb_status ehdlb_bandwidth_probe(int32_t kind, const void* src, void* dst, size_t bytes, const int32_t* dims,
                                   int32_t q, int32_t nf, void* hip_stream);

const char* ehdlb_last_error(const ehdlb_ctx* ctx);
void ehdlb_destroy(ehdlb_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* EHDLB_H */
