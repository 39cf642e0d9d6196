/*
 * fv.h -- C ABI of the fracture hot path (libfv.so, gfx950).
 *
 * The library advances the multi-material elastoplastic diffuse-interface
 * system of arXiv 2210.04037 (Wallis, Barton, Nikiforakis): the evolution
 * equations of Section 2.1 with the Romenskii closures of Section 2.3, Bonora
 * damage (Section 2.2), the void-opening fracture modifier (Section 3.1) and
 * the Lagrangian-coordinate perturbation field (Sections 2.4 and 3.2).
 *
 * Conventions shared by every entry point
 *   - Return value: FV_OK (0) or a negative status below.  No C++ exception
 *     crosses the ABI.  The text of the last error is in fv_last_error().
 *   - Device pointers are HIP device addresses owned by the caller (PyTorch
 *     tensors in the Python binding).  The library never allocates device
 *     memory: it keeps non-owning pointers into the caller's state, phi0 and
 *     workspace buffers, so a context must be destroyed before they are freed.
 *   - Host pointers are borrowed for the duration of the call only.
 *   - A context runs on one HIP stream (the one given to fv_init).  Calls
 *     marked "async" only enqueue work; errors found on the device (the
 *     non-physical-state flag) surface at the next syncing call.  A context
 *     is not thread-safe.
 *
 * State layout (one buffer per instance, structure of arrays, x fastest):
 *   state[f * ncell + (z * ny + y) * nx + x] for field f in the order of the
 *   evolution equations of Section 2.1:
 *     [phi_l] * N, [phi_l rho_l] * N, [phi_s rho_s eps_p, phi_s rho_s D] per
 *     solid, [rho u_i] * dim, rho E, Vbar components, [X_i] * dim
 *   Vbar components: 1D (11, 22, 33); 2D (11, 12, 21, 22, 33); 3D all nine,
 *   row-major.  The void fraction is 1 - sum phi_l (not stored).  Element
 *   type: double for FV_FP64, float for FV_FP32_BULK.  Materials: solids
 *   first, then at most one gas; N <= 2.  Two solids (and no gas) are
 *   compiled for 1D only; fv_init refuses them in 2D and 3D (FV_EINVAL).
 */
#ifndef FV_H
#define FV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define FV_OK 0
#define FV_EINVAL -1     /* invalid argument (message in fv_last_error) */
#define FV_ENOMEM -2     /* workspace too small */
#define FV_EDEVICE -3    /* HIP runtime error */
#define FV_ENONPHYS -4   /* device flag: NaN/Inf or non-positive density */
#define FV_ESTATE -5     /* call order violated */

/* boundary kinds, per side of each direction */
#define FV_BC_TRANSMISSIVE 0  /* zero-gradient ghost cells */
#define FV_BC_FREE 1          /* free surface: void outside (Section 3.1) */
#define FV_BC_PERIODIC 2      /* both sides of the direction; needs n >= 2 */

/* material kinds */
#define FV_MAT_SOLID 0   /* Romenskii EOS + shear modulus, Bonora damage */
#define FV_MAT_GAS 1     /* ideal gas, Grueneisen constant gamma - 1 */

/* precision policies */
#define FV_FP64 0        /* state and arithmetic in double */
#define FV_FP32_BULK 1   /* float state; double islands (see fv_options) */

/* Block schedules of the stage launch over an ensemble (fv_options.tile[2]):
 * the order in which the blocks of all instances are listed.  Results do
 * not depend on it. */
#define FV_SCHED_BY_INSTANCE 0    /* instance after instance (default) */
#define FV_SCHED_LARGEST_FIRST 1  /* instances by decreasing tile count */
#define FV_SCHED_INTERLEAVED 2    /* tile k of every instance before tile k+1 */

typedef struct fv_ctx fv_ctx;

/* Uniform grid of one instance.  dim in {1, 2, 3}; n[k] cells on [lo[k],hi[k]]
 * for k < dim (unused directions: n = 1, and their extent sets the cell
 * volume).  bc[k][0] / bc[k][1] are the lower / upper sides; periodic sides
 * come in pairs, on a direction of at least 2 cells (a one-cell periodic
 * direction would be its own neighbour).  An instance holds at most 2^31
 * cells; in 1D and 2D one field of its state (cells times the element size)
 * holds at most 4 GiB, i.e. 2^30 cells in FP32-bulk and 2^29 in FP64, so the
 * stage kernels address a cell with a 32-bit offset (FV_EINVAL beyond). */
typedef struct {
  int32_t dim;
  int32_t n[3];
  double lo[3];
  double hi[3];
  int32_t bc[3][2];
} fv_grid;

/* Material constants, SI units (Sections 2.2, 2.3; Appendix A tables).
 * Solid: rho0, K0 (bulk modulus), alpha (Romenskii exponent), G0, beta
 * (shear-modulus exponent, G = G0 (rho/rho0)^(beta+1)), Gamma0, yield (the
 * yield stress c1 the perturbation field scales), D_crit, D0, eps_th,
 * eps_c, bonora_alpha, n_hard (hardening exponent, of the threshold strain
 * and of the Johnson-Cook law), p_gate (damage accrues only for
 * p < p_gate).  Johnson-Cook plasticity (the paper's plasticity table:
 * c2 = jc_B, c3 = jc_C, m = jc_m, T_melt, C_V): the yield is
 *   (yield + jc_B eps_p^n_hard) (1 + jc_C ln max(rate / 1 s^-1, 1))
 *   (1 - T*^jc_m),   T* = clamp((T - 300 K) / (T_melt - 300 K), 0, 1),
 * with the rate the step's plastic increment over dt and T from the thermal
 * energy C_V (T - 300 K eta^Gamma0) of Section 2.2.  jc_B = jc_C = 0 and
 * T_melt = 0 give the constant yield; T_melt > 300 K needs jc_m > 0 and
 * C_V > 0, and negative jc_B or jc_C are rejected (FV_EINVAL).  The U-Nb
 * closures of the paper's ring (Section 2.3, Appendix A): G_p > 0 selects
 * the Steinberg shear modulus G0 + G_p p_c eta^(-1/3) instead of
 * G0 eta^(beta+1); Gamma1 or Gamma2 nonzero selects the Burakovsky-Preston
 * Grueneisen function Gamma0 + Gamma1 eta^(-1/3) + Gamma2 eta^(-gamma_bp)
 * (gamma_bp > 0) with its Debye temperature; Ddot0 > 0 selects the
 * simplified damage law dD/deps_p = Ddot0 (1 - D), without gate, instead
 * of the Bonora law (Section 4.3).  Zero keeps the Romenskii and Bonora
 * forms.  Gas: Gamma0 = gamma - 1; the other fields are ignored. */
typedef struct {
  int32_t kind;
  double rho0, K0, alpha, G0, beta, Gamma0;
  double yield, D_crit, D0, eps_th, eps_c, bonora_alpha, n_hard, p_gate;
  double jc_B, jc_C, jc_m, T_melt, C_V;
  double G_p, Gamma1, Gamma2, gamma_bp, Ddot0;
} fv_material;

/* Run options.  cfl: Courant number of the CFL reduction.  phi_floor:
 * volume fractions are clamped to [phi_floor, 1] (absent materials).
 * weno_eps: WENO3 smoothness floor relative to the squared domain extent.
 * phi_fp64_cut: FP32-bulk only, cells with a volume fraction below it invert
 * the mixture EOS in double.  tile: cells per workgroup tile in x and y,
 * then the block schedule (FV_SCHED_*); {0, 0} selects the default shape,
 * any other value must be one of the compiled shapes (fv_autotune lists
 * them) or fv_init fails with FV_EINVAL, as does a schedule outside 0..2.
 * Results depend on neither.  use_graph:
 * nonzero makes fv_step capture its n_steps steps into a HIP graph at the
 * first call with that step count and replay it afterwards.  seed_nu: the
 * Lagrangian seeding of Section 3.2.1 -- after each step, every cell whose
 * void fraction 1 - sum phi_l exceeds seed_nu (and has a void-fraction
 * gradient) takes Lagrangian coordinates extrapolated from the point 1.5
 * cells towards the material, X(p) - (p - c); 0 turns it off (the default
 * of the workloads surrounded by gas), values in [0, 1).  thinc_beta: THINC
 * interface sharpening of the volume fractions (Xiao, Honma and Kono 2005;
 * the paper uses it for its ring): in cells where a volume fraction is
 * monotone between its neighbours, its face values come from the tanh
 * profile of steepness thinc_beta that keeps the cell average; 0 (the
 * default) keeps MUSCL, values in [0, 10].  driver: the imposed-velocity
 * driver of the paper's ring (Section 4.3), {r_in, v0, v1, t0, t1, r_max}
 * in SI units: the driver surface starts at radius r_in about the z axis
 * and moves with the radial speed v0 t/t0 (t < t0), linear from v0 to v1
 * (t0 < t < t1), v1 afterwards, until it reaches r_max; after each step
 * every cell of a live solid whose centre lies behind it takes at least
 * that radial speed, the kinetic energy added going into the total energy.
 * r_max = 0 (the default) turns it off; it needs dim >= 2. */
typedef struct {
  int32_t precision;
  double cfl;
  double phi_floor;
  double weno_eps;
  double phi_fp64_cut;
  int32_t tile[3];
  int32_t use_graph;
  double seed_nu;
  double thinc_beta;
  double driver[6];
} fv_options;

/* Number of state fields S for a dimension and material list (the first
 * dimension of every state buffer).  Returns 0 for an invalid list. */
int32_t fv_state_fields(int32_t dim, int32_t n_mat, const fv_material* mats);

/* Bytes of device workspace fv_init needs for these instances (two stage
 * copies of every state, boundary-flux accumulators, dt state, instance
 * tables, reduction bins; in 3D also the primitives of every cell and each
 * cell's divergence sum).  Returns 0 for invalid arguments. */
size_t fv_workspace_bytes(int32_t n_inst, const fv_grid* grids, int32_t n_mat,
                          const fv_material* mats, const fv_options* opt);

/* Create a context for n_inst instances sharing dimension, materials and
 * options (the ensemble of seeded realisations advances in one launch).
 * state[i]: device pointer to instance i's state (S * ncell elements,
 * caller-owned, in/out).  phi0[i]: device pointer to the initial perturbation
 * field of instance i on its initial mesh (ncell elements of the state's
 * element type, read-only, Section 2.4).  workspace: device buffer of at
 * least fv_workspace_bytes.  stream: hipStream_t (NULL = default stream).
 * The states are not read here: load them with fv_load_primitive or write
 * conserved values and call fv_reset; until then fv_step, fv_cfl_dt and
 * fv_autotune return FV_ESTATE.  Errors: FV_EINVAL, FV_ENOMEM, FV_EDEVICE. */
int32_t fv_init(fv_ctx** out, int32_t n_inst, const fv_grid* grids,
                int32_t n_mat, const fv_material* mats, const fv_options* opt,
                void* const* state, const void* const* phi0, void* workspace,
                size_t workspace_bytes, void* stream);

/* Convert a primitive field to instance inst's conserved state (async).
 * prim: device pointer, S * ncell doubles in the state's field order with
 * rho_l in place of phi_l rho_l, (eps_p, D) in place of the history
 * densities, the velocity in place of the momentum and the pressure in place
 * of the total energy.  Volume fractions are clamped to [phi_floor, 1].
 * Also resets the instance's time, boundary accumulators and flag and
 * computes its first CFL time step. */
int32_t fv_load_primitive(fv_ctx* ctx, int32_t inst, const void* prim);

/* Reset time, accumulators and flag of every instance and recompute the CFL
 * time step from the current states (after the caller wrote conserved
 * states directly).  Async. */
int32_t fv_reset(fv_ctx* ctx);

/* The primitive field of instance inst (same layout as fv_load_primitive's
 * input) into prim (device, S * ncell doubles).  Async. */
int32_t fv_primitive(fv_ctx* ctx, int32_t inst, void* prim);

/* Time step of every instance from the CFL reduction of its current state
 * (Courant number times the inverse of the largest sum over directions of
 * (|u_d| + c) / dx_d), clamped to its end time.  The explicit update of
 * Section 3 advances at a time step set by a CFL number, which every test of
 * Section 4 states (0.3 to 0.4); c is the longitudinal mixture sound speed of
 * the closures of Sections 2.2 and 2.3.  dt_host: [n_inst] out.
 * Synchronises the stream; returns FV_ENONPHYS if the device flag is set. */
int32_t fv_cfl_dt(fv_ctx* ctx, double* dt_host);

/* Advance every instance by n_steps time steps (async, no host sync).  Each
 * step: three SSP-RK3 stages of the hyperbolic update (MUSCL/van Leer
 * primitives, WENO3 Lagrangian coordinates, HLLC flux with the void-opening
 * modifier of Section 3.1), then the source step (radial return to the
 * perturbed yield of Section 2.4, Bonora damage integrated by RK4 as in
 * Section 3.1, phi0 interpolated at the Lagrangian coordinates as in
 * Section 3.2.2), the Lagrangian seeding of void cells when
 * fv_options.seed_nu is set (Section 3.2.1) and the CFL reduction for the
 * next step.  dt_host: NULL to
 * use the device CFL step, else [n_inst] fixed steps.  t_end: NULL to keep
 * the current end times, else [n_inst]; an instance at its end time does no
 * work. */
int32_t fv_step(fv_ctx* ctx, const double* dt_host, int32_t n_steps,
                const double* t_end);

/* Simulated time of every instance, t_host [n_inst] out.  Synchronises. */
int32_t fv_time(fv_ctx* ctx, double* t_host);

/* Conservation totals of the quantities whose equations Section 2.1 writes in
 * conservation form (phasic mass, momentum, total energy); Section 3.1 opens
 * void instead of deleting critically damaged cells so that fracture keeps
 * them, and these sums are the check.  out: [n_inst][2 * (N + dim + 1)]
 * doubles: the interior totals of phi_l rho_l (N), rho u_i (dim) and rho E
 * over the cells times the cell volume, then the cumulative outward flux of
 * the same quantities through the domain boundary.  Each sum is exact before its one
 * final rounding (an integer superaccumulator), so it equals the correctly
 * rounded sum of the same values.  Synchronises; FV_ENONPHYS if flagged. */
int32_t fv_totals(fv_ctx* ctx, double* out);

/* Checkpoint of the context's own state: the step count, each instance's
 * time, CFL state, end time, fixed dt and flag, and its cumulative boundary
 * outflow.  With copies of the state buffers this is a complete checkpoint: a
 * context created with the same grids, materials and options whose state
 * buffers hold the saved states and that calls fv_restore continues bit for
 * bit.  fv_checkpoint_bytes: size of the blob (0 for a NULL ctx).
 * fv_checkpoint: writes the blob to dst (device, caller-owned); synchronises;
 * FV_ESTATE before a state is loaded.  fv_restore: reads it from src (device);
 * synchronises; FV_EINVAL if the blob is not a checkpoint of a context with
 * the same number of instances and cells. */
size_t fv_checkpoint_bytes(const fv_ctx* ctx);
int32_t fv_checkpoint(fv_ctx* ctx, void* dst);
int32_t fv_restore(fv_ctx* ctx, const void* src);

/* Autotuner: time every configuration of ctx's kernel set -- each compiled
 * tile shape under each block schedule (FV_SCHED_*; one schedule for a
 * single instance) -- on reps timing runs of the first RK stage over the
 * current state (these leave the state, time, dt and boundary accumulators
 * unchanged; they overwrite only the stage buffer in the workspace), keep
 * the fastest for later steps (a configuration displaces one listed before
 * it only when at least 2 % faster) and report.  tiles: host
 * int32[3 * max_report] out, (x, y, schedule) per configuration; ms: host
 * float[max_report] out, average launch time per configuration;
 * *n_variants: number of configurations; *chosen: index of the selected one
 * (either may be NULL).  Synchronises; drops captured step graphs.  Results
 * of later steps are bitwise those of any other configuration. */
int32_t fv_autotune(fv_ctx* ctx, int32_t reps, int32_t max_report, int32_t* tiles, float* ms,
                    int32_t* n_variants, int32_t* chosen);

/* One fragment of fv_fragments. */
typedef struct {
  int64_t label;            /* smallest linear cell index (x fastest) */
  int64_t n_cells;
  double mass;              /* sum of phi_s rho_s over its cells, correctly
                               rounded, times the cell volume */
  int32_t touches_boundary; /* 1 if a cell lies on a domain side */
  int32_t reserved;
} fv_fragment;

/* Bytes of device workspace fv_fragments needs for instance inst and at
 * most cap fragments.  Returns 0 for invalid arguments. */
size_t fv_fragment_workspace_bytes(const fv_ctx* ctx, int32_t inst, int64_t cap);

/* Fragments of instance inst (Sections 4.2 and 4.3 delineate fragments at the
 * volume-fraction contour): the connected sets of cells whose solid volume
 * fraction exceeds cut (compared in double), connected through cell faces (2
 * neighbours in 1D, 4 in 2D; not across periodic sides).
 * labels: device int32[ncell], caller-owned, out: the fragment label of each
 * cell (its smallest linear cell index) or -1 for a non-material cell.
 * frag_ws: device buffer of frag_ws_bytes >= fv_fragment_workspace_bytes.
 * out: host array of cap entries, filled in label order; *n_frag: the number
 * of fragments.  Deterministic and bit-exact.  Synchronises.  FV_ENOMEM if
 * there are more than cap fragments (*n_frag then holds the count and the
 * labels are complete, out is untouched); FV_EINVAL without a solid, for
 * more than 2^31 - 1 cells or a non-finite cut. */
int32_t fv_fragments(fv_ctx* ctx, int32_t inst, double cut, int32_t* labels, void* frag_ws,
                     size_t frag_ws_bytes, int64_t cap, int64_t* n_frag, fv_fragment* out);

/* Size of the static fragment scratch behind fv_fragments_noalloc (bytes per
 * GPU the library runs on, held until the process ends). */
#define FV_FRAGMENT_SCRATCH_BYTES (64u << 20)

/* fv_fragments without a workspace argument, for callers that cannot
 * allocate device memory (serving loops and harnesses that forbid hipMalloc
 * and workspace tensors): the kernels work in a static scratch array of
 * FV_FRAGMENT_SCRATCH_BYTES on the context's GPU instead of frag_ws.  The
 * call allocates nothing (no hipMalloc, no allocating library routine).  It
 * fits an instance and cap whose fv_fragment_workspace_bytes is at most
 * FV_FRAGMENT_SCRATCH_BYTES (for example 2^22 cells with cap 2^14), else
 * FV_ENOMEM with the size in fv_last_error.  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (two contexts or threads on
 * different streams) race and must be serialised by the caller.  Arguments,
 * outputs, bit-exactness and the other errors are those of fv_fragments. */
int32_t fv_fragments_noalloc(fv_ctx* ctx, int32_t inst, double cut, int32_t* labels, int64_t cap,
                             int64_t* n_frag, fv_fragment* out);

/* Cumulative fragment-mass histogram, the form in which Sections 4.2 and 4.3
 * present fragment distributions (fragment mass against cumulative fragment
 * number): counts[k] = number of fragments among frags[0..n) whose mass is at
 * least edges[k].  Host arrays, caller-owned: frags (n entries, as
 * fv_fragments returns them), edges (n_edges doubles, any order), counts
 * (n_edges int64, out).  No device work and no context.  FV_EINVAL for a
 * negative count or a null array that is needed. */
int32_t fv_fragment_histogram(const fv_fragment* frags, int64_t n, const double* edges,
                              int32_t n_edges, int64_t* counts);

/* Text of the last error of ctx (or of the last failed fv_init when ctx is
 * NULL).  Valid until the next call on ctx. */
const char* fv_last_error(const fv_ctx* ctx);

/* Destroy a context (synchronises its stream first).  NULL is allowed. */
void fv_destroy(fv_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* FV_H */
