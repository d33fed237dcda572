/*
 * sph.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot path
 * of adaptive-resolution weakly-compressible SPH (Muta & Ramachandran,
 * "Efficient and accurate adaptive resolution for weakly-compressible SPH",
 * arXiv 2107.01276): variable-h neighbour search, the pairwise rate loop,
 * the predict-evaluate-correct step and the split/merge adaptation driven by
 * background particles.
 *
 * Conventions for every call:
 *   - Particle data are structure-of-arrays in device memory owned by the
 *     caller; each array holds at least `capacity` entries and entries
 *     [0, n) are live.  Rows of a neighbour list and particle indices are
 *     "slots": positions in these arrays.
 *   - Positions, velocities, pressure, density, smoothing length and
 *     reference mass are double.  Mass is an int64 number of quanta `mq`;
 *     the mass of a particle is mq * mass_q exactly (mass_q is a power of
 *     two chosen so that every mq stays below 2^53 and the total over all
 *     particles below 2^63), which keeps total mass exactly conserved
 *     through splits and merges.
 *   - All work is issued on the context's stream in order.  Calls that
 *     return counts to the host (nnz, new particle count) synchronise that
 *     stream before returning; the others only enqueue work.
 *   - Scratch memory comes from the caller's workspace (sph_create); the
 *     library allocates no device memory.
 *   - Return value: SPH_OK (0) or a negative SPH_E_* code; sph_last_error()
 *     gives a message.  On error no caller-visible array has been modified
 *     unless the call's comment says otherwise.
 *   - 2D only; periodic axes use the minimum image.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SPH_OK = 0,
    SPH_E_INVAL = -1,     /* bad argument or configuration */
    SPH_E_CAPACITY = -2,  /* result does not fit the caller's arrays */
    SPH_E_NOMEM = -3,     /* workspace too small */
    SPH_E_DEVICE = -4,    /* HIP runtime error */
    SPH_E_NONFINITE = -5, /* NaN or Inf found in the state */
    SPH_E_AGAIN = -6      /* serving pool full: retry later */
};

enum { SPH_FP64 = 0, SPH_FP32 = 1 };             /* pair arithmetic precision */
/* Particle kinds (section 2.2): fluid; solid = dummy wall particles of the
 * Adami et al. wall treatment; inlet and outlet particles of an open
 * channel. */
enum { SPH_FLUID = 0, SPH_SOLID = 1, SPH_INLET = 2, SPH_OUTLET = 3 };

/* Run configuration.  Physical constants follow section 2 of the paper:
 * rho0, c_s, nu, alpha_e (eq. edac-alpha), the kernel support 3h (eq.
 * kernel).  Adaptation constants follow section 3: split_alpha and
 * split_eps (section 3.1), m_max = mmax_f m_ref and m_min = mmin_f m_ref
 * (section 3.3), merge_iters and shift_iters (section 3.2), hdx = C of
 * h = C (m/rho)^(1/2) (section 3.1).  Background constants follow section
 * 3.3: C_r, ds_min, ds_max, N_r and the number of h-smoothing + shifting
 * repetitions. */
typedef struct sph_config {
    int32_t precision;      /* SPH_FP64 or SPH_FP32 */
    int32_t periodic[2];    /* per axis: 1 = periodic */
    double lo[2], hi[2];    /* domain box; periodic axes wrap into [lo, hi) */
    double h_lo, h_hi;      /* expected smoothing-length range; sizes the grid.
                               Results never depend on it: any h is handled,
                               h far outside only costs time. */
    double rho0, cs, nu, alpha_e, hdx, u_ref;
    double body_force[2];
    double split_alpha, split_eps, mmax_f, mmin_f;
    double mass_q;          /* fluid mass quantum: masses are mq * mass_q with
                               int64 mq; choose it so that every mq stays
                               below 2^53 (exact in double) and the sum over
                               all particles below 2^63, e.g. 2^-40 of the
                               largest mass */
    int32_t merge_iters, shift_iters;
    double cr, ds_min, ds_max, n_r;
    int32_t bg_smooth_iters;
    double bg_mass_q;       /* background mass quantum */
    double wall_accel[2];   /* a_w of eq. (bc-pre): acceleration of the solid
                               particles (0 for a stationary body) */
    int32_t list_k;         /* columns of the rate passes' neighbour list
                               (0 = 256); longer rows fall back to a cell walk */
    int32_t lean;           /* 1: workspace without the adaptation buffers;
                               sph_adapt, sph_bg_update, sph_mref_lookup and
                               sph_inout then return SPH_E_INVAL */
    double list_skin;       /* in [0, 1]: the rate passes' list holds pairs
                               closer than (1 + skin) 3 max(h_i, h_j) and is
                               reused while every particle moved less than
                               1.5 skin h_i (results are unchanged: the exact
                               predicate is re-applied); 0 rebuilds it at
                               every evaluation without a host round trip */
    int32_t io_mode;        /* inlet/outlet rule of the boundary pass
                               (section 2.2): 0 = the inlet keeps its
                               velocity and takes the Shepard average of the
                               fluid pressure, the outlet takes the Shepard
                               averages of u, v, p (zero gradient);
                               1 = the non-reflecting characteristic rule of
                               Lastiwka et al.: about the reference state
                               io_ref = (u_r, v_r, p_r) and rho0 c_s, with
                               J2 = rho0 c (u - u_r) + (p - p_r) and
                               J3 = -rho0 c (u - u_r) + (p - p_r), the inlet
                               (upstream, flow along +x) takes J2 = 0, J3 and
                               v = v_r; the outlet takes J3 = 0, J2 and v
                               from the Shepard averages of the fluid; then
                               p = p_r + (J2 + J3)/2 and
                               u = u_r + (J2 - J3)/(2 rho0 c) */
    double io_ref[3];       /* (u_r, v_r, p_r) of io_mode 1 */
    /* The per-iteration schedule of sph_step (the algorithm of section 3.4): */
    double dt;              /* time step; 0 = eq. (timestep) with h_min = h_lo,
                               U = u_ref (sph_timestep) */
    double sol_k;           /* solution adaptivity (section 3.3): background
                               particles with Shepard-averaged |omega| above
                               sol_k max|omega| are refined at every
                               background update; 0 = off */
    int32_t n_adapt;        /* split, merge, shift and h update every n_adapt
                               iterations (0 = never) */
    int32_t n_bg;           /* background update every n_bg iterations (0 =
                               never) */
    int32_t bg_passes;      /* passes of each background update (1 suffices
                               for small motions, section 3.3) */
    int32_t csr_k;          /* entries per particle of capacity of the
                               internal neighbour lists of the adaptation
                               (0 = 160); a call that needs more returns
                               SPH_E_NOMEM and names the csr_k that fits.
                               The background update walks the cells and has
                               no such limit. */
} sph_config;

/* Caller-owned particle set (device pointers, see conventions). kind may be
 * NULL (all fluid). */
typedef struct sph_particles {
    int64_t n, capacity;
    double *x, *y, *u, *v, *p, *rho, *h, *mref;
    int64_t *mq;
    int32_t *kind;
} sph_particles;

/* Neighbour lists in CSR form (device arrays): row_ptr[n+1], col[nnz_cap].
 * Row i holds every j with |r_i - r_j| < 3 max(h_i, h_j), i itself
 * included, in ascending order. nnz is written (host) by the call. */
typedef struct sph_csr {
    int64_t *row_ptr;
    int32_t *col;
    int64_t nnz_cap;
    int64_t nnz;
} sph_csr;

/* Outputs of one rate evaluation (device arrays of length >= n, slot
 * order). Any pointer may be NULL to skip that field. */
typedef struct sph_rates_out {
    double *rho, *beta, *pavg, *nnb, *dxs, *dys, *dpdt, *dudt, *dvdt;
} sph_rates_out;

/* Index map of one adaptation (sph_adapt).  origin and sat are device
 * arrays of length >= capacity; the counters are written on the host. */
typedef struct sph_adapt_map {
    int64_t *origin;    /* new slot -> pre-adaptation slot it descends from */
    int32_t *sat;       /* 1 for the six off-centre children of a split */
    int64_t n_split;    /* particles split */
    int64_t n_required; /* size needed by the split (capacity check) */
    int64_t n_merged[8];/* merged pairs per merge iteration */
} sph_adapt_map;

/* Open-boundary zones of section 2.2 along x: inlet particles occupy
 * [x_in - len_in, x_in), outlet particles [x_out, x_out + len_out). */
typedef struct sph_inout_params {
    double x_in, len_in, x_out, len_out;
} sph_inout_params;

/* Result of sph_inout.  origin is a device array of length >= capacity;
 * the counters are written on the host. */
typedef struct sph_inout_map {
    int64_t *origin;      /* new slot -> old slot (the source, for an inlet copy) */
    int64_t n_appended;   /* inlet copies appended (= inlet -> fluid) */
    int64_t n_deleted;    /* outlet particles removed */
    int64_t n_to_outlet;  /* fluid -> outlet */
    int64_t n_required;   /* size the update needs (capacity check) */
} sph_inout_map;

/* Background particles of section 3.3 (device arrays, caller-owned). */
typedef struct sph_background {
    int64_t n, capacity;
    double *x, *y, *h, *ds, *mref;
    int32_t *mask;
    int64_t *mq;
} sph_background;

/* Scalar diagnostics (host), section 4.1: kinetic energy, volume error
 * sum(m/rho), linear momentum, total mass in quanta, extreme speed. */
typedef struct sph_diag {
    double ke, vol, mom_x, mom_y, umax;
    int64_t mq_total, n;
} sph_diag;

typedef struct sph_ctx sph_ctx;

/* Library version (major*10000 + minor*100 + patch). */
int sph_version(void);

/* Bytes of device workspace sph_create needs for `capacity` particles. */
size_t sph_workspace_bytes(const sph_config *cfg, int64_t capacity);

/* Creates a context on the current HIP device.  `workspace` (device,
 * >= sph_workspace_bytes, 256-byte aligned) is owned by the caller and must
 * outlive the context.  `stream` is a hipStream_t (NULL = default stream).
 * Errors: SPH_E_INVAL (bad config), SPH_E_NOMEM (workspace too small). */
int sph_create(const sph_config *cfg, int64_t capacity, void *workspace,
               size_t workspace_bytes, void *stream, sph_ctx **out);
void sph_destroy(sph_ctx *ctx);
/* Message of the last error of ctx; with ctx NULL, that of the calling
 * thread's last failed sph_rates_noalloc. */
const char *sph_last_error(const sph_ctx *ctx);
int sph_set_stream(sph_ctx *ctx, void *stream);

/* Neighbour search (paper section 2: kernel support 3h; symmetric because
 * the rates of eqs. edac:sph and mom-sph use W(h_i) and W(h_j)).  Builds
 * the search structure for `ps`; if `out` is non-NULL also writes the CSR.
 * Distances use the minimum image on periodic axes and are compared as
 * dx*dx + dy*dy < (3 max(h_i,h_j))^2 in double precision.
 * SPH_E_CAPACITY if nnz > out->nnz_cap (out->nnz = required, col untouched).
 * Synchronises when `out` is non-NULL. */
int sph_build_neighbors(sph_ctx *ctx, const sph_particles *ps, sph_csr *out);

/* One rate evaluation on the given state (section 2): pass A = summation
 * density (eq. sd-gather), beta (eq. beta), neighbour count and average
 * pressure (eq. pavg), limited shifting (eqs. shift-deltar, shift-limit);
 * pass B = EDAC pressure rate (eq. edac:sph) and momentum (eq. mom-sph).
 * Pair arithmetic in the configured precision.  dt enters through the
 * transport-velocity term (eq. shift-tvf).
 * When ps->kind is non-NULL, a boundary pass (section 2.2) runs first: over
 * its fluid neighbours, with the Shepard weights W(r, (h_b + h_f)/2) of eq.
 * (shepard), every solid particle gets p by eq. (bc-pre) (g = body_force,
 * a_w = wall_accel, rho_f = ps->rho, the stored density) and the no-slip
 * ghost velocity 2 u_b - u^ of eq. (bc-wall), which the viscous term uses
 * (the solid's own u, its prescribed velocity, is what the pressure
 * equation sees); inlet particles get the Shepard average of p; outlet
 * particles get the Shepard averages of u, v and p.  These values are
 * written into ps->p (and ps->u, ps->v of outlet particles).  A boundary
 * particle with no fluid neighbour keeps its values. */
int sph_rates(sph_ctx *ctx, const sph_particles *ps, double dt, sph_rates_out *out);

/* Launch schedule of the FP32 rate passes and of the neighbour-list build:
 * the variants compiled into the library, picked at run time (by a tuner
 * that times them on the caller's workload).  The results do not depend on
 * it beyond the order of the FP32 partial sums.  A new context starts with
 * {4, 5, 2, 2, 4, 4}.  The FP64 passes keep one fixed schedule. */
typedef struct sph_schedule {
    int32_t a_lanes;    /* pass A work-items per particle: 2, 4 or 8 */
    int32_t a_waves;    /* pass A minimum waves per SIMD the register
                           allocation must allow: 1 (the compiler's choice),
                           4 or 5 (the last spills to scratch) */
    int32_t b_lanes;    /* pass B work-items per particle: 1, 2 or 4 */
    int32_t b_unroll;   /* pass B row entries loaded ahead per lane: 2 or 4 */
    int32_t b_waves;    /* pass B minimum waves per SIMD: 1 or 4 */
    int32_t list_lanes; /* list build work-items per particle: 2, 4 or 8 */
} sph_schedule;

/* Sets the context's schedule; SPH_E_INVAL (schedule unchanged) for a
 * combination that is not compiled in. */
int sph_set_schedule(sph_ctx *ctx, const sph_schedule *sched);
/* Writes the context's schedule to *sched. */
int sph_get_schedule(const sph_ctx *ctx, sph_schedule *sched);

/* Time step of eq. (timestep): min(0.25 h_min / (U + c_s), 0.125 h_min^2 /
 * nu) with U = cfg->u_ref, c_s = cfg->cs, nu = cfg->nu (the second bound
 * is dropped for nu = 0); h_min <= 0 takes cfg->h_lo.  Returns 0 for an
 * invalid configuration. */
double sph_timestep(const sph_config *cfg, double h_min);

/* nsteps predict-evaluate-correct steps (eqs. int-pre, int-cor) of size dt,
 * neighbours rebuilt before each of the two evaluations per step.  Fluid
 * particles are integrated; solid particles stay in place; inlet and outlet
 * particles move with their own velocity (u^n for the half step, the
 * half-step boundary value for the full step).  Every evaluation runs the
 * boundary pass of sph_rates and stores its summation density in ps->rho,
 * which the next boundary pass reads.  Updates x, y, u, v, p and rho in
 * place; non-fluid particles end with their half-step boundary values. */
int sph_pec(sph_ctx *ctx, sph_particles *ps, double dt, int32_t nsteps);

/* nsteps iterations of the algorithm of section 3.4.  Before iteration it
 * (the context's counter, 0 at creation; sph_set_iteration sets it, and
 * sph_import sets it to the checkpoint's step), when it > 0:
 *   (i)  every cfg->n_bg iterations, when bg and solids are given, the
 *        background is updated (cfg->bg_passes passes of sph_bg_update with
 *        solids; with cfg->sol_k > 0 those of sph_bg_update_solution over
 *        ps, which refine the background where the fluid's vorticity is
 *        above sol_k of its maximum);
 *   (ii) every cfg->n_adapt iterations, when bg is given, the fluid is
 *        adapted as sph_adapt does (m_ref from the background, which the
 *        update of (i) already moved; split, merge, shift and Taylor
 *        correction, h update).
 * Then the iteration takes one predict-evaluate-correct step of size
 * cfg->dt (eq. timestep when 0), followed, when io is given, by the
 * inlet/outlet update of sph_inout.  The initialisation (items 1 and 2 of
 * the algorithm: the background's initial passes and the first
 * adaptations) is the caller's, with sph_bg_update and sph_adapt.  Runs of
 * steps between updates are enqueued at once with the guards of
 * sph_step_inout (one host round trip per run).  Needs a workspace with
 * the adaptation buffers when bg or io is given.  diag (may be NULL)
 * receives sph_diagnostics of the final state.  The results are those of
 * the separate calls in that order.  On error the iterations before the
 * failing one stay applied.  Synchronises. */
int sph_step(sph_ctx *ctx, sph_particles *ps, sph_background *bg, const sph_particles *solids,
             const sph_inout_params *io, int32_t nsteps, sph_diag *diag);
int sph_set_iteration(sph_ctx *ctx, int64_t it);
int64_t sph_iteration(const sph_ctx *ctx);

/* Fluid reference mass from the background (section 3.3 and the algorithm of
 * section 3.4, item 4): m_ref,i = min of the background m_ref within
 * 3 max(h_i, h_b); if none is in range, that of the nearest background
 * particle (lowest slot on ties).  Writes ps->mref. */
int sph_mref_lookup(sph_ctx *ctx, const sph_particles *ps, const sph_background *bg);

/* Adaptation (section 3; algorithm of section 3.4 items 5-7): split every
 * fluid particle with m > mmax_f m_ref into 7 (section 3.1), merge mutually
 * closest pairs merge_iters times (section 3.2), shift shift_iters times
 * with the Taylor correction (eq. shift-correct), then set h from the mean
 * neighbour mass.  If bg is non-NULL, m_ref is looked up first.
 * Two-phase: when the split needs more than ps->capacity slots, returns
 * SPH_E_CAPACITY with map->n_required set and the state untouched.
 * SPH_E_NOMEM when the neighbour list of a shift or of the h update needs
 * more than cfg->csr_k entries per particle of capacity (the message names
 * the csr_k that fits); the split and merges have then been applied.
 * Updates ps->n on the host.  Synchronises. */
int sph_adapt(sph_ctx *ctx, sph_particles *ps, const sph_background *bg, sph_adapt_map *map);

/* Background update (section 3.3 steps 1-4), `passes` times: mark background
 * particles near solids, grade sizes by C_r, split, then smooth h (eq.
 * h-smoothing) and shift.  Solution adaptivity: when phi (a device array
 * over the background as it is at the call) is non-NULL, particles with
 * phi > phi_thresh get a mark that lasts the whole call (their split
 * children keep it) and are refined like particles near a body; without
 * phi no particle is marked.  mask becomes 0, 1 (near a solid) or 3
 * (marked).  Updates bg->n.  *nsplit receives the number of splits.
 * The sweeps walk the cells of the background's own neighbour build, so a
 * background particle may have any number of neighbours; their sums over
 * neighbours (log-sizes, h_j, shift terms) are compensated (a TwoSum
 * cascade), which makes the update a function of the particle set, not of
 * the slot order.  SPH_E_CAPACITY when a split needs more than
 * bg->capacity slots (bg->n then holds the count before that split).
 * Synchronises. */
int sph_bg_update(sph_ctx *ctx, sph_background *bg, const sph_particles *solids,
                  const double *phi, double phi_thresh, int32_t passes, int64_t *nsplit);

/* Passes of the background initialisation of section 3.3: from particles
 * at ds_max, the update is repeated 3 ceil(ln(ds_max / ds_min) / ln C_r)
 * times (three per size level).  Returns 0 for a configuration without a
 * valid range (ds_min <= 0, ds_max < ds_min or C_r <= 1). */
int32_t sph_bg_init_passes(const sph_config *cfg);

/* Vorticity of every particle (solution adaptivity, section 3.3):
 * omega_i = sum_j (m_j/rho_j) [(v_j - v_i) dW/dx - (u_j - u_i) dW/dy] at
 * h_i over N(i), with the stored density.  omega: device array >= n. */
int sph_vorticity(sph_ctx *ctx, const sph_particles *ps, double *omega);

/* Background update with solution adaptivity (section 3.3): |omega| of the
 * fluid particles (kind 0) is carried to every background particle b by the
 * Shepard average of eq. (shepard) over the fluid particles within
 * 3 max(h_b, h_i), with W(r, (h_b + h_i)/2) (0 when none); background
 * particles with phi_b > k_frac max|omega| are then treated as boundary
 * background particles, as those near `solids` are, and the update of
 * sph_bg_update runs (`passes` times).  *omega_max (may be NULL) receives
 * max|omega|.  Synchronises. */
int sph_bg_update_solution(sph_ctx *ctx, sph_background *bg, const sph_particles *solids,
                           const sph_particles *fluid, double k_frac, int32_t passes,
                           int64_t *nsplit, double *omega_max);

/* Inlet/outlet update (section 2.2), to be called after a step.  On the
 * kinds before the call: an inlet particle with x >= x_in becomes fluid and
 * a copy of it (every field, kind inlet) is appended at x - len_in; a fluid
 * particle with x >= x_out becomes an outlet particle; an outlet particle
 * with x >= x_out + len_out is deleted.  Deleted slots are removed by stable
 * compaction; copies follow in ascending order of their source slot.
 * Requires ps->kind.  map->origin is written only when slots change
 * (n_appended or n_deleted > 0).  Two-phase: SPH_E_CAPACITY with
 * map->n_required set and the state untouched when the result exceeds
 * ps->capacity.  Updates ps->n.  Synchronises. */
int sph_inout(sph_ctx *ctx, sph_particles *ps, const sph_inout_params *io, sph_inout_map *map);

/* ---- Serving pool: continuous batching of independent simulations ------
 * Beyond the paper, which runs one simulation at a time: many independent
 * fluid-only simulations (periodic or open boxes, no boundary particles, no
 * adaptation) resident on one GPU and advanced together.  A pool owns host
 * bookkeeping, one stream and its graph; its device memory is the caller's
 * arena.  The resident simulations share one set of structure-of-arrays
 * buffers carved from the arena: each holds a contiguous range of particle
 * slots and a range of the cell-table region (first fit; freed ranges
 * coalesce).  sph_pool_step advances every resident simulation by one
 * predict-evaluate-correct step of its own dt (eqs. int-pre, int-cor, the
 * rates of section 2, the neighbour list rebuilt at every evaluation) with
 * one launch per kernel for all of them: each launch's blocks are dealt to
 * the simulations, and each block reads its simulation's descriptor (grid,
 * dt, rho0, c_s, nu, alpha_e, body force, mass quantum).  The step of the
 * resident set is captured into one HIP graph when the set changes and
 * replayed.  FP64 and FP32 simulations are two groups in the same graph.
 * A simulation's result is bit for bit that of sph_step on a context with
 * lean = 1, list_skin = 0 and list_k = 64, alone or in any mix.
 * Admission and retirement happen between steps.  Single-threaded use. */
typedef struct sph_pool sph_pool;

typedef struct sph_pool_stats {
    int64_t slots_total, slots_used, largest_free; /* particle slots */
    int64_t tables_total, tables_used;             /* cell-table entries */
    int64_t resident;      /* simulations */
    int64_t particles;     /* resident particles */
    int64_t max_resident;  /* simulations the pool can hold at once */
    double last_step_ms;   /* device time per step of the last sph_pool_step */
} sph_pool_stats;

/* Arena bytes one simulation of n particles with this configuration takes
 * (its particle slots, cell tables and digit-histogram tile). */
size_t sph_pool_footprint(const sph_config *cfg, int64_t n);

/* arena: device memory (256-byte aligned, at least 1 MiB) owned by the
 * caller, outliving the pool; max_sims in [1, 1024] simulations resident at
 * once.  About 1/16 of the arena holds cell tables and the rest particle
 * slots of about 630 bytes each.  Errors: SPH_E_INVAL, SPH_E_NOMEM (arena
 * too small for max_sims), SPH_E_DEVICE. */
int sph_pool_create(void *arena, size_t arena_bytes, int32_t max_sims, sph_pool **out);
void sph_pool_destroy(sph_pool *pool);
const char *sph_pool_last_error(const sph_pool *pool);

/* Admits a simulation whose initial state is `init` (device arrays x, y, u,
 * v, p, rho, h, mq; kind must be NULL) with time step dt and the
 * configuration's constants.  The copies are enqueued on the pool's stream
 * after the work enqueued on `stream` (a hipStream_t, NULL = default) before
 * the call; init's arrays must stay unchanged until the next sph_pool_step
 * returns.  SPH_E_AGAIN (nothing changed) when no free range holds the
 * particles or the cell tables, or max_sims are resident.  Writes the
 * simulation's id.  cfg->list_skin as in a context: 0 builds the
 * simulation's neighbour list at every evaluation; a skin keeps its sorted
 * order and list until one of its particles moved by 1.5 skin h (checked on
 * the device at every evaluation), independently of the other residents,
 * so its states are the bits a lean context with that configuration gives. */
int sph_pool_admit(sph_pool *pool, const sph_config *cfg, const sph_particles *init, double dt,
                   void *stream, int32_t *sim_id);

/* Advances every resident simulation by nsteps steps.  Returns when they
 * are done. */
int sph_pool_step(sph_pool *pool, int32_t nsteps);

/* Per simulation: the device time per step of the last sph_pool_step (every
 * resident simulation advanced in it), steps taken, and interacting ordered
 * pairs evaluated (sum over evaluations of |N(i)| - 1; for a retired
 * simulation, the total at retirement).  Any pointer may be NULL. */
int sph_pool_sim_stats(sph_pool *pool, int32_t sim_id, double *last_ms, int64_t *steps,
                       int64_t *pair_evals);

/* Copies a simulation's state (x, y, u, v, p, rho, h, mq; NULL fields are
 * skipped) into dst (device arrays, capacity >= n), on the pool's stream
 * after the work enqueued on `stream` before the call; later work on
 * `stream` sees the copies. */
int sph_pool_read(sph_pool *pool, int32_t sim_id, sph_particles *dst, void *stream);

/* Removes a simulation; later admissions reuse its ranges. */
int sph_pool_retire(sph_pool *pool, int32_t sim_id);

int sph_pool_info(sph_pool *pool, sph_pool_stats *out);

/* nsteps of { sph_step with nsteps = 1, then sph_inout }, with the same
 * results as those calls in sequence; the inlet/outlet round trip also
 * carries the list check of the next step.  The map's counters are summed
 * over the steps and map->origin is the composition of the steps' maps
 * (new slot -> slot before the call), written only when some step moved a
 * slot.  A capacity error stops at the step that needed it (earlier steps
 * stay applied; ps->n is current).  Synchronises. */
int sph_step_inout(sph_ctx *ctx, sph_particles *ps, double dt, int32_t nsteps,
                   const sph_inout_params *io, sph_inout_map *map);

/* Force on the solid particles, section 2.3, eq. (force-sph): one
 * evaluation of the current state (neighbours, the boundary pass, which
 * writes p, and u, v of outlet particles, of the non-fluid slots in place
 * as sph_rates does, and pass A), then, over every solid particle i and its
 * fluid neighbours j, in FP64:
 *   f_p    = -sum_i m_i sum_j m_j (P_i gradW(r_ij, h_i) + P_j gradW(r_ij, h_j))
 *   f_visc =  sum_i m_i (1/beta_i) sum_j m_j 4 nu / (rho_i + rho_j)
 *                       (r_ij . gradW_ij) / (r_ij^2 + eta_i) (u~_i - u_j)
 * with P = p / (rho^2 beta) (the unreduced pressure), gradW_ij the average
 * of the gradients at h_i and h_j, and u~_i the solid's ghost velocity.
 * The densities, beta and masses come from pass A in the context's
 * precision.  force (host, 8 doubles): f_p,x, f_p,y, f_visc,x, f_visc,y,
 * then the sums of the magnitudes of their terms (a scale for rounding
 * errors).  Drag and lift coefficients, eq. (cdcl), are these forces
 * divided by rho0 U^2 L / 2.  Needs kind and rho (the stored density);
 * SPH_E_INVAL otherwise.  The totals are summed in a fixed order (the same
 * bits on every call with the same input).  Synchronises. */
int sph_body_force(sph_ctx *ctx, sph_particles *ps, double *force);

/* Prescribed rigid motion of a body between steps (moving bodies, section
 * 3.3; the wall acceleration a_w of eq. bc-pre): every solid particle
 * (kind 1) is translated by disp (wrapped on periodic axes) and takes the
 * velocity vel, and the boundary passes of later evaluations use acc as the
 * wall acceleration a_w (it replaces the config's wall_accel for this
 * context).  disp, vel, acc: host arrays of two doubles.  Needs kind;
 * SPH_E_INVAL without it or with non-finite values.  Does not synchronise.
 * A neighbour list held across calls is re-checked at the next evaluation,
 * so moved solids are seen. */
int sph_move_solids(sph_ctx *ctx, sph_particles *ps, const double disp[2], const double vel[2],
                    const double acc[2]);

/* Checkpoint and resume.  A checkpoint is a host byte buffer: a 64-byte
 * header (bytes 0-7 "SPHCKPT1"; int32 version 1 at 8; int32 0 at 12; int64 n
 * at 16; double mass quantum at 24; int64 step and double time, the
 * caller's, at 32 and 40; zeros to 64), then over [0, n) the arrays x, y,
 * u, v, p, rho, h, mref (double), mq (int64) and kind (int32), each
 * contiguous, in that order (mref and kind are zero when ps has none).
 * Little-endian, as on the device.  A state resumed from it steps exactly
 * as the original (with list_skin 0 bit for bit; a reusable list may
 * otherwise order the pair sums differently). */
size_t sph_export_bytes(int64_t n);
/* Writes ps (x, y, u, v, p, rho, h, mq required) with step and time into
 * host_buf (>= sph_export_bytes(ps->n) bytes).  Synchronises. */
int sph_export(sph_ctx *ctx, const sph_particles *ps, int64_t step, double time, void *host_buf,
               size_t bytes);
/* Reads a checkpoint into ps and sets ps->n; *step and *time (may be NULL)
 * receive the caller's values.  Everything is checked before anything is
 * written: SPH_E_INVAL for a bad header, a buffer shorter than its n needs,
 * a mass quantum other than the context's (the ledger's quanta would mean
 * other masses) or non-fluid kinds when ps has no kind array;
 * SPH_E_CAPACITY when n exceeds ps->capacity; SPH_E_NONFINITE when a value
 * is NaN or infinite.  Synchronises. */
int sph_import(sph_ctx *ctx, sph_particles *ps, const void *host_buf, size_t bytes,
               int64_t *step, double *time);

/* Scalar diagnostics over [0, n).  Returns SPH_E_NONFINITE (with *out still
 * written) when a particle holds a NaN or infinite x, y, u, v, p, rho or h:
 * the check for a state that has blown up; SPH_E_INVAL (with *out written,
 * mq_total not meaningful) when a mass is negative or the ledger total
 * does not fit int64 (a mass quantum too fine for this many particles).
 * Synchronises. */
int sph_diagnostics(sph_ctx *ctx, const sph_particles *ps, sph_diag *out);

/* Profiling: bits 0-3 of `on` select the kernels to bracket with HIP events
 * on the context's stream (1 "pass_a", 2 "pass_b", 4 "build" (neighbour
 * sort and tables), 8 "list" (rate-pass list)); bits 8-15 give a sampling
 * period p (0 or 1: every launch; p: every p-th launch of each selected
 * kernel); 0 turns profiling off.  sph_profile_read synchronises and
 * returns the total milliseconds and the count of the bracketed launches of
 * the named kernel since the last reset. */
int sph_profile_enable(sph_ctx *ctx, int32_t on);
int sph_profile_read(sph_ctx *ctx, const char *kernel, double *ms, int64_t *launches);
int sph_profile_reset(sph_ctx *ctx);

/* ---- Rate evaluation that allocates nothing -----------------------------
 * For callers that cannot allocate device memory or create a context: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same evaluation as sph_rates (same kernels and results as
 * a context created with lean = 1 and list_skin = 0; the configuration's
 * lean and list_skin are ignored), on the current HIP device, enqueued on
 * `stream` (a hipStream_t of that device, NULL = default stream).  The
 * caller passes the particles and the outputs (as for sph_rates); scratch
 * memory is a static device array of SPH_NOALLOC_SCRATCH_BYTES that every
 * GPU the library runs on holds until the process ends.  The call
 * allocates nothing (no hipMalloc or hipFree, no host mailbox) and does not
 * synchronise.  Calls on one GPU share its array: calls that overlap on
 * the device (other streams, other threads) race; calls on one stream are
 * ordered.  Errors: SPH_E_NOMEM when the particles need more scratch than
 * the array holds (sph_rates_noalloc_bytes gives the need; about 1.5 KB
 * per particle at the default list width plus the cell tables, so some
 * 40,000 particles fit), SPH_E_INVAL for bad arguments, SPH_E_DEVICE for a
 * HIP error; sph_last_error(NULL) then gives the message (per thread).  On
 * error nothing has been written. */
#define SPH_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
size_t sph_rates_noalloc_bytes(const sph_config *cfg, int64_t n);
int sph_rates_noalloc(const sph_config *cfg, const sph_particles *ps, double dt,
                      sph_rates_out *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SPH_H */
