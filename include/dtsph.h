/*
 * dtsph.h - C-ABI of libdtsph.so, the MI355X (gfx950) hot path of dual-time
 * EDAC SPH with particles frozen in pseudo-time.
 *
 * The library advances weakly-compressible SPH particle state (positions r,
 * velocities V, pressures p) by real time steps of the dual-time scheme of
 * Ramachandran, Muta & Ramakrishna, "Dual-Time Smoothed Particle Hydrodynamics
 * for Incompressible Fluid Simulation" (arXiv:1904.00861):
 *   - Algorithm 2 ("Fixed particles in pseudo-time") gives the structure of a
 *     real step: a rate pass and predictor (eq. v0, eq. r0), the pseudo-time
 *     loop (eqs. pkstar_frozen, vkp1_frozen, pkp1_frozen with the frozen
 *     eq. dv_dtau_exact) run until the stop test of section 3.4 (eq. conv and
 *     the stall rule after it), then the position update eq. r-update;
 *   - the rates are the SPH sums of section 3.2: eq. dp-dtau-frozen-edac for
 *     the pressure and eq. mom-sph-frozen for the momentum, with the Monaghan
 *     artificial viscosity eq. mom-av / eq. av-phiij and the Morris viscous
 *     term, over neighbours within the support of a quintic spline kernel;
 *   - walls use the boundary condition of Adami et al. (2012) with the wall
 *     pressure kept non-negative, as section 3.2 describes.
 *   - particle shifting with a Taylor correction (section 3.5) runs after the
 *     corrector for the sims that ask for it; particles moving in pseudo-time
 *     (Algorithm 1) and the steady-state solve (sections 2.3 and 3.3) are
 *     per-sim variants of the same loop.
 *
 * Every numerical step runs in HIP kernels on the GPU. Many independent
 * simulations ("sims") can share one context and advance together.
 *
 * Conventions
 *   - Every call returns an int status (DTSPH_OK = 0, positive = warning,
 *     negative = error) unless stated otherwise. No C++ exception crosses the
 *     ABI. After an error, dtsph_last_error() describes it.
 *   - Particles are in "caller order": sim 0's fluid particles, then sim 0's
 *     walls, then sim 1's fluid, sim 1's walls, and so on. Per-particle vectors
 *     are float64 [n][3] row-major (three components even in 2D; the unused one
 *     is ignored on input and written as 0).
 *   - Pointers in state views are DEVICE pointers (HIP/torch device memory of
 *     the context's GPU). Pointers marked "host" are host memory.
 *   - The caller owns every pointer it passes; the library keeps none of them
 *     after the call returns. The context owns its internal (cell-ordered)
 *     copy of the state and all scratch memory, allocated at creation.
 *   - All GPU work is ordered on the stream given at creation. Calls that
 *     return reports synchronise that stream before returning.
 *   - One context must not be used from two threads at once.
 */
#ifndef DTSPH_H
#define DTSPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define DTSPH_OK 0
#define DTSPH_WARN_MAXITER 1 /* >= 1 sim stopped at max_iter; state valid      */
#define DTSPH_EINVAL (-1)    /* invalid argument / description / call order    */
#define DTSPH_ENOMEM (-2)    /* device allocation failed                       */
#define DTSPH_EHIP (-3)      /* HIP runtime error                               */
#define DTSPH_ENONFINITE (-4)/* NaN/Inf in a residual; state undefined         */
#define DTSPH_EOVERFLOW (-5) /* neighbour list capacity exceeded (raise
                                max_neighbors) or a cell holds > 4096 particles;
                                particle state undefined, recreate the context */

/* ---- precision of the pair sums ------------------------------------------
 * DTSPH_FP64: every quantity in float64 (the plain path).
 * DTSPH_FP32: pair sums, velocities and pressure rates in float32 on
 *   32-bit fixed-point positions (exact periodic wrap-around); positions,
 *   pressure, the pseudo-time pressure accumulation and the residual
 *   reductions stay float64.                                               */
#define DTSPH_FP64 0
#define DTSPH_FP32 1

/* ---- stop reasons (dtsph_iter_report.reason) ----------------------------
 * Section 3.4: the loop stops when both residuals are below tol (CONVERGED),
 * or each is below tol or stalled - its last stall_window values spread by
 * less than stall_rel of their maximum (STALLED) - or at max_iter. */
#define DTSPH_RUNNING 0
#define DTSPH_CONVERGED 1
#define DTSPH_STALLED 2
#define DTSPH_MAXITER 3
#define DTSPH_NONFINITE 4
#define DTSPH_FIXED 5 /* fixed_iters reached (stop test disabled) */

/* ---- one simulation ------------------------------------------------------
 * Physical inputs of one sim. Uniform density rho0 (the density is held fixed,
 * section 3), mass and smoothing length for all its particles.
 *   dim            2 or 3
 *   max_neighbors  capacity of each particle's neighbour list, at most 8000;
 *                  0 = estimate 1.5 x the lattice count of the support + 8
 *   h, kappa       smoothing length and support radius kappa*h (quintic: 3)
 *   rho0, mass     density and particle mass
 *   vref, beta     reference speed and beta = c / vref (section 3.4)
 *   nu             kinematic viscosity (Morris term)
 *   nu_e           EDAC diffusivity; <= 0 selects h c / 16 (eq. nu_edac)
 *   alpha, eps_av  artificial viscosity (eq. mom-av) and its regulariser
 *   eta            Morris regulariser (0.01 in the paper)
 *   g              body force per unit mass
 *   dt, dtau       real step; pseudo step (<= 0 selects dt / beta)
 *   tol            convergence tolerance epsilon of eq. conv
 *   max_iter       iteration cap (1000 in the paper)
 *   stall_window   iterations in the stall test (0..8; the paper says 3 or 4)
 *   stall_rel      relative spread of the stall test (0.05)
 *   conv_norm      0: mean residuals (the paper); 1: max residuals
 *   edac_reg_literal  1: EDAC diffusion denominator r^2 + h^2 as printed,
 *                  0: r^2 + eta h^2 (the Morris form of the viscous term)
 *   edac_rho_literal  1: keep the printed extra 1/rho_j in the EDAC term
 *   lo, hi         domain box. Periodic axes: the period [lo, hi); needs
 *                  kappa*h < (hi-lo)/2. Other axes: the cell grid's extent;
 *                  particles outside it are clamped into edge cells.
 *   periodic       per axis 0/1
 *   shift          1: particle shifting with Taylor correction after the
 *                  corrector (section 3.5, eqs. shift, shift-deltar,
 *                  shift-correct; free-surface particles are not shifted)
 *   shift_r, shift_n  shifting coefficient 1 + shift_r (W_ij / W(h))^shift_n;
 *                  the printed form is shift_r = 1, shift_n = 1 (n in 1..8)
 *   steady         1: steady-state solve (sections 2.3 and 3.3): pressure rate
 *                  eq. dp-dtau-frozen (no EDAC term), momentum eq. mom-steady
 *                  (no real-time term; minus the convective sum
 *                  sum_j (V_i . gradW_ij)(V_i + V_j) m/rho, a wall giving its
 *                  ghost velocity); particles never move. A real step
 *                  (dtsph_step, or predict / pseudo_iterate / correct) is then
 *                  one run of the pseudo-time loop from the current state,
 *                  started with the steady pressure rate there, whose end state
 *                  becomes the new state (V^{n-1} <- V^n, V^n <- V^K, p <- p^K);
 *                  eq. conv uses dt as given. Needs shift = 0. Steady and
 *                  time-accurate sims may share a context.
 *   move           particles in pseudo-time (sections 2.1 and 3.1, Algorithm
 *                  1): 0 frozen (Algorithm 2); 1 moving, r^{k+1/2} = r^k +
 *                  dtau/2 Vtilde^k, r^{k+1} = r^{k+1/2} + dtau/2 Vtilde^{k+1},
 *                  Vtilde^{k+1} = dt dV/dtau (eqs. rkstar, rkp1, vtilde), with
 *                  the advective terms Vtilde_i . sum_j (p_i + p_j) m/rho gradW
 *                  in the pressure rate (rho_i times the printed eq. dp-dtau
 *                  term, which is grad(p)/rho) and sum_j (Vtilde_i . gradW_ij)
 *                  (V_i + V_j) m/rho in the momentum rate (eq. discrete_ME),
 *                  over the lists of r^(0); 2 as 1 with the lists recomputed at
 *                  every r^{k+1/2} (from candidate lists: a particle moving
 *                  more than 0.45 skin from r^(0) inside one loop raises
 *                  EOVERFLOW). The loop's motion is discarded by eq. r-update.
 *                  Needs steady = 0.                                      */
typedef struct dtsph_sim_desc {
    int32_t dim;
    int32_t max_neighbors;
    double h, kappa;
    double rho0, mass;
    double vref, beta;
    double nu, nu_e;
    double alpha, eps_av, eta;
    double g[3];
    double dt, dtau;
    double tol;
    int32_t max_iter, stall_window;
    double stall_rel;
    int32_t conv_norm, edac_reg_literal;
    int32_t edac_rho_literal, reserved0;
    double lo[3], hi[3];
    int32_t periodic[3], reserved1;
    int32_t shift, shift_n;
    double shift_r;
    int32_t steady, move;
} dtsph_sim_desc;

/* ---- state views (device pointers, caller order, n = all particles) -----
 * Between steps the state is (x, v, v_prev, p) = (r^n, V^n, V^{n-1}, p^n).
 * For walls, v is the prescribed wall velocity (walls never move), v_prev is
 * ignored, and p (output only) is the last wall pressure.
 * Inside a step, after dtsph_predict and until dtsph_correct, the pseudo-time
 * state is also defined: x_iter = r^(0) (frozen positions), v_iter = V^k,
 * p_iter = p^k, dpdtau = (dp/dtau)^k; x, v, v_prev, p still hold r^n, V^n,
 * V^{n-1}, p^n.
 * dtsph_set_state: x, v, v_prev, p are required. If x_iter is non-NULL, all
 *   four in-loop pointers are required and the context enters the in-loop
 *   phase (ready for dtsph_pseudo_iterate); otherwise the between-steps phase.
 * dtsph_get_state: any pointer may be NULL (not written). In-loop pointers are
 *   only valid in the in-loop phase (DTSPH_EINVAL otherwise).              */
typedef struct dtsph_state_view {
    double *x;      /* [n][3] */
    double *v;      /* [n][3] */
    double *v_prev; /* [n][3] */
    double *p;      /* [n]    */
    double *x_iter; /* [n][3] */
    double *v_iter; /* [n][3] */
    double *p_iter; /* [n]    */
    double *dpdtau; /* [n]    (walls: 0) */
} dtsph_state_view;

/* ---- per-sim report of one pseudo-time loop (host memory) ---------------
 * iters: iterations run; reason: DTSPH_* stop reason; rp_*, rv_*: the last
 * iteration's residuals of eq. conv, mean |dp/dtau| dt/(rho0 c^2) and mean
 * |Vtilde|/vref with Vtilde = dt dV/dtau (eq. vtilde), and the same with
 * max instead of mean; pairs: fluid-row neighbour pairs per iteration.     */
typedef struct dtsph_iter_report {
    int32_t iters;
    int32_t reason;
    double rp_mean, rv_mean, rp_max, rv_max;
    int64_t pairs;
} dtsph_iter_report;

/* ---- timing of the pair pass (host memory; dtsph_set_option TIMING) ----- */
typedef struct dtsph_timing {
    int64_t pass_launches;  /* pseudo-iteration pair-pass launches timed (every
                               n-th, see DTSPH_OPT_TIMING)                   */
    double pass_ms;         /* summed duration (HIP events on the ctx stream) */
    int64_t pass_pairs;     /* neighbour pairs those launches evaluated       */
    int64_t pass_particles; /* fluid particles those launches updated         */
    int64_t wall_launches;
    double wall_ms;
    int64_t build_launches; /* full builds timed: keys, sort, gather, lists   */
    double build_ms;
    int64_t build_particles;/* particles those builds sorted                  */
    int64_t filter_launches;/* list filters timed (exact lists re-derived from
                               the candidate lists without a sort)           */
    double filter_ms;
    /* counted on every call (timing on or off), reset with the timers:       */
    int64_t full_builds;    /* sorts + neighbour-list builds                  */
    int64_t list_filters;   /* exact lists filtered from candidate lists      */
    double last_max_shift;  /* largest particle shift of the last shifting    */
    double last_disp;       /* largest |r^{n+1} - r^(0)| of the last loop     */
    int64_t spec_tries;     /* speculative ends of step queued (see
                               DTSPH_OPT_SPECULATE) and how many of them ran */
    int64_t spec_hits;
    int64_t tail_launches;  /* persistent tail launches (DTSPH_OPT_TAIL_LOOP 1) */
} dtsph_timing;

/* ---- sizes (host memory) ------------------------------------------------- */
typedef struct dtsph_info {
    int64_t n, n_fluid, n_wall;
    int64_t n_cells;        /* fluid cells of all sims (wall cells: as many)  */
    int32_t n_sims, precision;
    int32_t nbr_capacity;   /* neighbour list capacity per particle           */
    int32_t block;          /* pair-pass workgroup size                       */
    int32_t lanes;          /* lanes per particle in the pair pass            */
    int32_t reserved;
    int64_t device_bytes;   /* bytes of the context's device arrays          */
} dtsph_info;

/* ---- cell-ordered layout of a build (host memory; dtsph_build_cells) -----
 * keys          int32[n]: cell key of each slot (slot = position in the sorted
 *               order; fluid keys of every sim first, then wall keys)
 * caller_index  int32[n]: caller index of the particle in each slot
 * cell_start    int64[2 * n_cells + 1]: first slot of each key; key k holds
 *               slots [cell_start[k], cell_start[k+1]) (n_cells: dtsph_info)
 * Any pointer may be NULL (not written).                                   */
typedef struct dtsph_cells_view {
    int32_t *keys;
    int32_t *caller_index;
    int64_t *cell_start;
} dtsph_cells_view;

typedef struct dtsph_ctx dtsph_ctx;

/* Create a context for n_sims simulations. sims, n_fluid, n_wall: host
 * arrays of n_sims entries (n_fluid[s] >= 1, n_wall[s] >= 0). precision:
 * DTSPH_FP64 or DTSPH_FP32. hip_stream: hipStream_t to order work on (NULL:
 * the default stream). Uses the current HIP device. On success *out owns all
 * device memory; release with dtsph_destroy. Errors: EINVAL (bad description,
 * kappa*h >= L/2 on a periodic axis, dt/dtau <= 0, ...), ENOMEM, EHIP; on
 * error *out is NULL and dtsph_last_error(NULL) describes it.             */
int dtsph_create(const dtsph_sim_desc *sims, const int64_t *n_fluid, const int64_t *n_wall,
                 int32_t n_sims, int32_t precision, void *hip_stream, dtsph_ctx **out);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid device allocation): dtsph_create without any
 * allocation of device memory, mapped or pinned host memory, streams or events.
 * Arguments, checks and the resulting context are those of dtsph_create, except:
 *   - every device array of the context lives in the library's static device
 *     scratch of DTSPH_STATIC_SCRATCH_BYTES per GPU (held until the process
 *     ends); ENOMEM if the context needs more (dtsph_workspace_bytes tells how
 *     much a regular context of the same sims uses; roughly 0.8 kB per particle
 *     in FP32, 1 kB in FP64: ~65k particles);
 *   - one static context per GPU at a time: EINVAL while another one holds the
 *     device's scratch (dtsph_destroy releases it). Its contents are whatever
 *     the last static context left; creation clears what must start at zero.
 *     Static contexts on one GPU must not overlap in time;
 *   - the per-sim reports reach the host by a copy after a stream
 *     synchronisation instead of through mapped memory (same results);
 *   - options that would allocate are refused (EINVAL): PAIR_CACHE, GRAPHS,
 *     TIMING (HIP events), and so are dtsph_set_workspace and dtsph_autotune.
 * The context object itself is ordinary host memory. Results are identical to
 * a dtsph_create context's, bit for bit.                                     */
#define DTSPH_STATIC_SCRATCH_BYTES 67108864 /* 64 MiB */
int dtsph_create_static(const dtsph_sim_desc *sims, const int64_t *n_fluid, const int64_t *n_wall,
                        int32_t n_sims, int32_t precision, void *hip_stream, dtsph_ctx **out);

/* Free the context and its device memory (synchronises its stream). NULL ok. */
void dtsph_destroy(dtsph_ctx *ctx);

/* Text of the last error of ctx (or of the last failed dtsph_create if ctx is
 * NULL). Valid until the next call on ctx. Never NULL.                     */
const char *dtsph_last_error(const dtsph_ctx *ctx);

/* Load / read the particle state (see dtsph_state_view). set_state
 * invalidates the cell lists. On a periodic axis every position (x, and
 * x_iter when given) must lie in [lo, hi), the interval the step keeps them in.
 * Errors: EINVAL (NULL required pointer, wrong phase for in-loop fields, a
 * periodic coordinate outside [lo, hi): the state is then not usable and must
 * be set again), EHIP.                                                      */
int dtsph_set_state(dtsph_ctx *ctx, const dtsph_state_view *state);
int dtsph_get_state(dtsph_ctx *ctx, const dtsph_state_view *state);

/* Cell-linked list and neighbour lists at the current positions (r^n
 * between steps, r^(0) in the loop): cell key per particle, counting sort by
 * cell (ties in caller order), cell-start table, and each particle's exact
 * neighbour list N(i) = { j != i : |r_ij| < kappa h } (minimum image on
 * periodic axes; fluid rows take fluid and wall j, wall rows fluid j only).
 * The predicate is evaluated in float64 without fused multiply-add, so the
 * sets equal those of any implementation of that formula. The lists are
 * needed once per position change: at r^n and at r^(0) in each step; the
 * pseudo-time loop reuses them (frozen particles). A build also keeps
 * candidate lists of radius kappa*h + skin (skin = 0.3 h; 0.25 h with
 * particle shifting); since
 * r^{n+1} - r^(0) = dt/2 (V^{n+1} - V^(0)), the loop knows how far particles
 * will move, and the lists at r^{n+1} are then the candidates filtered by
 * the same exact predicate (no sort) whenever that distance is below 0.4 skin.
 * Other calls build on demand; calling it explicitly is optional. out: NULL,
 * or host arrays that receive the cell-ordered layout (dtsph_cells_view) of
 * the lists in use, which the call builds if the positions changed since the
 * last build. Errors: EOVERFLOW (capacity; the message names the needed
 * max_neighbors), EHIP.                                                     */
int dtsph_build_cells(dtsph_ctx *ctx, const dtsph_cells_view *out);

/* Predictor of Algorithm 2 (between-steps -> in-loop phase): wall pass and
 * rate pass at (r^n, V^n, p^n) with dV/dtau = 0, then eq. v0 and eq. r0 in
 * float64 (positions wrapped into periodic boxes), p^(0) = p^n and
 * (dp/dtau)^0 = D^n. Errors: EINVAL (already in-loop), EOVERFLOW, EHIP.     */
int dtsph_predict(dtsph_ctx *ctx);

/* Pseudo-time loop of Algorithm 2 at the frozen positions r^(0) (in-loop
 * phase, stays in it). Each iteration: p^{k+1/2} = p^k + dtau/2 (dp/dtau)^k;
 * wall pass at (V^k, p^{k+1/2}); one pair pass giving (dp/dtau)^{k+1/2} and
 * the momentum right side; dV/dtau from the frozen eq. dv_dtau_exact (BDF2
 * real-time derivative); V^{k+1} = V^k + dtau dV/dtau; p^{k+1} = p^{k+1/2} +
 * dtau/2 (dp/dtau)^{k+1/2}; float64 residual reduction and stop test per
 * sim. fixed_iters > 0: run exactly that many iterations (no stop test);
 * 0: run until every sim stops. rep: host array of n_sims reports, or NULL.
 * Returns OK, WARN_MAXITER, ENONFINITE, EINVAL (not in-loop), EHIP.        */
int dtsph_pseudo_iterate(dtsph_ctx *ctx, int32_t fixed_iters, dtsph_iter_report *rep);

/* Corrector of Algorithm 2 (in-loop -> between-steps phase): eq. r-update
 * r^{n+1} = r^n + dt/2 (V^n + V^{n+1}) in float64 (wrapped), V^{n-1} <- V^n,
 * V^n <- V^{n+1}, p^n <- p^K. Errors: EINVAL (not in-loop), EHIP.           */
int dtsph_correct(dtsph_ctx *ctx);

/* n_steps real steps of Algorithm 2 (predict, pseudo-iterate until each sim
 * stops, correct) from the between-steps phase. reps: host array of
 * n_steps * n_sims reports (step-major) or NULL. Returns the worst status. */
int dtsph_step(dtsph_ctx *ctx, int32_t n_steps, dtsph_iter_report *reps);

/* Test API: the exact neighbour sets N(i) at the current positions (the
 * definition given at dtsph_build_cells), one row per particle.
 * sim: -1 for every particle of the context (rows and entries in caller
 * indices, m = n); or s in [0, n_sims) for sim s alone (rows of its fluid
 * then its walls, entries relative to its first particle, m = n_fluid[s] +
 * n_wall[s]; no pair crosses sims). offsets: host int64[m + 1]; nbrs: host
 * int32[cap] receiving each row in ascending index; *needed (host) receives
 * the pair count. If nbrs is NULL or cap < *needed only offsets and needed
 * are written. Builds if needed. Errors: EINVAL (sim out of range, NULL
 * offsets or needed), EOVERFLOW, EHIP.                                      */
int dtsph_neighbor_list(dtsph_ctx *ctx, int32_t sim, int64_t *offsets, int32_t *nbrs, int64_t cap,
                        int64_t *needed);

/* Options (value semantics per option). Errors: EINVAL.                    */
#define DTSPH_OPT_TIMING 1     /* n >= 1: time every n-th pair-pass, wall-pass
                                  and build launch with HIP events; -1: the
                                  first pair and wall pass of every loop
                                  (whole workload, queued behind the build)
                                  and every build; 0: off                  */
#define DTSPH_OPT_RESET_TIMING 2
#define DTSPH_OPT_CHUNK 3      /* iterations launched between stop checks (>=1) */
#define DTSPH_OPT_BLOCK 4      /* pair-pass workgroup size: 64, 128 or 256    */
#define DTSPH_OPT_XCD_REMAP 5  /* 1: map consecutive tiles to one XCD (default) */
#define DTSPH_OPT_LANES 6      /* lanes per particle in the pair pass: 1, 2, 4, 8
                                  (default: smallest giving >= 512k threads)  */
#define DTSPH_OPT_SKIN 7       /* candidate-list skin in thousandths of h, at
                                  most the default (300; 250 for sims with
                                  shifting) (0: rebuild the cell lists at
                                  every position change)                     */
#define DTSPH_OPT_CELL_DIV 8   /* cell side >= (kappa h + skin) / value, value
                                  in {1, 2, 3} (default 2); the search visits
                                  +-value cells per axis                      */
#define DTSPH_OPT_NBR_LANES 9  /* lanes per particle of the neighbour-list
                                  build: 1, 2, 4, 8 (0: automatic)           */
#define DTSPH_OPT_GRAPHS 10    /* 1: dtsph_step records the segment from the
                                  rate pass to the first chunk of pseudo-
                                  iterations as a HIP graph (one per launch
                                  configuration, at most 16, kept by the
                                  context) and replays it; 0 (default): plain
                                  launches, which measured faster on MI355X
                                  for every workload here. Steps with a timed
                                  pair-pass launch run plainly.               */
#define DTSPH_OPT_PAIR_CACHE 11 /* cached pair coefficients (the paper's
                                  suggestion in the performance part of
                                  section 4): the first pseudo-iteration of a
                                  loop stores {G r_ij, F_ij} per neighbour-list
                                  entry (with artificial viscosity also
                                  r_ij / (r^2 + eps h^2)) and later iterations
                                  read them instead of the positions; a context
                                  of steady sims keeps them from loop to loop.
                                  0 (default): recompute; 1: always; 2: when
                                  the loop is expected to run >= 3 iterations
                                  (the previous loop's count or the fixed
                                  count) and the last loop's pairs need at most
                                  32 MiB of coefficients (streaming them from
                                  HBM is slower than recomputing; they pay
                                  only while they stay in the last-level
                                  cache). Results equal recomputation to
                                  rounding. Contexts whose EDAC or artificial-
                                  viscosity regulariser differs from eta h^2
                                  recompute. Enabling allocates cap x n
                                  entries of 16 B in FP32, 32 B in FP64 (with
                                  artificial viscosity 8 / 16 B more in 2D,
                                  16 / 32 B in 3D), which adds to
                                  dtsph_workspace_bytes; between steps only. */
#define DTSPH_OPT_SPECULATE 12 /* 1: dtsph_step queues the corrector
                                  and the next step's rate pass (with shifting:
                                  the shift kernels instead of the rate pass)
                                  behind a device gate (every sim stopped, no
                                  non-finite residual, candidate lists still
                                  valid) before it waits for the loop's
                                  reports; when the gate is closed they do
                                  nothing and the step ends as with 0. Off for
                                  contexts with graphs or more than 64 sims,
                                  and while recent gates mostly stayed closed.
                                  Results are identical. 0 (default): with the
                                  cut loop schedule most chunks do not end the
                                  loop, and speculation measured no faster.   */
#define DTSPH_OPT_FILTER_LANES 13 /* lanes per particle of the candidate-list
                                  filter: 1, 2, 4, 8 (0: automatic)           */
#define DTSPH_OPT_ABS32_POSITIONS 14 /* ablation of the FP32 path (0 default):
                                  1 rounds every coordinate to float32 before
                                  the pair passes see it, i.e. float32
                                  separations of absolute coordinates instead
                                  of exact fixed-point ones; no effect in FP64 */
#define DTSPH_OPT_NBR_TILES 15 /* neighbour-list build of 2D contexts: 1
                                  one workgroup per strip of cells stages the
                                  positions of the strip's neighbourhood in
                                  LDS and builds its particles' lists from
                                  there; 0 (default) one lane group per
                                  particle reading positions from global
                                  memory. Same lists either way; 3D contexts
                                  and periodic axes with fewer than 2m+3
                                  cells always use the latter. The
                                  autotuner times both.                      */
#define DTSPH_OPT_TAIL_LOOP 16 /* schedule of a batch's pseudo-time loop,
                                  bit-identical results in every case:
                                  0: chunks of plain launches, the first as
                                  long as the last loop's longest;
                                  1 (default): the first chunk ends where, by
                                  the last loop's per-sim counts, the sims
                                  still iterating hold at most a quarter of
                                  the tiles; later launches cover only those
                                  sims' tiles, and a small remainder (each
                                  sim at most 128 pair-pass tiles) runs the
                                  rest of its loop in one persistent
                                  cooperative launch (per-sim barriers on
                                  the device, no host round trip per chunk;
                                  not with moving or steady sims, separate
                                  regularisers, cached pair coefficients or
                                  in static contexts);
                                  2: as 1 without the persistent launch.   */
#define DTSPH_OPT_TAIL_SPIN 17 /* polls of a tail launch's barrier word before
                                  a waiting workgroup gives up (>= 1; 0
                                  restores the default, 4194304, several
                                  seconds). A wait that gives up leaves the
                                  launch, its sims publish no report, and the
                                  call returns DTSPH_EHIP with the particle
                                  state undefined; small values exist to test
                                  that path.                                 */
int dtsph_set_option(dtsph_ctx *ctx, int32_t option, int64_t value);

/* Autotuner of the launch shapes. Between steps only (EINVAL in the loop).
 * Builds the cell lists if needed, picks the cell subdivision m in {1, 2, 3}
 * together with the neighbour kernel (lanes per particle 1, 2, 4, 8, or the
 * staged-tile kernel where it applies) by timing full builds of every pair
 * (they only reorder the state), then times
 * the rate pass of the predictor (it writes only scratch between steps, so the state is unchanged)
 * for every lanes-per-particle in {1, 2, 4, 8} and workgroup size in {64, 128,
 * 256}, timed as the best of three windows of `repeats` launches (<= 0: 5),
 * and keeps the fastest for this context; then the lanes per particle (1, 2,
 * 4, 8) of the candidate filter, timed the same way. The choice is cached per process by (dim, precision, walls,
 * artificial viscosity, fluid-count bucket) and applied to later contexts of
 * the same kind. out (host, may be NULL) receives every timing.             */
typedef struct dtsph_tune_entry {
    int32_t lanes, block;
    double us; /* duration of one pass launch (best window's mean) */
} dtsph_tune_entry;

typedef struct dtsph_tune_report {
    int32_t lanes, block; /* the pair-pass choice */
    double us;
    int32_t n_entries, reserved;
    dtsph_tune_entry entries[12];
    int32_t nbr_lanes, filter_lanes; /* lanes per particle of the neighbour-list
                                        build and of the candidate filter */
    double nbr_us, filter_us;
    int32_t cell_div;                /* cell subdivision and its full-build time */
    int32_t nbr_tiles;               /* 1: the staged-tile neighbour kernel */
    double build_us;
} dtsph_tune_report;

int dtsph_autotune(dtsph_ctx *ctx, int32_t repeats, dtsph_tune_report *out);

int dtsph_get_timing(const dtsph_ctx *ctx, dtsph_timing *out);
int dtsph_get_info(const dtsph_ctx *ctx, dtsph_info *out);

/* Caller-supplied device memory (for callers whose allocator owns all device
 * memory, e.g. a caching allocator). dtsph_workspace_bytes writes the number of
 * bytes that holds every device array of the context (state, cell tables,
 * neighbour lists, partials; fixed at creation). dtsph_set_workspace moves all
 * of them into `dev` (device memory of the context's device, 256-byte aligned,
 * at least that many bytes), copying their contents on the context's stream
 * and freeing the library's own allocations; dev == NULL moves them back into
 * library allocations. The caller owns `dev` and must keep it alive and
 * untouched until the context is destroyed or another workspace is set; a new
 * workspace must not overlap the current one. Allowed at any point, also inside
 * the pseudo-time loop; synchronises the stream. The context still owns a small
 * block of mapped host memory (reports) and its events.
 * Errors: EINVAL (NULL ctx/bytes, misaligned or non-device memory, overlap),
 * ENOMEM (bytes too small, or library allocation failed with dev == NULL),
 * EHIP; on error the context keeps its previous memory and state.            */
int dtsph_workspace_bytes(const dtsph_ctx *ctx, size_t *bytes);
int dtsph_set_workspace(dtsph_ctx *ctx, void *dev, size_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* DTSPH_H */
