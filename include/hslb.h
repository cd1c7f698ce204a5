/*
 * hslb.h -- C ABI of libhslb.so: the time step of the lattice Boltzmann method
 * for inhomogeneous hard-sphere fluids (Melchionna and Marini Bettolo Marconi,
 * "Lattice Boltzmann method for inhomogeneous fluids") on one AMD Instinct MI355X
 * (gfx950) GPU.
 *
 * The problem the calls state is the paper's: a D3Q19 lattice (section
 * "Methods and Results") carrying a hard-sphere fluid between two flat walls
 * normal to z with halfway bounce-back (subsection "Numerical validation"),
 * periodic in x and y (and in z when there are no walls), driven by a uniform
 * external field parallel to the walls, evolved by the forward-Euler
 * propagation of equation (10) with the second-order equilibrium (11) and the
 * isothermal hard-sphere momentum-transfer term C^(1) of equation (12).
 *
 * Conventions shared by every call:
 *  - Node order: node = x + nx*(y + ny*z).  Scalar fields are [N] arrays,
 *    vector fields [3][N] (component-major), populations [Q][N] (Q = 19, or 39
 *    with HSLB_D3Q39), where
 *    N = nx*ny*nz counts solid wall layers too.
 *  - Host arrays are caller-owned, FP64, and copied during the call; the
 *    library never keeps a host pointer.  The library owns all device memory.
 *  - Units: lattice units, particle mass m = 1, k_B T = v_T^2 = 1/3 (2/3 on
 *    the 39-velocity lattice).
 *  - Every call returns int: HSLB_OK (0) or a negative HSLB_E* code; no call
 *    aborts or throws.  hslb_last_error() gives a message for the last failure.
 *  - A context is used by one host thread at a time.  Work is queued on the
 *    context's HIP stream; calls that return host data synchronise it.
 *
 * D3Q19 velocity order (index i: c_i):
 *   0:(0,0,0) 1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1) 6:(0,0,-1)
 *   7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0) 11:(1,0,1) 12:(-1,0,-1)
 *   13:(1,0,-1) 14:(-1,0,1) 15:(0,1,1) 16:(0,-1,-1) 17:(0,1,-1) 18:(0,-1,1)
 */
#ifndef HSLB_H
#define HSLB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HSLB_OK = 0,
    HSLB_EINVAL = -1,    /* bad parameters or fields */
    HSLB_ENOMEM = -2,    /* device or host allocation failed */
    HSLB_EDEVICE = -3,   /* HIP runtime error */
    HSLB_EUNSTABLE = -4, /* watchdog: non-finite state or mass drift */
    HSLB_ESTATE = -5,    /* call out of order (e.g. step before init) */
    HSLB_ENOSURR = -6    /* surrogate force requested without weights */
};

enum { HSLB_FP64 = 0, HSLB_FP32 = 1 }; /* population storage precision */

/* Contact value of the pair correlation as a function of the coarse-grained
 * packing fraction eta (section "Methods and Results", Fischer-Methfessel
 * prescription): HSLB_G2_PAPER is the printed closure
 * (1 - eta/2 + eta^2/4)/(1 - eta)^3, HSLB_G2_CS the Carnahan-Starling contact
 * value (1 - eta/2)/(1 - eta)^3. */
enum { HSLB_G2_PAPER = 0, HSLB_G2_CS = 1 };

/* Interaction force: the exact shell sum of equation (12), the learned
 * surrogate (with the exact sum as periodic judge), or none. */
enum { HSLB_FORCE_EXACT = 0, HSLB_FORCE_SURROGATE = 1, HSLB_FORCE_OFF = 2 };

/* Velocity set.  HSLB_D3Q19 (0) is the paper's 19-velocity lattice with the
 * second-order equilibrium (11) and k_B T = v_T^2 = 1/3.  HSLB_D3Q39 is the
 * higher-order Hermite basis the paper names as the alternative to the wall
 * regulariser and as the route to high Knudsen numbers (discussion of the
 * validation, and conclusions): the 39-velocity quadrature of degree 7 with
 * integer velocities, k_B T = v_T^2 = 2/3 (also in the force's k_B T and its
 * current coefficient), the equilibrium (11) carried to third order in u, and
 * a collision that keeps only the h^(2) and h^(3) projections of the
 * non-equilibrium part (off-basis contributions removed):
 *   f_i <- f_eq,i + (1 - 1/tau) w_i [h2_i : a2 / (2 v_T^4) + h3_i : a3 / (6 v_T^6)]
 *          + w_i c_i . F / v_T^2,   a_l = sum_i h_l(c_i) (f_i - f_eq,i).
 * Its population order is: 0 rest; 1-6 +-x, +-y, +-z; 7-14 (1,1,1), (-1,-1,-1),
 * (1,1,-1), (-1,-1,1), (1,-1,1), (-1,1,-1), (-1,1,1), (1,-1,-1); 15-20 +-2x,
 * +-2y, +-2z; 21-32 (2,2,0), (-2,-2,0), (2,-2,0), (-2,2,0), (2,0,2), (-2,0,-2),
 * (2,0,-2), (-2,0,2), (0,2,2), (0,-2,-2), (0,2,-2), (0,-2,2); 33-38 +-3x, +-3y,
 * +-3z.  A link that would cross a wall plane is reversed where it meets the
 * plane and lands on a node (halfway bounce-back for links up to length 3).
 * D3Q39 contexts are FP64 only, need nx, ny >= 3, nz >= 3 when z is periodic
 * and at least 3 fluid layers in a slit, and take no solid mask, learned force
 * or batch. */
enum { HSLB_D3Q19 = 0, HSLB_D3Q39 = 39 };

typedef struct {
    int32_t nx, ny, nz;       /* full grid, solid wall layers included */
    int32_t wall_lo, wall_hi; /* solid layers at the z ends; both 0: z periodic.
                                 Walls sit halfway between the last solid and the
                                 first fluid layer. */
    int32_t sigma;            /* hard-sphere diameter in lattice units, 2..8;
                                 nx, ny >= sigma + 2 */
    double tau;               /* BGK relaxation time, > 1/2 */
    double accel[3];          /* external force per particle g; the momentum
                                 source is n g (equation (1)'s field term) */
    int32_t g2_model;         /* HSLB_G2_* */
    int32_t wall_reg;         /* 1: wall factor 1 - exp(-d_w/sigma) on the
                                 density-current term (section "Methods and
                                 Results"); 0: off */
    int32_t precision;        /* HSLB_FP64 or HSLB_FP32 */
    int32_t force_mode;       /* HSLB_FORCE_* */
    int32_t surr_check_every; /* surrogate mode: exact judge every K steps */
    double surr_tol;          /* surrogate mode: residual threshold */
    /* Optional mean-field attraction, the generalisation to attractive forces
     * named in the paper's conclusions (0: off).  In equilibrium the paper ties
     * C^(1) to density functional theory (C^(1) = -n grad dF_exc/dn, section
     * "Theory"); a mean-field attractive functional adds to the force
     *   Phi(r)    = -att_eps sum_o exp(-|o|^2 / att_range^2) n(r + o),
     *   C1_att(r) = -n(r) [Phi(r + e_a) - Phi(r - e_a)] / 2  (each axis a),
     * o over the cube |o_x|, |o_y|, |o_z| <= ceil(3 att_range), n = 0 on solid
     * layers and beyond the walls, periodic images along periodic axes.  The
     * bulk pressure gains -(att_eps/2) (sum_o exp(-|o|^2/att_range^2)) n^2.
     * att_range in (0, 10] when att_eps != 0.  Not with the learned force or
     * the batch. */
    double att_eps;
    double att_range;
    int32_t lattice;          /* HSLB_D3Q19 (0) or HSLB_D3Q39 */
    /* 1: the non-isothermal terms the paper derives beside equation (12) and
     * then drops by taking T constant (section "Methods and Results"), on the
     * 39-velocity lattice only.  k_B = m = 1; the temperature is
     * n T = (1/3) sum_i f_i |c_i - u|^2 and v_T^2 = T(r) at the receiving node.
     *   C^(1) = -v_T^2 sigma^2 4 pi n sum_q W_q s_q sum_k alpha_k G_k
     *           [n' - chi kappa s.(j' - n' u) + n' (T' - T) / (2 v_T^2)],
     *   C^(2) = v_T^2 sigma^2 4 pi n sum_q W_q sum_k alpha_k G_k
     *           [-s.(j' - n' u) / 2 + n' (T' - T) / (sqrt(pi) v_T)],
     * with the quadrature, interpolation and midpoint closure of the isothermal
     * term; C^(2) is the energy gained per unit volume and step.  The
     * equilibrium is the Maxwellian at (n, u, T) expanded through h^(3) about
     * T0 = 2/3; the sources are w_i [c.F/T0 + ((c.F)(c.u) - T0 F.u)/T0^2 +
     * C2 (c^2 - 3 T0)/(3 T0^2)], so that momentum gains F and energy
     * F.u + C2.  Walls are adiabatic (bounce-back). */
    int32_t thermal;
} hslb_params;

typedef struct hslb_ctx hslb_ctx;

/* Validate *p and allocate a context on the current HIP device.
 * Errors: HSLB_EINVAL (bad parameters; *out untouched), HSLB_ENOMEM,
 * HSLB_EDEVICE.  Release with hslb_destroy. */
int hslb_create(const hslb_params *p, hslb_ctx **out);

/* Free every device and host resource of the context.  NULL is ignored. */
void hslb_destroy(hslb_ctx *ctx);

/* Message of the last failing call on ctx (library-owned, valid until the next
 * call on ctx); a static message when ctx is NULL. */
const char *hslb_last_error(const hslb_ctx *ctx);

/* Queue all later work on the given hipStream_t (NULL: the context's own
 * stream).  The caller keeps ownership of the stream. */
int hslb_set_stream(hslb_ctx *ctx, void *hip_stream);

/* Initial state: populations set to the local equilibrium (11) of the density
 * n[N] and velocity u[3][N] (u may be NULL for rest).  Values on solid layers
 * are ignored and treated as 0.  Errors: HSLB_EINVAL if a fluid n is negative
 * or non-finite or a fluid u non-finite. */
int hslb_init(hslb_ctx *ctx, const double *n, const double *u);

/* Thermal contexts (hslb_params.thermal = 1): the initial state at the
 * equilibrium of (n, u, T), T[N] positive on fluid nodes (NULL: T0 = 2/3
 * everywhere; hslb_init does the same).  Errors: HSLB_ESTATE on a context
 * that is not thermal, HSLB_EINVAL as hslb_init or for a non-positive T. */
int hslb_init_thermal(hslb_ctx *ctx, const double *n, const double *u, const double *T);

/* Thermal contexts: temperature T[N] and energy source C^(2) Q[N] of the
 * current state (0 on solid layers); either pointer may be NULL, not both. */
int hslb_thermal_fields(hslb_ctx *ctx, double *T, double *Q);

/* Advance nsteps time steps of equation (10): moments, coarse-grained density,
 * midpoint contact values, hard-sphere force (12) (plus the mean-field
 * attraction when att_eps != 0) plus n g, BGK collision with
 * the first-order source, streaming with halfway bounce-back.  Asynchronous;
 * launch errors are returned here, a failing watchdog (see
 * hslb_set_watchdog) returns HSLB_EUNSTABLE.  Errors: HSLB_ESTATE before init,
 * HSLB_EINVAL for nsteps < 0. */
int hslb_step(hslb_ctx *ctx, int64_t nsteps);

/* Wait for all queued work of the context. */
int hslb_sync(hslb_ctx *ctx);

/* Capture, without running them, every HIP graph that later hslb_step calls
 * replay (both population buffers as the starting one, every replay length),
 * so that a timed or latency-critical hslb_step does no graph capture or
 * instantiation.  Contexts that step eagerly (learned force, kernel timing on,
 * graphs off) have nothing to capture.  The state does not change.
 * Errors: HSLB_ESTATE before init, HSLB_EDEVICE. */
int hslb_prepare(hslb_ctx *ctx);

/* Number of steps taken since init (or since the last set_populations). */
int hslb_step_count(const hslb_ctx *ctx, int64_t *steps);

/* Moments of the current populations (equation (8)): n[N] and u[3][N] with
 * u = j/n (0 where n = 0, and on solid nodes).  Either pointer may be NULL. */
int hslb_moments(hslb_ctx *ctx, double *n, double *u);

/* Layer profiles accumulated in FP64 on the GPU: n_z[nz] = mean of n over the
 * layer, u_z[3][nz] = (sum of j over the layer)/(sum of n) (0 on empty layers).
 * Either pointer may be NULL. */
int hslb_profiles(hslb_ctx *ctx, double *n_z, double *u_z);

/* Total force F[3][N] = C^(1) + n g at the current state (0 on solid nodes),
 * as the next step would apply it. */
int hslb_force(hslb_ctx *ctx, double *F);

/* Coarse-grained packing fraction eta_bar[N] = (pi sigma^3/6) times the mean
 * density over the lattice nodes of the closed ball of radius sigma/2, at the
 * current state. */
int hslb_eta_bar(hslb_ctx *ctx, double *eta_bar);

/* Solid mask solid[N] (host, nonzero: solid node), beyond the wall layers;
 * call before hslb_init.  Solid nodes carry n = j = 0; a population heading
 * into one returns reversed to its node (halfway bounce-back, as at the walls
 * of section "Numerical validation"); the wall factor of a fluid node uses
 * d_w = (distance to the nearest solid node centre, wall layers included,
 * periodic images along periodic axes) - 1/2, which is the halfway-plane
 * distance of flat walls.  With FP32 storage the reference tables are then
 * kept FP32-representable, so solid nodes hold exact zeros.  Checkpoints do
 * not hold the mask: set it on the new context before hslb_init, then load.
 * Errors: HSLB_ESTATE after hslb_init or on a batch, HSLB_EINVAL with the
 * learned force or a NULL mask. */
int hslb_set_solid(hslb_ctx *ctx, const uint8_t *solid);

/* Mean-field attraction potential Phi[N] (see hslb_params.att_eps) at the
 * current state, solid layers included; all zero when the attraction is off. */
int hslb_attraction_potential(hslb_ctx *ctx, double *phi);

/* Populations f[Q][N] (Q = 19 or 39, see hslb_params.lattice) of the current
 * state, and their replacement.
 * set_populations zeroes solid nodes, resets the step counter and rebuilds the
 * storage reference from the given populations; in HSLB_FP32 contexts the
 * values pass through FP32 storage (for a bitwise resume use the raw
 * checkpoint below). */
int hslb_get_populations(hslb_ctx *ctx, double *f);
int hslb_set_populations(hslb_ctx *ctx, const double *f);

/* Raw checkpoint of a single lattice: the populations in storage precision,
 * the per-layer reference table and the step counters, so that a run resumed
 * from it continues bit for bit.  hslb_checkpoint_size gives the byte count of
 * the caller-owned buffer; hslb_checkpoint_load needs an initialised context
 * of the same grid, precision and lattice (HSLB_EINVAL otherwise). */
int hslb_checkpoint_size(hslb_ctx *ctx, int64_t *bytes);
int hslb_checkpoint_save(hslb_ctx *ctx, void *buf);
int hslb_checkpoint_load(hslb_ctx *ctx, const void *buf);

/* Watchdog: every `every` steps (0: off) check that the state is finite and
 * that the total mass drifts by at most tol (relative) from its value at init;
 * hslb_step returns HSLB_EUNSTABLE at the first failing check, with the step
 * count at that check available from hslb_step_count.  A single lattice starts
 * with every = 1000 and tol = 1e-3, so that a diverging run (the scheme is
 * unstable above a packing fraction that depends on sigma and tau) stops
 * instead of stepping on in non-finite values; a batch starts with it off. */
int hslb_set_watchdog(hslb_ctx *ctx, int64_t every, double tol);

/* Storage of the populations: f_i is kept as f_i - w_i nref(z), with nref the
 * mean density of the layer the population was streamed from, so that FP32
 * storage resolves the deviations from the layered state rather than the
 * layered state itself.  Every `every` steps (FP32 default 50, FP64 default
 * 0 = never) one step moves nref to the current layer means.  The values of
 * the populations are the same either way up to storage rounding. */
int hslb_set_shift_period(hslb_ctx *ctx, int64_t every);

/* Replay steps from a captured HIP graph (1, default) or launch kernels one by
 * one (0).  Both give bitwise identical results. */
int hslb_set_graph(hslb_ctx *ctx, int32_t enable);

/* Collide kernel of the step (the shell sum of eq. (12) with the BGK update):
 * 0 (default) reads the shell fields from global memory; 1 stages the (n, j)
 * entries and contact values of the layer, and the (n, j) entries of the xz
 * face diagonals, of each 64 x 4 tile of a layer through LDS wherever the
 * lattice allows it (FP32 storage, nx a multiple of 64 and ny of 4, no solid
 * mask, hard-sphere force on; else the default kernel runs).  Both give
 * bitwise identical results; on the 256^3 bulk at sigma 6 the staged kernel
 * takes about as long as the default one, on the sigma-8 slit longer.
 * Errors: HSLB_EINVAL (null context). */
int hslb_set_collide_tiles(hslb_ctx *ctx, int32_t enable);

/* Per-kernel timing with HIP events on the context's stream.  When enabled
 * (and graphs off), hslb_step brackets every kernel launch with events;
 * hslb_kernel_times fills names/total milliseconds/launch counts for up to
 * `cap` kernels and sets *count. */
int hslb_set_kernel_timing(hslb_ctx *ctx, int32_t enable);
int hslb_kernel_times(hslb_ctx *ctx, int32_t cap, char (*names)[32], double *total_ms,
                      int64_t *launches, int32_t *count);

/* Wall-clock milliseconds per step and fluid-node updates per second / 1e6
 * over the last hslb_step call (measured with HIP events around the call). */
int hslb_get_timings(hslb_ctx *ctx, double *ms_per_step, double *mlups);

/* ---- Batched ensembles ------------------------------------------------------
 * Many independent slits (each its own grid, walls, sigma, tau, field, packing)
 * advanced together: every phase of the step is one persistent launch whose
 * grid walks a work list spanning all slits, and steps replay K at a time from
 * one captured HIP graph.  The slits' problems are the single-lattice one of
 * this header; a batch context accepts hslb_step, hslb_sync, hslb_get_timings,
 * hslb_set_graph, hslb_set_kernel_timing, hslb_set_stream and hslb_destroy.
 *
 * hslb_batch_create: slits[nslits] validated as for hslb_create, all with the
 *   same precision and no surrogate force.  Errors as hslb_create (the message
 *   names the failing slit).
 * hslb_batch_init: initial state of one slit, arrays of that slit's size (see
 *   hslb_init).  Every slit must be initialised before the first step.
 * hslb_batch_profiles: layer profiles of one slit (see hslb_profiles).
 * hslb_batch_finite: flags[nslits] = 1 where the slit's state is finite
 *   (unstable slits diverge independently of the others).
 * hslb_batch_set_config: persistent grid of grid_per_cu blocks per compute
 *   unit for every phase; work in slit order (order 0) or grouped by sigma
 *   (order 1).
 * hslb_batch_set_launch / hslb_batch_get_launch: the same with separate grids
 *   for the four field phases (moments, row sums, ball sums, contact values)
 *   and for the collide phase; the active configuration.
 * hslb_batch_autotune: times 12 launch configurations over `steps` steps
 *   each: one grid of 1, 2, 4, 8, 16, 32 blocks per CU for every phase (slit
 *   order); then the best phase grid with the five other collide grids; then
 *   the best of these with the work grouped by sigma.  Keeps the fastest
 *   (*choice = its index), writes the microseconds per step of up to `cap`
 *   candidates in that order; the state is restored.  When the environment
 *   variable HSLB_TUNE_CACHE names a file, a configuration stored there for
 *   the same device, storage precision and slit list (geometry and sigma of
 *   every slit, in order) is applied without timing (*choice = -1,
 *   us_per_step[0] = its stored time); otherwise the result is added to the
 *   file (a JSON object, one entry per line). */
int hslb_batch_create(const hslb_params *slits, int32_t nslits, hslb_ctx **out);
int hslb_batch_init(hslb_ctx *ctx, int32_t slit, const double *n, const double *u);
int hslb_batch_profiles(hslb_ctx *ctx, int32_t slit, double *n_z, double *u_z);
int hslb_batch_finite(hslb_ctx *ctx, int32_t *flags);
int hslb_batch_set_config(hslb_ctx *ctx, int32_t grid_per_cu, int32_t order);
int hslb_batch_set_launch(hslb_ctx *ctx, int32_t phase_grid_per_cu, int32_t collide_grid_per_cu, int32_t order);
int hslb_batch_get_launch(hslb_ctx *ctx, int32_t *phase_grid_per_cu, int32_t *collide_grid_per_cu, int32_t *order);
int hslb_batch_autotune(hslb_ctx *ctx, int32_t steps, int32_t *choice, double *us_per_step,
                        int32_t cap);

/* ---- Learned force ---------------------------------------------------------
 * Not in the paper: a 3-D convolutional network replaces the exact interaction
 * force C1 of eq. (12) between periodic exact checks.  Network: three 5x5x5
 * convolutions with bias, 1 -> 32 -> 32 -> 3 channels, exact GELU after the
 * first two; input the packing-fraction field pi sigma^3 n / 6; output F_hat
 * with C1 ~= F_hat v_T^2 (6/pi)^2 4 pi / sigma^4.  x and y wrap, z wraps
 * without walls and reads zero beyond walled arrays.  The input, weights and
 * hidden activations are rounded to bfloat16 for the BF16 matrix cores, with
 * FP32 accumulation, biases and activations.
 *
 * Weights: HSLB_CNN_NWEIGHTS FP32 values, canonical order W1[32][1][125],
 * b1[32], W2[32][32][125], b2[32], W3[3][32][125], b3[3]; tap
 * t = (dz+2)*25 + (dy+2)*5 + (dx+2), conv(x)[co][r] = sum W[co][ci][t] x[ci][r + d_t].
 *
 * A context created with force_mode HSLB_FORCE_SURROGATE (nx % 32 == 0,
 * ny % 4 == 0, surr_check_every >= 1, surr_tol > 0, else HSLB_EINVAL) steps
 * as follows once weights are loaded (hslb_step before that: HSLB_ENOSURR):
 *   - every surr_check_every steps (step index % K == 0) an exact step that
 *     also judges the force the surrogate path would apply at that state,
 *     pred = fs F_hat(n) + delta_prev (HSLB_SURR_CORRECTED), fs F_hat(n)
 *     (HSLB_SURR_PLAIN) or delta_prev (HSLB_SURR_FROZEN; delta_prev is 0
 *     at the first check after init or a mode change), by its residual
 *     r = |pred - C1|_2 / |C1|_2 over the fluid nodes, and then keeps the
 *     correction delta = C1 - fs F_hat (C1 itself without the network);
 *   - otherwise, if the last check had r <= surr_tol, a step with
 *     C1 = fs F_hat(n_t) + delta (corrected), fs F_hat(n_t) (plain) or the
 *     frozen exact force delta of the last check without the network (frozen,
 *     the no-network ablation); if r > surr_tol, exact steps until the next
 *     check.  The first check after init, hslb_set_populations, a checkpoint
 *     load or new weights has no previous correction.
 * hslb_surrogate_stats: checks done, exact fallback steps, last and largest
 * residual.  hslb_surrogate_force: fs F_hat [3][N] of the current state
 * (host, caller-owned).  Weight arrays are caller-owned and copied.
 * hslb_surrogate_set_components: the components of F_hat the network drives,
 * bits x = 1, y = 2, z = 4 (default 7; 0 or above 7: HSLB_EINVAL).  A component
 * outside the mask is 0 in F_hat everywhere, so that the corrected path keeps
 * it at the exact value of the last check (as the frozen mode does) while the
 * network moves the others; 4 is the wall-normal variant for slits, whose
 * in-plane force balances the driving field, orders of magnitude below the
 * layering force the network learns.  Like a mode change it drops the
 * previous correction. */
#define HSLB_CNN_NWEIGHTS 144067
enum { HSLB_SURR_CORRECTED = 0, HSLB_SURR_PLAIN = 1, HSLB_SURR_FROZEN = 2 };
int hslb_surrogate_set_weights(hslb_ctx *ctx, const float *w, int64_t nw);
int hslb_surrogate_get_weights(hslb_ctx *ctx, float *w, int64_t nw);
int hslb_surrogate_set_mode(hslb_ctx *ctx, int32_t mode);
int hslb_surrogate_set_components(hslb_ctx *ctx, int32_t mask);
int hslb_surrogate_stats(hslb_ctx *ctx, int64_t *checks, int64_t *fallback_steps, double *last_residual,
                         double *max_residual);
int hslb_surrogate_force(hslb_ctx *ctx, double *F);

/* Training of the learned force from snapshot files.
 * hslb_surrogate_save_snapshot writes the current state of a context (FP32 or
 *   FP64, exact or surrogate force mode, nx % 32 == 0, ny % 4 == 0, hard-sphere
 *   term on) to the file `path`: its network input bf16(pi sigma^3 n / 6) and
 *   its exact C1 / fs without the external field, the training pair of
 *   hslb_trainer_add_snapshot.  Format: the 8 bytes "HSLBSNP1", int32 nx, ny,
 *   nz, wall_lo, wall_hi, sigma, then uint16 x[N] and float target[3][N]
 *   (little endian).
 * hslb_surrogate_train trains the network of a surrogate-mode context on every
 *   file named *.hsnap in snapshot_dir (taken in byte order of their names):
 *   `epochs` passes of one Adam step per snapshot (as hslb_trainer_train), the
 *   learning rate lr halved after each pass, each pass over a permutation of
 *   the snapshots drawn by Fisher-Yates from splitmix64 seeded with
 *   0x48534c42 + pass, swapping entry i with entry (splitmix64 output mod
 *   (i + 1)) for i = count - 1 down to 1.  Training starts from the context's
 *   weights (hslb_surrogate_set_weights; HSLB_ENOSURR without) and leaves the
 *   trained weights loaded, as hslb_surrogate_set_weights would;
 *   *final_loss (nullable) is the mean loss of the last pass.  Errors:
 *   HSLB_ESTATE (not a surrogate context), HSLB_EINVAL (no snapshot files, a
 *   malformed file, epochs < 1, lr <= 0), HSLB_ENOMEM, HSLB_EUNSTABLE (a loss
 *   is not finite; the context's weights are then left unchanged). */
int hslb_surrogate_save_snapshot(hslb_ctx *ctx, const char *path);
int hslb_surrogate_train(hslb_ctx *ctx, const char *snapshot_dir, int32_t epochs, double lr,
                         double *final_loss);

/* Training of the learned force on the GPU.  A trainer holds up to
 * capacity_nodes nodes of snapshots (14 bytes per node of device memory), each
 * of at most max_snapshot_nodes nodes: the network input of a lattice state
 * and its target C1 / fs (exact force without the external field).
 *   hslb_trainer_add_snapshot: from a context's current state (FP32 or FP64,
 *     exact or surrogate force mode; nx % 32 == 0, ny % 4 == 0);
 *   hslb_trainer_add_snapshot_host: from host arrays eta[N] (network input
 *     before rounding) and target[3][N]; walls as in hslb_params;
 *   hslb_trainer_set_weights: FP32 master weights (resets Adam);
 *   hslb_trainer_eval / _grad: loss = mean over fluid nodes and the 3
 *     components of (F_hat - target)^2, the raw output F_hat [3][N] and the
 *     gradient [HSLB_CNN_NWEIGHTS] (each output nullable);
 *   hslb_trainer_step: one Adam step (beta 0.9, 0.999, eps 1e-8) on snapshot k.
 * Gradients: bfloat16 operands (activations, activation gradients), FP32
 * accumulation.  Errors: HSLB_EINVAL, HSLB_ENOMEM (store full), HSLB_ENOSURR
 * (no weights), HSLB_EDEVICE; the message is in hslb_trainer_last_error. */
typedef struct hslb_trainer hslb_trainer;
int hslb_trainer_create(int64_t capacity_nodes, int64_t max_snapshot_nodes, hslb_trainer **out);
void hslb_trainer_destroy(hslb_trainer *tr);
const char *hslb_trainer_last_error(const hslb_trainer *tr);
int hslb_trainer_add_snapshot(hslb_trainer *tr, hslb_ctx *ctx, int32_t *index);
int hslb_trainer_add_snapshot_host(hslb_trainer *tr, int32_t nx, int32_t ny, int32_t nz, int32_t wall_lo,
                                   int32_t wall_hi, const double *eta, const double *target, int32_t *index);
int hslb_trainer_count(hslb_trainer *tr, int32_t *count);
int hslb_trainer_set_weights(hslb_trainer *tr, const float *w, int64_t nw);
int hslb_trainer_get_weights(hslb_trainer *tr, float *w, int64_t nw);
int hslb_trainer_eval(hslb_trainer *tr, int32_t snapshot, double *loss, float *out);
int hslb_trainer_grad(hslb_trainer *tr, int32_t snapshot, double *loss, float *grad);
int hslb_trainer_step(hslb_trainer *tr, int32_t snapshot, double lr, double *loss);
/* n Adam steps on the snapshots order[0..n) in turn; *mean_loss = the mean
 * of their losses (each taken before its step).  HSLB_EUNSTABLE if a loss is
 * not finite. */
int hslb_trainer_train(hslb_trainer *tr, const int32_t *order, int32_t n, double lr, double *mean_loss);

/* One network operation on host data (nx % 32 == 0, ny % 4 == 0, zper: z
 * periodic).  All host arrays are FP32, channel-major [c][N]; values that feed
 * a convolution are rounded to bfloat16 first; w in canonical order.
 *   FWD1: in x[N]          -> out z1[32][N], a1[32][N]    (a = bf16(GELU(z)))
 *   FWD2: in a1[32][N]     -> out z2[32][N], a2[32][N]
 *   FWD3: in a2[32][N]     -> out F_hat[3][N]
 *   DX3:  in g[3][N], aux z2[32][N]   -> out da2[32][N], dz2 = bf16(da2 GELU'(z2))
 *   DX2:  in dz2[32][N], aux z1[32][N] -> out da1[32][N], dz1
 *   DW1:  in x[N], aux dz1[32][N]     -> out dW1[32*125], db1[32]
 *   DW2:  in a1[32][N], aux dz2[32][N] -> out dW2[32*32*125], db2[32]
 *   DW3:  in a2[32][N], aux g[3][N]    -> out dW3[3*32*125], db3[3]
 * (da = transposed convolution of the gradient; dW, db as the weight and bias
 * gradients of the layer.)  Message in hslb_trainer_last_error(NULL). */
enum { HSLB_CNN_FWD1 = 0, HSLB_CNN_FWD2, HSLB_CNN_FWD3, HSLB_CNN_DX3, HSLB_CNN_DX2, HSLB_CNN_DW1, HSLB_CNN_DW2,
       HSLB_CNN_DW3 };
int hslb_cnn_op(int32_t op, int32_t nx, int32_t ny, int32_t nz, int32_t zper, const float *w, const float *in,
                const float *aux, float *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the total
 * force F[3][N] = C^(1) + n g of the density n[N] and velocity u[3][N] (u may
 * be NULL: rest) on the lattice *p, as hslb_force returns it for an FP64
 * context initialised with hslb_init(n, u) (the same kernels, on the local
 * equilibrium of (n, u)).  n, u and F are caller-owned DEVICE arrays of FP64
 * in the node order of this header; the work is queued on hip_stream (NULL:
 * the null stream) and the call returns without synchronising.  *p must be
 * an FP64 19-velocity lattice with the exact force or none and no attraction.
 * Every intermediate (populations, moment fields, contact values, tables)
 * lives in one fixed device-resident array of HSLB_FORCE_NOALLOC_BYTES per GPU
 * (64 MiB, held from the first call on that GPU until the process ends),
 * enough for about 200 000 nodes at sigma 8: a lattice that needs more is
 * rejected with HSLB_EINVAL.  The call allocates nothing.  All calls on one
 * GPU share the array and it keeps the last call's contents (each call
 * clears what it reads), so calls that overlap on one GPU race.  Errors:
 * HSLB_EINVAL (parameters, size, null n or F), HSLB_EDEVICE; the message is in
 * hslb_last_error(NULL). */
#define HSLB_FORCE_NOALLOC_BYTES (64ll << 20)
int hslb_force_noalloc(const hslb_params *p, const double *n, const double *u, double *F, void *hip_stream);

/* Device-to-device copy of `bytes` bytes, repeated `iters` times on a private
 * stream: *gbps = 2 * bytes * iters / elapsed (read + write).  The reference
 * for the achievable HBM bandwidth and the calibration kernel ("k_copy") of the
 * traffic counters.  Allocates and frees its own two buffers. */
int hslb_copy_bandwidth(int64_t bytes, int32_t iters, double *gbps);

#ifdef __cplusplus
}
#endif

#endif /* HSLB_H */
