/*
 * lbm.h -- C-ABI of the MI355X lattice Boltzmann stream-collide library
 * (liblbm.so, hand-written HIP kernels for gfx950).
 *
 * The library advances the particle populations f_i of a lattice Boltzmann
 * simulation: BGK collision to the quadratic equilibrium (paper Sec. 2,
 * eqs. LBM-BGK, tau, feq), streaming (eq. streaming), the boundary treatment
 * of Sec. 3.5 (halfway bounce-back with a moving-wall term, Zou-He velocity /
 * pressure faces, equilibrium outflow, solid cells), the moments rho and u
 * (eqs. density, velocity), and the discrete adjoint of the step (the
 * gradients that the paper obtains from automatic differentiation of `step`,
 * Sec. 3.6 and Sec. 6).
 *
 * Conventions
 *  - Lattices: D2Q9, D3Q19, D3Q27 (Fig. "lattice").  Direction 0 is the rest
 *    vector; 1..Q-1 follow the figure's order.
 *  - Grid: nx * ny * nz cells, fields in (x, y, z) C order with z fastest
 *    (2-D: nz = 1 or 0, y fastest), as the paper's arrays (Sec. 3.3).  Every
 *    cell is a fluid node unless flagged solid; the six domain faces are
 *    halfway outside the outermost cell layer.  N = nx*ny*nz < 2^31.
 *  - Units: dx = dt = 1, cs^2 = 1/3, omega = 1/tau, nu = (tau - 1/2)/3.
 *  - Pointers are device pointers unless marked host.  The caller owns every
 *    pointer it passes; it must stay valid until the work enqueued on the
 *    context's stream has completed.  Nothing is retained after return except
 *    copies the library makes itself.
 *  - All calls are ordered on the context's HIP stream (lbm_set_stream); calls
 *    that return host data synchronise that stream.
 *  - Errors: 0 on success, a negative LBM_E* code otherwise; no exception or
 *    abort crosses the ABI.  lbm_last_error() returns a thread-local message
 *    for the last failing call of this thread.  Argument checks run before any
 *    device work, so a rejected call has no effect.  An asynchronous device
 *    fault surfaces as LBM_EDEVICE at the next synchronising call.
 *  - A context belongs to one host thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define LBM_OK            0
#define LBM_EINVAL       -1   /* bad argument */
#define LBM_ENOMEM       -2   /* device (or host) allocation failed */
#define LBM_EDEVICE      -3   /* HIP runtime / device error */
#define LBM_ESTATE       -4   /* call not valid in the context's current state */
#define LBM_EUNSUPPORTED -5   /* valid request this library does not implement */

/* ---- lattices (Fig. "lattice") ------------------------------------------ */
#define LBM_D2Q9  0
#define LBM_D3Q19 1
#define LBM_D3Q27 2

/* ---- face boundary types (Sec. 3.5; Sec. 3.4 for periodic) --------------- */
#define LBM_PERIODIC        0  /* must be set on both faces of an axis */
#define LBM_WALL            1  /* halfway bounce-back; tangential u = moving wall */
#define LBM_ZOUHE_VELOCITY  2  /* Zou-He non-equilibrium bounce-back, velocity u */
#define LBM_ZOUHE_PRESSURE  3  /* Zou-He, density rho (u normal to the face) */
#define LBM_EQ_OUTFLOW      4  /* missing populations = feq(rho, u of the cell) */
#define LBM_REG_VELOCITY    5  /* regularized (Latt et al. 2008), velocity u: rho as for Zou-He; the whole
                                  cell rebuilt from feq and the regularized non-equilibrium momentum flux */
#define LBM_REG_PRESSURE    6  /* regularized, density rho (u normal to the face) */

/* ---- storage / arithmetic types (Sec. 3.7 "computation/storage" pairs) --- */
#define LBM_F64  0
#define LBM_F32  1
#define LBM_F16  2
#define LBM_BF16 3

/* ---- collision models ----------------------------------------------------- */
#define LBM_BGK 0  /* eq. LBM-BGK (default) */
#define LBM_KBC 1  /* KBC entropic multi-relaxation (D2Q9 / D3Q27) */

/* ---- streaming patterns --------------------------------------------------- */
#define LBM_INPLACE 0  /* one buffer, AA access pattern (Bailey et al. 2009) */
#define LBM_DOUBLE  1  /* two buffers, push streaming */
#define LBM_PULL    2  /* two buffers, pull streaming: every step gathers from the
                          neighbours and writes the cell's own slots (the first
                          step after an init / load is the local in-place step) */

/*
 * One face of the box.  Faces are ordered -x, +x, -y, +y, -z, +z.
 *  type : LBM_PERIODIC / LBM_WALL / LBM_ZOUHE_VELOCITY / LBM_ZOUHE_PRESSURE /
 *         LBM_EQ_OUTFLOW / LBM_REG_VELOCITY / LBM_REG_PRESSURE.
 *  u    : wall velocity (LBM_WALL; its normal component must be 0) or inlet
 *         velocity (LBM_ZOUHE_VELOCITY, LBM_REG_VELOCITY).
 *  rho  : face density (LBM_ZOUHE_PRESSURE, LBM_REG_PRESSURE, LBM_EQ_OUTFLOW); must be > 0 there.
 * Rules (else LBM_EINVAL): periodic on both faces of an axis or on neither;
 * Zou-He / regularized / outflow faces on at most one axis, that axis at least 2 cells
 * long; for 2-D lattices the z faces are ignored.
 */
typedef struct {
    int32_t type;
    int32_t reserved;
    double  u[3];
    double  rho;
} lbm_face;

typedef struct {
    lbm_face face[6];
} lbm_bc;

/*
 * Options; set before the first lbm_init_equilibrium.
 *  storage : LBM_F64, LBM_F32 (default), LBM_F16, LBM_BF16.  Populations are
 *            stored as the deviation h_i = f_i - w_i rho0 (F64/F32) or as
 *            h_i / w_i (F16/BF16, rounded to nearest even) -- the
 *            renormalisation around zero that the paper notes single
 *            precision needs (Sec. 4.1).
 *  compute : LBM_F64 (only with F64 storage) or LBM_F32 (others).
 *  pattern : LBM_INPLACE (default), LBM_DOUBLE or LBM_PULL.  All three give
 *            bitwise-equal states.  LBM_PULL takes twice the memory of
 *            LBM_INPLACE and writes only aligned, cell-local addresses: on boxes
 *            of more than ~10^8 cells it runs faster than the in-place pattern,
 *            whose neighbour step writes Z-shifted addresses.
 *  rho0    : reference density (default 1).
 */
typedef struct {
    int32_t storage;
    int32_t compute;
    int32_t pattern;
    int32_t reserved;
    double  rho0;
} lbm_options;

typedef struct lbm_ctx lbm_ctx;

/*
 * Velocity set of a lattice (Sec. 3.2, Fig. "lattice"): c receives Q rows of
 * 3 int32 components in caller axes (2-D: (cx, cy, 0)), w the Q weights
 * (the textbook values by |c|^2; the paper does not print them).  Both are
 * host pointers of the caller, either may be NULL.  Returns Q, or LBM_EINVAL
 * for an unknown lattice.  No device work.
 */
int lbm_lattice_info(int lattice, int32_t *c, double *w);

/* Thread-local text of the last error of this thread ("" if none). */
const char *lbm_last_error(void);

/* Library version string. */
const char *lbm_version(void);

/*
 * Create a single-domain context (Sec. 3.2 lattice choice, Sec. 3.3 domain,
 * Sec. 3.5 boundary setup).  lattice: LBM_D2Q9/D3Q19/D3Q27; nx, ny >= 1;
 * nz >= 1 for 3-D, nz in {0, 1} for D2Q9 (the paper's nz = 0 for 2-D);
 * tau > 1/2 (nu > 0, eq. tau); bc: host pointer, copied; NULL = all periodic.
 * Does no device work: the state is allocated on the current HIP device by the
 * first lbm_init_equilibrium.  Returns NULL on error (see lbm_last_error).
 */
lbm_ctx *lbm_create(int lattice, int nx, int ny, int nz, double tau, const lbm_bc *bc);

/*
 * Create a batch of independent domains of one lattice that advance together
 * (the batching the paper gets from vmap, Sec. 3.1 / Sec. 6.1).  n >= 1;
 * nx, ny, nz, tau: host arrays of n; bcs: host array of n lbm_bc (NULL = all
 * periodic).  Per-domain fields are packed back to back; lbm_batch_offsets
 * gives each domain's first cell.  Returns NULL on error.
 */
lbm_ctx *lbm_create_batch(int lattice, int n, const int *nx, const int *ny, const int *nz,
                          const double *tau, const lbm_bc *bcs);

/* off: host array of n+1 int64; off[d] = first packed cell of domain d, off[n] = total cells. */
int lbm_batch_offsets(const lbm_ctx *ctx, int64_t *off);

/*
 * Work decomposition of a batch.  A batch is stepped as a list of tiles of
 * `tile` consecutive cells of one domain, one workgroup each; with
 * persistent = 1, n steps run as one cooperative launch whose resident
 * workgroups stride over the tiles with a grid barrier between steps, else
 * one launch per step.  By default the first lbm_step / lbm_capture_graph
 * times tile in {64, 128, 256} x both launch modes on a copy of the state
 * (restored afterwards) and keeps the fastest, caching the choice in the file
 * named by LBM_AUTOTUNE_CACHE (default ~/.cache/lbm_mi355x_autotune.txt);
 * LBM_AUTOTUNE=0 skips the timing.  lbm_batch_tuning(ctx, tile, persistent)
 * fixes the choice (tile 0 keeps the tile, persistent -1 keeps the mode;
 * 0 and -1 together return to automatic).  lbm_batch_config reports it.
 * Batch domains hold fewer than 2^24 cells each and use the in-place pattern;
 * solid cells and partial bounce-back are single-domain features.
 */
int lbm_batch_tuning(lbm_ctx *ctx, int tile, int persistent);
int lbm_batch_config(const lbm_ctx *ctx, int *tile, int *persistent);

/* Free everything the context owns (synchronises its stream).  NULL is a no-op. */
void lbm_destroy(lbm_ctx *ctx);

/* opt: host pointer.  LBM_ESTATE after the state exists, or when the compute
 * type would change while a force field or curved links are set. */
int lbm_set_options(lbm_ctx *ctx, const lbm_options *opt);

/*
 * Change tau and the faces' velocities / densities of a single-domain context
 * (the face types must stay the same).  bc: host pointer or NULL (faces
 * unchanged).  Invalidates a recorded tape and captured graphs.  Checked like
 * lbm_create.
 */
int lbm_set_params(lbm_ctx *ctx, double tau, const lbm_bc *bc);

/*
 * The HIP stream that orders every later call of this context (the paper
 * leaves ordering and asynchronous dispatch of `step` to JAX, Sec. 3.1; here
 * the caller names the stream, normally torch's current one).
 * hip_stream: a hipStream_t (NULL = the null stream); not owned.  Drops a
 * captured graph.  LBM_EINVAL for a NULL context.
 */
int lbm_set_stream(lbm_ctx *ctx, void *hip_stream);

/*
 * Solid cells: the solid part of the boundary mask of Sec. 3.5 (interior
 * obstacles; a fluid cell whose neighbour x - c_i is solid takes f_i by
 * halfway bounce-back, Fig. "mask").  flags: N
 * bytes, nonzero = solid; host (on_device = 0) or device (1).  Copied.  NULL
 * clears.  Valid before or after init; solid cells report rho0, u = 0.
 */
int lbm_set_solid(lbm_ctx *ctx, const uint8_t *flags, int on_device);

/*
 * Curved walls: interpolated bounce-back (Bouzidi, Firdaouss & Lallemand
 * 2001), the paper's no-slip condition for curved geometries (Sec. 4.3), on
 * links from fluid cells into the solid cells of lbm_set_solid.  Link k: the
 * fluid cell cell[k] (flat index in the caller's (x, y, z) order), the
 * direction dir[k] (lbm_lattice_info order) whose neighbour cell + c_dir is a
 * solid cell, and the fraction q[k] in (0, 1] of the link's length at which
 * the wall cuts it.  After every step the population that comes back along
 * -c_dir is the value the bounce geometry interpolates, with
 * order = 1 (linear) or 2 (quadratic) Lagrange weights:
 *   q < 1/2 : the post-collision field f*_dir at s = 2q - 1 from the cells
 *             cell, cell - c_dir (and cell - 2 c_dir);
 *   q >= 1/2: the returning field at the cell from the turned population
 *             (at s = 2q - 1, value f*_dir(cell)) and f*_-dir at cell (and at
 *             cell - c_dir).
 * q = 1/2 is halfway bounce-back.  A link whose cell - c_dir is not a fluid
 * cell keeps halfway bounce-back; a quadratic link whose cell - 2 c_dir is
 * not one uses the linear weights.  Walls at rest.  lbm_forces then sums
 * the momentum exchange of Mei, Yu, Shyy & Luo over these links,
 * (f*_dir(cell, t) + f_-dir(cell, t+1)) c_dir.
 *   n     : number of links (0 clears them; the pointers may then be NULL);
 *   cell, dir, q : host arrays of n, copied (each (cell, dir) at most once);
 *   order : 1 or 2.
 * LBM_EINVAL for an out-of-range or solid cell, a direction whose neighbour
 * (periodic faces wrap) is not a solid cell, q outside (0, 1], a repeated
 * link, an unknown order, or n > 0 without solid cells; LBM_EUNSUPPORTED on
 * batch contexts and for a link whose interpolation cells wrap onto its own
 * cell (a periodic axis shorter than 3 cells).  lbm_set_solid drops the
 * links; lbm_backward returns LBM_EUNSUPPORTED while links are set.  Drops a
 * captured graph.
 */
int lbm_set_curved_links(lbm_ctx *ctx, int64_t n, const int64_t *cell, const int32_t *dir, const double *q,
                         int order);

/*
 * Partial bounce-back solid fraction s in [0, 1] per cell (gray LBM, Walsh,
 * Burwinkle & Saar 2009 -- an addition to the paper): after collision,
 * f_i <- (1 - s) f*_i + s f_opp(i) with the pre-collision opposite population.
 * s: N float32, host (on_device = 0) or device (1); copied; NULL clears.
 * s = 0 everywhere is bitwise the plain BGK step.
 */
int lbm_set_solid_fraction(lbm_ctx *ctx, const float *s, int on_device);

/*
 * f <- feq(rho, u) at every fluid cell (eq. feq), allocating the state on
 * first use.  rho: N values, u: D x N values (component-major: u_x plane,
 * then u_y, then u_z), both device pointers of `dtype` (LBM_F64 or LBM_F32);
 * NULL rho = rho0, NULL u = 0.  Resets the step counter to 0.
 */
int lbm_init_equilibrium(lbm_ctx *ctx, const void *rho, const void *u, int dtype);

/*
 * Advance n >= 0 time steps (collide, stream, boundary fill; Sec. 3.6),
 * asynchronously on the context's stream.  If a tape is recording, the state
 * is checkpointed every K steps.  Batch contexts advance every domain.
 */
int lbm_step(lbm_ctx *ctx, int n);

/* Number of completed steps since the last init / load. */
int64_t lbm_time(const lbm_ctx *ctx);

/*
 * Moments of the current state (eqs. density, velocity): rho (N values) and
 * u (D x N, component-major), device pointers of `dtype` (LBM_F64 or LBM_F32);
 * either may be NULL.  Solid cells get rho0 and 0.  sums_host (nullable, host)
 * receives {mass, P_x, P_y, P_z, kinetic energy 1/2 sum rho|u|^2} over fluid
 * cells, summed in FP64 in a fixed order (deterministic); for a batch context
 * it receives 5 values per domain.  A non-NULL sums_host synchronises.
 */
int lbm_moments(lbm_ctx *ctx, void *rho, void *u, int dtype, double *sums_host);

/*
 * Momentum-exchange force (Ladd; Mei et al. on curved links) of the most
 * recent step: the momentum the
 * fluid handed to the solid cells and to each wall face while streaming into
 * them -- the drag / lift sums of the paper's obstacle flows (Sec. 4.3).  For
 * every fluid cell x and direction i whose neighbour x + c_i is solid or
 * across a wall face, the link contributes (f°_i(x, t) + f_opp(i)(x, t+1)) c_i,
 * with f_opp(i)(x, t+1) = f°_i + 6 w_opp rho0 (c_opp . u_w) under halfway
 * bounce-back and the interpolated value on curved links
 * (lbm_set_curved_links).  In a closed domain
 * the fluid momentum changes over the step by exactly minus the sum of all
 * these forces.
 * out: host double[21], overwritten: out[0..2] force on the solid cells,
 * out[3 + 3 f + a] force on face f (f = -x, +x, -y, +y, -z, +z), axis a,
 * caller axes (2-D: faces -x, +x, -y, +y and axes x, y; the rest 0); a link
 * across several wall faces counts for the lowest-index one.  Summed in FP64
 * in a fixed order (deterministic).  Synchronises.  LBM_ESTATE before the
 * first step after init / load; LBM_EUNSUPPORTED on batch contexts.
 */
int lbm_forces(lbm_ctx *ctx, double *out);

/*
 * lbm_forces for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same 21 FP64 sums
 * (same layout, caller axes), written to the caller's device buffer out_dev
 * (21 doubles) on the context's stream, with no allocation and no
 * synchronisation; the caller reads it after the stream's work.  The per-block
 * partial sums go to a fixed scratch array of 3.4 MB that each GPU holds for
 * the life of the process (rows of up to 16384 x 4096 step-kernel workgroups
 * plus curved-link blocks; larger grids get LBM_EINVAL -- use lbm_forces).
 * The scratch is shared by every call on a GPU: calls that overlap on one GPU
 * (other streams, other threads) race and must be ordered by the caller.  The
 * partial sums are added in a fixed order (per pass of 16384 rows, then the
 * passes), so the result is deterministic; it differs from lbm_forces only in
 * that summation order.  Errors as lbm_forces; LBM_EINVAL for a NULL out_dev.
 */
int lbm_forces_noalloc(lbm_ctx *ctx, double *out_dev);

/*
 * Body force by the exact-difference method (Sec. 4.4 and 6.1, after Kupershtokh, the
 * forcing of the paper's turbulent channel and of its neural corrector): from
 * the next step on, every fluid cell's relaxed populations gain
 * feq_i(rho, u + eps F / rho) - feq_i(rho, u), before any partial bounce-back
 * mix, with F = force + field(x) and u, rho the cell's moments before the
 * force.  lbm_moments keeps reporting u = j / rho (the method's physical
 * velocity is u + eps F / (2 rho)).
 *   force : host double[D] (caller axes), the uniform part; NULL = 0.
 *   field : device pointer or NULL: D planes of N values (component-major,
 *           cells in the order of lbm_moments' output), float for FP32 /
 *           FP16 / BF16 storage, double for FP64 storage.  Read by every later
 *           step: the caller keeps it allocated until the force is replaced
 *           or the context destroyed, and may update it between steps on the
 *           context's stream.  While a field is set, lbm_set_options may not
 *           change the compute type (LBM_ESTATE).
 *   eps   : scale on both parts (the paper's epsilon; 1 for a plain force).
 * A zero force with no field (or eps = 0) switches the force off.  The taped
 * adjoint (lbm_backward, lbm_backward_force) differentiates through the force
 * as set when it runs: keep it unchanged over the taped steps.  LBM_EINVAL for
 * a non-finite force or eps; LBM_EUNSUPPORTED on batch contexts.  Drops a
 * captured graph.
 */
int lbm_set_force(lbm_ctx *ctx, const double *force, const void *field, double eps);

/*
 * Collision model for the following steps (Sec. 2 lists BGK, MRT, cumulant,
 * regularized and KBC collisions; Sec. 4 runs KBC on D2Q9 and D3Q27).
 * LBM_KBC (Karlin, Bosch & Chikatamarla 2014): f - feq splits into a shear part ds -- the deviatoric non-equilibrium
 * momentum flux P, carried by the axis velocities ((P_aa - tr P / D) / 2 each)
 * and the face diagonals (c_a c_b P_ab / 4) -- and the rest dh; the step takes
 * f*_i = f_i - beta (2 ds_i + gamma dh_i), beta = 1 / (2 tau),
 * gamma = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh> with <x|y> = sum x_i y_i / feq_i
 * (the minimiser of the quadratic entropy; BGK when dh = 0 or tau = 1).
 * LBM_EINVAL for an unknown model; LBM_EUNSUPPORTED for KBC on D3Q19, on batch
 * contexts or with a partial bounce-back field; lbm_backward differentiates
 * KBC steps (gamma's dependence on the state included) except with a body
 * force or regularized faces.  Drops a captured graph.
 */
int lbm_set_collision(lbm_ctx *ctx, int model);

/*
 * Start recording a tape for lbm_backward -- the in-memory checkpointing
 * (Sec. 3.7) that differentiating unrolled steps needs (Sec. 3.6, Sec. 6.1):
 * a bit-exact checkpoint of the
 * state now and every K >= 1 steps after it.  The segment between
 * checkpoints is recomputed during the backward pass.  LBM_ENOMEM if the
 * checkpoints for max_steps steps plus a K-state recompute ring do not fit.
 */
int lbm_tape_begin(lbm_ctx *ctx, int K, int max_steps);

/* Stop recording (the tape stays available to lbm_backward). */
int lbm_tape_end(lbm_ctx *ctx);

/* Drop the tape and free its memory. */
int lbm_tape_free(lbm_ctx *ctx);

/*
 * Identity of the context's current tape: a number that grows by one with
 * every lbm_tape_begin on this context (the first tape is 1); 0 when no tape
 * is held, -1 for a NULL context.  A caller that records a tape and runs its
 * backward later (an autograd node, Sec. 6.1's unrolled training) keeps this
 * number and checks it before lbm_backward: a different value means another
 * recording replaced its tape.
 */
int64_t lbm_tape_id(const lbm_ctx *ctx);

/*
 * Discrete adjoint of the recorded steps (the gradient the paper obtains from
 * jax.grad through `step`, Sec. 3.6), seeded at the final state by a loss
 * L(rho, u) of the final moments:
 *   dL_drho : N values, dL_du : D x N values (component-major), device
 *             pointers of `dtype` (LBM_F64 / LBM_F32); either may be NULL (= 0).
 * Outputs (each nullable; all accumulate nothing -- they are overwritten):
 *   dL_ds    : device float32[N], gradient w.r.t. the solid fraction s
 *              (zero if no s field is set);
 *   dL_dtau  : host double[n_domains], gradient w.r.t. each domain's tau;
 *   dL_duw   : host double[n_domains * 6 * 3], gradient w.r.t. each face's
 *              wall velocity (moving LBM_WALL faces only: a wall at rest
 *              takes no moving-wall term, and its entries are 0, as are
 *              those of other faces).
 * The forward state is left unchanged.  Synchronises.  LBM_ESTATE without a
 * tape, if the state moved since the tape ended, or if lbm_set_params,
 * lbm_set_solid, lbm_set_solid_fraction, lbm_set_force or lbm_set_collision
 * was called after the tape began (the recorded steps no longer match the
 * parameters the adjoint would use); LBM_EUNSUPPORTED with curved links,
 * and with regularized faces or the KBC collision on a batch context or with
 * a body force (their transposes cover single domains without one; KBC also
 * not with regularized faces).
 */
int lbm_backward(lbm_ctx *ctx, const void *dL_drho, const void *dL_du, int dtype,
                 float *dL_ds, double *dL_dtau, double *dL_duw);

/*
 * lbm_backward plus the gradients with respect to the body force of
 * lbm_set_force (Sec. 6.1: training a corrector force through unrolled steps):
 *   dL_dfield : device pointer or NULL: D x N values of `dtype` (component-
 *               major, caller axes, the field's layout), overwritten with
 *               dL/dfield(x) = eps sum_t sum_i lambda_i dfeq_i/dm at
 *               m = j + eps F (lambda: the adjoint of the post-collision values);
 *   dL_dforce : host double[D] or NULL: gradient with respect to the uniform
 *               part, the FP64 fixed-order sum of dL_dfield over the cells.
 * eps is that of the last lbm_set_force (1 if none); with no force set the
 * gradients are taken at F = 0.  The adjoint accumulates dL/dF in the compute
 * type (FP64 storage: FP64, otherwise FP32).  LBM_EUNSUPPORTED on batch
 * contexts when either output is requested; otherwise as lbm_backward.
 */
int lbm_backward_force(lbm_ctx *ctx, const void *dL_drho, const void *dL_du, int dtype,
                       float *dL_ds, double *dL_dtau, double *dL_duw,
                       void *dL_dfield, double *dL_dforce);

/*
 * The compiled step loop (the paper JIT-compiles `step` with JAX, Sec. 3.1):
 * capture n_steps >= 1 steps into a HIP graph that lbm_graph_launch replays
 * with one launch (batch and single contexts).  The graph reads the state at
 * launch time; it is invalidated by lbm_init_equilibrium / lbm_load /
 * lbm_set_* calls.
 */
int lbm_capture_graph(lbm_ctx *ctx, int n_steps);
int lbm_graph_launch(lbm_ctx *ctx);

/*
 * Checkpoint / resume (Sec. 3.7): lbm_state_bytes gives the size of the
 * opaque image; lbm_save copies it to host memory (synchronises), lbm_load
 * restores it (bit-exact; the step counter and pattern parity included).
 */
size_t lbm_state_bytes(const lbm_ctx *ctx);
int lbm_save(lbm_ctx *ctx, void *host, size_t bytes);
int lbm_load(lbm_ctx *ctx, const void *host, size_t bytes);

/* Wait for all work of the context; returns LBM_EDEVICE on a device fault. */
int lbm_sync(lbm_ctx *ctx);

/*
 * Streaming copy of `bytes` bytes from src to dst on `hip_stream` (device
 * pointers, 16-byte aligned, bytes a multiple of 16): the bandwidth probe that
 * measures the achievable HBM copy rate, the empirical roofline ceiling.
 */
int lbm_copy_probe(void *dst, const void *src, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
