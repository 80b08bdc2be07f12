/*
 * libxfdtd — one time step of the 3D staggered-grid (Yee) FDTD Maxwell solver
 * whose Faraday update uses the extended stencil of Blinne et al.,
 * "A Systematic Approach to Numerical Dispersion in Maxwell Solvers"
 * (arXiv:1710.06829), built for AMD Instinct MI355X (gfx950).
 *
 * Operations and where the paper defines them:
 *   - extended difference D*_a with per-axis alpha, beta, delta: Sec. 2,
 *     the D* equation; consistency condition eq.(alpha);
 *   - Faraday update with D* and Ampere update with the Yee difference D:
 *     App. A, eq. update1-6 (vacuum, J = 0);
 *   - dispersion relation and stability bound: Sec. 3, eq. dispersion_relation
 *     and eq. constraints; phase and group velocity: Sec. 5;
 *   - divergence constraints: Sec. 2.1, eq. divstarb and eq. divE.
 *
 * Conventions (all functions):
 *   - c = 1: dt is in the same length unit as dx, dy, dz.
 *   - Periodic boundaries on all three axes.
 *   - A field is a contiguous array of nz*ny*nx values, x fastest:
 *     element (i, j, k) is at index (k*ny + j)*nx + i.  Six separate arrays,
 *     in the order Ex, Ey, Ez, Bx, By, Bz, all of the handle's dtype.
 *     Element (i, j, k) of a component sits at the staggered site of the
 *     update equations: Ex (i+1/2, j, k), Ey (i, j+1/2, k), Ez (i, j, k+1/2),
 *     Bx (i, j+1/2, k+1/2), By (i+1/2, j, k+1/2), Bz (i+1/2, j+1/2, k).
 *   - The state is (E^n, B^{n-1/2}); a step is the Faraday update followed by
 *     the Ampere update, giving (E^{n+1}, B^{n+1/2}).
 *   - coeffs[12] = { alpha_x, beta_xy, beta_xz, delta_x,
 *                    alpha_y, beta_yx, beta_yz, delta_y,
 *                    alpha_z, beta_zx, beta_zy, delta_z },
 *     beta_ab being the a-derivative's taps shifted along b (Sec. 2).
 *     All 12 are used as given; alpha is not re-derived.
 *   - Device memory (fields, scratch, k-vectors, outputs marked "device") is
 *     owned by the caller and must stay valid while work that uses it may run.
 *     The library allocates only small internal buffers (reduction partials)
 *     and frees them in xfdtd_destroy.
 *   - Every function returns XFDTD_OK (0) or a negative status; the message
 *     of the last failure on the calling thread is xfdtd_last_error().
 *     Argument errors are reported before any GPU work is queued.  An
 *     asynchronous GPU error is reported by the next call that synchronises.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Work is queued on the stream given to xfdtd_bind (a hipStream_t; NULL
 *     is the default stream).  Functions that return host values synchronise
 *     that stream; the others return as soon as the work is queued.
 */
#ifndef XFDTD_H
#define XFDTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xfdtd_s *xfdtd_t;

/* Grid: cell counts (each >= 1, each <= 2^30, nx*ny*nz <= 4e9, and
 * nx*ny <= 2^28 because z-planes are addressed with 32-bit offsets) and
 * spacings (each > 0, finite). */
typedef struct {
    int64_t nx, ny, nz;
    double dx, dy, dz;
} xfdtd_grid;

enum { XFDTD_F32 = 1, XFDTD_F64 = 2 };

enum {
    XFDTD_OK = 0,
    XFDTD_EINVAL = -1,     /* bad argument (size, pointer, dtype, value) */
    XFDTD_EUNSTABLE = -2,  /* dt beyond the stability bound, or F_min < 0 */
    XFDTD_ENONFINITE = -3, /* a non-finite value was found */
    XFDTD_EHIP = -4,       /* a HIP runtime call failed */
    XFDTD_ESTATE = -5      /* call not valid in the handle's state */
};

/* Warning bits returned by xfdtd_flags(). */
enum { XFDTD_WARN_ALPHA = 1 /* coefficients do not satisfy eq.(alpha) to 1e-12 */ };

/* Version of this interface (incremented on incompatible change). */
int xfdtd_abi_version(void);

/* Message of the last failure on the calling thread ("" if none). */
const char *xfdtd_last_error(void);

/*
 * Stability of a coefficient set (eq. constraints, Sec. 3).
 * Computes F_min and F_max of F(k) = sum_a s_a^2 A_a over the whole zone
 * 0 <= k_a d_a <= pi (exactly, by enumerating the stationary points of F as a
 * quadratic in sin^2(k_a d_a / 2)), then dt_max = 1/sqrt(F_max).
 * Host only; any output pointer may be NULL.  Returns XFDTD_EUNSTABLE if
 * F_max <= 0 (no finite bound) — dt_max is then +inf.
 */
int xfdtd_cfl_limit(const xfdtd_grid *g, const double coeffs[12],
                    double *dt_max, double *f_min, double *f_max);

/* Fill alpha_x, alpha_y, alpha_z of coeffs in place from eq.(alpha):
 * alpha_a = 1 - 2 beta_ab - 2 beta_ac - 3 delta_a.  Host only. */
int xfdtd_consistent_alpha(double coeffs[12]);

/*
 * Create a solver for grid g, time step dt and coefficients coeffs.
 * dtype is XFDTD_F32 or XFDTD_F64 (the type of the fields and of the
 * arithmetic).  Fails with XFDTD_EUNSTABLE if dt^2 F_max > 1 or F_min < 0
 * (tolerance 1e-12 relative) unless allow_unstable is non-zero.
 * The folded weights dt*coef/d_a are computed in double and rounded once to
 * dtype (xfdtd_get_weights reports them).  On success *out owns a handle that
 * must be released with xfdtd_destroy.  No GPU work is queued.
 */
int xfdtd_create(const xfdtd_grid *g, double dt, const double coeffs[12], int dtype,
                 int allow_unstable, xfdtd_t *out);

/* Release a handle (NULL is ignored).  Waits for the handle's queued work. */
void xfdtd_destroy(xfdtd_t h);

/* Warning bits (XFDTD_WARN_*) of a handle. */
int xfdtd_flags(xfdtd_t h);

/*
 * Bind device memory and a stream.
 *   fields[6]  : device pointers Ex, Ey, Ez, Bx, By, Bz (nz*ny*nx elements each,
 *                handle dtype, 16-byte aligned).  They hold the state and receive
 *                the result of every stepping call.
 *   scratch[6] : device arrays of the same size, or NULL.  With scratch the
 *                time loop uses the fused out-of-place step (ping-pong between
 *                fields and scratch); without it, the in-place unfused pair.
 *                Scratch contents are undefined after any call.
 *   stream     : hipStream_t (NULL = default stream).
 * Arrays must not overlap each other.  May be called again to rebind.
 */
int xfdtd_bind(xfdtd_t h, void *const fields[6], void *const scratch[6], void *stream);

/* Faraday update in place on the bound B (App. A, eq. update1-3):
 * B^{n+1/2} = B^{n-1/2} + dt (D* x E^n) with the signs of the paper. */
int xfdtd_step_faraday(xfdtd_t h);

/* Ampere update in place on the bound E (eq. update4-6, J = 0):
 * E^{n+1} = E^n + dt (D x B^{n+1/2}). */
int xfdtd_step_ampere(xfdtd_t h);

/*
 * The Ampere update with a current source (App. A eq. update4-6 with the
 * mu_0 J term, in the library's units c = mu_0 = 1):
 *   E^{n+1} = E^n + dt (D x B^{n+1/2}) - dt J^{n+1/2},
 * in place on the bound fields.  J: three device arrays (Jx, Jy, Jz) of the
 * handle's dtype and grid shape, at the staggered sites of Ex, Ey, Ez;
 * caller-owned, read only, and must not overlap the bound E arrays
 * (XFDTD_EINVAL).  dt is rounded once to the dtype.  A hook for
 * particle codes: the discrete continuity D.E^{n+1} - D.E^n = -dt D.J holds
 * exactly (up to rounding).  Asynchronous on the bound stream.
 */
int xfdtd_step_ampere_current(xfdtd_t h, const void *const J[3]);

/* n >= 0 full steps (Faraday then Ampere each); the result is in the bound
 * fields when the queued work completes.  With scratch arrays bound, FP32
 * handles advance two steps per pass over the fields by default (see
 * xfdtd_set_steps_per_pass).  Runs of 32 steps or more replay a HIP graph of
 * 32 steps captured on the first such call (again when the bound arrays,
 * stream or launch configuration change); XFDTD_GRAPH=0 at xfdtd_create
 * launches every step directly.  Both orders of launches give bitwise the
 * same result. */
int xfdtd_run(xfdtd_t h, int64_t n);

/*
 * Steps per pass of xfdtd_run (with scratch arrays bound):
 *   1: one fused step per launch (reads and writes the state once per step:
 *      48 B per cell-update in FP32, 96 B in FP64);
 *   2: two chained steps per launch (the leapfrog of App. A eq. update1-6
 *      applied twice in one z-march: the state is read and written once per
 *      two steps, 24 B per cell-update in FP32, 48 B in FP64).  The second
 *      step's inputs are formed on chip, redundantly on a 4-cell halo of each
 *      tile (32 x 8 or 32 x 16 output tiles in FP32, 24 x 8 in FP64); every
 *      cell's arithmetic is the one-step kernel's, so the results are
 *      bitwise the same as with 1.
 * Default 2 for FP32 grids of at least 2^23 cells, else 1 (override with
 * XFDTD_STEPS_PER_PASS=1 or 2 at xfdtd_create); xfdtd_tune chooses between
 * them per grid.  XFDTD_EINVAL for other values.  Host only.
 */
int xfdtd_set_steps_per_pass(xfdtd_t h, int steps);

/* Launch configuration of the two-step kernel for this handle, and the steps
 * per pass xfdtd_run uses (1 or 2): tile width and height of its output tiles
 * (32 x 8 or 32 x 16 in FP32, 24 x 8 in FP64), z-planes per workgroup,
 * workgroups per launch.  Any pointer may be NULL.  Until xfdtd_tune is
 * called the tile height and z-planes come from the grid, overridable with
 * XFDTD_BLK_TILE_Y (FP32: 8 or 16) and XFDTD_BLK_ZCHUNK read at
 * xfdtd_create.  Host only. */
int xfdtd_launch_config2(xfdtd_t h, int *steps_per_pass, int *tile_x, int *tile_y, int *zchunk,
                         int *workgroups);

/*
 * Folded weights actually used, as doubles exactly equal to the dtype values.
 * w[0..14]: per axis a (x, y, z), five values
 *   { dt*(alpha_a+delta_a)/d_a, dt*delta_a/d_a, dt*beta_a,t1/d_a, dt*beta_a,t2/d_a,
 *     dt/d_a }
 * (t1, t2 the transverse axes in coefficient order).  The extended difference
 * is applied in the equivalent form
 *   D*_a X = [(alpha+delta) g(p) + delta (g(p+e_a) + g(p-e_a))
 *             + sum_t beta_at (g(p+e_t) + g(p-e_t))] / d_a,
 *   g(q) = X[q+e_a] - X[q],
 * which is an exact rewrite of the Sec. 2 definition (the delta pair
 * X[p+2e_a] - X[p-e_a] is the sum of three consecutive g).  nw receives 15.
 */
int xfdtd_get_weights(xfdtd_t h, double w[15], int *nw);

/* Launch configuration of the fused step for this handle: tile width (64 or
 * 32 columns), tile height (rows of the (x, y) tile), z-planes per workgroup,
 * and workgroups per launch.  Any pointer may be NULL.  Until xfdtd_tune is
 * called the choice depends on grid and dtype only: 32-column tiles for
 * boxes at most 96 wide that they cover with fewer loaded columns (e.g.
 * nx = 96), overridable with the XFDTD_TILE_X / XFDTD_TILE_Y / XFDTD_ZCHUNK
 * environment variables read at xfdtd_create.  Results are bitwise the same
 * for every configuration. */
int xfdtd_launch_config(xfdtd_t h, int *tile_x, int *tile_y, int *zchunk, int *workgroups);

/* Autotunes the launch configuration of xfdtd_run for this handle: times
 * the fused step's tile widths 64 and 32, tile heights 8 and 16 (FP32; 4 and
 * 8 for FP64) and the two-step kernel's tiles (32 x 8 and 32 x 16 in FP32,
 * 24 x 8 in FP64),
 * each with a few z-chunk lengths, with launches that alternate between the
 * scratch arrays and a temporary copy of the state (allocated for the call
 * and freed before it returns; the memory pattern of xfdtd_run, whose every
 * launch reads what the previous one wrote), or that read the bound fields
 * and write the scratch arrays when that copy cannot be allocated (the state
 * is unchanged either way); keeps the
 * fastest per step (setting the steps per pass) and caches it per (grid size,
 * dtype, device); force = 1 re-times, otherwise a cached choice is taken.
 * best_ms (nullable) receives the best time per step (-1 when taken from the
 * cache).  With XFDTD_TUNE_CACHE=<file> in the environment the choice also
 * persists across processes: a grid not tuned in this process is looked up
 * in the file (lines "<gpu arch>/<CUs> single:<f32|f64>:<nx>x<ny>x<nz>
 * <steps per pass> <tile_x> <tile_y> <z-chunk>", the last one for a key
 * wins, lines this handle cannot launch are ignored) and every timed choice
 * is appended; xfdtd_batch_tune does the same with "batch:<shapes>" keys
 * (and "batchadj:<shapes>" for the batched adjoint's tiling).
 * File errors never fail a tuning.  Requires bound fields and scratch arrays
 * (XFDTD_ESTATE otherwise); synchronises the stream.  Results are bitwise the
 * same for every configuration. */
int xfdtd_tune(xfdtd_t h, int force, double *best_ms);

/*
 * Dispersion of the scheme at n wave vectors (Sec. 3 and Sec. 5), on the GPU.
 *   k     : device, n x 3 doubles (k_x, k_y, k_z) in radians per length unit.
 *   omega : device, n doubles: principal branch of sin(omega dt/2)/dt = sqrt(F(k)).
 *   vph   : device, n doubles or NULL: omega/|k| (NaN at k = 0).
 *   vg    : device, n x 3 doubles or NULL: d omega / d k.
 *   stream: hipStream_t for the work.
 * Entries with dt^2 F outside [0, 1] get NaN and the call returns
 * XFDTD_EUNSTABLE (after synchronising the stream).  Arithmetic in double.
 */
int xfdtd_dispersion(const xfdtd_grid *g, double dt, const double coeffs[12],
                     const double *k, int64_t n, double *omega, double *vph, double *vg,
                     void *stream);

/*
 * Dispersion norm f_w of Sec. 4 (eq. norm), c = 1:
 *   f_w = prod_a d_a  integral over [0, pi/d_a]^dims of w(k) (omega(k) - |k|)^2,
 * by the midpoint rule with n points per axis, on the GPU (FP64).
 *   dims  : 3, or 2 for the k_z = 0 plane (the paper's 2D tables; the
 *           product then runs over d_x d_y).
 *   weight: XFDTD_WEIGHT_UNIT (w = 1) or XFDTD_WEIGHT_AXIS,
 *           w = exp(-sum_{t = y, z} (k_t d_t / width)^2) (Sec. 5.2,
 *           eq. norm_x_axis with width 0.1: propagation close to the x axis).
 *   f     : host, the norm.  grad: host, 13 doubles or NULL: d f_w / d coeffs
 *           (12, coefficient order) then d f_w / d dt, from the closed-form
 *           derivative of omega.
 * Only the spacings of g are used.  If any sample has dt^2 F outside (0, 1)
 * (omega undefined or on the stability boundary) f is NaN and the call
 * returns XFDTD_EUNSTABLE.  Synchronises `stream`; allocates two small device
 * buffers per call.
 */
enum { XFDTD_WEIGHT_UNIT = 0, XFDTD_WEIGHT_AXIS = 1 };
int xfdtd_dispersion_norm(const xfdtd_grid *g, double dt, const double coeffs[12], int dims, int64_t n,
                          int weight, double width, double *f, double grad[13], void *stream);

/*
 * Minimisation of f_w over a family of stencils (Sec. 4: bounded, from a grid
 * of starting points, under the stability constraints of eq. constraints,
 * 0 <= F and dt^2 F <= 1 over the zone, dims-dimensional).
 * The stencil is affine in the free parameters x[0..nparam):
 *   q = base + map x  (q: the 12 coefficients, then dt; map row-major 13 x 8),
 * then, if alpha_rule != 0, alpha_a = 1 - 2 beta_at1 - 2 beta_at2 - 3 delta_a
 * (eq. alpha).  dt_mode 0 takes dt = q[12]; dt_mode 1 takes
 * dt = x[dt_param] * (stability bound of the stencil), x[dt_param] in (0, 1].
 * The box lo <= x <= hi is the search space; the search starts from the
 * centres of a grid of starts^nparam cells of the box and runs a projected
 * quasi-Newton iteration (at most max_iter steps each) that rejects unstable
 * stencils.  Outputs (host): x_out[nparam], the 12 coefficients, dt, f_w and
 * (if non-NULL) the number of norm evaluations.  Returns XFDTD_EUNSTABLE if
 * no starting point is stable.  Synchronises `stream`.
 */
typedef struct {
    int32_t nparam;      /* 1..8 */
    int32_t alpha_rule;  /* nonzero: alpha from eq. alpha after the map */
    int32_t dt_mode;     /* 0 or 1, see above */
    int32_t dt_param;    /* dt_mode 1: the parameter that scales the bound */
    double base[13];
    double map[13 * 8];
    double lo[8], hi[8];
    int32_t dims;        /* norm: 2 or 3 */
    int32_t weight;      /* norm: XFDTD_WEIGHT_* */
    double width;        /* norm: XFDTD_WEIGHT_AXIS width */
    int64_t n;           /* norm: midpoints per axis */
    int32_t starts;      /* starting points per parameter, 1..64, starts^nparam <= 4096 */
    int32_t max_iter;    /* per start, 1..1e5 */
} xfdtd_stencil_problem;
int xfdtd_optimize_stencil(const xfdtd_grid *g, const xfdtd_stencil_problem *p, double x_out[8],
                           double coeffs_out[12], double *dt_out, double *f_out, int *evals_out,
                           void *stream);

/*
 * Divergence diagnostics of the bound fields (eq. divstarb, eq. divE).
 *   div_star_b : device, nz*ny*nx of the handle dtype, or NULL: D*.B at the
 *                cell centres, element (i,j,k) at (i+1/2, j+1/2, k+1/2).
 *   div_e      : device, same size, or NULL: D.E at the nodes (i, j, k).
 * Queued on the handle's stream.
 */
int xfdtd_divergence(xfdtd_t h, void *div_star_b, void *div_e);

/*
 * max |D*.B - ref_b| and max |D.E - ref_e| over the grid, reduced on the GPU
 * (ref arrays as written by xfdtd_divergence, or NULL for zero).
 * Also checks the six fields for non-finite values.  Synchronises the stream.
 * out[0] = max |D*.B - ref_b|, out[1] = max |D.E - ref_e|,
 * out[2] = number of non-finite field values.  Returns XFDTD_ENONFINITE when
 * out[2] > 0 (out is still filled).
 */
int xfdtd_divergence_max(xfdtd_t h, const void *ref_b, const void *ref_e, double out[3]);

/*
 * Failure detection: xfdtd_run in blocks of `every` steps, each followed by
 * the non-finite check of xfdtd_divergence_max (one read of the six fields
 * and a stream synchronisation per block).  Stops after the first block
 * that leaves a non-finite value and returns XFDTD_ENONFINITE; *done
 * (nullable) receives the steps completed either way.  n >= 0 and
 * every >= 1, else XFDTD_EINVAL; other errors as xfdtd_run.
 */
int xfdtd_run_checked(xfdtd_t h, int64_t n, int64_t every, int64_t *done);

/*
 * Reverse-mode differentiation (adjoint of the step; not in the paper: the
 * transposes of its update equations).  The forward step is
 *   B' = B + K E   (Faraday increment, extended difference D*),
 *   E' = E + L B'  (Ampere increment, Yee difference),
 * so its adjoint maps (lE', lB') to
 *   mu = lB' + L^T lE',  lE = lE' + K^T mu,  lB = mu,
 * and adds <mu, (dK/dcoeff) E> to the gradient of each of the 12 coefficients
 * (all 12 treated as independent inputs, alpha included).
 *
 * One reverse step on the handle's stream:
 *   lam_in[6]  : device, dL/d(E^{n+1}, B^{n+1/2}) (Ex..Bz), read only.
 *   lam_out[6] : device, receives dL/d(E^n, B^{n-1/2}); each array must be
 *                disjoint from every lam_in, e_n and other lam_out array
 *                (checked on the host: XFDTD_EINVAL).
 *   e_n[3]     : device, the step's primal input E^n.
 *   grad       : device, 12 doubles; this step's coefficient gradient is added.
 * Arrays have the handle's grid and dtype.  Requires xfdtd_bind (for the
 * stream; the bound fields are not touched).  The adjoint's tiling (64 or 32
 * columns, 4 or 8 rows, z-chunk) is chosen at xfdtd_create like the fused
 * step's and can be overridden with XFDTD_ADJ_TILE_X / XFDTD_ADJ_TILE_Y /
 * XFDTD_ADJ_ZCHUNK; lam_out is bitwise the same for every tiling, the
 * gradient up to the summation order of its FP64 partial sums.  A box one
 * plane deep (nz = 1) takes a one-pass kernel instead of the z-march (same
 * lam_out bitwise), whose workgroups each cover up to 16 tiles and sum
 * their gradient terms once (the partial-sum slots stay one per tile: each
 * launch writes every slot, the others of a workgroup as zero).
 */
int xfdtd_adjoint_step(xfdtd_t h, void *const lam_in[6], void *const lam_out[6],
                       const void *const e_n[3], double *grad);

/*
 * The adjoint step of xfdtd_adjoint_step for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid hipMalloc.  Same arguments, operation and
 * results (bitwise) as xfdtd_adjoint_step; the per-workgroup FP64 gradient
 * sums of the launch go to a static device array of the library (16384
 * workgroups x 12 doubles = 1.5 MiB, one copy per GPU, held until the process
 * ends) instead of a buffer the handle allocates on first use.  Each call
 * overwrites the slots it uses, so nothing needs clearing between calls, but
 * calls that overlap on one GPU (other streams, other threads, other
 * handles) share that array and race: serialise them.  XFDTD_EINVAL when the
 * handle's adjoint launch has more than 16384 workgroups or the current
 * device is not the handle's.  Calls no hipMalloc or hipFree; the first call
 * on a device looks up the array's device address.
 */
int xfdtd_adjoint_step_noalloc(xfdtd_t h, void *const lam_in[6], void *const lam_out[6],
                               const void *const e_n[3], double *grad);

/*
 * Checkpointed gradient of n steps.  The forward pass stores the state every
 * `seg` steps (seg <= 0 selects ceil(sqrt(2 n))) and the E fields of the last
 * two segments; the backward pass recomputes every earlier segment from its
 * checkpoint, keeping the E of each of its steps, and runs the adjoint steps
 * in reverse.  It recomputes segment m - 1 on a second (internal) stream
 * while it reverses segment m, so it holds two sets of E snapshots.
 * Memory: ceil(n/seg) + 2 states plus 2 (seg - 1) E fields (seg - 1 when
 * seg >= n: one segment, nothing to recompute).
 *
 * xfdtd_grad_workspace: bytes of device workspace for (n, seg).
 * xfdtd_grad_forward:   n steps from the bound fields; the final state is in
 *                       the bound fields, checkpoints in ws (caller-owned,
 *                       ws_bytes >= the workspace size, 256-byte aligned,
 *                       disjoint from the bound fields).
 * xfdtd_grad_backward:  lam[6] (device, handle dtype) holds dL/d(final state)
 *                       on entry and dL/d(initial state) on return; grad
 *                       (host, 12 doubles) receives dL/dcoeffs.  ws must be
 *                       the workspace filled by xfdtd_grad_forward on this
 *                       handle with the same n and seg; the six lam arrays are
 *                       disjoint from each other and from ws.  It overwrites
 *                       the E snapshots in ws, so it consumes that forward
 *                       pass: another backward needs another forward.  The
 *                       handle remembers which workspaces hold an unconsumed
 *                       forward pass (its last 64) and rejects any other ws,
 *                       n or seg with XFDTD_EINVAL.  Synchronises the stream.
 * Argument errors are XFDTD_EINVAL, found on the host before any device work.
 */
int xfdtd_grad_workspace(xfdtd_t h, int64_t n, int64_t seg, uint64_t *bytes);
int xfdtd_grad_forward(xfdtd_t h, int64_t n, int64_t seg, void *ws, uint64_t ws_bytes);
int xfdtd_grad_backward(xfdtd_t h, int64_t n, int64_t seg, void *ws, uint64_t ws_bytes,
                        void *const lam[6], double grad[12]);

/*
 * Instrumentation (not part of the method): what a handle has run, an
 * algorithmic-bytes model and optional device timing.
 *
 * xfdtd_stats fields (counted since xfdtd_create or the last reset):
 *   run_calls, steps    xfdtd_run calls and the steps they advanced;
 *   in_place_steps      of those, unfused in-place steps (a Faraday and an
 *                       Ampere launch each);
 *   fused_launches      one-step out-of-place launches;
 *   two_step_launches   two-step launches (two steps each), so that
 *                       steps = in_place_steps + fused_launches
 *                               + 2 two_step_launches;
 *   graph_replays, graph_captures   of xfdtd_run's 32-step graph;
 *   tunes               xfdtd_tune calls that timed candidates;
 *   grad_forward_steps  steps of xfdtd_grad_forward;
 *   adjoint_steps       adjoint steps (xfdtd_grad_backward,
 *                       xfdtd_adjoint_step, xfdtd_adjoint_step_noalloc);
 *   recomputed_steps    forward steps recomputed by xfdtd_grad_backward;
 *   model_bytes         algorithmic HBM bytes of all these steps: 12 values
 *                       per cell per forward step (run, checkpointed forward,
 *                       recompute; each component read and written once) and
 *                       15 per adjoint step, at the handle's dtype size;
 *   elapsed_ms          with timing on: device time from the start of the
 *                       first xfdtd_run after the reset to the end of the
 *                       last (gaps between calls included); else -1;
 *   gcells_per_s        with timing on: steps x cells / elapsed, in
 *                       Gcell-updates/s; else -1.
 * xfdtd_get_stats: fills *out (host); synchronises the stream when timing is
 *     on and a run was timed.  xfdtd_reset_stats: zeroes the counters and
 *     sets timing on (1) or off (0); with timing on each xfdtd_run records a
 *     device event before and after its work (not inside a capture of the
 *     caller's stream).  XFDTD_EINVAL for a null argument.
 * XFDTD_LOG=1 in the environment prints configuration and tuning decisions
 * (creation, tuning winners, graph captures, gradient schedules, batch work
 * lists) to stderr; run, tune, gradient passes and each backward segment's
 * recompute and adjoint are marked as roctx ranges (rocprofv3
 * --marker-trace).
 */
typedef struct xfdtd_stats {
    int64_t run_calls, steps, in_place_steps, fused_launches, two_step_launches;
    int64_t graph_replays, graph_captures, tunes;
    int64_t grad_forward_steps, adjoint_steps, recomputed_steps;
    double model_bytes, elapsed_ms, gcells_per_s;
} xfdtd_stats;
int xfdtd_get_stats(xfdtd_t h, xfdtd_stats *out);
int xfdtd_reset_stats(xfdtd_t h, int timing);

/*
 * Batches: m independent periodic boxes of any sizes, each with its own
 * coefficients and time step (each box obeys the conventions above), advanced
 * together.  A step is one launch of a persistent kernel over a work list of
 * (box, tile) items; xfdtd_batch_run captures its n launches once into a HIP
 * graph and replays it.  Not thread-safe per handle.
 *
 * xfdtd_batch_create: grids[m], dts[m], coeffs[m*12]; validated like
 *     xfdtd_create (stability per box unless allow_unstable).
 * xfdtd_batch_bind: fields[m*6] and scratch[m*6] (device, box-major, Ex..Bz
 *     per box, handle dtype, 16-byte aligned, no overlaps); stream as in
 *     xfdtd_bind.  Builds the work list (small internal device buffers).
 * xfdtd_batch_tune: times a candidate set of launch configurations (tile
 *     height 4/8/16 (16: FP32), 32-column tiles as well when a box's nx
 *     leaves a 64-column tile at most half used, z-split 1/2/4 and the
 *     z-split of the step cost model below, persistent grid of 1x/2x the CU
 *     count or one workgroup per work-list slot; for FP32 also the two-step
 *     kernel on 32 x 8 and 32 x 16 tiles with z-split 1, 2 or 0) with
 *     launches that alternate between the scratch arrays and a temporary
 *     copy of the state (allocated for the call; without it, launches that
 *     read the state and write the scratch arrays), keeps the fastest per
 *     step, and caches it per set of box shapes (force = 1
 *     re-times).  It then times the batched adjoint's tilings for the
 *     gradient passes the same way (the state read as lambda and primal E,
 *     the scratch arrays written): the tile width of the column-count rule
 *     below and, where that is 32, 64 as well; the default tile height and,
 *     for FP32 32-column tiles, 12; z-split 1-4 and the model's; each box's
 *     items dispatched as one run or in runs of a few tiles.  best_ms (nullable)
 *     receives the forward's best time per step (-1 when taken from the
 *     cache; the adjoint's choice is then also taken from the cache if it
 *     holds one, else the model below chooses).  Synchronises the stream.
 *     A failure while timing the forward candidates keeps the previous
 *     forward configuration; a failure while timing the adjoint's keeps the
 *     new forward configuration and leaves the adjoint's tiling to the
 *     model; either returns the error.
 * xfdtd_batch_set_config / get_config: choose / report the configuration:
 *     tile_x 64 or 32, tile_y 4, 8 or 16 (16: FP32 only), zsplit 0..1024
 *     (zsplit >= 1: each box is cut into z-chunks of ceil(nz / zsplit) >= 4
 *     planes; 0: each box gets 1 to 4 chunks, chosen on the host by a
 *     list-scheduling model of the work list below), grid >= 0 (0 = one
 *     workgroup per work-list slot); nitems = work-list length in slots (0
 *     before binding): the tiles x z-chunks of every box, dealt to the 8
 *     XCDs in runs of neighbouring tiles with balanced plane counts, each
 *     XCD's share longest first, padded with empty slots where an XCD's
 *     share is short.  XFDTD_EINVAL for any other value.  The untuned
 *     default: tile_x 32 only when every box has nx <= 32, tile_y 8, the
 *     z-split minimising max(total plane iterations / resident workgroups,
 *     longest work item), grid 0, one step per launch.
 * A batch whose boxes are all one plane deep (nz = 1) steps on plane
 *     kernels (64 x 16 tiles in FP32, 64 x 8 in FP64, one step per launch)
 *     whatever the tiling and steps per pass set; get_config and
 *     get_steps_per_pass report those, and the tuner times only the grid.
 *     Its adjoint takes the one-pass kernel, a work item being up to 16
 *     tiles of one box.
 * xfdtd_batch_run: n >= 0 steps of every box through the cached graph (the
 *     graph is re-captured when n or the configuration changes); the result
 *     is in the bound fields when the queued work completes.
 * xfdtd_batch_run_eager: the same launches without a graph.
 */
typedef struct xfdtd_batch_s *xfdtd_batch_t;
int xfdtd_batch_create(const xfdtd_grid *grids, const double *dts, const double *coeffs, int64_t m,
                       int dtype, int allow_unstable, xfdtd_batch_t *out);
void xfdtd_batch_destroy(xfdtd_batch_t b);
int xfdtd_batch_bind(xfdtd_batch_t b, void *const *fields, void *const *scratch, void *stream);
int xfdtd_batch_tune(xfdtd_batch_t b, int force, double *best_ms);
int xfdtd_batch_set_config(xfdtd_batch_t b, int tile_x, int tile_y, int zsplit, int grid);
int xfdtd_batch_get_config(xfdtd_batch_t b, int *tile_x, int *tile_y, int *zsplit, int *grid, int *nitems);
int xfdtd_batch_run(xfdtd_batch_t b, int64_t n);
int xfdtd_batch_run_eager(xfdtd_batch_t b, int64_t n);

/*
 * Steps per launch of a batch's run (as xfdtd_set_steps_per_pass for one
 * box): 1, or 2 for the two-step kernel (the leapfrog of App. A eq.
 * update1-6 applied twice per pass over each box's fields; FP32, tiling
 * 32 x 8 or 32 x 16 set by xfdtd_batch_set_config or the tuner), bitwise the
 * same results.  xfdtd_batch_tune also times two-step candidates and sets
 * this; xfdtd_batch_set_config resets it to 1 for tilings the two-step kernel
 * does not have.  XFDTD_EINVAL otherwise.  Host only.
 */
int xfdtd_batch_set_steps_per_pass(xfdtd_batch_t b, int steps);
int xfdtd_batch_get_steps_per_pass(xfdtd_batch_t b, int *steps);

/*
 * The batched adjoint's launch configuration, chosen by each
 * xfdtd_batch_grad_backward and by xfdtd_batch_tune (all 0 before either):
 * tile_x 32 or 64; tile_y 4, 8, or 12 (FP32 32-column tiles only); zsplit,
 * the z-chunks per box; nslots, its dispatch slots.  The tiling is the one
 * xfdtd_batch_tune timed fastest for the batch's shapes; untuned, the tile
 * width is 32 where the forward runs 32-column tiles or every box is at most
 * 96 wide and 32-column tiles load fewer columns in all (64 otherwise), and
 * the height and z-split those of a
 * list-scheduling model of the work list (tile positions x planes per item).
 * XFDTD_EINVAL for a null handle.  Host only.
 */
int xfdtd_batch_get_adjoint_config(xfdtd_batch_t b, int *tile_x, int *tile_y, int *zsplit, int *nslots);

/*
 * Batched checkpointed gradients: the single-box schedule of
 * xfdtd_grad_forward / xfdtd_grad_backward for every box of the batch at once
 * (same n and seg for all boxes), one batched launch per step.  As there,
 * the backward pass recomputes segment m - 1 of every box on a second
 * (internal) stream while it reverses segment m, and each workspace holds two
 * sets of E snapshots (one when seg >= n).
 *   bytes[m] / ws[m] / ws_bytes[m] : one workspace per box (device,
 *       256-byte aligned, caller-owned), sized by xfdtd_batch_grad_workspace.
 *   lam[m*6] : device, dL/d(final state) of each box in, dL/d(initial state)
 *       out (box-major, Ex..Bz).
 *   grad : host, m*12 doubles, dL/dcoeffs of each box.
 * The forward steps run on the batch's one-step configuration; the adjoint
 * steps on a tiling of their own, chosen per backward pass
 * (xfdtd_batch_get_adjoint_config).  The results do not depend on either
 * tiling: the adjoint fields are bitwise those of single-box runs and the
 * coefficient gradients differ from them only in the order of the FP64
 * workgroup sums.
 * The forward leaves the final states in the bound fields.  Both synchronise
 * the stream and allocate small internal buffers (launch descriptors).  The
 * backward consumes the forward pass like xfdtd_grad_backward: it needs the
 * same ws list, n and seg as an unconsumed forward on this batch, else
 * XFDTD_EINVAL.
 * Workspaces must be disjoint from each other and (forward) from the bound
 * fields and scratch arrays; (backward) the lambda arrays from each other and
 * from the workspaces.  Violations are XFDTD_EINVAL before any device work.
 */
int xfdtd_batch_grad_workspace(xfdtd_batch_t b, int64_t n, int64_t seg, uint64_t *bytes);
int xfdtd_batch_grad_forward(xfdtd_batch_t b, int64_t n, int64_t seg, void *const *ws,
                             const uint64_t *ws_bytes);
int xfdtd_batch_grad_backward(xfdtd_batch_t b, int64_t n, int64_t seg, void *const *ws,
                              const uint64_t *ws_bytes, void *const *lam, double *grad);

#ifdef __cplusplus
}
#endif
#endif /* XFDTD_H */
