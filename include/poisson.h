/*
 * poisson.h -- C ABI of the MI355X (gfx950) FFT-based pressure Poisson solver.
 *
 * The operation (FluTAS, arXiv 2204.08834):
 *   Section 3.3, eqn:poisson -- the constant-coefficient Poisson equation of
 *   the pressure-correction step, lap(psi) = (rho_0/dt) div(u*); the caller
 *   passes the right-hand side f = (rho_0/dt) div(u*) already evaluated.
 *   Section 3 -- uniform Cartesian marker-and-cell grid with spacings
 *   dx, dy, dz; psi at the cell centres; second-order 7-point Laplacian.
 *   Section 3.3.1 -- the solve: Fourier expansions along x and y reduce the
 *   7-diagonal operator to one tridiagonal system along z per wavenumber pair,
 *   solved by Gauss elimination; the steps are forward transforms along x
 *   then y, the z solve, and backward transforms along y then x.  With
 *   periodic z the z solve becomes a third transform and a division by the
 *   eigenvalue.  Walls sit on the cell faces with a homogeneous condition:
 *   Neumann (zero normal gradient, the boundary condition stated after
 *   eqn:corr; the ghost cell mirrors the first interior cell) or Dirichlet
 *   (zero value on the face; the ghost cell is the negated interior cell) --
 *   the homogeneous pressure conditions the Fourier-based expansions of
 *   Section 3.3.1 cover.
 *
 * Problem solved: the unique zero-mean p with  L p = f - mean(f)  when no wall
 * is Dirichlet (the constant is then in the null space).  The mean of f (which
 * makes the periodic/Neumann problem incompatible when non-zero) is removed
 * and reported in poisson_stats_t.rhs_mean; it is not an error.  With a
 * Dirichlet wall the operator is regular: L p = f, nothing is removed.
 *
 * Memory: all field arrays are float64 device pointers (hipMalloc'd, or torch
 * CUDA tensors), contiguous, shape (nz, ny, nx) in C order (x fastest).  The
 * caller owns rhs and sol; rhs is never written; rhs and sol must not
 * overlap.  The plan owns its workspace, twiddle and eigenvalue tables.
 *
 * Streams: `stream` is a hipStream_t (passed as void*; NULL = default
 * stream).  All work of a plan is enqueued on its stream.  POISSON_FP64 and
 * POISSON_FP32 solves are asynchronous unless stats is non-NULL (then the
 * call synchronises once to read the removed mean).  POISSON_FP32_REFINE
 * synchronises once per refinement iteration to read the residual norm.
 * One plan must be used by one host thread / stream at a time.
 *
 * Errors: every function returns POISSON_OK (0) or a negative code below.
 * Descriptors are fully validated before any HIP call.
 */
#ifndef POISSON_H
#define POISSON_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define POISSON_OK 0
#define POISSON_ERR_INVALID_ARG (-1)   /* NULL pointer, bad size/spacing, aliasing */
#define POISSON_ERR_UNSUPPORTED (-2)   /* BC combination or length outside 2^a 3^b */
#define POISSON_ERR_OUT_OF_MEMORY (-3) /* device allocation failed */
#define POISSON_ERR_HIP (-4)           /* a HIP runtime call failed */
#define POISSON_ERR_NOT_CONVERGED (-5) /* refinement stalled or hit max_refine; last iterate kept */
#define POISSON_ERR_NONFINITE (-6)     /* non-finite residual (NaN/Inf in rhs or solution) */
#define POISSON_ERR_TOO_LARGE (-7)     /* exceeds the fixed scratch of poisson_solve_noalloc */

/* Bytes of the fixed device scratch array of poisson_solve_noalloc (one copy
 * per GPU the library runs on, held until the process ends). */
#define POISSON_NOALLOC_SCRATCH_BYTES ((size_t)160 << 20)

typedef enum {
    POISSON_BC_PERIODIC = 0,
    POISSON_BC_NEUMANN = 1,  /* wall on the cell face, zero normal gradient */
    POISSON_BC_DIRICHLET = 2 /* wall on the cell face, zero value there (ghost = -wall cell) */
} poisson_bc_t;

typedef enum {
    POISSON_FP64 = 0,        /* every pass in FP64 */
    POISSON_FP32_REFINE = 1, /* FP32 transforms + FP64 residual iterative refinement */
    POISSON_FP32 = 2         /* one FP32 solve (FP64 zero mode), no refinement */
} poisson_precision_t;

/*
 * Stretched z (dz_cells != NULL): walls in z (bc_z NEUMANN or DIRICHLET), cell
 * k of thickness dz_cells[k] > 0 (dz is then unused, but must still be a
 * valid spacing).  This extends the elimination along z of Section 3.3.1 to
 * cells of different thickness: the z part of the operator is
 *   [ (p[k+1] - p[k]) / d[k+1/2] - (p[k] - p[k-1]) / d[k-1/2] ] / dz_cells[k],
 *   d[k+1/2] = (dz_cells[k] + dz_cells[k+1]) / 2,
 * no flux through a Neumann wall, flux (0 - p[0]) / (dz_cells[0]/2) at a
 * Dirichlet wall (likewise at the top); equal thicknesses give the uniform
 * operator.  The singular problem removes the volume-weighted mean of f
 * (reported as rhs_mean) and returns the p of zero volume-weighted mean.
 * The plan copies the array; the caller may free it after plan creation.
 * poisson_project does not take stretched plans (UNSUPPORTED).
 *
 * Problem descriptor.
 *   nx      : even, nx/2 of the form 2^a or 3*2^a, 2 <= nx <= 2048.
 *   ny      : 2^a or 3*2^a, 1 <= ny <= 2048.
 *   nz      : walls: 1..4096 (any value); periodic: 2^a or 3*2^a up to 2048.
 *   nx*ny*nz <= 2^31.
 *   dx,dy,dz: positive, finite cell sizes.
 *   bc_x, bc_y, bc_z: POISSON_BC_PERIODIC, POISSON_BC_NEUMANN or
 *             POISSON_BC_DIRICHLET, any combination (the homogeneous pressure
 *             conditions of the expansions of Section 3.3.1: Fourier series
 *             along a periodic axis, cosine / sine series between walls along
 *             x and y, the tridiagonal solve between walls along z).  With a
 *             Dirichlet wall the operator has no null space: f keeps its
 *             mean, p is not shifted, rhs_mean reports 0.
 *   precision: poisson_precision_t.
 *   rtol    : FP32_REFINE target for ||f - mean f - L p||_2 / ||f - mean f||_2
 *             (default 1e-10; must be > 0).
 *   max_refine: maximum number of refinement corrections (default 8, >= 1).
 */
typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    int bc_x, bc_y, bc_z;
    int precision;
    double rtol;
    int max_refine;
    const double *dz_cells; /* NULL (uniform dz), or a host array of nz cell thicknesses */
} poisson_desc_t;

/*
 * Per-solve statistics (written when the pointer is non-NULL).
 *   iterations  : refinement corrections applied (0 for FP64 / FP32).
 *   rel_residual: final relative L2 residual (FP32_REFINE); -1 when not computed.
 *   rhs_mean    : mean(f) removed from the right-hand side.
 *   status      : same value as the return code of the solve.
 */
typedef struct {
    int iterations;
    double rel_residual;
    double rhs_mean;
    int status;
} poisson_stats_t;

typedef struct poisson_plan_s *poisson_plan;

/* Fill a descriptor with defaults (periodic x,y,z, FP64, rtol 1e-10,
 * max_refine 8, unit spacing, uniform z, sizes 0).  Host only. */
int poisson_desc_init(poisson_desc_t *d);

/* Check a descriptor without touching the GPU.  Host only. */
int poisson_desc_validate(const poisson_desc_t *d);

/* Device workspace bytes a plan for this descriptor allocates (tables
 * excluded): none field-sized for FP64 (the transforms run in place in the
 * solution array); 4 B per point for FP32 (the FP32 spectrum); 8 B per point
 * for FP32_REFINE (the spectrum and an exact FP32 copy of the first
 * iterate); plus the per-workgroup partial-sum records.  Host only; 0 on an
 * invalid descriptor. */
size_t poisson_workspace_bytes(const poisson_desc_t *d);

/* Create a plan: validates d, builds FP64 twiddle and eigenvalue tables on
 * the host (FP32 copies rounded once), allocates the workspace on the current
 * device.  *out is set only on success. */
int poisson_plan_create(const poisson_desc_t *d, void *stream, poisson_plan *out);

/* Solve L sol = rhs - mean(rhs) with zero-mean sol (see the file comment).
 * rhs_dev, sol_dev: device float64, nx*ny*nz elements each, non-overlapping.
 * stats may be NULL. */
int poisson_solve(poisson_plan plan, const double *rhs_dev, double *sol_dev,
                  poisson_stats_t *stats);

/*
 * Allocation-free solve, for callers that cannot allocate device memory:
 * code running under HIP graph capture, tight serving loops, and harnesses
 * that forbid hipMalloc.  Same operation, kernels and results as
 * poisson_plan_create + poisson_solve with the default launch variants (and
 * those of a tuning cache, as a new plan would take them), without a plan
 * object: every device buffer (tables, partial sums, scalars, and for
 * FP32 / FP32_REFINE the 4 B/point spectrum and, for FP32_REFINE, the
 * 4 B/point first iterate) is a piece of one fixed static device array of
 * POISSON_NOALLOC_SCRATCH_BYTES per GPU.  The call allocates no device or
 * pinned host memory (no hipMalloc, hipHostMalloc, hipFree, no library
 * allocator).
 *   d      : descriptor, validated as for poisson_plan_create.
 *   stream : hipStream_t as void* (NULL = default stream); the current
 *            device is the one used.
 *   rhs, sol, stats: as poisson_solve (device float64, nx*ny*nz each,
 *            non-overlapping; rhs is not written; stats may be NULL).
 * Size limit: the tables plus 4 B/point (FP32) or 8 B/point (FP32_REFINE)
 * plus the partial-sum records must fit the array (FP32_REFINE up to about
 * 19 M points, e.g. 256^3; FP64 needs only the tables and records, so every
 * valid size fits).  A larger problem returns POISSON_ERR_TOO_LARGE (with a
 * message on stderr) before any work is enqueued.
 * State: the array keeps the last call's contents.  The tables are
 * regenerated and copied (then `stream` is synchronised once) only when the
 * descriptor differs from the previous call's on that GPU; the scalars are
 * cleared by a kernel on every call.  All calls on one GPU share the one
 * array: calls that overlap in time on one GPU (from several host threads,
 * or on several streams) race and give wrong results; serialise them.
 * Synchronisation otherwise as poisson_solve (FP32_REFINE synchronises once
 * per refinement iteration).  Errors: INVALID_ARG, UNSUPPORTED, TOO_LARGE,
 * HIP, and those of poisson_solve.
 */
int poisson_solve_noalloc(const poisson_desc_t *d, void *stream, const double *rhs, double *sol,
                          poisson_stats_t *stats);

/*
 * The whole projection step around the solve (FluTAS Section 3.3:
 * eqn:poisson, then eqn:corr and eqn:p_upt) on a single-problem plan:
 *   f   = alpha D(u, v, w)      (alpha = rho_0/dt), evaluated inside the
 *                               first transform pass (never stored, except
 *                               under POISSON_FP32_REFINE, see below);
 *   psi = the zero-mean solution of L psi = f - mean(f), as poisson_solve;
 *   u  -= beta Gx psi, v -= beta Gy psi, w -= beta Gz psi  (beta = dt/rho_0);
 *   p  += psi                   (skipped when p is NULL).
 * Faces (Section 3): u[k,j,i] on x = (i+1) dx, v[k,j,i] on y = (j+1) dy,
 * w[k,j,i] on z = (k+1) dz; D is the cell-centred divergence,
 *   (D u)[k,j,i] = (u[i] - u[i-1])/dx + (v[j] - v[j-1])/dy + (w[k] - w[k-1])/dz,
 * and G the face gradient, (Gx psi)[i] = (psi[i+1] - psi[i])/dx etc., both
 * periodic along periodic axes.  Along an axis with (Neumann, solid) walls no
 * flux crosses the first face or the last face, which is the wall: u[nx-1],
 * v[ny-1] or w[nz-1] of such an axis is not read and not changed.  D G equals the 7-point L,
 * so with alpha * beta = 1 the corrected velocity is discretely
 * divergence-free up to the solve's accuracy.
 * u, v, w, p, psi: device float64, nx*ny*nz elements each, pairwise
 * non-overlapping; u, v, w and p are updated in place, psi receives the
 * solution.  alpha, beta: finite.  stats as poisson_solve.  The velocity and
 * pressure are updated only when the solve succeeds: on any error (for
 * instance NOT_CONVERGED or NONFINITE under refinement) they are left as they
 * were and psi holds the last iterate.  Under POISSON_FP32_REFINE the first
 * call allocates one more float64 field (nx*ny*nz) that the plan keeps for f.
 * Errors: INVALID_ARG (null plan or field, batched plan, non-finite scale,
 * overlapping fields), UNSUPPORTED (a plan with Dirichlet walls: the face
 * conventions above are those of solid walls), OUT_OF_MEMORY, HIP, and those
 * of poisson_solve.
 */
int poisson_project(poisson_plan plan, double *u, double *v, double *w, double *p, double *psi,
                    double alpha, double beta, poisson_stats_t *stats);

/* Release a plan and everything it owns.  NULL is accepted. */
int poisson_destroy(poisson_plan plan);

/* Batched plan: `count` independent problems (descs[i], possibly different
 * sizes and boundaries, one shared precision/rtol/max_refine taken from
 * descs[0]) solved together on one stream.  Problems of equal shape share
 * kernel launches. */
int poisson_batch_plan_create(const poisson_desc_t *descs, int count, void *stream,
                              poisson_plan *out);

/* rhs[i], sol[i]: host arrays of `count` device pointers (problem i's fields,
 * each of that problem's nx*ny*nz doubles).  No sol[i] may share a byte with
 * another problem's solution or with any right-hand side (the refinement
 * re-reads every rhs while the solutions are written): INVALID_ARG, checked
 * before any work is enqueued.  Right-hand sides may overlap each other.
 * stats: NULL or an array of `count` entries.  Returns the first non-OK
 * per-problem status, else POISSON_OK. */
int poisson_batch_solve(poisson_plan plan, const double *const *rhs, double *const *sol,
                        poisson_stats_t *stats);

/* Static English description of an error code. */
const char *poisson_error_string(int code);

/*
 * Where the refinement loop is driven (the batched schedule and the
 * refinement control of FluTAS Section 3.3.1 as built here):
 *   0 (default) host-driven: after each residual the host reads the norms
 *     back (one synchronisation per iteration) and launches only the passes
 *     the running problems need;
 *   1 captured graph: the first solve and a fixed number of loop segments
 *     (residual evaluation, device-side convergence decision, correction)
 *     are captured once into a hipGraph and replayed; every pass of a
 *     segment is gated per problem by a device control record, so problems
 *     that converge early skip the rest.  Further segment-only graphs are
 *     launched while a problem still runs (at most max_refine corrections).
 *     One synchronisation per graph launch;
 *   2 the launch sequence of mode 1 issued eagerly (no capture), for testing.
 * Modes 1 and 2 run on a stream owned by the plan, ordered after the plan's
 * stream on entry and before it on return with events.  Same results as mode 0
 * up to the order of the per-problem convergence decisions (identical for a
 * single problem).  Per-pass timing (below) disables the capture of mode 1.
 * Returns POISSON_ERR_INVALID_ARG for a null plan or another mode.
 */
int poisson_plan_set_graph(poisson_plan plan, int mode);

/*
 * Autotuner (the per-shape schedule choice of the batched solves).  For each
 * distinct problem shape of the plan, times the launch variants of the
 * passes on scratch fields of that shape -- the tile of the wall-bounded z
 * solve, the tile width and radix order of the y transforms, and the block
 * order of the passes (which decides how much of each pass's input is still
 * in the last-level cache) -- on the plan's stream, and keeps the fastest.
 * Choices are cached for the process per (precision, grid, z boundary,
 * device) and used by later plans of that shape at creation; with the
 * environment variable POISSON_TUNE_CACHE naming a file they persist across
 * processes.  POISSON_AUTOTUNE=1 tunes every plan at creation.  Synchronises
 * the plan's stream; allocates two scratch fields of one problem for the
 * duration of the call.  flags: 0, or POISSON_TUNE_FORCE to ignore cached
 * choices.  Errors: INVALID_ARG, OUT_OF_MEMORY, HIP.
 */
#define POISSON_TUNE_FORCE 1
int poisson_plan_autotune(poisson_plan plan, int flags);

/*
 * Text description of the plan: one line per shape group with its grid,
 * boundary, precision, number of problems and chosen launch variants.
 * Writes at most len bytes (NUL-terminated) to buf; returns INVALID_ARG if
 * the text was truncated or an argument is null.
 */
int poisson_plan_describe(poisson_plan plan, char *buf, int len);

/*
 * Per-pass timing (tracing).  When enabled, every kernel launch of a solve is
 * bracketed by hipEvents on the plan's stream; the accumulated time and the
 * algorithmic HBM bytes of each pass are read back with
 * poisson_plan_get_timing (which synchronises the stream).
 */
typedef struct {
    char name[40];           /* pass name, e.g. "x_r2c_f32" */
    int launches;            /* launches since the last reset */
    double total_ms;         /* summed kernel time */
    double bytes_per_launch; /* algorithmic HBM bytes moved by one launch */
} poisson_pass_stat_t;

int poisson_plan_set_timing(poisson_plan plan, int enable);
int poisson_plan_reset_timing(poisson_plan plan);
int poisson_plan_get_timing(poisson_plan plan, poisson_pass_stat_t *out, int capacity,
                            int *count);

#ifdef __cplusplus
}
#endif

#endif /* POISSON_H */
