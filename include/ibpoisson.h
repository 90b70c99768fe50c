/*
 * libibpoisson -- staggered-grid pressure Poisson solver for AMD Instinct
 * MI355X (gfx950).  C ABI: plain pointers and sizes only.
 *
 * The problem (paper: eq. ``elliptic`` of the fractional-step method, its
 * boundary-condition paragraph after eq. ``pressure``, and the FFT solver of
 * the "Fluid domain" parallelisation subsection): on a grid of nx * ny * nz
 * pressure cells, periodic and uniform in x (length Lx) and z (length Lz) and
 * wall-bounded with arbitrary spacing in y, find phi with
 *
 *     L_h phi = rhs - m,      sum_cells V phi = 0,
 *
 * where L_h = D G is the second-order staggered 7-point Laplacian with
 * homogeneous Neumann conditions at the two y walls, V = dx dz dyf_j is the
 * cell volume and m = sum V rhs / sum V is the volume-weighted mean of rhs
 * (zero for a right-hand side that is the divergence of a velocity field
 * with zero wall-normal velocity at the walls; otherwise it is removed and
 * reported).  The caller applies the 1/(alpha dt) scale and any mass source
 * q of eq. ``elliptic``: the library solves exactly what it is given.
 *
 * Method: real FFT along x, complex FFT along z, one tridiagonal system per
 * horizontal wavenumber pair along y (the (0,0) mode by FP64 flux
 * integration), inverse FFTs.
 *
 * Layout: every field is C-ordered [ny][nz][nx] (x fastest, y slowest), FP64,
 * device memory, 16-byte aligned.  x and z cell centres are at (i + 1/2) dx
 * and (k + 1/2) dz; y pressure points are the midpoints of the ny + 1 face
 * coordinates passed to ibp_plan_create.
 *
 * Execution: argument checks are synchronous and happen before anything is
 * enqueued.  Solves are asynchronous on the given stream (NULL = the
 * device's default stream); they never synchronise, allocate or
 * copy to the host, so a solve sequence can be captured in a hipGraph.  A
 * plan owns one workspace: solves with one plan must not overlap on two
 * streams.  Nothing aborts, exits or throws across this interface.
 */
#ifndef IBPOISSON_H
#define IBPOISSON_H

#include <stddef.h>

#include <hip/hip_runtime_api.h>   /* hipStream_t */

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibp_plan_s* ibp_plan_t;

typedef enum {
  IBP_SUCCESS = 0,
  IBP_ERROR_INVALID_VALUE = 1,    /* null pointer, bad geometry, misaligned or aliased buffers */
  IBP_ERROR_UNSUPPORTED_SIZE = 2, /* grid size outside what the kernels support (see ibp_check_dims) */
  IBP_ERROR_OUT_OF_MEMORY = 3,    /* device allocation failed, or caller workspace too small */
  IBP_ERROR_HIP = 4,              /* a HIP runtime call failed (no device, launch failure, ...) */
  IBP_ERROR_INTERNAL = 5          /* unexpected internal failure (C++ exception caught) */
} ibp_status_t;

typedef enum {
  IBP_FP64 = 0,            /* FP64 transforms and line solves: the direct solve */
  IBP_MIXED = 1,           /* FP32 transforms and FP32 line solves, FP64 (0,0) mode, FP64
                              residual and update, iterative refinement to rtol */
  IBP_MIXED_F64SWEEP = 2,  /* as IBP_MIXED, but the line-solve arithmetic is FP64 on the
                              FP32 spectral data (storage and transforms stay FP32) */
  IBP_MIXED_F64INV = 3     /* FP32 forward transforms (FP32 half spectrum); the line solve
                              reads it and solves in FP64 into an FP64 half spectrum, and
                              the inverse transforms run in FP64.  Rounding at or after the
                              line solve is what the wall rows of the stencil amplify most;
                              without it one correction reaches 1e-10 where IBP_MIXED needs
                              two (single plans only: ibp_solve_batched solves such plans
                              one after another) */
} ibp_precision_t;

#define IBP_HISTORY_MAX 16

typedef struct {
  int iterations;       /* refinement corrections applied after the initial solve (0 for FP64) */
  int converged;        /* FP64: 1.  Mixed: 1 = rel_residual <= rtol reached; 2 = stopped before
                           rtol because the iterate reached the FP64 floor (backward_error <=
                           8 unit roundoffs: no further correction can lower the residual, as on
                           strongly stretched grids whose FP64 residual floor lies above rtol);
                           0 = max_iters corrections did neither */
  int nonfinite_input;  /* a NaN/Inf (or FP64 overflow) was met in rhs or in a residual */
  int reserved;
  double rel_residual;  /* ||rhs - m - L_h phi||_2 / ||rhs - m||_2 in FP64 (NaN for FP64 solves) */
  double removed_mean;  /* m, the removed volume-weighted mean of rhs */
  double rhs_norm;      /* ||rhs - m||_2 (mixed) */
  double residual_norm; /* ||rhs - m - L_h phi||_2 (mixed) */
  /* Mixed forms (NaN for FP64 solves), all of the returned iterate: */
  double rel_residual_vw;  /* volume-weighted ||V r||_2 / ||V (rhs - m)||_2, V the cell volumes */
  double backward_error;   /* ||r||_inf / (||L_h||_inf ||phi||_inf + ||rhs - m||_inf) */
  int history_len;         /* entries of residual_history */
  int reserved2;
  double residual_history[IBP_HISTORY_MAX];   /* rel_residual after k = 0, 1, ... corrections
                                                 (k = 0: the initial FP32 solve) */
} ibp_info_t;

/* Host-only size check (touches no GPU).  Even nx <= 4096 (transformed as
 * nx/2 complex pairs) or odd nx <= 2048 (as nx complex values); nz <= 4096;
 * 2 <= ny <= 1536.  Any prime factors are accepted, but then the x
 * transform length <= 1024 or nz <= 2047 for that direction: lines of at
 * most 1024 points with a prime factor above 11 (e.g. the paper's 632 = 8 x
 * 79 and 501 = 3 x 167 points) take a chirp convolution held in registers,
 * longer ones a slower direct-sum or convolution stage in LDS; the mixed
 * forms' residual passes take the LDS stages.  Returns IBP_SUCCESS or
 * IBP_ERROR_UNSUPPORTED_SIZE (IBP_ERROR_INVALID_VALUE for nx, nz < 1). */
ibp_status_t ibp_check_dims(int nx, int ny, int nz);

/* Create a plan for one grid.  y_nodes: HOST pointer to ny + 1 finite,
 * strictly increasing wall-normal face coordinates (walls at y_nodes[0] and
 * y_nodes[ny]); copied, the caller keeps ownership.  Lx, Lz: finite, > 0.
 * Builds the FP64 y-operator coefficients, the closed-form eigenvalues
 * lambda_x(kx) = -(4/dx^2) sin^2(pi kx/nx), lambda_z(kz) likewise, the FFT
 * twiddles, and allocates the device tables and the default workspace on
 * the current device.  Precision defaults to IBP_FP64.  On failure *plan is
 * set to NULL. */
ibp_status_t ibp_plan_create(ibp_plan_t* plan, int nx, int ny, int nz, double Lx, double Lz,
                             const double* y_nodes);

/* Free the plan's device tables and owned workspace (not a caller workspace).
 * NULL is accepted.  Waits for nothing: the caller must make sure no solve
 * with this plan is still running. */
ibp_status_t ibp_plan_destroy(ibp_plan_t plan);

/* Wall condition of the pressure correction at a y wall.  The paper's
 * default configuration has homogeneous Neumann conditions at both walls
 * (boundary-condition paragraph after eq. ``pressure``): then L_h is
 * singular, the volume-weighted mean of rhs is removed (ibp_info_t.removed_mean)
 * and phi has zero volume-weighted mean.  Its ``neumann_velocity`` outlet
 * option gives the upper wall a homogeneous Dirichlet condition (phi = 0 on
 * the wall face, half a cell from the nearest centre); with a Dirichlet wall
 * the problem is non-singular, nothing is removed and phi is unique. */
typedef enum { IBP_BC_NEUMANN = 0, IBP_BC_DIRICHLET = 1 } ibp_bc_t;

/* Set the conditions at the lower (y = y_nodes[0]) and upper wall; a new
 * plan has Neumann at both.  Rewrites the plan's coefficient tables
 * (synchronous); batches built on the plan must be rebuilt. */
ibp_status_t ibp_plan_set_bc(ibp_plan_t plan, ibp_bc_t lower, ibp_bc_t upper);

/* Select the precision form.  rtol: relative residual target of the mixed
 * forms (> 0, e.g. 1e-10); max_iters: maximum refinement corrections after
 * the initial FP32 solve, 0..64.  Both are ignored for IBP_FP64. */
ibp_status_t ibp_plan_set_precision(ibp_plan_t plan, ibp_precision_t precision, double rtol,
                                    int max_iters);

/* Bytes of device workspace a solve with this plan needs (any precision). */
ibp_status_t ibp_plan_workspace_size(ibp_plan_t plan, size_t* bytes);

/* Hand the plan a caller-owned device workspace of at least
 * ibp_plan_workspace_size bytes, 256-byte aligned (e.g. from PyTorch's
 * allocator); the plan frees its own workspace and uses this one until the
 * plan is destroyed or another workspace is set.  Passing NULL re-allocates
 * an owned workspace.  Too small -> IBP_ERROR_OUT_OF_MEMORY. */
ibp_status_t ibp_plan_set_workspace(ibp_plan_t plan, void* device_ptr, size_t bytes);

/* Solve L_h phi = rhs - m (see top).  rhs, phi: device pointers to
 * nx*ny*nz doubles, [ny][nz][nx], 16-byte aligned.  rhs is read-only.
 * phi may alias rhs (in-place) for IBP_FP64 only; in the mixed forms rhs is
 * read again by every refinement pass, so any overlap returns
 * IBP_ERROR_INVALID_VALUE.  Enqueued on `stream` (NULL: the default stream); call
 * on the device the plan was created on. */
ibp_status_t ibp_solve(ibp_plan_t plan, const double* rhs, double* phi, hipStream_t stream);

/* ibp_solve for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid allocation):
 * the same solve, but its workspace (half spectrum, row and plane sums, norm
 * partials, control block) is a static device array of the library, 32 MiB
 * per GPU, held from the library's first use of that GPU until the process
 * ends, instead of the plan's own workspace.  Calls no hipMalloc, hipFree or
 * other allocating routine (the array's address is looked up once per
 * device).  Plans whose workspace (ibp_plan_workspace_size) exceeds 32 MiB
 * return IBP_ERROR_UNSUPPORTED_SIZE: FP64 grids up to about 2 million
 * half-spectrum coefficients, e.g. 128 x 128 x 128.  Every such call on one
 * GPU uses the same array and leaves its contents there: calls that overlap
 * on one GPU (two streams or threads) race, and ibp_get_info after this call
 * reports the state the array holds, valid until the next such call on the
 * GPU.  Always the separate-pass schedule, without per-pass profiling
 * events.  Arguments, layout and errors as ibp_solve. */
ibp_status_t ibp_solve_scratch(ibp_plan_t plan, const double* rhs, double* phi, hipStream_t stream);

/* Solve `count` independent problems, problem i with plans[i], rhs[i],
 * phi[i] (each as in ibp_solve; HOST arrays of plans and device pointers).
 * The plans must be distinct (each owns its workspace).  All work is
 * enqueued on `stream`.
 *
 * When every plan is on the current device with the same precision
 * (IBP_FP64 or IBP_MIXED) and, for IBP_MIXED, the same max_iters, the grids
 * are solved together: each stage of the solve is one launch covering all
 * grids (in groups of IBP_BATCH_MAX), through a batch the library builds for
 * that sequence of plans and keeps until one of them is destroyed.  Building
 * it (the first call with a given sequence, or after a plan's precision or
 * workspace changed) allocates and synchronises; later calls do neither.
 * Callers that capture graphs from the first call build the batch
 * explicitly with ibp_batch_create.  Otherwise the plans are solved one after
 * another on `stream`.  The batched stages use the general mixed-radix
 * transforms for every grid, so results can differ from ibp_solve's in the
 * last bits for grids that ibp_solve transforms with its power-of-two
 * kernels. */
ibp_status_t ibp_solve_batched(const ibp_plan_t* plans, int count, const double* const* rhs,
                               double* const* phi, hipStream_t stream);

/* ---------------------------------------------------------------- batches
 * Many uneven grids solved together (one launch per stage covering every
 * grid).  A batch records per-grid arguments (tables, workspaces, shapes) in
 * a device table; the right-hand sides and solutions are given per call. */
#define IBP_BATCH_MAX 64
typedef struct ibp_batch_s* ibp_batch_t;

/* Build a batch over plans[0..count) (1 <= count <= IBP_BATCH_MAX; distinct
 * plans on the current device, all IBP_FP64 or all IBP_MIXED with one
 * max_iters; else IBP_ERROR_INVALID_VALUE or IBP_ERROR_UNSUPPORTED_SIZE for a
 * precision form that batches do not support).  Allocates and synchronises.
 * The plans must outlive the batch; changing a plan's precision or workspace
 * afterwards makes ibp_batch_solve return IBP_ERROR_INVALID_VALUE. */
ibp_status_t ibp_batch_create(const ibp_plan_t* plans, int count, ibp_batch_t* out);

/* Solve problem i of the batch with rhs[i], phi[i] (HOST arrays of device
 * pointers, as in ibp_solve).  Asynchronous on `stream`; never allocates,
 * synchronises or copies to the host, so it can be captured in a graph.
 * Per-grid state is read with ibp_get_info on the grid's plan. */
ibp_status_t ibp_batch_solve(ibp_batch_t batch, const double* const* rhs, double* const* phi, hipStream_t stream);

/* Line-solve columns per block of the batch's stage launches (2, 4, 8 or 16;
 * capped by the LDS budget).  Used by the batch autotuner. */
ibp_status_t ibp_batch_set_ycols(ibp_batch_t batch, int cols);

/* Schedule of the batch's solves.  1: the whole batched solve (every stage
 * of every grid, and for IBP_MIXED every refinement pass) is one persistent
 * launch: each grid is pinned to one XCD, whose blocks take the stages'
 * blocks from a queue in dependency order and overlap the stages of
 * different grids.  0 (the default): one launch per stage covering every
 * grid, measured faster on MI355X for batches of 32..192-point grids.  The
 * persistent schedule is available when every grid's x and z lines fit the
 * small transform tiles (nx/2 and nz up to 1024) and the tallest grid has at
 * most 384 rows (512 with 64-lane line solves of 8 rows); otherwise
 * IBP_ERROR_UNSUPPORTED_SIZE for enable = 1.  ibp_batch_autotune times both.
 * Results are bitwise the same under both. */
ibp_status_t ibp_batch_set_persistent(ibp_batch_t batch, int enable);

/* Free the batch's device table (the plans are untouched).  NULL accepted. */
ibp_status_t ibp_batch_destroy(ibp_batch_t batch);

/* ---------------------------------------------------------------- autotuning
 * Work splits chosen by timing: how many rows, columns or lines each block
 * of a stage takes.  They change which block computes what, never the
 * arithmetic, so solutions are bitwise the same under every choice. */
typedef struct {
  int xdiv;          /* x-stage rows per block = the largest tile's / xdiv (batches, FP64) */
  int zdiv;          /* z-stage columns per block = the largest tile's / zdiv (general z transform) */
  int ycols;         /* line-solve columns per block */
  int tried;         /* configurations timed */
  double ms;         /* time of one solve with the chosen configuration (HIP events) */
  double ms_before;  /* time of one solve with the configuration in place before tuning */
  int persistent;    /* batches: 1 = the persistent schedule was chosen (ibp_batch_set_persistent) */
  int lag;           /* batches, persistent: diagonal interleave of the grids' stages in a queue */
  int chunk;         /* batches, persistent: work items a block claims at once */
  int xsmall;        /* plans: general x transform in the small (1) or large (0) LDS tile; -1: no choice */
  int zsmall;        /* plans: the same for the general z transform */
  int reserved;
} ibp_tune_t;

/* Time solves of rhs into phi (device pointers as in ibp_solve; phi is
 * overwritten with the solution) over the plan's tunable configurations and
 * keep the fastest: the LDS tile (small or large) of the general x and z
 * transforms, z columns and line-solve columns per block.  Synchronises
 * `stream`; not for use under graph capture.
 *
 * Tuning cache: when the environment variable IBP_TUNE_CACHE names a file,
 * every tuned choice is appended to it as one JSON line keyed by the device
 * architecture, the grid dimensions and the precision form, e.g.
 *   {"key": "gfx950/plan/512x384x512/0", "xdiv": 1, "zdiv": 1, "ycols": 8,
 *    "xsmall": -1, "zsmall": -1, "persistent": 0, "lag": 1, "chunk": 8, "ms": 1.67}
 * (batches: "gfx950/batch/<precision>.<max_iters>/<nx>x<ny>x<nz>,..." over
 * their grids in order).  A key found there is applied without a search
 * (tried = 0), and ibp_plan_create, ibp_plan_set_precision and
 * ibp_batch_create apply it by themselves.  The last line of a key wins. */
ibp_status_t ibp_plan_autotune(ibp_plan_t plan, const double* rhs, double* phi, hipStream_t stream, ibp_tune_t* out);

/* The same for a batch (x rows, z columns and line-solve columns per block
 * of its stage launches; the x split is tuned for IBP_FP64 batches only,
 * because the mixed forms' norm partials follow it). */
ibp_status_t ibp_batch_autotune(ibp_batch_t batch, const double* const* rhs, double* const* phi, hipStream_t stream,
                                ibp_tune_t* out);

/* Wait for the plan's last solve and report its state (iterations,
 * convergence, non-finite flag, residuals, removed mean). */
ibp_status_t ibp_get_info(ibp_plan_t plan, ibp_info_t* out);

/* Discrete divergence of a staggered velocity field on the plan's grid (the
 * div u* of eq. ``elliptic``): f[j][k][i] = (u[j][k][i+1]-u[j][k][i])/dx +
 * (v[j+1][k][i]-v[j][k][i])/dyf_j + (w[j][k+1][i]-w[j][k][i])/dz, periodic in
 * x and z.  u, w: [ny][nz][nx] on the x and z faces at x = i dx, z = k dz;
 * v: [ny+1][nz][nx] on the y faces (rows 0 and ny are the walls); f:
 * [ny][nz][nx].  Device pointers, asynchronous on `stream`. */
ibp_status_t ibp_divergence(ibp_plan_t plan, const double* u, const double* v, const double* w,
                            double* f, hipStream_t stream);

/* One substep of the fractional-step method around the solve (paper, eqs.
 * ``elliptic``, ``velsolen`` and ``pressure``).
 *
 * ibp_solve_divergence: solve lap(phi) = (div u* - q) / alpha_dt with the
 * right-hand side built from the provisional velocity (u, v, w laid out as
 * for ibp_divergence) and the mass sources q ([ny][nz][nx], NULL for none);
 * alpha_dt > 0.  With IBP_FP64 and rhs_out == NULL the right-hand side is
 * assembled inside the first transform pass and never stored (one field
 * write and read fewer than ibp_divergence + ibp_solve).  Otherwise it is
 * written to rhs_out ([ny][nz][nx], required for the mixed forms, whose
 * refinement passes read it again) and solved as by ibp_solve.  Device
 * pointers, 16-byte aligned; asynchronous on `stream`. */
ibp_status_t ibp_solve_divergence(ibp_plan_t plan, const double* u, const double* v, const double* w,
                                  const double* q, double alpha_dt, double* rhs_out, double* phi, hipStream_t stream);

/* Projection and pressure update in one pass over the cells:
 *   u -= alpha_dt * G phi (x, y and z faces; at a Neumann wall the normal
 *   velocity is unchanged, at a Dirichlet wall G is the one-sided difference
 *   over the half cell to the wall value 0),
 *   p += phi - visc * L_h phi   (visc = alpha_dt / (2 Re) with implicit
 *   viscous terms, 0 with explicit ones; p may be NULL to skip it).
 * u, v, w, p are updated in place; phi is read.  Asynchronous on `stream`. */
ibp_status_t ibp_project(ibp_plan_t plan, const double* phi, double alpha_dt, double visc, double* u, double* v,
                         double* w, double* p, hipStream_t stream);

/* Factored implicit viscous solve (paper: eq. ``nstime_discr`` with
 * Crank-Nicolson viscous terms, split into direction-wise tridiagonal solves,
 * Thomas with a Sherman-Morrison correction along the two periodic
 * directions; "Fluid domain" parallelisation subsection):
 *   field <- (1 - beta L_y)^-1 (1 - beta L_z)^-1 (1 - beta L_x)^-1 field,
 * beta = alpha dt / (2 Re).  L_x, L_z: periodic uniform second differences.
 * L_y: the wall-normal second difference with the velocity wall conditions,
 * the complement of the plan's pressure-correction ones (ibp_plan_set_bc):
 * prescribed velocity (zero increment) at a Neumann wall of the plan, zero
 * normal gradient at a Dirichlet wall.
 *
 * IBP_AT_CELLS: a field [ny][nz][nx] at the y cell centres (u on the x faces,
 *   w on the z faces, cell-centred scalars); a prescribed-velocity wall is a
 *   zero value on the wall face, half a cell from the first centre.
 * IBP_AT_YFACES: the wall-normal component, [ny+1][nz][nx] on the y faces;
 *   rows 1..ny-1 are solved across the interior faces
 *   ((v[j+1]-v[j])/dyf_j - (v[j]-v[j-1])/dyf_{j-1}) / dyc_j and rows 0 and
 *   ny are set to zero (the increment vanishes on the walls).  Needs
 *   prescribed velocity at both walls (the plan's walls both Neumann). */
typedef enum { IBP_AT_CELLS = 0, IBP_AT_YFACES = 1 } ibp_location_t;

/* Factors the line operators of all three directions for `beta` (finite,
 * >= 0) on the host in FP64 and uploads them (synchronous; allocates the
 * plan's factor tables on first use).  Must be called again after
 * ibp_plan_set_bc.  IBP_ERROR_UNSUPPORTED_SIZE for lines longer than 1536. */
ibp_status_t ibp_helmholtz_set(ibp_plan_t plan, double beta);

/* Applies the factored solve in place to `field` (device pointer, 16-byte
 * aligned, layout as above): three passes, each reading and writing the field
 * once.  Asynchronous on `stream`, no allocation or host copy (graph
 * capturable).  IBP_ERROR_INVALID_VALUE if ibp_helmholtz_set has not been
 * called since the plan's last change of wall conditions, or for
 * IBP_AT_YFACES without prescribed velocity at both walls. */
ibp_status_t ibp_helmholtz(ibp_plan_t plan, double* field, ibp_location_t where, hipStream_t stream);

/* Per-pass timing.  While enabled, every kernel launch of ibp_solve is
 * bracketed by two HIP events recorded on the solve's stream (a few
 * microseconds of overhead per launch; not for graph capture). */
typedef struct {
  char name[32];           /* pass name, e.g. "x_r2c", "z_fwd", "y_solve", "z_inv", "x_c2r" */
  int launches;            /* launches since profiling was enabled or last queried */
  int reserved;
  double total_ms;         /* summed event-measured duration of those launches */
  double bytes_per_launch; /* algorithmic HBM bytes of one launch: every input element
                              read once and every output element written once */
} ibp_pass_stat_t;

ibp_status_t ibp_plan_set_profiling(ibp_plan_t plan, int enable);

/* Waits for the recorded events, writes up to `max` pass entries to `stats`
 * (HOST array) and their number to *count, and resets the counters. */
ibp_status_t ibp_plan_get_profile(ibp_plan_t plan, int max, int* count, ibp_pass_stat_t* stats);

/* Static, never NULL. */
const char* ibp_status_string(ibp_status_t status);

/* Library version as major*10000 + minor*100 + patch. */
int ibp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IBPOISSON_H */
