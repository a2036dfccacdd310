/*
 * bhx.h - biharmonic field extension on AMD Instinct MI355X (gfx950).
 *
 * The library solves the extension problem of Sec. 2 of Moroney, Lusmore,
 * McCue and McElwain, "Extending fields in a level set method by solving a
 * biharmonic equation":
 *
 *   - a field F is known at the grid nodes where the level-set function
 *     phi < 0 (the known set K; the region definitions of Sec. 3 use a strict
 *     inequality, so phi == 0 and NaN are unknown);
 *   - at every other node (the unknown set U) the 13-point discrete
 *     biharmonic equation, eq. (12), must hold; near the edges of the grid
 *     the stencil uses two ghost layers whose values follow the boundary rule
 *     of each axis (Algorithm 1 pads the array for Dirichlet conditions;
 *     Sec. 3.1 and 3.2 describe the Neumann and periodic variants);
 *   - the unknowns solve the symmetric positive definite system
 *     A_UU u = -A_UK F_K (Sec. 2.2) by matrix-free preconditioned conjugate
 *     gradients, the preconditioner being the fast Poisson solver on the whole
 *     rectangle: embed the residual (zero at K), transform, divide by the
 *     squared eigenvalues of the discrete Laplacian, transform back, restrict
 *     (Algorithm 1; cosine transforms for Neumann axes, Fourier (Hartley)
 *     transforms for periodic axes, sine transforms for Dirichlet axes).
 *
 * Conventions for every entry point:
 *   - Arrays are float64, contiguous, row-major with x fastest:
 *     a[j*nx + i], 0 <= i < nx, 0 <= j < ny.  phi and F are DEVICE pointers
 *     owned by the caller (for instance torch tensors on the same device).
 *   - F is in/out.  Values at known nodes are read and never written
 *     (bit-exact).  Values at unknown nodes on input are ignored (the solve
 *     starts from zero, as Algorithm 1 does) and on return hold the
 *     extension.
 *   - The stencil is the paper's unscaled integer stencil; the grid spacing h
 *     cancels from the system and from the relative residual, so h is only
 *     validated (finite, > 0).
 *   - The stopping test is ||b - A_UU x||_2 <= tol * ||b||_2 on the recursive
 *     residual, followed by one check of the true residual computed with
 *     compensated (double-double) arithmetic; if that check fails the solve
 *     restarts from the true residual (up to the iteration limit).
 *   - Return values: 0 = BHX_OK; > 0 = warning, F holds the last iterate;
 *     < 0 = error, F untouched.  Nothing is thrown across this interface.
 *   - Entry points that take a stream enqueue their GPU work on it; they
 *     synchronise with it before returning (stats are valid on return).
 *     Calls on one handle are serialised by a lock inside the handle.
 *   - Boundary rules: Neumann, periodic and Dirichlet axes, one rule per axis.
 *     A Dirichlet axis of n nodes is transformed through a DFT of length
 *     2(n+1) (its odd extension) or, for 1024 <= n <= 2046, through a
 *     chirp-z transform of n+1 points; either must fit LDS like any
 *     transform: n <= 2047 in FP64 and FP32 (in three dimensions the y and z
 *     axes take n <= 1023 or n = 2047); otherwise BHX_ERR_ARG.
 */
#ifndef BHX_H
#define BHX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary rule of one axis. */
enum {
  BHX_NEUMANN = 0,    /* half-sample even reflection: g[-1]=f[0], g[-2]=f[1]; DCT-II */
  BHX_PERIODIC = 1,   /* wrap-around: g[-1]=f[n-1], g[-2]=f[n-2]; Hartley (DFT) */
  BHX_DIRICHLET = 2   /* Algorithm 1: g[-1]=0, g[-2]=-f[0]; DST-I */
};
/* Both axes packed into one int: low nibble x axis, next nibble y axis. */
#define BHX_BC(bx, by) ((bx) | ((by) << 4))
/* Three axes (three-dimensional entry points): third nibble z axis. */
#define BHX_BC3(bx, by, bz) ((bx) | ((by) << 4) | ((bz) << 8))

/* Status codes. */
enum {
  BHX_OK = 0,
  BHX_NOT_CONVERGED = 1,   /* iteration limit reached; F holds the last iterate   */
  BHX_ERR_ARG = -1,        /* invalid argument (sizes < 4, bad bc, tol not in (0,1),
                              h not finite or <= 0, null pointer, count < 1)        */
  BHX_ERR_SINGULAR = -2,   /* no known node and no Dirichlet axis: the system is
                              singular (constants are in the null space)           */
  BHX_ERR_NONFINITE = -3,  /* a known value inside the stencil reach of an unknown
                              node is NaN or infinite (the right-hand side is not
                              finite)                                              */
  BHX_ERR_NOMEM = -4,      /* device or pinned host allocation failed              */
  BHX_ERR_HIP = -5,        /* a HIP runtime call failed                            */
  BHX_BUSY = -6,           /* engine: the request does not fit right now           */
  BHX_ERR_BREAKDOWN = -7   /* the iteration produced a non-finite or non-positive
                              curvature (should not happen for valid input); F holds
                              the last finite iterate                              */
};

/* Precision of the preconditioner (transforms and spectral scaling). */
enum {
  BHX_PREC_FP64 = 0,       /* everything float64, standard PCG                     */
  BHX_PREC_FP32 = 1        /* transforms and scaling in float32, stencil, dots and
                              recurrences in float64; flexible (Polak-Ribiere) PCG */
};

typedef struct {
  int precision;    /* BHX_PREC_FP64 or BHX_PREC_FP32                              */
  int maxit;        /* iteration limit; 0 -> 50 * max(nx, ny)                       */
  int precond;      /* 1 = spectral fast Poisson preconditioner, 0 = none (plain CG) */
  int accurate;     /* 1 = outer defect correction: inner solves to tol_inner
                         relative to a compensated true residual until the true
                         residual meets tol                                         */
  double tol_inner; /* inner tolerance for accurate mode; 0 -> 1e-8                 */
  int flexible;     /* -1 = default (standard), 0 = standard beta = r.z / r_old.z_old,
                         1 = Polak-Ribiere beta (flexible PCG, for a preconditioner
                         that varies between applications)                          */
  int chunk;        /* iterations per captured graph between convergence checks;
                         0 -> 32; an odd value is rounded up to even                 */
  int rows;         /* packed complex rows (two grid rows each) per transform work
                         item; 0 = automatic (autotuner or built-in policy: as many as
                         fit, fewer while the instance alone supplies under two items
                         per CU); -1 = as many as fit (the engine's default, whose
                         launches are shared by many requests)                        */
  int occupancy;    /* persistent blocks per CU of the transform passes; 0 = auto   */
  int autotune;     /* 1 = choose the launch schedule (packed rows per transform work
                         item, persistent-grid occupancy per pass, iterations per
                         graph) by timing short trial solves of this batch's shape on
                         first use, cached per handle; 0 = built-in policy           */
  int profile;      /* bit mask of iteration passes to time: each launch of such a
                         pass carries start/stop events recorded by its dispatch
                         (kernel execution time; the iterations are then launched
                         directly, not from a graph): bit 0 stencil, 1 row-forward,
                         2 column, 3 row-inverse; results in bhx_stats.pass_ms /
                         pass_launches; 0 = off                                      */
  int warm_start;   /* 1 = the values of F at the unknown nodes on input are the
                         first iterate x0 (e.g. the previous time step's extension);
                         the stopping rule stays ||b - A x|| <= tol ||b||; a start
                         that already meets it returns with 0 iterations and F
                         unchanged; a non-finite start gives BHX_ERR_NONFINITE.
                         0 = x0 = 0 (Algorithm 1), input values at U are ignored    */
  int solver;       /* 0 = preconditioned conjugate gradients (Algorithm 1);
                         1 = sparse direct (Sec. 2.2): banded Cholesky of A_UU on the
                         GPU with the unknowns numbered line by line, then refinement
                         with the compensated residual until ||b - A u|| <= tol ||b||
                         (bhx_stats.iterations = refinement solves).  Two dimensions,
                         FP64, at most one periodic axis (both periodic: BHX_ERR_ARG).
                         The lines run along y (grid columns) when y is periodic or
                         when x is the longer non-periodic axis, else along x, so a
                         periodic axis never couples the first and last lines; band
                         storage is about 8 (64 + w) bytes per unknown, w the band
                         width (about twice the unknowns per line).  Fields sharing phi in one
                         bhx_extend_fields call share one factorisation.  Not for
                         the serving engine or three dimensions (BHX_ERR_ARG).       */
  int transform;    /* form of the preconditioner's 1-D transforms (two dimensions):
                         1 = FFT family: radix-4/2 cores in LDS, Bluestein's chirp-z for
                         lengths without one;
                         2 = dense where both axes have at most 512 nodes: each 1-D
                         transform a product with its basis matrix on the matrix cores
                         (v_mfma_f64_16x16x4 / v_mfma_f32_16x16x4), the basis entries
                         generated from a table in LDS; the FFT family otherwise;
                         0 = built-in choice: the FFT family (faster at every size
                         measured); with autotune = 1 the autotuner also times dense-
                         wherever-possible for the batch and keeps it if faster.  The
                         two forms' results agree to rounding.                        */
} bhx_opts;

typedef struct {
  int status;              /* per-instance status code (see above)                 */
  int iterations;          /* conjugate-gradient iterations (matrix-vector products) */
  int restarts;            /* number of true-residual restarts                       */
  int n_unknown;           /* |U|                                                    */
  double rel_residual;     /* recursive ||r|| / ||b|| at exit                         */
  double true_rel_residual;/* compensated ||b - A_UU x|| / ||b|| at exit             */
  double seconds;          /* host wall time of the call that produced this record   */
  double pass_ms[4];       /* summed event-timed duration of each profiled pass       */
  int pass_launches[4];    /* launches counted in pass_ms (iterations that did work)  */
} bhx_stats;

typedef struct bhx_handle bhx_handle;
typedef struct bhx_engine bhx_engine;

/* Fill *o with defaults (FP64, spectral, maxit 0, chunk 0, flexible -1). */
void bhx_default_opts(bhx_opts* o);

/* Create / destroy a handle bound to HIP device `device`.  The handle owns
 * transform tables, a growable device workspace and captured graphs.
 * Returns BHX_OK, BHX_ERR_ARG (null out, device < 0 or >= the device
 * count) or BHX_ERR_HIP (no usable HIP device; bhx_last_error() says why).
 * Processes that also use another HIP runtime (PyTorch bundles one) must
 * load it first, so that this library binds to that runtime. */
int bhx_create(bhx_handle** out, int device);
void bhx_destroy(bhx_handle* h);

/* Single extension with the library's default handle on device 0, the null
 * stream and default options (FP64 PCG).  Blocks until done.  `bc` is
 * BHX_BC(bx, by).  Returns a status code. */
int bhx_extend(const double* phi, double* F, int nx, int ny, double h, int bc, double tol);

/* Single extension with explicit handle, options (NULL -> defaults), stream
 * (a hipStream_t passed as void*, NULL -> null stream) and stats (may be
 * NULL). */
int bhx_extend_ex(bhx_handle* hd, const double* phi, double* F, int nx, int ny, double h,
                  int bc, double tol, const bhx_opts* o, void* stream, bhx_stats* out);

/* Capacity of the static device array behind bhx_extend_noalloc, per device. */
#define BHX_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* bhx_extend_ex for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * The call allocates no device or pinned memory: every buffer of the solve
 * (descriptors, transform tables, control block, workspace vectors) lives in
 * one static device array of the library of BHX_NOALLOC_SCRATCH_BYTES per
 * device, whose address bhx_create looks up once per device.  The caller
 * passes phi and F as for bhx_extend_ex (device pointers, caller-owned);
 * arguments, options, statuses and stats are those of bhx_extend_ex, with
 * these differences:
 *   - a problem whose workspace, tables and descriptors exceed the array
 *     (about 1.3 million nodes in FP64: 1024 x 1024 fits, 2048 x 2048 does
 *     not) returns BHX_ERR_ARG, F untouched, bhx_last_error() saying the
 *     bytes needed and the limit;
 *   - opts.autotune, opts.profile and opts.solver = 1 return BHX_ERR_ARG;
 *   - iteration chunks are launched directly (no captured graphs), so a
 *     solve may take a little longer than with bhx_extend_ex; the kernels
 *     and their order are the same, and so is the result, bit for bit.
 * All calls on one device share that device's array, and each call leaves
 * it holding its own state: calls are serialised by a lock per device in
 * this process, and must not overlap with each other on one device in any
 * other way (each process has its own copy).  Synchronises with the stream
 * before returning. */
int bhx_extend_noalloc(bhx_handle* hd, const double* phi, double* F, int nx, int ny, double h,
                       int bc, double tol, const bhx_opts* o, void* stream, bhx_stats* out);

/* `count` independent extensions of mixed sizes and boundary rules solved
 * together: each pass of every iteration is one launch over the tiles of all
 * unfinished instances; instances retire independently.  phi, F are host
 * arrays of `count` device pointers; nx, ny, h, bc, tol are host arrays of
 * `count` values; out (may be NULL) receives `count` records.  Returns
 * BHX_OK if every instance converged, the first negative per-instance code
 * if any instance failed, else BHX_NOT_CONVERGED.  Argument errors in any
 * instance reject the whole call before any GPU work. */
int bhx_extend_batched(bhx_handle* hd, int count, const double* const* phi, double* const* F,
                       const int* nx, const int* ny, const double* h, const int* bc,
                       const double* tol, const bhx_opts* o, void* stream, bhx_stats* out);

/* `nfields` fields known on the same region (one phi, e.g. the components of
 * a velocity, or a field and its gradient components in a level-set step)
 * extended in one batched solve: F is a host array of `nfields` device
 * pointers, each (ny, nx) like phi; one tolerance for all; out (may be NULL)
 * receives `nfields` records.  Each result is bit-identical to the same field
 * solved alone with bhx_extend_ex and the same options (warm_start applies to
 * every field).  Returns as bhx_extend_batched. */
int bhx_extend_fields(bhx_handle* hd, int nfields, const double* phi, double* const* F, int nx,
                      int ny, double h, int bc, double tol, const bhx_opts* o, void* stream,
                      bhx_stats* out);

/* Device bytes the library needs for one instance (workspace vectors, mask,
 * partial sums, control block), excluding phi and F.  Host-only; 0 for
 * invalid arguments. */
size_t bhx_workspace_bytes(int nx, int ny, int bc, const bhx_opts* o);

/* ---- Three dimensions (Sec. 3, Example 2) -------------------------------
 * The same extension on an nx x ny x nz grid: arrays (nz, ny, nx), x fastest,
 * a[(k*ny + j)*nx + i]; the operator is the square of the negative 7-point
 * Laplacian, the 25-point discrete biharmonic operator, with two ghost
 * layers per face by each axis' rule; the preconditioner transforms along x,
 * y and z and divides by (lambda_x + lambda_y + lambda_z)^2.  bc =
 * BHX_BC3(bx, by, bz).  nx, ny, nz >= 4, each a supported transform length,
 * and nx*ny*nz < 2^31.  Options, stopping rule, statuses and the handling of
 * F are those of bhx_extend_ex (warm_start included). */
int bhx_extend3d(bhx_handle* hd, const double* phi, double* F, int nx, int ny, int nz, double h,
                 int bc, double tol, const bhx_opts* o, void* stream, bhx_stats* out);
/* Device bytes of one three-dimensional instance; 0 for invalid arguments. */
size_t bhx_workspace_bytes3d(int nx, int ny, int nz, int bc, const bhx_opts* o);

/* ---- Serving engine: continuous batching of requests --------------------
 * The engine owns a worker thread and a stream on `device`.  Requests are
 * admitted while their workspace fits in `hbm_budget` bytes and a slot is
 * free (at most `max_slots` in flight); admitted requests join the running
 * batch at the next iteration-chunk boundary, so their work overlaps with
 * requests already on the device.  phi and F stay owned by the caller and
 * must stay valid until the request completes. */
int bhx_engine_create(bhx_engine** e, int device, size_t hbm_budget, int max_slots,
                      const bhx_opts* o);
/* Non-blocking.  Returns BHX_OK and the request id, BHX_BUSY if the request
 * cannot be admitted now (budget or slots; retry later), BHX_ERR_ARG for
 * invalid arguments or a request that could never fit the budget. */
int bhx_engine_submit(bhx_engine* e, const double* phi, double* F, int nx, int ny, double h,
                      int bc, double tol, uint64_t* id);
/* Collect up to `max` finished requests: ids[i], st[i]; *n_done receives the
 * count.  Non-blocking. */
int bhx_engine_poll(bhx_engine* e, uint64_t* ids, bhx_stats* st, int max, int* n_done);
/* Number of requests admitted and not yet collected by poll. */
int bhx_engine_inflight(bhx_engine* e);
/* Kernel timing of an engine created with bhx_opts.profile != 0 (a bit mask
 * of iteration passes: bit 0 stencil, 1 row-forward, 2 column, 3
 * row-inverse; such an engine launches its iteration chunks directly with
 * dispatch-recorded start/stop events around the selected passes instead of
 * replaying captured graphs).  For each pass p (arrays of 4, caller-owned
 * host memory): ms[p] the summed kernel execution time of its launches,
 * launches[p] their number, unknown_nodes[p] and nodes[p] the sums over those
 * launches of the unknown and of all nodes of the requests each launch
 * worked on (a request counts in the launches of the iterations it ran).
 * reset != 0 zeroes the sums after reading.  Returns BHX_OK or BHX_ERR_ARG. */
int bhx_engine_profile(bhx_engine* e, double* ms, long long* launches, double* unknown_nodes,
                       double* nodes, int reset);
/* Stops the worker after in-flight requests finish and frees everything. */
void bhx_engine_destroy(bhx_engine* e);

/* Diagnostic: apply one operator of the iteration to a device vector `in`
 * (float64, nx*ny) with the known set taken from phi (phi < 0):
 *   op 0: out = R A R^T in - the masked 13-point operator of eq. (12):
 *         values of `in` at known nodes are treated as 0, and out is 0 there;
 *   op 1: out = the fast Poisson preconditioner of Algorithm 1 applied to
 *         `in` restricted to the unknown nodes (embed with zeros at K,
 *         transform, divide by (lambda_x + lambda_y)^2 with 0 for a zero
 *         eigenvalue, transform back, restrict), in the given precision.
 * `precision`: bits 0-3 the preconditioner's precision (BHX_PREC_*), bits
 * 4-7 the transform form (bhx_opts.transform).  Synchronises with the
 * stream.  Returns a status code. */
int bhx_debug_apply(bhx_handle* hd, int op, const double* phi, const double* in, double* out,
                    int nx, int ny, int bc, int precision, void* stream);
/* bhx_debug_apply in three dimensions: op 0 the masked 25-point operator,
 * op 1 the three-axis preconditioner; bc = BHX_BC3(bx, by, bz). */
int bhx_debug_apply3d(bhx_handle* hd, int op, const double* phi, const double* in, double* out,
                      int nx, int ny, int nz, int bc, int precision, void* stream);

/* Human-readable name of a status code (static storage). */
const char* bhx_status_string(int status);

/* Description of the last HIP failure on the calling thread (the runtime
 * call, its source location and HIP's message); "" if none. */
const char* bhx_last_error(void);

/* Library version string (static storage). */
const char* bhx_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BHX_H */
