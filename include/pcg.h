/*
 * pcg.h -- C ABI of libpcg, a matrix-free, vertical-line-preconditioned
 * conjugate gradient solver for anisotropic 3D elliptic problems on flat
 * tensor-product grids, after Mueller, Guo, Scheichl and Shi,
 * "Matrix-free GPU implementation of a preconditioned conjugate gradient
 * solver for anisotropic elliptic PDEs" (arXiv 1302.7193).
 *
 * The operator is the cell-centred finite-volume discretisation of
 *     -div(K grad u) + u = f,   K = diag(K_h, K_h, K_v),
 * on n_x * n_y vertical columns of n_z levels (Sec. 3.1, eqs.
 * ModelEqnCubedSphere, DiagonalMatrix, TridiagonalMatrix): each column block
 * A_T is tridiagonal and the coupling to a horizontal neighbour is diagonal.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.  Every field vector holds n = n_x*n_y*n_z values with cell (i,j,k)
 *   at index l = (i*n_y + j)*n_z + k: vertical columns are contiguous, k = 0
 *   is the lowest (finest) level (Sec. 3.2, eq. GlobalColumnReprConversion;
 *   Sec. 6.1, eq. MemoryMappingCPU).  Batched vectors stack right-hand sides:
 *   index s*n + l for right-hand side s.
 * Memory.  Vector arguments are device pointers (HIP device memory of the
 *   device that was current when the problem was created), owned by the
 *   caller, 16-byte aligned (PCG_E_INVALID otherwise), never retained after
 *   return.
 *   Host pointers are accepted only where the argument name ends in _host,
 *   for descriptor, option, tuning and result structs, and where the
 *   description says host array (the widths of
 *   pcg_problem_create_stretched, the pointer array of pcg_stream_probe).
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the default
 *   stream).  pcg_apply/pcg_precond/pcg_csr_* are asynchronous on it;
 *   pcg_solve and pcg_solve_batched block until the solve has finished.
 * Errors.  Every call returns a pcg_status; nothing aborts or throws across
 *   the ABI.  Arguments are validated before any launch; HIP failures map
 *   to PCG_E_DEVICE.  pcg_last_error() returns the calling thread's last
 *   message.  A problem handle may be used by one host thread at a time;
 *   the server API is thread-safe.
 * Numbers.  FP64 entry points compute in FP64.  FP32 entry points store
 *   vectors and evaluate the stencil and line solves in FP32; every dot
 *   product is accumulated in FP64 and every Krylov scalar is FP64.
 */
#ifndef PCG_H
#define PCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PCG_OK = 0,
    PCG_E_INVALID = -1,   /* bad argument or descriptor; nothing launched  */
    PCG_E_NOMEM = -2,     /* workspace / arena / budget too small          */
    PCG_E_DEVICE = -3,    /* HIP runtime error                             */
    PCG_E_NOCONV = -4,    /* max_iter reached; the result is still filled  */
    PCG_E_BREAKDOWN = -5, /* <p,Ap> <= 0, <r,z> <= 0 or a non-finite value */
    PCG_E_AGAIN = -6,     /* request still queued or running               */
    PCG_E_CANCELLED = -7  /* request cancelled before it ran               */
} pcg_status;

typedef enum { PCG_BC_DIRICHLET = 0, PCG_BC_PERIODIC = 1 } pcg_bc;
typedef enum { PCG_F64 = 0, PCG_F32 = 1 } pcg_dtype;
typedef enum { PCG_PREC_FP64 = 0, PCG_PREC_MIXED = 1 } pcg_precision;

/* Grid and coefficients.  Horizontal cells are dx*dy, the n_z levels span
 * height H with geometric grading dz[k+1] = grading*dz[k] (finest at k = 0;
 * Sec. 3.1 asks for the finest spacing near the ground).  Top and bottom
 * faces are Dirichlet (u = 0); each horizontal direction is Dirichlet or
 * periodic.  Dirichlet faces use the half-cell distance.  Periodic
 * directions need at least 3 cells.  1 <= n_z <= 1024. */
typedef struct {
    int32_t nx, ny, nz;
    double dx, dy;
    double height;
    double grading;
    double k_h, k_v;
    int32_t bc_x, bc_y; /* pcg_bc */
} pcg_problem_desc;

typedef struct {
    double rtol;          /* stop when ||r|| / ||r0|| < rtol ...              */
    double atol;          /* ... or ||r|| < atol (Alg. InterleavedPCG)       */
    int32_t max_iter;     /* FP64: iterations; MIXED: inner iterations total */
    int32_t precision;    /* pcg_precision                                    */
    double inner_rtol;    /* MIXED: relative tolerance of each FP32 inner solve */
    int32_t max_outer;    /* MIXED: refinement steps (FP64 residuals)         */
    int32_t fused;        /* 1: two fused sweeps per iteration (Sec. 4.3);
                             0: separate operator, preconditioner and BLAS-1
                                kernels (standard PCG, Sec. 4.1)             */
    int32_t graph_chunk;  /* >0: iterations per captured HIP graph replay;
                             0: direct launches; -1: adaptive (last count)  */
    int32_t profile;      /* 1: time every fused kernel with HIP events
                             (event records between the launches, or event
                             nodes inside the graph chunks); single
                             right-hand side; fills the *_kernel_* fields;
                             2: kernel A only (half the events; the
                             precond fields stay 0)                        */
    int32_t true_residual;/* 1: also compute ||b - A x|| / ||r0|| in FP64    */
    int32_t x0_zero;      /* 1: start from x0 = 0 without reading x          */
    int32_t preconditioner; /* PCG_PRECOND_LINE (default), _MG or _RBGS       */
    int32_t mg_levels;    /* MG: at most this many levels (0: every level the
                             grid allows; 1: line-Jacobi sweeps only)        */
} pcg_solve_opts;

/* Preconditioners.  LINE: the vertical line preconditioner (one tridiagonal
 * solve per column, Sec. 4.1-4.2).  MG: one V-cycle of a tensor-product
 * multigrid built on it, the extension the paper names as its next step
 * (Sec. 1, Sec. 8): only the horizontal grid is coarsened (2 x 2 cells
 * merged per level while n_x and n_y are even and the halves have >= 4
 * cells), coarse operators are the same discretisation on the coarse grid,
 * prolongation copies a coarse column to its four children and restriction
 * sums them, the smoother is vertical-line Jacobi damped by 0.8 with one
 * pre- and one post-smoothing sweep (4 sweeps on the coarsest level).  The
 * V-cycle is symmetric positive definite, so the same CG applies.  MG runs
 * in the fused iteration only (fused = 1; FP64 or mixed precision).
 * RBGS: the block-SOR alternative of Sec. 4.1 (the same column solves plus
 * one more sparse product): symmetric block Gauss-Seidel over the vertical
 * columns ordered red-black by horizontal position (i + j even: red), one
 * forward and one backward sweep, relaxation factor 1.  Needs an even
 * number of cells in every periodic direction (PCG_E_INVALID otherwise);
 * fused iteration only.
 *
 * AUTO chooses by the anisotropy ratio gamma^2 = (K_v / (H/n_z)^2) /
 * (K_h / dx^2) of the descriptor (dx: desc->dx; for stretched grids the
 * mean x width) and the size, from time-to-solution measured on MI355X:
 * MG when gamma^2 <= 300 and n >= 2^22 unknowns (its fixed cost per level
 * pays off only on large grids), else RBGS when gamma^2 <= 1e4 and
 * red-black ordering applies, else LINE; the unfused iteration always
 * takes LINE.  pcg_result.preconditioner reports the choice. */
enum { PCG_PRECOND_LINE = 0, PCG_PRECOND_MG = 1, PCG_PRECOND_RBGS = 2, PCG_PRECOND_AUTO = 3 };

typedef struct {
    int32_t status;            /* pcg_status of the solve                    */
    int32_t iterations;        /* FP64: iterations; MIXED: inner iterations  */
    int32_t outer_iterations;  /* MIXED: FP64 residual evaluations - 1       */
    int32_t launches;          /* kernel launches issued                     */
    double rel_res_recursive;  /* recursive ||r|| / ||r0|| at exit           */
    double rel_res_true;       /* FP64 ||b - A x|| / ||r0|| (if requested;
                                  always for MIXED), else -1                 */
    double r0_norm;            /* ||b - A x0||                               */
    double elapsed_ms;         /* host wall time of the call                 */
    double ms_apply_kernel;    /* profile: summed time of fused apply kernel */
    double ms_precond_kernel;  /* profile: summed time of fused precond kernel */
    int32_t n_apply_kernel;    /* profile: launches timed                    */
    int32_t n_precond_kernel;
    int32_t preconditioner;    /* the preconditioner used (AUTO resolved)    */
    int32_t reserved;
} pcg_result;

typedef struct pcg_problem pcg_problem; /* opaque */
typedef struct pcg_server pcg_server;   /* opaque */

/* Default options: rtol 1e-8, atol 0, max_iter 10000, FP64, inner_rtol 3e-5,
 * max_outer 20, fused, graph_chunk -1, no profiling, no true residual, x0
 * read from x, the line preconditioner (mg_levels 0). */
void pcg_default_opts(pcg_solve_opts *opts);

/* Fill a descriptor for the unit square (dx = 1/n_x, dy = 1/n_y), height 1,
 * K_h = 1 and K_v set from the anisotropy ratio
 *     gamma2 = (K_v / dzbar^2) / (K_h / dx^2),  dzbar = height / n_z,
 * i.e. the vertical/horizontal coupling ratio at the mean vertical spacing
 * (Sec. 3, eq. Anisotropy).  bc applies to both horizontal directions. */
pcg_status pcg_desc_from_ratio(int32_t nx, int32_t ny, int32_t nz, double grading,
                               double gamma2, int32_t bc, pcg_problem_desc *out);

/* Validate desc and precompute, on the current device, the vertical
 * coefficient vectors a, b, c, d of length n_z (Sec. 3.1, eq.
 * TridiagonalMatrix; Sec. 4.2: only O(n_z) numbers describe the vertical
 * discretisation) and the LU factors of the column block for each of the
 * at most nine column classes (number of Dirichlet side faces).  Allocates
 * a few KiB of device memory owned by the handle. */
pcg_status pcg_problem_create(const pcg_problem_desc *desc, pcg_problem **out);

/* The same operator on a stretched tensor-product horizontal grid: cell
 * (i, j) is x_widths[i] by y_widths[j] (host arrays of n_x and n_y positive
 * finite values, copied; desc->dx and desc->dy are not used).  The
 * horizontal geometry enters the method only through |T| and the face
 * weights alpha_{T,T'} (Sec. 3.1, eqs. DiagonalMatrix / TridiagonalMatrix;
 * Sec. 4.2), which the kernels rebuild per column from these widths: the
 * distance between neighbouring centres is the mean of their widths (half a
 * width at a Dirichlet wall, the first and last cells across a periodic
 * seam).  Every column block now differs, so the line solve factorises it in
 * the kernel instead of using per-class factors.  Errors as
 * pcg_problem_create, and PCG_E_INVALID for a NULL or non-positive width. */
pcg_status pcg_problem_create_stretched(const pcg_problem_desc *desc, const double *x_widths,
                                        const double *y_widths, pcg_problem **out);
void pcg_problem_destroy(pcg_problem *p);

/* Bytes of device workspace pcg_solve needs for these options
 * (opts may be NULL for the defaults).  nrhs >= 1 for pcg_solve_batched. */
size_t pcg_workspace_bytes(const pcg_problem *p, const pcg_solve_opts *opts, int32_t nrhs);

/* y = A x, matrix-free: the 7-point stencil is rebuilt from the column
 * coefficient vectors and per-column geometry (Sec. 4.2, eq. for the
 * sparse matrix-vector product).  x and y: n values of dtype; must not
 * overlap.  Asynchronous on stream. */
pcg_status pcg_apply(pcg_problem *p, int32_t dtype, const void *x, void *y, void *stream);

/* z = M^{-1} r where M is A without the couplings between vertical columns:
 * one tridiagonal solve per column (Sec. 4.1 and eq.
 * MatrixFreeTridiagonalSystem).  r and z: n values of dtype; either the
 * same vector (in place) or not overlapping at all (PCG_E_INVALID for a
 * partial overlap).  Asynchronous on stream. */
pcg_status pcg_precond(pcg_problem *p, int32_t dtype, const void *r, void *z, void *stream);

/* Multigrid preconditioner alone: z = B r for one V-cycle B (see
 * PCG_PRECOND_MG) over at most mg_levels levels (0: all).  r and z: n values
 * of dtype, not overlapping each other or the workspace.  workspace: at
 * least pcg_mg_bytes(p, dtype, mg_levels) bytes of device memory (16-byte
 * aligned) for the coarse levels and one fine-level vector.  pcg_mg_levels: the number of levels the grid allows.
 * Asynchronous on stream. */
int32_t pcg_mg_levels(const pcg_problem *p);
size_t pcg_mg_bytes(const pcg_problem *p, int32_t dtype, int32_t mg_levels);
pcg_status pcg_mg_precond(pcg_problem *p, int32_t dtype, const void *r, void *z,
                          int32_t mg_levels, void *workspace, size_t workspace_bytes,
                          void *stream);

/* Block Gauss-Seidel preconditioner alone: z = M^{-1} r for the symmetric
 * red-black block Gauss-Seidel M (see PCG_PRECOND_RBGS).  r and z: n values
 * of dtype, not overlapping.  Asynchronous on stream. */
pcg_status pcg_rbgs_precond(pcg_problem *p, int32_t dtype, const void *r, void *z, void *stream);

/* Solve A x = b.  b, x: n FP64 values; x holds x0 on entry and the solution
 * on return.  workspace: at least pcg_workspace_bytes(p, opts, 1) bytes of
 * device memory (contents destroyed).  b, x and the workspace must not
 * overlap (PCG_E_INVALID).  FP64 precision runs the loop-fused
 * iteration of Alg. InterleavedPCG (or, with fused = 0, standard PCG);
 * MIXED runs FP32 inner solves inside FP64 iterative refinement, with the
 * residual b - A x and the update of x in FP64.  Blocks until done.
 * Returns PCG_OK, PCG_E_NOCONV or PCG_E_BREAKDOWN with result filled, or an
 * argument/device error. */
pcg_status pcg_solve(pcg_problem *p, const double *b, double *x, void *workspace,
                     size_t workspace_bytes, const pcg_solve_opts *opts,
                     pcg_result *result, void *stream);

/* pcg_solve without a workspace argument and without any device memory
 * allocation in the call, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * The workspace is a fixed scratch array inside the library, 64 MiB per
 * device, held for the life of the process: enough for an FP64 solve of
 * about two million unknowns (less with the multigrid preconditioner's
 * coarse levels); larger solves return PCG_E_NOMEM with a message giving
 * the bytes needed.  Kernels, launch parameters and results are those of
 * pcg_solve with the same options run with graph_chunk = 0 (direct
 * launches, bitwise the same as graph chunks); graph_chunk and profile are
 * ignored.  Every call on one device shares that device's scratch: calls
 * that overlap in time on one device (from several host threads, or on
 * several streams) race and must not be made.  b, x, opts, result and
 * errors as pcg_solve.  Blocks until done. */
pcg_status pcg_solve_noalloc(pcg_problem *p, const double *b, double *x,
                             const pcg_solve_opts *opts, pcg_result *result, void *stream);

/* Solve A x_s = b_s for nrhs right-hand sides sharing one operator, all
 * advanced together by single launches that cover every right-hand side
 * (each with its own scalars and exit test; finished ones drop out).
 * b, x: nrhs*n FP64 values (index s*n + l).  results: nrhs entries (host).
 * workspace: pcg_workspace_bytes(p, opts, nrhs). */
pcg_status pcg_solve_batched(pcg_problem *p, int32_t nrhs, const double *b, double *x,
                             void *workspace, size_t workspace_bytes,
                             const pcg_solve_opts *opts, pcg_result *results, void *stream);

/* Launch parameters of the column kernels for one precision.
 *   lanes_per_column  L: a column is handled by L lanes of a 64-wide
 *                     wavefront, each owning ceil(n_z/L) (rounded up to a
 *                     power of two, at most 16) consecutive levels; the
 *                     line solve combines the L pieces with an in-wave
 *                     scan (DPP moves within rows of 16 lanes, then across
 *                     rows; the sub-structuring of Sec. 6.1).
 *                     Power of two, 1 <= L <= 64, 16*L >= n_z.
 *   block_cap         workgroups per right-hand side (>= 1, <= 65536; default
 *                     16384); each walks a contiguous range of column tiles.
 *                     Workspace sizes depend on it: query pcg_workspace_bytes
 *                     after changing the tuning.
 *   reduction         0: the last workgroup of each reduction totals the
 *                     partial sums and performs the scalar step inside the
 *                     kernel (device-scope fences in every workgroup);
 *                     1: a separate one-workgroup launch does it.
 * Both reductions add the same numbers in the same order; changing L or
 * block_cap changes the summation order (results stay within rounding).
 * lanes_per_column_prec / block_cap_prec: L and the block cap of the
 * line-solve kernels (kernel B of the fused iteration, pcg_precond), which
 * read and write whole columns independently of the other kernels and
 * usually prefer fewer lanes per column (shorter scans). */
typedef struct {
    int32_t lanes_per_column;
    int32_t block_cap;
    int32_t reduction;
    int32_t lanes_per_column_prec;   /* the same two for the kernels dominated */
    int32_t block_cap_prec;          /* by the line solve (kernel B, pcg_precond) */
} pcg_tuning;

pcg_status pcg_get_tuning(const pcg_problem *p, int32_t dtype, pcg_tuning *out);
pcg_status pcg_set_tuning(pcg_problem *p, int32_t dtype, const pcg_tuning *t);

/* Tuning cache: launch parameters keyed by (GPU architecture, uniform or
 * stretched horizontal grid, n_x, n_y, n_z, dtype, nrhs).  Loaded on first
 * use from tuning_cache.txt next to libpcg.so (regenerate it with
 * python -m paper_1302_7193_amd.make_tuning_cache), or from the file
 * named by the PCG_TUNING_CACHE environment
 * variable (empty: none).  A solve of nrhs right-hand sides uses the entry
 * for its shape unless the problem's tuning was set explicitly
 * (pcg_set_tuning, pcg_autotune); pcg_get_tuning reports the tuning a
 * one-right-hand-side solve would use.  pcg_autotune adds its result to the
 * in-memory table; pcg_tuning_cache_save writes the table (path NULL: the
 * default file); pcg_tuning_cache_load merges a file into it. */
pcg_status pcg_tuning_cache_load(const char *path);
pcg_status pcg_tuning_cache_save(const char *path);

/* Autotuner: times kernels A and B of the fused iteration (each with its
 * reduction, over nrhs right-hand sides, on synthetic vectors) for every
 * supported lanes_per_column, a ladder of block caps and both reduction
 * modes; keeps the three fastest launch shapes of each kernel per mode,
 * times the nine pairs together and takes the fastest pair for (p, dtype);
 * records it in the tuning cache for (shape, dtype, nrhs) and returns it in
 * best (may be NULL).  A set-up utility: it allocates (and frees) its own
 * device scratch of about 5 vectors of nrhs*n values of dtype.  Blocks. */
pcg_status pcg_autotune(pcg_problem *p, int32_t dtype, int32_t nrhs, void *stream,
                        pcg_tuning *best);

/* Assembled-CSR comparator (Sec. 6.2): bytes for the CSR arrays of dtype
 * (values of dtype, int32 column indices, int32 row offsets), a device-side
 * assembly into buf, and y = A x from it (y must not overlap x or buf).
 * Not used by the solver. */
size_t pcg_csr_bytes(const pcg_problem *p, int32_t dtype);
pcg_status pcg_csr_build(pcg_problem *p, int32_t dtype, void *buf, size_t bytes, void *stream);
pcg_status pcg_csr_apply(pcg_problem *p, int32_t dtype, const void *buf, const void *x,
                         void *y, void *stream);

/* ------------------------------------------------------------ serving --
 * Continuous batching of independent solves with different grids and
 * coefficients.  pcg_submit queues a request and returns at once; worker
 * threads (max_active of them, one HIP stream each) admit queued requests in
 * arrival order whenever a worker is idle and the request's device bytes
 * (pcg_request_bytes) keep the admitted total within hbm_budget_bytes and
 * fit in the caller's device arena; an admitted request is copied in, solved
 * by the fused iteration from x0 = 0 (HIP-graph-captured chunks), copied out
 * and its memory released, which admits the next.  Requests overlap on the
 * device.  A request's arithmetic depends only on its own descriptor and
 * options, so its result is the same alone and in any mix.  The library
 * allocates no device memory for requests beyond the arena (it does create
 * small per-shape problem tables).  All server calls are thread-safe. */
typedef struct {
    size_t hbm_budget_bytes; /* admitted requests' bytes stay within this (and the arena) */
    int32_t max_active;      /* requests solved concurrently, 1..64                  */
    int32_t batched;         /* 0: one worker thread and stream per active request;
                                1: one scheduler whose every launch advances all
                                   active requests (see below)                   */
} pcg_server_opts;

typedef struct {
    uint64_t submitted, completed, cancelled, rejected;
    int32_t queued, active;
    size_t bytes_in_use, peak_bytes_in_use;
    int32_t peak_active;     /* most requests running on the device at once */
    int32_t reserved;
} pcg_server_stats;

/* Batched mode (batched = 1): continuous batching with shared launches.  One
 * scheduler thread runs ticks; in each, the requests at that stage get their
 * FP64 refinement residual, then a few iterations of the two fused kernels,
 * then the refinement update (or the FP64 exit correction), each step one
 * launch over all of them in which every request keeps its own grid,
 * tables, vectors, solver state and partial sums.  Requests that arrive
 * while others run join at the next tick (admitted by budget and arena as
 * above, up to max_active at once); finished ones leave.  Requests take a
 * served launch shape (4 levels per lane in FP32, 2 in FP64), so a result
 * equals that request served alone, in any mix, but may differ from
 * pcg_solve's within rounding.  It covers the line preconditioner (AUTO
 * resolving to it) on grids with n_z = 4, 8, 16, 32, 64 or 128; other
 * requests are rejected (PCG_E_INVALID).  FP64 requests report
 * rel_res_true = -1. */

/* Device bytes one request needs: b, x and its workspace (0 if invalid). */
size_t pcg_request_bytes(const pcg_problem_desc *desc, const pcg_solve_opts *opts);

/* arena: caller-owned device memory, 256-byte aligned, arena_bytes long;
 * it must outlive the server.  Starts the worker threads on the current
 * device. */
pcg_status pcg_server_create(const pcg_server_opts *opts, void *arena, size_t arena_bytes,
                             pcg_server **out);

/* Queue a solve.  b_host (read) and x_host (written) are host arrays of
 * n FP64 values that must stay valid until pcg_poll/pcg_wait reports the
 * ticket finished (pinned memory makes the copies faster).  opts may be
 * NULL (defaults); the solve always starts from x0 = 0.  PCG_E_NOMEM if the
 * request can never fit the budget or the arena. */
pcg_status pcg_submit(pcg_server *s, const pcg_problem_desc *desc, const pcg_solve_opts *opts,
                      const double *b_host, double *x_host, uint64_t *ticket);

/* As pcg_submit with b and x in device memory (n FP64 values each, 16-byte
 * aligned, caller-owned, valid until the ticket is finished): nothing is
 * copied and only the workspace (pcg_workspace_bytes) is taken from the
 * arena and counted against the budget.  The solve is ordered after the
 * work queued on `stream` (the producer of b) at the time of the call; x is
 * final when pcg_poll/pcg_wait reports the ticket finished. */
pcg_status pcg_submit_device(pcg_server *s, const pcg_problem_desc *desc,
                             const pcg_solve_opts *opts, const double *b_dev, double *x_dev,
                             void *stream, uint64_t *ticket);

/* PCG_E_AGAIN while queued or running; otherwise the solve's status with
 * *out filled (elapsed_ms = submission to completion) and the ticket
 * released; PCG_E_CANCELLED for a cancelled request. */
pcg_status pcg_poll(pcg_server *s, uint64_t ticket, pcg_result *out);
pcg_status pcg_wait(pcg_server *s, uint64_t ticket, pcg_result *out); /* blocking poll */

/* Cancel a request that is still queued (PCG_E_AGAIN once it runs). */
pcg_status pcg_cancel(pcg_server *s, uint64_t ticket);
pcg_status pcg_server_query(pcg_server *s, pcg_server_stats *out);

/* Cancels queued requests, waits for running ones, stops the workers. */
void pcg_server_destroy(pcg_server *s);

/* HBM bandwidth probe: the paper rates its memory-bound kernels by their
 * global-memory bandwidth as a fraction of the quoted peak (Sec. 5); this
 * measures what a kernel that only streams attains, the practical ceiling
 * beside that peak.  One kernel streams n_read (1..4) vectors in and n_write
 * (1..3) out, each `bytes` long (a positive multiple of 16), 16 bytes per
 * lane and access, with the nontemporal hint on no access (nontemporal = 0),
 * on every access (1), on every access but the reads of the first vector
 * (2: kernel A's pattern, whose stencil input is re-read as neighbour
 * columns) or on every access but the writes of the last vector (3: kernel
 * B's, whose z the next kernel reads).  vectors: host array of n_read + n_write device pointers
 * (16-byte aligned, caller-owned), the read ones first; a written vector may
 * not overlap any other.  Written vector k receives sum_i v_i * 2^-(i+k)
 * elementwise.  blocks: workgroups (0: 16384), each streaming one contiguous
 * range.  Asynchronous on `stream` (current device); the caller times it.
 * The mixes of the solver's kernels: 4 in / 3 out (kernel A), 2 / 2
 * (kernel B), 1 / 1 (copy).  PCG_E_INVALID for bad arguments. */
pcg_status pcg_stream_probe(int32_t n_read, int32_t n_write, void *const *vectors, size_t bytes,
                            int32_t nontemporal, int64_t blocks, void *stream);

/* Thread-local message of the last failing call (NUL-terminated, truncated
 * to n bytes); returns the full length. */
size_t pcg_last_error(char *buf, size_t n);

#ifdef __cplusplus
}
#endif
#endif /* PCG_H */
