/*
 * femh.h -- C ABI of the MI355X (gfx950) nodal-hexahedral H-field
 * finite element scattering solver.
 *
 * The method (Vollaire, Nicolas, Nicolas, "Parallel computing for the
 * finite element method", section 2, eqs. (1)-(4)): the total magnetic
 * field H of a time-harmonic scattering problem, three complex components
 * per node of a structured box of first-order (8-node trilinear)
 * hexahedra, satisfies
 *
 *     int (1/eps_r) curl W . curl H + s int div W div H
 *       - k0^2 int mu_r W . H + int_{S_ext} W . g_ABC(H)
 *     = int_{S_ext} W . [ g_ABC(H_i) - n x curl H_i ],
 *
 * with the second-order Engquist-Majda condition of eq. (3),
 * g_ABC(H) = j k0 H_t - (j / 2k0) lap_t H_t, on outer faces tagged ABC,
 * the grad-div penalty of eq. (2) with weight s, and PEC elements removed
 * (PEC is a natural condition for H).  The discrete system is a
 * complex-symmetric (A = A^T, not Hermitian) matrix of 3x3 blocks, one
 * block per pair of nodes sharing an active element, solved by conjugate
 * gradients with diagonal preconditioning (section 3.1.5), read for a
 * complex-symmetric matrix as COCG (unconjugated bilinear form).
 *
 * Conventions shared by every call:
 *   - Every call returns a femh_status (0 = success, < 0 = error) unless
 *     noted.  femh_last_error() returns a message for the calling thread's
 *     last failing call.
 *   - Input arrays are copied (or fully consumed) before the call returns;
 *     the caller may free them afterwards.  Output buffers are owned and
 *     sized by the caller.
 *   - "device pointer" means memory of the context's device, readable and
 *     writable by kernels on the context's stream.
 *   - Unless a call says it is asynchronous, it returns after its device
 *     work on the context's stream has completed.
 *   - Handles own their device memory; destroy(NULL) is a no-op.
 *   - One context (and its problems) must not be used by two threads at
 *     once.  The server calls are the exception: they are thread-safe.
 *   - Element arrays are [nz][ny][nx] (x fastest).  Active nodes are the
 *     nodes of at least one non-PEC element, numbered in lexicographic grid
 *     order (x fastest).  Unknown index = 3 * node + component (x, y, z).
 *   - Complex numbers are interleaved (re, im) pairs: femh_c128 in FP64,
 *     and pairs of float for complex64 device vectors.
 */
#ifndef FEMH_H
#define FEMH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } femh_c128;

typedef enum {
  FEMH_OK = 0,
  FEMH_E_INVALID = -1,        /* bad argument or descriptor */
  FEMH_E_NONFINITE = -2,      /* NaN/Inf in an input */
  FEMH_E_OOM = -3,            /* device allocation failed / over budget */
  FEMH_E_DEVICE = -4,         /* HIP runtime error, or no usable gfx950 device */
  FEMH_E_NOT_CONVERGED = -5,  /* iteration limit reached; best iterate returned */
  FEMH_E_BREAKDOWN = -6,      /* COCG breakdown (x^T A x or r^T z vanished) */
  FEMH_E_CANCELLED = -7,      /* server request cancelled */
  FEMH_E_PENDING = -8,        /* server request not finished yet */
  FEMH_E_NOT_FOUND = -9       /* unknown server ticket */
} femh_status;

/* Outer face tags, faces ordered -x, +x, -y, +y, -z, +z.  The two plane
 * conditions of section 3.1.3 are essential: on every active node of the
 * face the constrained components are fixed to zero by elimination (their
 * matrix rows and columns are those of the identity, their right-hand side
 * entries zero, so the matrix stays complex-symmetric); the other
 * components keep the natural condition.  A node on two such faces
 * collects both constraints. */
enum { FEMH_FACE_ABC = 0,      /* eq. (3) absorbing condition */
       FEMH_FACE_NATURAL = 1,  /* no surface term (a PEC wall for H) */
       FEMH_FACE_SYM = 2,      /* symmetry plane, n . H = 0 (eq. (6a)): the normal component fixed */
       FEMH_FACE_ANTISYM = 3   /* antisymmetry plane, n x H = 0 (eq. (6b)): the tangential ones fixed */ };

typedef enum { FEMH_FP64 = 0,          /* complex128 matrix and Krylov vectors */
               FEMH_MIXED = 1,         /* complex64 matrix and Krylov vectors (FP32 arithmetic),
                                          reliable updates into an FP64 iterate */
               FEMH_MIXED_MATRIX = 2   /* complex64 matrix, complex128 Krylov vectors,
                                          reliable updates against the FP64 matrix */ } femh_precision;

typedef enum { FEMH_PRECOND_JACOBI = 0,  /* z = D^-1 r, D = diag(A) (section 3.1.5.1) */
               FEMH_PRECOND_NONE = 1,
               FEMH_PRECOND_BIC0 = 2     /* block incomplete Cholesky (sections 3.1.5.2-3.1.5.3): the
                                            unknowns of precond_block consecutive nodes form a block,
                                            couplings between blocks are dropped, and each block keeps
                                            eq. (5)'s complex-symmetric IC(0) factor L L^T on the lower part
                                            of its 3x3-block pattern; z = (L L^T)^-1 r by eq. (6)'s forward
                                            and back substitution.  FEMH_FP64 single right-hand-side
                                            solves only (femh_solve, femh_solve_dev, femh_solve_rhs_dev,
                                            and servers without batch_rhs); the other precisions and the
                                            batched solver return FEMH_E_INVALID.  The factor is built on
                                            the device at the first such solve and kept with the problem
                                            (FEMH_E_BREAKDOWN if a pivot vanishes). */
} femh_precond;

/* Device memory provider.  alloc returns a device pointer of at least
 * `bytes` bytes (NULL on failure) usable on the context's stream; free
 * releases it.  A NULL femh_allocator means hipMalloc/hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} femh_allocator;

/* Problem statement of section 2: a box [origin, origin + (nx hx, ny hy,
 * nz hz)] of nx*ny*nz hexahedra. */
typedef struct {
  int32_t nx, ny, nz;          /* elements per axis, >= 1 */
  double h[3];                 /* element size per axis, > 0 */
  double origin[3];            /* minimum corner */
  const femh_c128* eps_r;      /* [nz][ny][nx] relative permittivity, nonzero; NULL = 1 */
  const femh_c128* mu_r;       /* [nz][ny][nx] relative permeability; NULL = 1 */
  const uint8_t* pec;          /* [nz][ny][nx], nonzero = element is PEC (removed); NULL = none */
  int32_t outer_face[6];       /* FEMH_FACE_* per outer face */
  double k0;                   /* free-space wavenumber, > 0 */
  double penalty_s;            /* grad-div penalty weight s >= 0 (eq. (2) gives none); 0 selects 1 */
  int32_t arrays_on_device;    /* 1: eps_r, mu_r, pec are device pointers, 0: host pointers */
  int32_t penalty_surface;     /* 0 (default): the penalty's surface integral of eq. (4) is dropped, and the matrix
                                  is complex-symmetric by construction.  1: that integral is assembled as printed,
                                  -s int (W . n)(div H) dS over the ABC outer faces and the faces between active
                                  and PEC elements, and the matrix is then averaged with its transpose as section
                                  3.1.4 does (A + (S + S^T) / 2; the right-hand side unchanged).  The paper-literal
                                  variant, for comparison: it no longer reproduces the incident wave in an empty
                                  box.  Not combined with symmetry or antisymmetry faces (FEMH_E_INVALID). */
} femh_problem_desc;

/* Incident plane wave H_i(r) = p exp(-j k0 d . r): |d| = 1, p . d = 0
 * (within 1e-9).  p is the H polarisation. */
typedef struct {
  double d[3];
  femh_c128 p[3];
} femh_plane_wave;

/* Solver options; a zero-initialised struct selects the defaults shown. */
typedef struct {
  int32_t precision;     /* femh_precision; default FEMH_FP64 */
  int32_t precond;       /* femh_precond; default Jacobi */
  double rtol;           /* stop at ||b - A x||_2 <= rtol ||b||_2 (FP64 true residual); default 1e-6 */
  int32_t max_iter;      /* Krylov iterations in total (inner ones for MIXED); default 200000 */
  int32_t precond_block; /* FEMH_PRECOND_BIC0: nodes per block, 1..512; default 4 (ignored otherwise) */
  double inner_rtol;     /* MIXED*: residual reduction between reliable updates; default 0.1
                            (FEMH_MIXED), 1e-3 (FEMH_MIXED_MATRIX) */
  int32_t max_outer;     /* MIXED: refinement steps; default 20 */
  int32_t check_every;   /* iterations queued between host convergence reads; default 32 */
} femh_solve_opts;

typedef struct {
  int32_t status;             /* femh_status of this right-hand side */
  int32_t iters;              /* Krylov iterations (inner ones for MIXED) */
  int32_t outer_iters;        /* refinement steps (MIXED), restarts (FP64) */
  int32_t reserved;
  double rel_residual;        /* final FP64 ||b - A x||_2 / ||b||_2 */
  double seconds;             /* device time of the solve (HIP events) */
} femh_solve_stats;

typedef struct {
  int64_t grid_nodes;         /* (nx+1)(ny+1)(nz+1) */
  int64_t n_nodes;            /* active nodes (block rows) */
  int64_t n_unknowns;         /* 3 * n_nodes */
  int64_t nnzb;               /* stored 3x3 blocks */
  int64_t device_bytes;       /* device memory held by the problem */
} femh_problem_info;

typedef struct femh_ctx femh_ctx;
typedef struct femh_problem femh_problem;
typedef struct femh_server femh_server;

/* ------------------------------------------------------------ context */

/* Open a context on HIP device `device` (must be gfx950).  `alloc` may be
 * NULL; `hip_stream` is a hipStream_t to launch on, or NULL for a stream
 * the context creates (default priority).  *out receives the handle. */
int femh_ctx_create(int device, const femh_allocator* alloc, void* hip_stream, femh_ctx** out);
void femh_ctx_destroy(femh_ctx* ctx);

/* Message of the calling thread's last failing call ("" if none).  The
 * string stays valid until the thread's next femh call. */
const char* femh_last_error(void);

/* Library version as major * 10000 + minor * 100 + patch. */
int femh_version(void);

/* ------------------------------------------------------ host-only checks */

/* Check a descriptor without touching the device: sizes, finite values,
 * face tags, eps_r != 0, k0 > 0, s >= 0; host arrays are scanned for
 * NaN/Inf.  Writes a message into msg[0..n) when it fails. */
int femh_validate_desc(const femh_problem_desc* desc, char* msg, size_t n);

/* Device bytes a problem plus the vectors of an nrhs-column solve of the
 * given precision will need.  Exact when the PEC mask is on the host, an
 * upper bound when it is on the device. */
int femh_estimate_bytes(const femh_problem_desc* desc, int32_t nrhs, int32_t precision,
                        int64_t* bytes);

/* Check incident waves: |d| = 1, p . d = 0, finite. */
int femh_validate_waves(int32_t nrhs, const femh_plane_wave* waves, char* msg, size_t n);

/* ---------------------------------------------------------- problems */

/* Number the active nodes, build the block pattern and assemble the
 * matrix (eqs. (1)-(4)) on the device: FP64 blocks, their complex64
 * rounding, and the Jacobi diagonal inverse.  Section 3.1.2's assembly by
 * degree of freedom is kept: every block row is computed by its owner from
 * the elements around the node, with no atomics and no symbolic phase on
 * the host. */
int femh_problem_create(femh_ctx* ctx, const femh_problem_desc* desc, femh_problem** out);
int femh_problem_get_info(const femh_problem* prob, femh_problem_info* info);
void femh_problem_destroy(femh_problem* prob);

/* A problem made from an already assembled matrix instead of a mesh: the
 * global system of section 3 in 3x3 block CSR form, so that the solver of
 * section 3.1.5 (Jacobi-preconditioned conjugate gradients read as COCG)
 * and its products can run on a matrix built elsewhere (an oracle, another
 * assembler).  nb block rows; row_ptr[nb + 1] with row_ptr[0] = 0 and
 * row_ptr[nb] = nnzb; col_idx[nnzb] strictly ascending within each row,
 * every row holding its diagonal block and at most 27 blocks (the
 * neighbourhood of a hexahedral-mesh node); vals[nnzb][3][3] complex128,
 * row-major blocks.  Host pointers, copied before the call returns.  The
 * complex64 values are the round-to-nearest copy, the Jacobi inverse is
 * 1 / the diagonal entries.  The problem has no mesh: femh_solve,
 * femh_solve_dev, femh_solve_batched_dev and femh_export_rhs return
 * FEMH_E_INVALID for it; femh_solve_rhs_dev, the products and the other
 * export hooks work (grid_nodes reads 0).  Errors: FEMH_E_INVALID for a
 * malformed pattern or a zero diagonal entry, FEMH_E_NONFINITE for a
 * NaN/Inf value, FEMH_E_OOM. */
int femh_import_bsr(femh_ctx* ctx, int64_t nb, int64_t nnzb, const int32_t* row_ptr, const int32_t* col_idx,
                    const femh_c128* vals, femh_problem** out);

/* Solve for nrhs incident waves.  H_out (host) receives
 * [nrhs][nz+1][ny+1][nx+1][3] complex128 total-field values at the grid
 * nodes (0 at nodes of PEC elements only); stats (host) receives nrhs
 * entries.  Returns FEMH_OK when every right-hand side converged, else the
 * first failing status; failed columns still hold their best iterate. */
int femh_solve(femh_problem* prob, int32_t nrhs, const femh_plane_wave* waves,
               const femh_solve_opts* opts, femh_c128* H_out, femh_solve_stats* stats);

/* As femh_solve, with H_out a device pointer of the same layout. */
int femh_solve_dev(femh_problem* prob, int32_t nrhs, const femh_plane_wave* waves,
                   const femh_solve_opts* opts, femh_c128* H_out_dev, femh_solve_stats* stats);

/* Solve A x = b for nrhs given right-hand sides (section 3.1.5's solver
 * on the assembled system, without the right-hand side of eq. (4) or the
 * grid scatter): b_dev and x_dev are device arrays [nrhs][n_unknowns]
 * complex128 in compact unknown order (3 * node + component); x_dev is
 * overwritten (the iteration starts from x = 0).  Each column runs the
 * single-right-hand-side solver of opts->precision, exactly as femh_solve
 * does for the assembled right-hand side.  Statuses as femh_solve. */
int femh_solve_rhs_dev(femh_problem* prob, int32_t nrhs, const femh_c128* b_dev, const femh_solve_opts* opts,
                       femh_c128* x_dev, femh_solve_stats* stats);

/* Batched right-hand sides: the nrhs (<= 64) columns advance together,
 * one block-sparse matrix times dense block (SpMM) per iteration, each
 * column with its own COCG scalars (section 3.1.5's conjugate gradient with
 * Jacobi preconditioning, applied per column).  Every column's iterate,
 * residual, direction and product are FP64.  opts->precision FEMH_FP64 (the
 * default) multiplies by the complex128 matrix; FEMH_MIXED and
 * FEMH_MIXED_MATRIX multiply by the complex64 matrix promoted inside FP64
 * products, with reliable updates against the FP64 matrix to opts->rtol.
 * opts->inner_rtol (default 1e-3) is the residual drop that triggers a
 * column's update (its true residual replaces the recurrence's).
 * Up to four right-hand sides use a narrow [n_unknowns][4] layout whose
 * product reads each matrix value once for all columns; five to eight run
 * as two such groups (four and the rest) stepped together, each column's
 * result identical to solving its group alone; more use the
 * [n_unknowns][64] layout.  Device memory: five complex128 blocks of that
 * layout.  H_out_dev as in femh_solve_dev. */
int femh_solve_batched_dev(femh_problem* prob, int32_t nrhs, const femh_plane_wave* waves,
                           const femh_solve_opts* opts, femh_c128* H_out_dev,
                           femh_solve_stats* stats);

/* ---------------------------------------------- inspection / bench hooks */

/* Copy the assembled FP64 matrix to host buffers: row_ptr[n_nodes + 1],
 * col_idx[nnzb] (ascending within a row), vals[nnzb][3][3] row-major
 * blocks.  Any pointer may be NULL to skip it. */
int femh_export_bsr(const femh_problem* prob, int32_t* row_ptr, int32_t* col_idx, femh_c128* vals);

/* Copy the complex64 matrix values [nnzb][3][3] (interleaved floats). */
int femh_export_bsr_c64(const femh_problem* prob, float* vals);

/* Right-hand sides of eq. (4) for nrhs waves, host buffer
 * [nrhs][n_unknowns] complex128. */
int femh_export_rhs(femh_problem* prob, int32_t nrhs, const femh_plane_wave* waves, femh_c128* b);

/* Jacobi diagonal inverse, host buffer [n_unknowns] complex128. */
int femh_export_jacobi(const femh_problem* prob, femh_c128* dinv);

/* The factor L of FEMH_PRECOND_BIC0 for blocks of nodes_per_block nodes
 * (eq. (5) inside each block), built on the device if the problem does not
 * hold it yet: scalar CSR over the n_unknowns rows, row_ptr[n_unknowns + 1],
 * col_idx[nnz] and vals[nnz] complex128, columns ascending within a row and
 * the diagonal entry last.  *nnz receives the entry count; with row_ptr,
 * col_idx and vals all NULL only the count is returned (call once to size
 * the buffers, then again to fill them).  Host pointers.  Errors:
 * FEMH_E_INVALID (nodes_per_block outside 1..512, NULL prob or nnz, or
 * more than 2^31 - 1 scalar entries in A, the range of the factor's 32-bit
 * row starts), FEMH_E_BREAKDOWN (a pivot vanished or is not finite),
 * FEMH_E_OOM. */
int femh_export_bic0(femh_problem* prob, int32_t nodes_per_block, int64_t* nnz, int32_t* row_ptr, int32_t* col_idx,
                     femh_c128* vals);

/* z = (L L^T)^-1 r with the FEMH_PRECOND_BIC0 factor for blocks of
 * nodes_per_block nodes (eq. (6)'s forward and back substitution inside
 * each block), the factor built if the problem does not hold it yet.  r_dev
 * and z_dev are device arrays [n_unknowns] complex128 (distinct).  The
 * application runs `reps` >= 1 times; *avg_seconds (may be NULL) receives
 * the mean kernel time measured with HIP events on the context's stream.
 * Errors as femh_export_bic0. */
int femh_bic0_apply_dev(femh_problem* prob, int32_t nodes_per_block, const femh_c128* r_dev, femh_c128* z_dev,
                        int32_t reps, double* avg_seconds);

/* y = A x on device vectors of n_unknowns complex entries: complex128 for
 * FEMH_FP64, complex64 with FP32 accumulation for FEMH_MIXED, the complex64
 * matrix times complex128 vectors for FEMH_MIXED_MATRIX.  The product
 * runs `reps` >= 1 times; *avg_seconds (may be NULL) receives the mean
 * kernel time measured with HIP events on the context's stream. */
int femh_spmv_dev(femh_problem* prob, int32_t precision, const void* x_dev, void* y_dev,
                  int32_t reps, double* avg_seconds);

/* As femh_spmv_dev with host vectors x, y [n_unknowns] complex128: for
 * FEMH_MIXED x is rounded to complex64 on the host, the complex64 product
 * runs on the device and y is widened back; the other precisions take the
 * complex128 vectors as they are.  The timing covers the device products
 * only, not the copies. */
int femh_spmv(femh_problem* prob, int32_t precision, const femh_c128* x, femh_c128* y, int32_t reps,
              double* avg_seconds);

/* Y = A X for ncols (1..64) columns: X and Y complex128 device arrays
 * [n_unknowns][ncols] (column index fastest), the batched solver's wide
 * product.  precision FEMH_FP64: the complex128 matrix, FP64 arithmetic;
 * FEMH_MIXED_MATRIX: the complex64 matrix promoted inside FP64 arithmetic,
 * or FP32 matrix-core products per 3x3 block summed in FP64 when tile kind
 * 1 is set (complex64 matrix whatever precision says).  Timing as
 * femh_spmv_dev. */
int femh_spmm_dev(femh_problem* prob, int32_t precision, int32_t ncols, const void* X_dev, void* Y_dev,
                  int32_t reps, double* avg_seconds);

/* y = A x (complex128) from the symmetric half store: the matrix is
 * complex-symmetric block by block (A_ba = A_ab^T), so each block row keeps
 * only its blocks with column <= row (the analogue of the paper's storage
 * #1, section 4.2) and reads the others transposed from the rows that store
 * them.  The store (about 52 % of the blocks plus an int32 per block) is
 * built on the first call and kept with the problem.  Timing as
 * femh_spmv_dev. */
int femh_spmv_half_dev(femh_problem* prob, const void* x_dev, void* y_dev, int32_t reps, double* avg_seconds);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): Y = A X
 * exactly as femh_spmm_dev with ncols = 64 (X, Y device arrays
 * [n_unknowns][64] complex128, column fastest; the same kernel, the
 * problem's tuned grid or, before any tuning, the default one, so Y is the
 * same bit for bit), but the product's partial sums and scalar block live in
 * a static device array of 4 MiB + 64 KiB that each GPU holds until the
 * process ends, and the call allocates nothing.  Only ncols = 64 is taken
 * (FEMH_E_INVALID otherwise): the narrower layouts need a staging copy.
 * Every call on one GPU shares that GPU's array, so calls that overlap on
 * one GPU (two threads, two streams) race: serialise them.  Returns after
 * the product has completed on the context's stream; no timing. */
int femh_spmm_noalloc_dev(femh_problem* prob, int32_t precision, int32_t ncols, const void* X_dev, void* Y_dev);

/* The wide SpMM shape the batched solver uses for this problem: *kind = 0
 * FP64 vector FMAs (the only kind the autotuner times, over grid sizes, on
 * the problem's first wide product, with that product's matrix), 1
 * matrix cores (FP32 products per 3x3 block; only when set explicitly), -1
 * not tuned yet; *blocks = workgroups of the launch. */
int femh_spmm_tile(const femh_problem* prob, int32_t* kind, int32_t* blocks);

/* Override the autotuner's choice (kind 0 or 1; blocks a positive multiple
 * of 8, at most 2048), e.g. to replay a shape tuned offline.  Kind 1 is
 * for well-conditioned systems: on indefinite ones its FP32 products can
 * stall the batched recurrence. */
int femh_spmm_set_tile(femh_problem* prob, int32_t kind, int32_t blocks);

/* Streaming copy of `bytes` bytes between two device buffers the library
 * allocates, `reps` times; *gbps receives (read + write bytes) / mean time.
 * The denominator for achieved-bandwidth figures. */
int femh_bw_probe(femh_ctx* ctx, int64_t bytes, int32_t reps, double* gbps);

/* Per-kernel event timing of the single-RHS solvers.  When enabled, every
 * solve records HIP events around every eighth matrix product it launches
 * (a sample, so that the events barely slow the solve being measured); the
 * totals accumulate until read.  spmv_seconds / spmv_launches receive the
 * sum of kernel times and the number of timed products that did work, per
 * kind (index 0 = FP64, 1 = complex64, 3 = complex64 matrix with complex128
 * vectors; index 2 stays 0: the batched SpMM is timed by femh_spmm_dev). */
int femh_profile_enable(femh_ctx* ctx, int32_t on);
int femh_profile_read(femh_ctx* ctx, double spmv_seconds[4], int64_t spmv_launches[4],
                      int32_t reset);

/* --------------------------------------------------------------- serving */

typedef struct {
  int64_t hbm_budget_bytes;   /* admission limit on resident problem bytes; 0 = 80 % of free */
  int32_t max_slots;          /* resident requests at once; 0 = 32 */
  int32_t chunk_iters;        /* iterations per slot per scheduling round; 0 = 32 */
  int32_t batch_rhs;          /* 1: a request's waves are solved in groups of up to four, one
                                 batched solve each (as femh_solve_batched_dev: FP64 directions,
                                 the complex128 matrix for FEMH_FP64, else the complex64 one);
                                 0: one single-RHS solve per wave (as femh_solve) */
  int32_t reserved;           /* must be 0 (FEMH_E_INVALID otherwise) */
} femh_server_opts;

typedef struct {
  int64_t submitted, completed, failed, cancelled, rejected;
  int64_t rhs_completed;
  double p50_seconds, p99_seconds;      /* submit -> result ready latency */
  double requests_per_second;           /* completed / span of first submit .. last completion */
  double rhs_per_second;
  int64_t peak_resident_bytes;
} femh_server_report;

/* A continuous-batching request loop on its own host thread: submitted
 * requests are admitted as memory (budget) and slots free up, assembled on
 * the device, and advanced in rounds of chunk_iters iterations interleaved
 * with every other resident request; finished requests retire and free
 * their memory at once. */
int femh_server_create(femh_ctx* ctx, const femh_server_opts* opts, femh_server** out);

/* Queue a request.  All inputs are copied (host pointers only).  A request
 * whose estimated footprint exceeds the whole budget is rejected with
 * FEMH_E_OOM.  *ticket identifies it.  Thread-safe. */
int femh_server_submit(femh_server* srv, const femh_problem_desc* desc, int32_t nrhs,
                       const femh_plane_wave* waves, const femh_solve_opts* opts,
                       uint64_t* ticket);

/* Wait up to timeout_ms (0 = do not wait, < 0 = forever) for a request.
 * On completion copies [nrhs][nz+1][ny+1][nx+1][3] into H_out (host, may be
 * NULL) and nrhs stats, forgets the ticket and returns the request's
 * status; FEMH_E_PENDING if still running.  Thread-safe. */
int femh_server_poll(femh_server* srv, uint64_t ticket, int32_t timeout_ms, femh_c128* H_out,
                     femh_solve_stats* stats);

/* Cancel a request; its slot and memory are released at the next round.
 * Other requests are unaffected.  Thread-safe. */
int femh_server_cancel(femh_server* srv, uint64_t ticket);

int femh_server_report_get(femh_server* srv, femh_server_report* out);

/* Stop the loop (pending requests are cancelled) and free everything. */
void femh_server_destroy(femh_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* FEMH_H */
