// Internal declarations of the femh library: device-side problem layout,
// solver scalar blocks, and the launchers the host code calls.  Kernels live
// in the .hip files; host orchestration in the .cpp files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "femh.h"

namespace femh {

// ----------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

// ------------------------------------------------------------------ log
// FEMH_LOG (environment, read once): 1 logs problem and factor builds, the
// end of every solve segment (recursive and true residual, the action
// taken) and the server's admissions; 2 also logs each chunk of iterations
// as its scalars are read back (a residual history at chunk granularity).
// Lines go to stderr, prefixed "[femh]".
int log_level();
void logf(int level, const char* fmt, ...);

#define FEMH_TRY_HIP(call)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      ::femh::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__,    \
                        __LINE__);                                                           \
      return FEMH_E_DEVICE;                                                                  \
    }                                                                                        \
  } while (0)

#define FEMH_TRY(call)            \
  do {                            \
    int s_ = (call);              \
    if (s_ != FEMH_OK) return s_; \
  } while (0)

// Faces: index f -> axis f / 2, side f % 2 (0 = minimum coordinate).
inline int face_axis(int f) { return f >> 1; }
inline int face_side(int f) { return f & 1; }

// ------------------------------------------------- device view of a problem
// Plain struct passed by value to kernels.
struct MeshDev {
  int nx, ny, nz;            // elements per axis
  double h[3], origin[3];
  double k0, s;
  int abc_mask;              // bit f set = outer face f carries the ABC
  int sym_mask;              // bit f set = outer face f is a symmetry plane (n . H = 0)
  int anti_mask;             // bit f set = outer face f is an antisymmetry plane (n x H = 0)
  int penalty_surface;       // 1: add the printed penalty surface term, averaged with its transpose
  const double2* eps;        // [ne] or null (= 1)
  const double2* mu;         // [ne] or null (= 1)
  const uint8_t* pec;        // [ne] or null (= none)
};

struct PatternDev {
  int32_t nn;                // active nodes = block rows
  int64_t nnzb;
  const int32_t* node_id;    // [grid nodes] -> active id or -1
  const int32_t* node_grid;  // [nn] -> grid node index
  const uint32_t* nbr_mask;  // [nn] 27-bit neighbour mask, bit = (dz+1)*9 + (dy+1)*3 + (dx+1)
  const int32_t* row_ptr;    // [nn + 1]
  const int32_t* col_idx;    // [nnzb]
  const int32_t* row_order;  // [nn] block-row order of the wide SpMM, or null (built on its first use)
};

// Block incomplete Cholesky factor (blocks of nodes_per_block consecutive
// nodes): L as scalar CSR (columns ascending, diagonal last), U = the strict
// upper part of L^T as scalar CSR, and 1 / l_uu.  Device pointers.
constexpr int kBicMaxNodesPerBlock = 512;
struct BicFactorDev {
  int64_t n = 0;               // unknowns (3 nn)
  int32_t rows_per_block = 0;  // 3 nodes_per_block
  int32_t nblk = 0;
  int32_t chunk_cap = 0;       // entries the application stages at a time (>= the longest row of L and U)
  const int32_t* lrp = nullptr;  // [n + 1]
  const int32_t* lcol = nullptr;
  const double2* lval = nullptr;
  const int32_t* urp = nullptr;  // [n + 1]
  const int32_t* ucol = nullptr;
  const double2* uval = nullptr;
  const double2* ldinv = nullptr;  // [n]
};

// COCG scalar block of one right-hand side, kept on the device so the
// host never waits inside an iteration.  Values that the iteration kernels
// both read and write are kept in two slots indexed by the parity of the
// iteration (a kernel argument), so no workgroup of a launch can observe a
// value another workgroup of the same launch writes.  Complex as double2.
struct CocgScalars {
  double2 rho[2];      // r^T z of the current iterate (single-reduction form: p^T A p of
                       // the last step), slot = parity
  double2 alpha, beta; // last step (beta also feeds cocg_pupdate_*)
  double rr;           // ||r||^2 after the last iteration (host view)
  double bb;           // ||b||^2 of the system being solved
  double tol2;         // stop when rr <= tol2 * bb
  double bd_tol;       // breakdown threshold (relative)
  double rr_max[2];    // largest ||r||^2 since the last reliable update, slot = parity
  double delta2;       // > 0: stop with done = 4 once rr <= delta2 * rr_max
  int32_t iters[2];    // iterations done, slot = parity
  int32_t max_iters;   // stop (not converged) at this count
  int32_t done;        // 0 running, 1 converged, 2 iteration limit, 3 breakdown,
                       // 4 residual dropped by delta: reliable update due
  int32_t iters_out;   // iterations done (host view)
  int32_t stop_par;    // slot of rho_{k-1} when the recurrence stopped
  uint32_t ticket[4];  // last-block counters of the once-per-segment kernels
};

// Per-column COCG scalars of a batched solve (up to 64 columns).  done[c]:
// 0 running, 1 converged (recursive), 2 iteration limit, 3 breakdown,
// 4 reliable update due, 5 finished, 6 finished without converging,
// 7 finished by breakdown.
struct BatchScalars {
  double2 rho[64], pq[64], alpha[64], beta[64];
  double rr[64], rr_max[64], tol2[64];
  int32_t done[64];
  int32_t iters[64];
  int32_t active;     // columns with done == 0
  int32_t max_iters;
  uint32_t ticket;
  int32_t pad;
  double delta2;
  double bd_tol;
};

// Host-written plan of one reliable update.  action[c]: 0 none, 1 replace
// the residual and keep the direction, 2 replace the residual and restart
// the direction, 3 finish with final_state[c].
struct BatchPlan {
  int32_t action[64];
  int32_t final_state[64];
  double tol2[64];    // recursive tolerance (absolute ||r||^2)
};

// SpMM tile choice: kind 0 = vector FMAs, 1 = matrix cores (both 64
// columns), 2 = narrow product (4 columns); blocks = grid.
struct BatchTile {
  int kind;
  int blocks;
};

// --------------------------------------------------------------- launchers
namespace k {

// ---- batched right-hand sides ([n][ld] complex layout, ld = 4 or 64)
int batched_blocks_for(int32_t nn, int n_cu, int per_cu);
int batched_vec_blocks(int64_t n, int ld);
// per-column partial sums are FP64: partials hold [blocks][ld][4] doubles
// The matrix times FP64 directions: the complex128 values when val64 is not
// null, else the complex64 values promoted, FP64 products.  tile.kind 0:
// vector FMAs (ld 64), 1: matrix cores, FP32 products per block of the
// complex64 matrix (ld 64), 2: narrow product (ld 4)
hipError_t bspmm(hipStream_t st, const PatternDev& pt, const float2* val32, const double2* val64, const double2* P,
                 double2* Q, double* partials, const BatchScalars* sc, BatchTile tile);
hipError_t bred_alpha(hipStream_t st, const double* partials, int nblocks, int ld, BatchScalars* sc);
hipError_t bupdate(hipStream_t st, int64_t n, int ld, const double2* dinv, double2* X, double2* R, const double2* P,
                   const double2* Q, double* partials, int blocks, const BatchScalars* sc);
hipError_t bred_beta(hipStream_t st, const double* partials, int nblocks, int ld, BatchScalars* sc);
hipError_t bpupdate(hipStream_t st, int64_t n, int ld, const double2* dinv, const double2* R, double2* P, int blocks,
                    const BatchScalars* sc, const int32_t* only);
hipError_t bresidual64(hipStream_t st, const PatternDev& pt, int ld, const double2* val, const double2* X,
                       const double2* B, double2* R, double* partials, int blocks, double* rr64,
                       const int32_t* mask);
hipError_t brescale(hipStream_t st, int64_t n, int ld, const double2* R, const double2* dinv, double2* P,
                    double* partials, int blocks, BatchScalars* sc, const BatchPlan* plan);
// Minimal-residual step (x += omega p, r -= omega A p, omega = (Ap)^H r /
// |Ap|^2) for the columns with plan->action == 2, whose P holds D^-1 r;
// run_all is a scalar block with active = 1 so the product always runs.
hipError_t bmr_step(hipStream_t st, const PatternDev& pt, int64_t n, int ld, const float2* val32,
                    const double2* val64, double2* X,
                    double2* R, const double2* P, double2* Q, double* partials, int blocks, BatchTile tile,
                    const BatchScalars* run_all, BatchScalars* sc, const BatchPlan* plan);
hipError_t to_block(hipStream_t st, int64_t n, int ld, int nrhs, const double2* b, double2* B);
// a scalar block that lets the products run (active = 1), written on the device
hipError_t product_scalars(hipStream_t st, BatchScalars* sc);
hipError_t from_block(hipStream_t st, int64_t n, int ld, int nrhs, const double2* X, double2* x);

// Exclusive prefix sum of n int32 (n >= 0); *total (device) gets the sum.
// tmp must hold scan_tmp_ints(n) ints.
int64_t scan_tmp_ints(int64_t n);
hipError_t exclusive_scan(hipStream_t st, const int32_t* in, int32_t* out, int64_t n,
                          int32_t* tmp, int32_t* total);

hipError_t check_materials(hipStream_t st, const double2* eps, const double2* mu, int64_t ne,
                           int32_t* flag);
hipError_t node_flags(hipStream_t st, const MeshDev& m, int32_t* flags);
hipError_t node_compact(hipStream_t st, const MeshDev& m, const int32_t* flags,
                        const int32_t* scan, int32_t* node_id, int32_t* node_grid);
hipError_t row_masks(hipStream_t st, const MeshDev& m, int32_t nn, const int32_t* node_id,
                     const int32_t* node_grid, uint32_t* mask, int32_t* counts);
hipError_t assemble(hipStream_t st, const MeshDev& m, const PatternDev& p, int32_t* col_idx,
                    double2* val64, float2* val32, double2* dinv64, float2* dinv32);
hipError_t rhs(hipStream_t st, const MeshDev& m, const PatternDev& p, int32_t nrhs,
               const femh_plane_wave* waves_dev, double2* b);
hipError_t scatter(hipStream_t st, const MeshDev& m, const PatternDev& p, int32_t nrhs,
                   const double2* x, double2* out);
hipError_t copy_probe(hipStream_t st, const float4* src, float4* dst, int64_t n);
// imported matrices: complex64 rounding of the values, and the Jacobi
// inverse from the diagonal blocks (*bad = 1 on a zero diagonal entry)
hipError_t round_c64(hipStream_t st, int64_t n, const double2* v64, float2* v32);
hipError_t dinv_from_blocks(hipStream_t st, int32_t nn, const int32_t* row_ptr, const int32_t* col_idx,
                            const double2* val64, double2* dinv64, float2* dinv32, int32_t* bad);

// ---- Krylov kernels
struct SpmvLaunch {
  int blocks;       // multiple of 8 (one share per XCD)
};
SpmvLaunch spmv_launch_for(int32_t nn, int n_cu);

// Symmetric half store: hpos[nnzb] per block slot (stored index, or
// -(index + 1) for the transpose of a stored block), hval[stored][9].
hipError_t spmv_half_c128(hipStream_t st, const PatternDev& p, const double2* hval, const int32_t* hpos,
                          const double2* x, double2* y, SpmvLaunch L);
hipError_t gather_half(hipStream_t st, int64_t nnzb, const int32_t* hpos, const double2* val, double2* hval);
hipError_t spmv_c128(hipStream_t st, const PatternDev& p, const double2* val, const double2* x,
                     double2* y, SpmvLaunch L);
hipError_t spmv_c64(hipStream_t st, const PatternDev& p, const float2* val, const float2* x,
                    float2* y, SpmvLaunch L);

// complex64 matrix times complex128 vector (values promoted, FP64 sums)
hipError_t spmv_m32(hipStream_t st, const PatternDev& p, const float2* val, const double2* x,
                    double2* y, SpmvLaunch L);

// COCG building blocks.  One iteration = spmv_dot (q = A p, per-workgroup
// partials of p^T q), update (every workgroup re-reduces those partials in
// a fixed order for alpha; x += alpha p, r -= alpha q; partials of r^T z,
// ||r||^2) and pupdate (re-reduces them: convergence / limit / breakdown /
// reliable-update decisions, beta, p = z + beta p).  `par` is the parity of
// the iteration (the host counts the iterations it queues); segment-start
// kernels write slot `par` of the iteration that follows them.  Partials
// hold 4 doubles per workgroup of the producing kernel.
hipError_t cocg_init_c128(hipStream_t st, int64_t n, const double2* b, const double2* dinv,
                          double2* x, double2* r, double2* p, CocgScalars* sc, void* partials,
                          int zero_x, int par);
hipError_t cocg_spmv_dot_c128(hipStream_t st, const PatternDev& pt, const double2* val,
                              const double2* p, double2* q, CocgScalars* sc, void* partials,
                              SpmvLaunch L);
hipError_t cocg_spmv_dot_m32(hipStream_t st, const PatternDev& pt, const float2* val,
                             const double2* p, double2* q, CocgScalars* sc, void* partials,
                             SpmvLaunch L);
hipError_t cocg_update_c128(hipStream_t st, int64_t n, const double2* dinv, double2* x,
                            double2* r, const double2* p, const double2* q, CocgScalars* sc,
                            const void* partials_in, int nin, void* partials_out, int par);
hipError_t cocg_pupdate_c128(hipStream_t st, int64_t n, const double2* dinv, const double2* r,
                             double2* p, CocgScalars* sc, const void* partials_in, int par);
// Single-reduction form of the FP64 COCG step: cocg_spmv_dot_c128 on z
// (w = A z, partials of z^T w) and sr_update_c128 make an iteration.
// sr_init: z = D^-1 r, p = s = 0, partials of r^T z, z^T s, ||r||^2,
// ||z||^2 into partials_out (8 values per workgroup, reduce_blocks_for(n)
// workgroups); slot par marks the first step.  sr_update: the step's scalars
// from the product's partials (partials_a, nin_a workgroups) and the previous
// update's or sr_init's (partials_b), then p, s, x, z and the next
// partials into partials_out, which must be a different buffer (the
// residual is carried as z; r is not written while iterating).
hipError_t sr_init_c128(hipStream_t st, int64_t n, const double2* r, const double2* dinv, double2* z,
                        double2* p, double2* s, CocgScalars* sc, void* partials_out, int par);
hipError_t sr_update_c128(hipStream_t st, int64_t n, const double2* dinv, double2* x, double2* z,
                          const double2* w, double2* p, double2* s, CocgScalars* sc,
                          const void* partials_a, int nin_a, const void* partials_b,
                          void* partials_out, int par);
// p = D^-1 r + beta p with beta from the scalar block (after a reliable update)
hipError_t cocg_apply_beta_c128(hipStream_t st, int64_t n, const double2* dinv, const double2* r,
                                double2* p, const CocgScalars* sc);

hipError_t cocg_spmv_dot_c64(hipStream_t st, const PatternDev& pt, const float2* val,
                             const float2* p, float2* q, CocgScalars* sc, void* partials,
                             SpmvLaunch L);
hipError_t cocg_update_c64(hipStream_t st, int64_t n, const float2* dinv, float2* x, float2* r,
                           const float2* p, const float2* q, CocgScalars* sc,
                           const void* partials_in, int nin, void* partials_out, int par);
hipError_t cocg_pupdate_c64(hipStream_t st, int64_t n, const float2* dinv, const float2* r,
                            float2* p, CocgScalars* sc, const void* partials_in, int par);
hipError_t cocg_apply_beta_c64(hipStream_t st, int64_t n, const float2* dinv, const float2* r,
                               float2* p, const CocgScalars* sc);
// workgroups of the update kernel (= partial count seen by pupdate)
int update_blocks_for(int64_t n);

// Reliable update of the complex64 recurrence: r = r64 * inv_s, z = D^-1 r;
// rho' = r^T z.  fresh = 1: p = z (restart).  fresh = 0: beta = rho' /
// (rho_{k-1} * ratio) for the direction kept in the old scaling (ratio =
// s_old / s_new); the caller then runs cocg_apply_beta_c64.  Writes slot
// `par`, sets tol2, clears done.
hipError_t cocg_rescale_c64(hipStream_t st, int64_t n, const double2* r64, double inv_s,
                            const float2* dinv, float2* r, float2* p, CocgScalars* sc,
                            void* partials, double ratio, double tol2, int fresh, int par);
// x64 += s * d32 and d32 = 0
hipError_t ir_fold(hipStream_t st, int64_t n, float2* d, double s, double2* x);
// FP64 reliable update after r was overwritten with the true residual:
// rho' = r^T D^-1 r, beta = rho' / rho_{k-1}; the caller runs
// cocg_apply_beta_c128.  Writes slot `par`.
hipError_t cocg_replace_c128(hipStream_t st, int64_t n, const double2* r, const double2* dinv,
                             CocgScalars* sc, void* partials, int par);

// r = b - A x (FP64) and ||r||^2 -> *rr_out (device), deterministic.
hipError_t residual_c128(hipStream_t st, const PatternDev& pt, const double2* val,
                         const double2* x, const double2* b, double2* r, double* partials,
                         uint32_t* ticket, double* rr_out, SpmvLaunch L);
// ||v||^2 of a device vector into *out (device), deterministic.
hipError_t norm2_c128(hipStream_t st, int64_t n, const double2* v, double* partials,
                      uint32_t* ticket, double* out);

int reduce_blocks_for(int64_t n);

// Block incomplete Cholesky (bic_kernels.hip).  Pattern: per-row entry
// counts of L, then columns and A's values at the scanned offsets; factor in
// place (one thread per block; *bad = 1 on a zero or non-finite pivot),
// writing ldinv; U from L (counts non-null: counts only, else fill at urp).
hipError_t bic_pattern_count(hipStream_t st, const PatternDev& p, int32_t nodes_per_block, int32_t* counts);
hipError_t bic_pattern_fill(hipStream_t st, const PatternDev& p, int32_t nodes_per_block, const double2* val,
                            const int32_t* lrp, int32_t* lcol, double2* lval);
hipError_t bic_factor(hipStream_t st, int64_t n, int32_t rows_per_block, int32_t nblk, const int32_t* lrp,
                      const int32_t* lcol, double2* lval, double2* ldinv, int32_t* bad);
hipError_t bic_upper(hipStream_t st, int64_t n, int32_t rows_per_block, const int32_t* lrp, const int32_t* lcol,
                     const double2* lval, int32_t* counts, const int32_t* urp, int32_t* ucol, double2* uval);
// z = (L L^T)^-1 r, one workgroup per block, then r^T z (re, im), ||r||^2,
// ||z||^2 summed in a fixed order into out[0..3] (stage: bic_stage_doubles
// doubles; ticket: a zeroed counter the launches leave zeroed).  Skipped
// when sc (may be null) has stopped.
size_t bic_stage_doubles(int32_t nblk);
hipError_t bic_apply(hipStream_t st, const BicFactorDev& f, const double2* r, double2* z, double* stage,
                     uint32_t* ticket, double* out, const CocgScalars* sc);
// Segment start from an application's totals: p = z, rho / ||r||^2 / start
// verdict into slot par.
hipError_t bic_init(hipStream_t st, int64_t n, const double2* z, double2* p, CocgScalars* sc, const double* sums,
                    int par);

}  // namespace k

// ------------------------------------------------------------- host objects
struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  femh_allocator alloc{};
  int n_cu = 256;
  bool profile = false;
  double prof_sec[4] = {0, 0, 0, 0};
  int64_t prof_cnt[4] = {0, 0, 0, 0};
  std::vector<hipEvent_t> ev_pool;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  void* pinned = nullptr;  // small pinned host buffer for scalar readback
  int64_t live_bytes = 0;
  void* scratch = nullptr;  // this device's copy of the allocation-free product's static scratch

  void* dmalloc(size_t bytes);
  void dfree(void* p);
};

struct Problem {
  Ctx* ctx = nullptr;
  MeshDev mesh{};
  PatternDev pat{};
  int faces[6] = {0, 0, 0, 0, 0, 0};
  int64_t grid_nodes = 0;
  // owned device memory
  double2* eps = nullptr;
  double2* mu = nullptr;
  uint8_t* pec = nullptr;
  int32_t* node_id = nullptr;
  int32_t* node_grid = nullptr;
  uint32_t* nbr_mask = nullptr;
  int32_t* row_ptr = nullptr;
  int32_t* col_idx = nullptr;
  double2* val64 = nullptr;
  float2* val32 = nullptr;
  double2* dinv64 = nullptr;
  float2* dinv32 = nullptr;
  int64_t dev_bytes = 0;
  k::SpmvLaunch spmv{};
  BatchTile tile{-1, 0};  // autotuned SpMM shape (kind -1 = not tuned yet)
  int32_t* row_order = nullptr;  // wide SpMM traversal order (device, [nn])
  int32_t* hpos = nullptr;        // symmetric half store: per block slot index (device, [nnzb])
  double2* hval64 = nullptr;      // symmetric half store values (device, [stored][9])
  int64_t n_half = 0;             // stored blocks
  bool imported = false;          // built by femh_import_bsr: pattern and values only, no mesh
  int32_t bic_nodes = 0;          // block incomplete Cholesky factor built for this block size (0: none)
  int64_t bic_nnz_l = 0;
  BicFactorDev bic{};
  std::vector<void*> bic_mem;     // the factor's device memory (freed on a rebuild)

  std::vector<void*> owned;
  void* alloc(size_t bytes);  // tracked allocation, freed with the problem
  ~Problem();
};

// Host-side helpers shared by the C API and the server.
int validate_desc(const femh_problem_desc* d, std::string& msg);
int validate_waves(int32_t nrhs, const femh_plane_wave* w, std::string& msg);
int64_t estimate_bytes(const femh_problem_desc* d, int32_t nrhs, int32_t precision);
// Extra device bytes of solving nrhs waves as batched groups of up to four.
int64_t estimate_batch_workspace(const femh_problem_desc* d, int32_t nrhs);
int problem_create(Ctx* ctx, const femh_problem_desc* d, Problem** out);
// A problem from a host block-CSR matrix (no mesh): validates the pattern,
// copies it and the complex128 values, derives the complex64 values and
// the Jacobi inverse.
int problem_import(Ctx* ctx, int64_t nb, int64_t nnzb, const int32_t* row_ptr, const int32_t* col_idx,
                   const femh_c128* vals, Problem** out);
femh_solve_opts opts_with_defaults(const femh_solve_opts* o);
// Options (after defaults) the solvers accept; batched: the columns of one
// batched solve (no block incomplete Cholesky there).
int check_solve_opts(const femh_solve_opts& o, bool batched, std::string& msg);
// Extra device bytes of FEMH_PRECOND_BIC0: the factor and, per right-hand
// side, the preconditioner's workspace.
int64_t estimate_bic_bytes(const femh_problem_desc* d, int32_t nrhs);

// Solve one right-hand side already assembled into b (device, FP64) into x
// (device, FP64).  Fills one stats entry.  Workspace is allocated inside.
int solve_single(Problem* P, const double2* b, double2* x, const femh_solve_opts& o,
                 femh_solve_stats* st);

// Batched solve of nrhs <= 64 right-hand sides b (device, [nrhs][n] FP64)
// into x (device, [nrhs][n] FP64): complex64 SpMM-COCG per column with
// per-column reliable updates into FP64.
int solve_batched(Problem* P, int nrhs, const double2* b, double2* x, const femh_solve_opts& o,
                  femh_solve_stats* st);
// Pick the SpMM tile for a problem (timed candidates), cached on the problem.
// Times the wide vector SpMM over grid sizes with the given matrix (val64
// non-null: complex128) unless the problem's tile is set; cached per (CU
// count, log2 of block rows, matrix precision).
int autotune_spmm(Problem* P, const double2* val64, const double2* Pv, double2* Qv, double* partials,
                  const BatchScalars* sc);
// Builds P->row_order (and P->pat.row_order) once per problem.
int ensure_row_order(Problem* P);
// Builds the symmetric half store (P->hpos, P->hval64) once per problem.
int ensure_half_store(Problem* P);
// Builds the block incomplete Cholesky factor for blocks of nodes_per_block
// nodes (kept until another block size is asked for).  FEMH_E_BREAKDOWN
// when a pivot vanishes or is not finite (no factor is kept).
int ensure_bic(Problem* P, int32_t nodes_per_block);

// Single-RHS solve as a non-blocking state machine (one code path for
// femh_solve and the server).  step() queues the work its phase allows and
// acts on readbacks that have landed; wait() blocks on the oldest one.
// Non-blocking batched solve of nrhs (<= 64) right-hand sides b (device,
// [nrhs][n]) into x: the state machine solve_batched drives to the end,
// and the serving loop interleaves with other requests.
struct BatchStepper;
BatchStepper* batch_stepper_create(Problem* P, int nrhs, const double2* b, double2* x, const femh_solve_opts& o);
int batch_stepper_step(BatchStepper* s, bool* progress);
bool batch_stepper_done(const BatchStepper* s);
void batch_stepper_wait(BatchStepper* s);
bool batch_stepper_iterating(const BatchStepper* s);  // past its set-up phases (iterating or done)
int batch_stepper_stats(const BatchStepper* s, femh_solve_stats* st);  // first failing status
void batch_stepper_destroy(BatchStepper* s);

struct Stepper;
Stepper* stepper_create(Problem* P, const double2* b, double2* x, const femh_solve_opts& o);
int stepper_step(Stepper* s, bool* progress);
bool stepper_done(const Stepper* s);
void stepper_wait(Stepper* s);
void stepper_stats(const Stepper* s, femh_solve_stats* st);
void stepper_destroy(Stepper* s);

}  // namespace femh
