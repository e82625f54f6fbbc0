// extern "C" entry points of libfemh (declared in include/femh.h).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using femh::Ctx;
using femh::Problem;

struct femh_ctx : Ctx {};
struct femh_problem : Problem {};

namespace femh {
const char* last_error();
}

namespace {

int copy_msg(const std::string& m, char* msg, size_t n) {
  if (msg && n) {
    std::strncpy(msg, m.c_str(), n - 1);
    msg[n - 1] = 0;
  }
  return 0;
}

// Static scratch of the allocation-free product (femh_spmm_noalloc_dev): the
// per-workgroup, per-column partial sums the wide product kernel writes (at
// most 2048 workgroups x 64 columns x 4 doubles) and one scalar block.  Each
// device holds its own copy until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returned for that device.
constexpr size_t kScratchPartials = (size_t)2048 * 64 * 4 * sizeof(double);
constexpr size_t kScratchBytes = kScratchPartials + 65536;
static_assert(sizeof(femh::BatchScalars) <= 65536, "scalar block exceeds its scratch slot");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// A pair of timing events, destroyed on every return path.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t create() {
    const hipError_t e = hipEventCreate(&a);
    return e != hipSuccess ? e : hipEventCreate(&b);
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

struct DevTmp {
  Ctx* c;
  void* p;
  DevTmp(Ctx* ctx, size_t bytes) : c(ctx), p(ctx->dmalloc(bytes)) {}
  ~DevTmp() {
    if (p) {
      (void)hipStreamSynchronize(c->stream);
      c->dfree(p);
    }
  }
};

}  // namespace

static int require_mesh(const femh_problem* prob) {
  if (prob->imported) {
    femh::set_error("the problem was imported as a matrix and has no mesh: solve with femh_solve_rhs_dev");
    return FEMH_E_INVALID;
  }
  return FEMH_OK;
}

static int check_opts(const femh_solve_opts& o, bool batched = false) {
  std::string m;
  const int st = femh::check_solve_opts(o, batched, m);
  if (st != FEMH_OK) femh::set_error("%s", m.c_str());
  return st;
}

extern "C" {

const char* femh_last_error(void) { return femh::last_error(); }

int femh_version(void) { return 10000; }

int femh_ctx_create(int device, const femh_allocator* alloc, void* hip_stream, femh_ctx** out) {
  femh::clear_error();
  if (!out) {
    femh::set_error("out is NULL");
    return FEMH_E_INVALID;
  }
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    femh::set_error("no HIP device available");
    return FEMH_E_DEVICE;
  }
  if (device < 0 || device >= count) {
    femh::set_error("device %d out of range (%d devices)", device, count);
    return FEMH_E_INVALID;
  }
  FEMH_TRY_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  FEMH_TRY_HIP(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    femh::set_error("device %d is %s; this library is built for gfx950 only", device, prop.gcnArchName);
    return FEMH_E_DEVICE;
  }
  // this device's copy of the allocation-free product's scratch (set-up,
  // once per context; the symbol's host-side name is not a device address)
  void* scratch_ptr = nullptr;
  FEMH_TRY_HIP(hipGetSymbolAddress(&scratch_ptr, HIP_SYMBOL(scratch)));
  femh_ctx* c = new femh_ctx();
  c->device = device;
  c->scratch = scratch_ptr;
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  if (alloc && alloc->alloc && alloc->free) c->alloc = *alloc;
  if (hip_stream) {
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      femh::set_error("hipStreamCreate failed");
      delete c;
      return FEMH_E_DEVICE;
    }
    c->own_stream = true;
  }
  if (hipHostMalloc(&c->pinned, 16384, hipHostMallocDefault) != hipSuccess) {
    femh::set_error("hipHostMalloc failed");
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return FEMH_E_DEVICE;
  }
  *out = c;
  return FEMH_OK;
}

void femh_ctx_destroy(femh_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int femh_validate_desc(const femh_problem_desc* desc, char* msg, size_t n) {
  femh::clear_error();
  std::string m;
  int st = femh::validate_desc(desc, m);
  copy_msg(m, msg, n);
  if (st != FEMH_OK) femh::set_error("%s", m.c_str());
  return st;
}

int femh_validate_waves(int32_t nrhs, const femh_plane_wave* waves, char* msg, size_t n) {
  femh::clear_error();
  std::string m;
  int st = femh::validate_waves(nrhs, waves, m);
  copy_msg(m, msg, n);
  if (st != FEMH_OK) femh::set_error("%s", m.c_str());
  return st;
}

int femh_estimate_bytes(const femh_problem_desc* desc, int32_t nrhs, int32_t precision, int64_t* bytes) {
  femh::clear_error();
  std::string m;
  int st = femh::validate_desc(desc, m);
  if (st != FEMH_OK) {
    femh::set_error("%s", m.c_str());
    return st;
  }
  if (!bytes || nrhs < 0 || (precision != FEMH_FP64 && precision != FEMH_MIXED && precision != FEMH_MIXED_MATRIX)) {
    femh::set_error("bad estimate arguments");
    return FEMH_E_INVALID;
  }
  *bytes = femh::estimate_bytes(desc, nrhs, precision);
  return FEMH_OK;
}

int femh_problem_create(femh_ctx* ctx, const femh_problem_desc* desc, femh_problem** out) {
  femh::clear_error();
  if (!ctx || !out) {
    femh::set_error("ctx and out must not be NULL");
    return FEMH_E_INVALID;
  }
  *out = nullptr;
  FEMH_TRY_HIP(hipSetDevice(ctx->device));
  Problem* P = nullptr;
  int st = femh::problem_create(ctx, desc, &P);
  if (st != FEMH_OK) return st;
  *out = static_cast<femh_problem*>(P);
  return FEMH_OK;
}

int femh_problem_get_info(const femh_problem* p, femh_problem_info* info) {
  if (!p || !info) {
    femh::set_error("NULL argument");
    return FEMH_E_INVALID;
  }
  info->grid_nodes = p->grid_nodes;
  info->n_nodes = p->pat.nn;
  info->n_unknowns = 3 * (int64_t)p->pat.nn;
  info->nnzb = p->pat.nnzb;
  info->device_bytes = p->dev_bytes;
  return FEMH_OK;
}

void femh_problem_destroy(femh_problem* p) {
  if (!p) return;
  (void)hipSetDevice(p->ctx->device);
  delete static_cast<Problem*>(p);
}

int femh_import_bsr(femh_ctx* ctx, int64_t nb, int64_t nnzb, const int32_t* row_ptr, const int32_t* col_idx,
                    const femh_c128* vals, femh_problem** out) {
  femh::clear_error();
  if (!ctx || !out) {
    femh::set_error("ctx and out must not be NULL");
    return FEMH_E_INVALID;
  }
  *out = nullptr;
  FEMH_TRY_HIP(hipSetDevice(ctx->device));
  Problem* P = nullptr;
  int st = femh::problem_import(ctx, nb, nnzb, row_ptr, col_idx, vals, &P);
  if (st != FEMH_OK) return st;
  *out = static_cast<femh_problem*>(P);
  return FEMH_OK;
}

int femh_solve_rhs_dev(femh_problem* prob, int32_t nrhs, const femh_c128* b_dev, const femh_solve_opts* opts,
                       femh_c128* x_dev, femh_solve_stats* stats) {
  femh::clear_error();
  if (!prob || !b_dev || !x_dev || !stats || nrhs < 1) {
    femh::set_error("prob, b, x and stats must not be NULL; nrhs >= 1");
    return FEMH_E_INVALID;
  }
  const femh_solve_opts o = femh::opts_with_defaults(opts);
  FEMH_TRY(check_opts(o));
  Ctx* c = prob->ctx;
  FEMH_TRY_HIP(hipSetDevice(c->device));
  const int64_t n = 3 * (int64_t)prob->pat.nn;
  int first_bad = FEMH_OK;
  for (int r = 0; r < nrhs; ++r) {
    int rc = femh::solve_single(prob, (const double2*)b_dev + r * n, (double2*)x_dev + r * n, o, &stats[r]);
    if (rc != FEMH_OK && rc != FEMH_E_NOT_CONVERGED && rc != FEMH_E_BREAKDOWN) return rc;
    if (rc != FEMH_OK && first_bad == FEMH_OK) first_bad = rc;
  }
  FEMH_TRY_HIP(hipStreamSynchronize(c->stream));
  return first_bad;
}

static int upload_waves(Ctx* c, int32_t nrhs, const femh_plane_wave* waves, DevTmp& dw) {
  if (!dw.p) {
    femh::set_error("device allocation failed (waves)");
    return FEMH_E_OOM;
  }
  FEMH_TRY_HIP(hipMemcpyAsync(dw.p, waves, sizeof(femh_plane_wave) * nrhs, hipMemcpyHostToDevice, c->stream));
  return FEMH_OK;
}

int femh_solve_dev(femh_problem* prob, int32_t nrhs, const femh_plane_wave* waves, const femh_solve_opts* opts,
                   femh_c128* H_out_dev, femh_solve_stats* stats) {
  femh::clear_error();
  if (!prob || !H_out_dev || !stats) {
    femh::set_error("prob, H_out and stats must not be NULL");
    return FEMH_E_INVALID;
  }
  FEMH_TRY(require_mesh(prob));
  std::string m;
  int st = femh::validate_waves(nrhs, waves, m);
  if (st != FEMH_OK) {
    femh::set_error("%s", m.c_str());
    return st;
  }
  const femh_solve_opts o = femh::opts_with_defaults(opts);
  FEMH_TRY(check_opts(o));
  Ctx* c = prob->ctx;
  FEMH_TRY_HIP(hipSetDevice(c->device));
  const int64_t n = 3 * (int64_t)prob->pat.nn;
  DevTmp dw(c, sizeof(femh_plane_wave) * nrhs);
  FEMH_TRY(upload_waves(c, nrhs, waves, dw));
  DevTmp db(c, 16 * n * nrhs), dx(c, 16 * n * nrhs);
  if (!db.p || !dx.p) {
    femh::set_error("device allocation failed (right-hand sides)");
    return FEMH_E_OOM;
  }
  double2* b = (double2*)db.p;
  double2* x = (double2*)dx.p;
  FEMH_TRY_HIP(femh::k::rhs(c->stream, prob->mesh, prob->pat, nrhs, (const femh_plane_wave*)dw.p, b));
  int first_bad = FEMH_OK;
  for (int r = 0; r < nrhs; ++r) {
    int rc = femh::solve_single(prob, b + r * n, x + r * n, o, &stats[r]);
    if (rc != FEMH_OK && rc != FEMH_E_NOT_CONVERGED && rc != FEMH_E_BREAKDOWN) return rc;
    if (rc != FEMH_OK && first_bad == FEMH_OK) first_bad = rc;
  }
  FEMH_TRY_HIP(femh::k::scatter(c->stream, prob->mesh, prob->pat, nrhs, x, (double2*)H_out_dev));
  FEMH_TRY_HIP(hipStreamSynchronize(c->stream));
  return first_bad;
}

int femh_solve(femh_problem* prob, int32_t nrhs, const femh_plane_wave* waves, const femh_solve_opts* opts,
               femh_c128* H_out, femh_solve_stats* stats) {
  femh::clear_error();
  if (!prob || !H_out || !stats || nrhs < 1) {
    femh::set_error("prob, H_out and stats must not be NULL; nrhs >= 1");
    return FEMH_E_INVALID;
  }
  FEMH_TRY(require_mesh(prob));
  Ctx* c = prob->ctx;
  const size_t bytes = sizeof(femh_c128) * 3 * (size_t)prob->grid_nodes * nrhs;
  DevTmp dh(c, bytes);
  if (!dh.p) {
    femh::set_error("device allocation failed (output)");
    return FEMH_E_OOM;
  }
  int rc = femh_solve_dev(prob, nrhs, waves, opts, (femh_c128*)dh.p, stats);
  if (rc != FEMH_OK && rc != FEMH_E_NOT_CONVERGED && rc != FEMH_E_BREAKDOWN) return rc;
  FEMH_TRY_HIP(hipMemcpyAsync(H_out, dh.p, bytes, hipMemcpyDeviceToHost, c->stream));
  FEMH_TRY_HIP(hipStreamSynchronize(c->stream));
  return rc;
}

int femh_solve_batched_dev(femh_problem* prob, int32_t nrhs, const femh_plane_wave* waves,
                           const femh_solve_opts* opts, femh_c128* H_out_dev, femh_solve_stats* stats) {
  femh::clear_error();
  if (!prob || !H_out_dev || !stats) {
    femh::set_error("prob, H_out and stats must not be NULL");
    return FEMH_E_INVALID;
  }
  if (nrhs < 1 || nrhs > 64) {
    femh::set_error("batched solve takes 1..64 right-hand sides (got %d)", nrhs);
    return FEMH_E_INVALID;
  }
  FEMH_TRY(require_mesh(prob));
  std::string m;
  int st = femh::validate_waves(nrhs, waves, m);
  if (st != FEMH_OK) {
    femh::set_error("%s", m.c_str());
    return st;
  }
  // FP64 directions and residuals in every case; FEMH_FP64 multiplies by
  // the complex128 matrix, any other precision by the complex64 matrix
  femh_solve_opts ob{};
  if (opts) ob = *opts;
  if (ob.precision != FEMH_FP64) ob.precision = FEMH_MIXED_MATRIX;
  // both recurrences are FP64: reliable updates every three decades
  if (ob.inner_rtol <= 0.0) ob.inner_rtol = 1e-3;
  const femh_solve_opts o = femh::opts_with_defaults(&ob);
  FEMH_TRY(check_opts(o, true));
  Ctx* c = prob->ctx;
  FEMH_TRY_HIP(hipSetDevice(c->device));
  const int64_t n = 3 * (int64_t)prob->pat.nn;
  DevTmp dw(c, sizeof(femh_plane_wave) * nrhs);
  FEMH_TRY(upload_waves(c, nrhs, waves, dw));
  DevTmp db(c, 16 * n * nrhs), dx(c, 16 * n * nrhs);
  if (!db.p || !dx.p) {
    femh::set_error("device allocation failed (right-hand sides)");
    return FEMH_E_OOM;
  }
  FEMH_TRY_HIP(femh::k::rhs(c->stream, prob->mesh, prob->pat, nrhs, (const femh_plane_wave*)dw.p, (double2*)db.p));
  int rc = femh::solve_batched(prob, nrhs, (const double2*)db.p, (double2*)dx.p, o, stats);
  if (rc != FEMH_OK && rc != FEMH_E_NOT_CONVERGED && rc != FEMH_E_BREAKDOWN) return rc;
  FEMH_TRY_HIP(femh::k::scatter(c->stream, prob->mesh, prob->pat, nrhs, (const double2*)dx.p, (double2*)H_out_dev));
  FEMH_TRY_HIP(hipStreamSynchronize(c->stream));
  return rc;
}

int femh_spmm_dev(femh_problem* p, int32_t precision, int32_t ncols, const void* X, void* Y, int32_t reps,
                  double* avg_seconds) {
  femh::clear_error();
  if (!p || !X || !Y || reps < 1 || ncols < 1 || ncols > 64 ||
      (precision != FEMH_FP64 && precision != FEMH_MIXED_MATRIX)) {
    femh::set_error("bad spmm arguments (precision FP64 or MIXED_MATRIX, 1 <= ncols <= 64, reps >= 1)");
    return FEMH_E_INVALID;
  }
  const double2* val64 = precision == FEMH_FP64 ? p->val64 : nullptr;
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  const int64_t n = 3 * (int64_t)p->pat.nn;
  const bool direct = ncols == 64;
  DevTmp xp(c, direct ? 16 : 16 * (size_t)n * 64), yp(c, direct ? 16 : 16 * (size_t)n * 64);
  DevTmp part(c, 2048 * 64 * 4 * sizeof(double)), scd(c, sizeof(femh::BatchScalars));
  if (!xp.p || !yp.p || !part.p || !scd.p) {
    femh::set_error("device allocation failed (spmm)");
    return FEMH_E_OOM;
  }
  const double2* Xd = (const double2*)X;
  double2* Yd = (double2*)Y;
  if (!direct) {
    FEMH_TRY_HIP(hipMemsetAsync(xp.p, 0, 16 * (size_t)n * 64, s));
    FEMH_TRY_HIP(hipMemcpy2DAsync(xp.p, 64 * 16, X, (size_t)ncols * 16, (size_t)ncols * 16, (size_t)n,
                                  hipMemcpyDeviceToDevice, s));
    Xd = (const double2*)xp.p;
    Yd = (double2*)yp.p;
  }
  femh::BatchScalars* hs = reinterpret_cast<femh::BatchScalars*>(c->pinned);
  std::memset(hs, 0, sizeof(*hs));
  hs->active = 1;
  FEMH_TRY_HIP(hipMemcpyAsync(scd.p, hs, sizeof(*hs), hipMemcpyHostToDevice, s));
  FEMH_TRY_HIP(hipStreamSynchronize(s));
  FEMH_TRY(femh::autotune_spmm(p, val64, Xd, Yd, (double*)part.p, (const femh::BatchScalars*)scd.p));
  EventPair ev;
  FEMH_TRY_HIP(ev.create());
  FEMH_TRY_HIP(hipEventRecord(ev.a, s));
  for (int i = 0; i < reps; ++i)
    FEMH_TRY_HIP(femh::k::bspmm(s, p->pat, p->val32, val64, Xd, Yd, (double*)part.p,
                                (const femh::BatchScalars*)scd.p, p->tile));
  FEMH_TRY_HIP(hipEventRecord(ev.b, s));
  FEMH_TRY_HIP(hipEventSynchronize(ev.b));
  float ms = 0;
  FEMH_TRY_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
  if (avg_seconds) *avg_seconds = ms * 1e-3 / reps;
  if (!direct)
    FEMH_TRY_HIP(hipMemcpy2DAsync(Y, (size_t)ncols * 16, yp.p, 64 * 16, (size_t)ncols * 16, (size_t)n,
                                  hipMemcpyDeviceToDevice, s));
  FEMH_TRY_HIP(hipStreamSynchronize(s));
  return FEMH_OK;
}

int femh_spmm_noalloc_dev(femh_problem* p, int32_t precision, int32_t ncols, const void* X, void* Y) {
  femh::clear_error();
  if (!p || !X || !Y || (precision != FEMH_FP64 && precision != FEMH_MIXED_MATRIX)) {
    femh::set_error("bad spmm arguments (precision FP64 or MIXED_MATRIX, X and Y non-NULL)");
    return FEMH_E_INVALID;
  }
  if (ncols != 64) {
    femh::set_error("the allocation-free product takes the [n_unknowns][64] layout only (got %d columns)", ncols);
    return FEMH_E_INVALID;
  }
  Ctx* c = p->ctx;
  if (!c->scratch) {
    femh::set_error("the context has no scratch address for its device");
    return FEMH_E_DEVICE;
  }
  FEMH_TRY_HIP(hipSetDevice(c->device));
  // the problem's tuned shape if it has one, else the untuned default (no
  // timing run: that would allocate events)
  femh::BatchTile t = p->tile.kind >= 0 ? p->tile : femh::BatchTile{0, femh::k::batched_blocks_for(p->pat.nn, c->n_cu, 8)};
  if (t.blocks < 8 || t.blocks > 2048) {
    femh::set_error("product grid of %d workgroups exceeds the scratch (at most 2048)", t.blocks);
    return FEMH_E_INVALID;
  }
  double* partials = reinterpret_cast<double*>(c->scratch);
  femh::BatchScalars* sc = reinterpret_cast<femh::BatchScalars*>(reinterpret_cast<char*>(c->scratch) + kScratchPartials);
  const double2* val64 = precision == FEMH_FP64 ? p->val64 : nullptr;
  FEMH_TRY_HIP(femh::k::product_scalars(c->stream, sc));
  FEMH_TRY_HIP(femh::k::bspmm(c->stream, p->pat, p->val32, val64, (const double2*)X, (double2*)Y, partials, sc, t));
  FEMH_TRY_HIP(hipStreamSynchronize(c->stream));
  return FEMH_OK;
}

int femh_spmm_tile(const femh_problem* p, int32_t* kind, int32_t* blocks) {
  if (!p || !kind || !blocks) {
    femh::set_error("NULL argument");
    return FEMH_E_INVALID;
  }
  *kind = p->tile.kind;
  *blocks = p->tile.blocks;
  return FEMH_OK;
}

int femh_spmm_set_tile(femh_problem* p, int32_t kind, int32_t blocks) {
  if (!p || (kind != 0 && kind != 1) || blocks < 8 || blocks > 2048 || blocks % 8) {
    femh::set_error("bad tile (kind 0/1, blocks a multiple of 8 in [8, 2048])");
    return FEMH_E_INVALID;
  }
  p->tile.kind = kind;
  p->tile.blocks = blocks;
  return FEMH_OK;
}

// ----------------------------------------------------------------- hooks
int femh_export_bsr(const femh_problem* p, int32_t* row_ptr, int32_t* col_idx, femh_c128* vals) {
  femh::clear_error();
  if (!p) {
    femh::set_error("prob is NULL");
    return FEMH_E_INVALID;
  }
  hipStream_t s = p->ctx->stream;
  FEMH_TRY_HIP(hipSetDevice(p->ctx->device));
  if (row_ptr) FEMH_TRY_HIP(hipMemcpyAsync(row_ptr, p->row_ptr, 4 * ((size_t)p->pat.nn + 1), hipMemcpyDeviceToHost, s));
  if (col_idx) FEMH_TRY_HIP(hipMemcpyAsync(col_idx, p->col_idx, 4 * (size_t)p->pat.nnzb, hipMemcpyDeviceToHost, s));
  if (vals) FEMH_TRY_HIP(hipMemcpyAsync(vals, p->val64, 144 * (size_t)p->pat.nnzb, hipMemcpyDeviceToHost, s));
  FEMH_TRY_HIP(hipStreamSynchronize(s));
  return FEMH_OK;
}

int femh_export_bsr_c64(const femh_problem* p, float* vals) {
  femh::clear_error();
  if (!p || !vals) {
    femh::set_error("NULL argument");
    return FEMH_E_INVALID;
  }
  hipStream_t s = p->ctx->stream;
  FEMH_TRY_HIP(hipMemcpyAsync(vals, p->val32, 72 * (size_t)p->pat.nnzb, hipMemcpyDeviceToHost, s));
  FEMH_TRY_HIP(hipStreamSynchronize(s));
  return FEMH_OK;
}

int femh_export_rhs(femh_problem* p, int32_t nrhs, const femh_plane_wave* waves, femh_c128* b) {
  femh::clear_error();
  if (!p || !b) {
    femh::set_error("NULL argument");
    return FEMH_E_INVALID;
  }
  FEMH_TRY(require_mesh(p));
  std::string m;
  int st = femh::validate_waves(nrhs, waves, m);
  if (st != FEMH_OK) {
    femh::set_error("%s", m.c_str());
    return st;
  }
  Ctx* c = p->ctx;
  const int64_t n = 3 * (int64_t)p->pat.nn;
  DevTmp dw(c, sizeof(femh_plane_wave) * nrhs);
  FEMH_TRY(upload_waves(c, nrhs, waves, dw));
  DevTmp db(c, 16 * n * nrhs);
  if (!db.p) {
    femh::set_error("device allocation failed");
    return FEMH_E_OOM;
  }
  FEMH_TRY_HIP(femh::k::rhs(c->stream, p->mesh, p->pat, nrhs, (const femh_plane_wave*)dw.p, (double2*)db.p));
  FEMH_TRY_HIP(hipMemcpyAsync(b, db.p, 16 * n * nrhs, hipMemcpyDeviceToHost, c->stream));
  FEMH_TRY_HIP(hipStreamSynchronize(c->stream));
  return FEMH_OK;
}

int femh_export_jacobi(const femh_problem* p, femh_c128* dinv) {
  femh::clear_error();
  if (!p || !dinv) {
    femh::set_error("NULL argument");
    return FEMH_E_INVALID;
  }
  FEMH_TRY_HIP(hipMemcpyAsync(dinv, p->dinv64, 48 * (size_t)p->pat.nn, hipMemcpyDeviceToHost, p->ctx->stream));
  FEMH_TRY_HIP(hipStreamSynchronize(p->ctx->stream));
  return FEMH_OK;
}

int femh_export_bic0(femh_problem* p, int32_t nodes_per_block, int64_t* nnz, int32_t* row_ptr, int32_t* col_idx,
                     femh_c128* vals) {
  femh::clear_error();
  if (!p || !nnz) {
    femh::set_error("prob and nnz must not be NULL");
    return FEMH_E_INVALID;
  }
  FEMH_TRY_HIP(hipSetDevice(p->ctx->device));
  FEMH_TRY(femh::ensure_bic(p, nodes_per_block));
  const int64_t n = 3 * (int64_t)p->pat.nn;
  const int64_t nz = p->bic_nnz_l;
  *nnz = nz;
  hipStream_t s = p->ctx->stream;
  if (row_ptr) FEMH_TRY_HIP(hipMemcpyAsync(row_ptr, p->bic.lrp, 4 * (size_t)(n + 1), hipMemcpyDeviceToHost, s));
  if (col_idx) FEMH_TRY_HIP(hipMemcpyAsync(col_idx, p->bic.lcol, 4 * (size_t)nz, hipMemcpyDeviceToHost, s));
  if (vals) FEMH_TRY_HIP(hipMemcpyAsync(vals, p->bic.lval, 16 * (size_t)nz, hipMemcpyDeviceToHost, s));
  FEMH_TRY_HIP(hipStreamSynchronize(s));
  return FEMH_OK;
}

int femh_bic0_apply_dev(femh_problem* p, int32_t nodes_per_block, const femh_c128* r, femh_c128* z, int32_t reps,
                        double* avg_seconds) {
  femh::clear_error();
  if (!p || !r || !z || reps < 1 || (const void*)r == (const void*)z) {
    femh::set_error("prob, r and z must not be NULL, r and z distinct; reps >= 1");
    return FEMH_E_INVALID;
  }
  Ctx* c = p->ctx;
  FEMH_TRY_HIP(hipSetDevice(c->device));
  FEMH_TRY(femh::ensure_bic(p, nodes_per_block));
  const size_t stage_bytes = 8 * femh::k::bic_stage_doubles(p->bic.nblk) + 256;
  DevTmp stage(c, stage_bytes), out(c, 64);
  if (!stage.p || !out.p) {
    femh::set_error("device allocation failed (application sums)");
    return FEMH_E_OOM;
  }
  double* st = (double*)stage.p;
  uint32_t* ticket = reinterpret_cast<uint32_t*>(st + femh::k::bic_stage_doubles(p->bic.nblk));
  FEMH_TRY_HIP(hipMemsetAsync(stage.p, 0, stage_bytes, c->stream));
  EventPair ev;
  FEMH_TRY_HIP(ev.create());
  FEMH_TRY_HIP(hipEventRecord(ev.a, c->stream));
  for (int i = 0; i < reps; ++i)
    FEMH_TRY_HIP(femh::k::bic_apply(c->stream, p->bic, (const double2*)r, (double2*)z, st, ticket, (double*)out.p,
                                    nullptr));
  FEMH_TRY_HIP(hipEventRecord(ev.b, c->stream));
  FEMH_TRY_HIP(hipEventSynchronize(ev.b));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, ev.a, ev.b);
  if (avg_seconds) *avg_seconds = ms * 1e-3 / reps;
  return FEMH_OK;
}

int femh_spmv_dev(femh_problem* p, int32_t precision, const void* x, void* y, int32_t reps, double* avg_seconds) {
  femh::clear_error();
  if (!p || !x || !y || reps < 1 ||
      (precision != FEMH_FP64 && precision != FEMH_MIXED && precision != FEMH_MIXED_MATRIX)) {
    femh::set_error("bad spmv arguments");
    return FEMH_E_INVALID;
  }
  Ctx* c = p->ctx;
  FEMH_TRY_HIP(hipSetDevice(c->device));
  EventPair ev;
  FEMH_TRY_HIP(ev.create());
  FEMH_TRY_HIP(hipEventRecord(ev.a, c->stream));
  for (int i = 0; i < reps; ++i) {
    if (precision == FEMH_FP64)
      FEMH_TRY_HIP(femh::k::spmv_c128(c->stream, p->pat, p->val64, (const double2*)x, (double2*)y, p->spmv));
    else if (precision == FEMH_MIXED_MATRIX)
      FEMH_TRY_HIP(femh::k::spmv_m32(c->stream, p->pat, p->val32, (const double2*)x, (double2*)y, p->spmv));
    else
      FEMH_TRY_HIP(femh::k::spmv_c64(c->stream, p->pat, p->val32, (const float2*)x, (float2*)y, p->spmv));
  }
  FEMH_TRY_HIP(hipEventRecord(ev.b, c->stream));
  FEMH_TRY_HIP(hipEventSynchronize(ev.b));
  float ms = 0;
  FEMH_TRY_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
  if (avg_seconds) *avg_seconds = ms * 1e-3 / reps;
  return FEMH_OK;
}

int femh_spmv(femh_problem* p, int32_t precision, const femh_c128* x, femh_c128* y, int32_t reps,
              double* avg_seconds) {
  femh::clear_error();
  if (!p || !x || !y || reps < 1 ||
      (precision != FEMH_FP64 && precision != FEMH_MIXED && precision != FEMH_MIXED_MATRIX)) {
    femh::set_error("bad spmv arguments");
    return FEMH_E_INVALID;
  }
  Ctx* c = p->ctx;
  FEMH_TRY_HIP(hipSetDevice(c->device));
  const int64_t n = 3 * (int64_t)p->pat.nn;
  const bool c64 = precision == FEMH_MIXED;
  const size_t vb = c64 ? 8 : 16;
  DevTmp dx(c, vb * n), dy(c, vb * n);
  if (!dx.p || !dy.p) {
    femh::set_error("device allocation failed (spmv vectors)");
    return FEMH_E_OOM;
  }
  std::vector<float2> h32;
  if (c64) {
    // complex64 vectors: the input rounded to nearest on the host
    h32.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) h32[i] = make_float2((float)x[i].re, (float)x[i].im);
    FEMH_TRY_HIP(hipMemcpyAsync(dx.p, h32.data(), vb * n, hipMemcpyHostToDevice, c->stream));
  } else {
    FEMH_TRY_HIP(hipMemcpyAsync(dx.p, x, vb * n, hipMemcpyHostToDevice, c->stream));
  }
  int rc = femh_spmv_dev(p, precision, dx.p, dy.p, reps, avg_seconds);
  if (rc != FEMH_OK) return rc;
  if (c64) {
    FEMH_TRY_HIP(hipMemcpyAsync(h32.data(), dy.p, vb * n, hipMemcpyDeviceToHost, c->stream));
    FEMH_TRY_HIP(hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < n; ++i) y[i] = femh_c128{(double)h32[i].x, (double)h32[i].y};
  } else {
    FEMH_TRY_HIP(hipMemcpyAsync(y, dy.p, vb * n, hipMemcpyDeviceToHost, c->stream));
    FEMH_TRY_HIP(hipStreamSynchronize(c->stream));
  }
  return FEMH_OK;
}

int femh_spmv_half_dev(femh_problem* p, const void* x, void* y, int32_t reps, double* avg_seconds) {
  femh::clear_error();
  if (!p || !x || !y || reps < 1) {
    femh::set_error("bad spmv arguments");
    return FEMH_E_INVALID;
  }
  FEMH_TRY_HIP(hipSetDevice(p->ctx->device));
  FEMH_TRY(femh::ensure_half_store(p));
  Ctx* c = p->ctx;
  EventPair ev;
  FEMH_TRY_HIP(ev.create());
  FEMH_TRY_HIP(hipEventRecord(ev.a, c->stream));
  for (int i = 0; i < reps; ++i)
    FEMH_TRY_HIP(femh::k::spmv_half_c128(c->stream, p->pat, p->hval64, p->hpos, (const double2*)x, (double2*)y,
                                         p->spmv));
  FEMH_TRY_HIP(hipEventRecord(ev.b, c->stream));
  FEMH_TRY_HIP(hipEventSynchronize(ev.b));
  float ms = 0;
  FEMH_TRY_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
  if (avg_seconds) *avg_seconds = ms * 1e-3 / reps;
  return FEMH_OK;
}

int femh_bw_probe(femh_ctx* c, int64_t bytes, int32_t reps, double* gbps) {
  femh::clear_error();
  if (!c || bytes < 16 || reps < 1 || !gbps) {
    femh::set_error("bad probe arguments");
    return FEMH_E_INVALID;
  }
  bytes &= ~(int64_t)15;
  FEMH_TRY_HIP(hipSetDevice(c->device));
  DevTmp a(c, bytes), b(c, bytes);
  if (!a.p || !b.p) {
    femh::set_error("device allocation failed (probe)");
    return FEMH_E_OOM;
  }
  FEMH_TRY_HIP(hipMemsetAsync(a.p, 0, bytes, c->stream));
  FEMH_TRY_HIP(femh::k::copy_probe(c->stream, (const float4*)a.p, (float4*)b.p, bytes / 16));
  EventPair ev;
  FEMH_TRY_HIP(ev.create());
  FEMH_TRY_HIP(hipEventRecord(ev.a, c->stream));
  for (int i = 0; i < reps; ++i) FEMH_TRY_HIP(femh::k::copy_probe(c->stream, (const float4*)a.p, (float4*)b.p, bytes / 16));
  FEMH_TRY_HIP(hipEventRecord(ev.b, c->stream));
  FEMH_TRY_HIP(hipEventSynchronize(ev.b));
  float ms = 0;
  FEMH_TRY_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
  *gbps = 2.0 * (double)bytes / (ms * 1e-3 / reps) / 1e9;
  return FEMH_OK;
}

int femh_profile_enable(femh_ctx* c, int32_t on) {
  if (!c) {
    femh::set_error("ctx is NULL");
    return FEMH_E_INVALID;
  }
  c->profile = on != 0;
  return FEMH_OK;
}

int femh_profile_read(femh_ctx* c, double sec[4], int64_t cnt[4], int32_t reset) {
  if (!c || !sec || !cnt) {
    femh::set_error("NULL argument");
    return FEMH_E_INVALID;
  }
  for (int i = 0; i < 4; ++i) {
    sec[i] = c->prof_sec[i];
    cnt[i] = c->prof_cnt[i];
    if (reset) {
      c->prof_sec[i] = 0;
      c->prof_cnt[i] = 0;
    }
  }
  return FEMH_OK;
}

}  // extern "C"
