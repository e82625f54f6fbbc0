// Host side of problem set-up: errors, contexts, descriptor validation,
// footprint estimates and on-device numbering + assembly.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace femh {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

int log_level() {
  static const int level = [] {
    const char* v = std::getenv("FEMH_LOG");
    return v ? std::atoi(v) : 0;
  }();
  return level;
}

void logf(int level, const char* fmt, ...) {
  if (log_level() < level) return;
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[femh] %s\n", buf);
}

void* Ctx::dmalloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~(size_t)255;
  void* p = nullptr;
  if (alloc.alloc) {
    p = alloc.alloc(bytes, alloc.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  return p;
}

void Ctx::dfree(void* p) {
  if (!p) return;
  if (alloc.free) alloc.free(p, alloc.user);
  else (void)hipFree(p);
}

void* Problem::alloc(size_t bytes) {
  void* p = ctx->dmalloc(bytes);
  if (p) {
    owned.push_back(p);
    dev_bytes += (int64_t)((bytes + 255) & ~(size_t)255);
  }
  return p;
}

Problem::~Problem() {
  if (ctx) {
    (void)hipStreamSynchronize(ctx->stream);
    for (void* p : owned) ctx->dfree(p);
    for (void* p : bic_mem) ctx->dfree(p);
  }
}

// ---------------------------------------------------------------- checks
static bool finite_c(const femh_c128& z) { return std::isfinite(z.re) && std::isfinite(z.im); }

int validate_desc(const femh_problem_desc* d, std::string& msg) {
  if (!d) {
    msg = "descriptor is NULL";
    return FEMH_E_INVALID;
  }
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) {
    msg = "nx, ny, nz must be >= 1";
    return FEMH_E_INVALID;
  }
  const int64_t ne = (int64_t)d->nx * d->ny * d->nz;
  const int64_t ng = (int64_t)(d->nx + 1) * (d->ny + 1) * (d->nz + 1);
  if (ng > (int64_t)1 << 30) {
    msg = "mesh too large (more than 2^30 grid nodes)";
    return FEMH_E_INVALID;
  }
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(d->h[a]) || !std::isfinite(d->origin[a])) {
      msg = "h and origin must be finite";
      return FEMH_E_NONFINITE;
    }
    if (!(d->h[a] > 0.0)) {
      msg = "element sizes h must be > 0";
      return FEMH_E_INVALID;
    }
  }
  if (!std::isfinite(d->k0) || !std::isfinite(d->penalty_s)) {
    msg = "k0 and penalty_s must be finite";
    return FEMH_E_NONFINITE;
  }
  if (!(d->k0 > 0.0)) {
    msg = "k0 must be > 0";
    return FEMH_E_INVALID;
  }
  if (d->penalty_s < 0.0) {
    msg = "penalty_s must be >= 0";
    return FEMH_E_INVALID;
  }
  for (int f = 0; f < 6; ++f)
    if (d->outer_face[f] < FEMH_FACE_ABC || d->outer_face[f] > FEMH_FACE_ANTISYM) {
      msg = "outer_face entries must be FEMH_FACE_ABC, _NATURAL, _SYM or _ANTISYM";
      return FEMH_E_INVALID;
    }
  if (d->penalty_surface != 0 && d->penalty_surface != 1) {
    msg = "penalty_surface must be 0 or 1";
    return FEMH_E_INVALID;
  }
  if (d->penalty_surface)
    for (int f = 0; f < 6; ++f)
      if (d->outer_face[f] == FEMH_FACE_SYM || d->outer_face[f] == FEMH_FACE_ANTISYM) {
        msg = "penalty_surface is not combined with symmetry or antisymmetry faces";
        return FEMH_E_INVALID;
      }
  if (d->arrays_on_device != 0 && d->arrays_on_device != 1) {
    msg = "arrays_on_device must be 0 or 1";
    return FEMH_E_INVALID;
  }
  if (!d->arrays_on_device) {
    if (d->eps_r)
      for (int64_t i = 0; i < ne; ++i) {
        if (!finite_c(d->eps_r[i])) {
          msg = "eps_r has a non-finite entry";
          return FEMH_E_NONFINITE;
        }
        if (d->eps_r[i].re == 0.0 && d->eps_r[i].im == 0.0) {
          msg = "eps_r has a zero entry";
          return FEMH_E_INVALID;
        }
      }
    if (d->mu_r)
      for (int64_t i = 0; i < ne; ++i)
        if (!finite_c(d->mu_r[i])) {
          msg = "mu_r has a non-finite entry";
          return FEMH_E_NONFINITE;
        }
    if (d->pec) {
      int64_t active = 0;
      for (int64_t i = 0; i < ne; ++i) active += d->pec[i] == 0;
      if (active == 0) {
        msg = "every element is PEC: no unknowns";
        return FEMH_E_INVALID;
      }
    }
  }
  return FEMH_OK;
}

int validate_waves(int32_t nrhs, const femh_plane_wave* w, std::string& msg) {
  if (nrhs < 1) {
    msg = "nrhs must be >= 1";
    return FEMH_E_INVALID;
  }
  if (!w) {
    msg = "waves is NULL";
    return FEMH_E_INVALID;
  }
  for (int r = 0; r < nrhs; ++r) {
    double dd = 0, pn = 0;
    double pdr = 0, pdi = 0;
    for (int c = 0; c < 3; ++c) {
      if (!std::isfinite(w[r].d[c]) || !finite_c(w[r].p[c])) {
        msg = "wave " + std::to_string(r) + " has a non-finite entry";
        return FEMH_E_NONFINITE;
      }
      dd += w[r].d[c] * w[r].d[c];
      pn += w[r].p[c].re * w[r].p[c].re + w[r].p[c].im * w[r].p[c].im;
      pdr += w[r].p[c].re * w[r].d[c];
      pdi += w[r].p[c].im * w[r].d[c];
    }
    if (std::fabs(dd - 1.0) > 1e-9) {
      msg = "wave " + std::to_string(r) + ": |d| must be 1";
      return FEMH_E_INVALID;
    }
    if (std::sqrt(pdr * pdr + pdi * pdi) > 1e-9 * std::fmax(1.0, std::sqrt(pn))) {
      msg = "wave " + std::to_string(r) + ": p must be orthogonal to d";
      return FEMH_E_INVALID;
    }
  }
  return FEMH_OK;
}

// Active nodes and stored blocks of a host PEC mask (exact), or their upper
// bounds when the mask is not on the host.
static void count_pattern(const femh_problem_desc* d, int64_t& nn, int64_t& nnzb) {
  const int nx = d->nx, ny = d->ny, nz = d->nz;
  const int64_t gx = nx + 1, gy = ny + 1, gz = nz + 1;
  const uint8_t* pec = d->arrays_on_device ? nullptr : d->pec;
  if (!pec) {
    nn = gx * gy * gz;
    // with no PEC element every pair of nodes within one element shares it
    nnzb = (3 * gx - 2) * (3 * gy - 2) * (3 * gz - 2);
    return;
  }
  auto act = [&](int64_t ex, int64_t ey, int64_t ez) -> bool {
    if (ex < 0 || ey < 0 || ez < 0 || ex >= nx || ey >= ny || ez >= nz) return false;
    return pec[ex + nx * (ey + ny * ez)] == 0;
  };
  nn = 0;
  nnzb = 0;
  for (int64_t k = 0; k < gz; ++k)
    for (int64_t j = 0; j < gy; ++j)
      for (int64_t i = 0; i < gx; ++i) {
        bool node_act = false;
        for (int dz = -1; dz <= 0 && !node_act; ++dz)
          for (int dy = -1; dy <= 0 && !node_act; ++dy)
            for (int dx = -1; dx <= 0 && !node_act; ++dx) node_act = act(i + dx, j + dy, k + dz);
        if (!node_act) continue;
        ++nn;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int64_t x0 = dx == 0 ? i - 1 : (dx > 0 ? i : i - 1), x1 = dx == 0 ? i : x0;
              const int64_t y0 = dy == 0 ? j - 1 : (dy > 0 ? j : j - 1), y1 = dy == 0 ? j : y0;
              const int64_t z0 = dz == 0 ? k - 1 : (dz > 0 ? k : k - 1), z1 = dz == 0 ? k : z0;
              bool sh = false;
              for (int64_t ez = z0; ez <= z1 && !sh; ++ez)
                for (int64_t ey = y0; ey <= y1 && !sh; ++ey)
                  for (int64_t ex = x0; ex <= x1 && !sh; ++ex) sh = act(ex, ey, ez);
              nnzb += sh;
            }
      }
}

static inline int64_t al(int64_t b) { return (b + 255) & ~(int64_t)255; }

int64_t estimate_bytes(const femh_problem_desc* d, int32_t nrhs, int32_t precision) {
  int64_t nn, nnzb;
  count_pattern(d, nn, nnzb);
  const int64_t ne = (int64_t)d->nx * d->ny * d->nz;
  const int64_t ng = (int64_t)(d->nx + 1) * (d->ny + 1) * (d->nz + 1);
  int64_t b = 0;
  if (d->eps_r) b += al(16 * ne);
  if (d->mu_r) b += al(16 * ne);
  if (d->pec) b += al(ne);
  b += al(4 * ng) + 3 * al(4 * nn) + al(4 * (nn + 1)) + al(4 * nnzb);
  b += al(144 * nnzb) + al(72 * nnzb) + al(48 * nn) + al(24 * nn);
  // per right-hand side: b and x (FP64), the solver's workspace (mixed: an
  // FP64 residual and four complex64 vectors; matrix-mixed: three FP64
  // vectors; FP64, in its single-reduction form: five), the partial-sum
  // buffers of 2048 workgroups x 4 doubles (FP64: five, two otherwise), the
  // scalar blocks, and the output grid
  const int64_t v64 = al(48 * nn), v32 = al(24 * nn);
  if (nrhs > 0) {
    const bool fp64 = precision == FEMH_FP64;
    const int64_t ws = precision == FEMH_MIXED ? v64 + 4 * v32 : (fp64 ? 5 : 3) * v64;
    const int64_t part = (fp64 ? 5 : 2) * al(8 * 2048 * 4) + 2 * al(1024);
    b += (int64_t)nrhs * (2 * v64 + ws + part) + al((int64_t)nrhs * 48 * ng);
  }
  b += 1 << 20;  // numbering scratch, scalars
  return b;
}

int64_t estimate_bic_bytes(const femh_problem_desc* d, int32_t nrhs) {
  int64_t nn, nnzb;
  count_pattern(d, nn, nnzb);
  // L and U hold at most 9 nnzb + 3 nn entries together (column + value),
  // plus their row starts and 1 / l_uu; per right-hand side the
  // preconditioned residual, a vector of ones, the direction update's
  // partial sums and the application's per-block sums (at most one block
  // per node)
  const int64_t factor = al(20 * (9 * nnzb + 3 * nn)) + 2 * al(12 * nn + 4) + al(48 * nn);
  const int64_t per_rhs = 2 * al(48 * nn) + al(8 * 2048 * 4) + al(32 * nn + 8 * 256 + 256);
  return factor + (int64_t)(nrhs > 0 ? nrhs : 0) * per_rhs;
}

int check_solve_opts(const femh_solve_opts& o, bool batched, std::string& msg) {
  char buf[160];
  if (o.precision != FEMH_FP64 && o.precision != FEMH_MIXED && o.precision != FEMH_MIXED_MATRIX) {
    std::snprintf(buf, sizeof buf, "unknown precision %d", o.precision);
    msg = buf;
    return FEMH_E_INVALID;
  }
  if (o.precond != FEMH_PRECOND_JACOBI && o.precond != FEMH_PRECOND_NONE && o.precond != FEMH_PRECOND_BIC0) {
    std::snprintf(buf, sizeof buf, "unknown preconditioner %d", o.precond);
    msg = buf;
    return FEMH_E_INVALID;
  }
  if (o.precond == FEMH_PRECOND_BIC0) {
    if (batched || o.precision != FEMH_FP64) {
      msg = "FEMH_PRECOND_BIC0 runs with single right-hand-side FEMH_FP64 solves only";
      return FEMH_E_INVALID;
    }
    if (o.precond_block < 1 || o.precond_block > kBicMaxNodesPerBlock) {
      std::snprintf(buf, sizeof buf, "precond_block must be 1..%d (got %d)", kBicMaxNodesPerBlock,
                    o.precond_block);
      msg = buf;
      return FEMH_E_INVALID;
    }
  }
  return FEMH_OK;
}

int64_t estimate_batch_workspace(const femh_problem_desc* d, int32_t nrhs) {
  int64_t nn, nnzb;
  count_pattern(d, nn, nnzb);
  // per group of up to four waves: five [unknowns][4] complex128 blocks,
  // the per-workgroup partial sums (2048 x 64 x 4 doubles) and small blocks
  const int64_t groups = (nrhs + 3) / 4;
  return groups * (5 * al(4 * 48 * nn) + (4 << 20) + (1 << 16));
}

// Symmetric half store of the complex-symmetric matrix (A_ba = A_ab^T per
// block): each row keeps its blocks with column <= row, a prefix of the
// row since columns ascend.  Slot k of row a with column b points at the
// stored block: row a's own (b <= a), or row b's block for column a read
// transposed (b > a).  Built on the host from the pattern.
int ensure_half_store(Problem* P) {
  if (P->hpos) return FEMH_OK;
  const int32_t nn = P->pat.nn;
  const int64_t nnzb = P->pat.nnzb;
  std::vector<int32_t> rp((size_t)nn + 1), ci((size_t)nnzb), hp((size_t)nnzb);
  FEMH_TRY_HIP(hipMemcpy(rp.data(), P->row_ptr, sizeof(int32_t) * (nn + 1), hipMemcpyDeviceToHost));
  FEMH_TRY_HIP(hipMemcpy(ci.data(), P->col_idx, sizeof(int32_t) * nnzb, hipMemcpyDeviceToHost));
  std::vector<int64_t> hrow((size_t)nn + 1, 0);
  for (int32_t a = 0; a < nn; ++a) {
    int32_t lower = 0;
    for (int32_t k = rp[a]; k < rp[a + 1] && ci[k] <= a; ++k) ++lower;
    hrow[a + 1] = hrow[a] + lower;
  }
  for (int32_t a = 0; a < nn; ++a)
    for (int32_t k = rp[a]; k < rp[a + 1]; ++k) {
      const int32_t b = ci[k];
      if (b <= a) {
        hp[k] = (int32_t)(hrow[a] + (k - rp[a]));
      } else {
        int32_t r = rp[b];
        while (r < rp[b + 1] && ci[r] != a) ++r;
        if (r == rp[b + 1]) {
          set_error("matrix pattern is not symmetric");
          return FEMH_E_INVALID;
        }
        hp[k] = -(int32_t)(hrow[b] + (r - rp[b])) - 1;
      }
    }
  int32_t* dpos = (int32_t*)P->alloc(sizeof(int32_t) * nnzb);
  double2* dval = (double2*)P->alloc(sizeof(double2) * 9 * (size_t)hrow[nn]);
  if (!dpos || !dval) {
    set_error("device allocation failed (half store)");
    return FEMH_E_OOM;
  }
  FEMH_TRY_HIP(hipMemcpy(dpos, hp.data(), sizeof(int32_t) * nnzb, hipMemcpyHostToDevice));
  FEMH_TRY_HIP(k::gather_half(P->ctx->stream, nnzb, dpos, P->val64, dval));
  FEMH_TRY_HIP(hipStreamSynchronize(P->ctx->stream));
  P->hpos = dpos;
  P->hval64 = dval;
  P->n_half = hrow[nn];
  return FEMH_OK;
}

// --------------------------------------------------------- problem create
static void fill_mesh(MeshDev& m, const femh_problem_desc* d) {
  m.nx = d->nx;
  m.ny = d->ny;
  m.nz = d->nz;
  for (int a = 0; a < 3; ++a) {
    m.h[a] = d->h[a];
    m.origin[a] = d->origin[a];
  }
  m.k0 = d->k0;
  m.s = d->penalty_s == 0.0 ? 1.0 : d->penalty_s;
  m.abc_mask = m.sym_mask = m.anti_mask = 0;
  m.penalty_surface = d->penalty_surface;
  for (int f = 0; f < 6; ++f) {
    if (d->outer_face[f] == FEMH_FACE_ABC) m.abc_mask |= 1 << f;
    if (d->outer_face[f] == FEMH_FACE_SYM) m.sym_mask |= 1 << f;
    if (d->outer_face[f] == FEMH_FACE_ANTISYM) m.anti_mask |= 1 << f;
  }
  m.eps = nullptr;
  m.mu = nullptr;
  m.pec = nullptr;
}

struct TmpBuf {
  Ctx* ctx;
  void* p = nullptr;
  TmpBuf(Ctx* c, size_t bytes) : ctx(c) { p = c->dmalloc(bytes); }
  ~TmpBuf() {
    if (p) {
      (void)hipStreamSynchronize(ctx->stream);
      ctx->dfree(p);
    }
  }
  template <typename T> T* as() { return reinterpret_cast<T*>(p); }
};

// ------------------------------------------- block incomplete Cholesky
static void drop_bic(Problem* P) {
  if (!P->bic_mem.empty()) (void)hipStreamSynchronize(P->ctx->stream);
  for (void* p : P->bic_mem) P->ctx->dfree(p);
  P->bic_mem.clear();
  P->bic = BicFactorDev{};
  P->bic_nodes = 0;
  P->bic_nnz_l = 0;
}

int ensure_bic(Problem* P, int32_t nodes_per_block) {
  // checked first: bic_nodes is 0 while no factor is held
  if (nodes_per_block < 1 || nodes_per_block > kBicMaxNodesPerBlock) {
    set_error("block incomplete Cholesky: nodes per block must be 1..%d (got %d)", kBicMaxNodesPerBlock,
              nodes_per_block);
    return FEMH_E_INVALID;
  }
  if (P->bic_nodes == nodes_per_block) return FEMH_OK;
  // the factor's row starts are 32-bit: bound its entries by A's scalar count
  if (P->pat.nnzb * 9 > (int64_t)INT32_MAX) {
    set_error("block incomplete Cholesky: %lld stored blocks exceed the factor's 32-bit row starts",
              (long long)P->pat.nnzb);
    return FEMH_E_INVALID;
  }
  drop_bic(P);
  Ctx* c = P->ctx;
  hipStream_t s = c->stream;
  const int64_t n = 3 * (int64_t)P->pat.nn;
  const int32_t rpb = 3 * nodes_per_block;
  auto take = [&](size_t bytes) -> void* {
    void* p = c->dmalloc(bytes > 0 ? bytes : 16);
    if (p) P->bic_mem.push_back(p);
    return p;
  };
  auto oom = [&]() {
    drop_bic(P);
    set_error("device allocation failed (block incomplete Cholesky factor)");
    return FEMH_E_OOM;
  };
  TmpBuf counts(c, 4 * (size_t)n), tmp(c, 4 * (size_t)k::scan_tmp_ints(n)), flag(c, 64);
  int32_t* lrp = (int32_t*)take(4 * ((size_t)n + 1));
  int32_t* urp = (int32_t*)take(4 * ((size_t)n + 1));
  double2* ldinv = (double2*)take(16 * (size_t)n);
  if (!counts.p || !tmp.p || !flag.p || !lrp || !urp || !ldinv) return oom();
  int32_t host[2] = {0, 0};
  // L's pattern and A's values on it
  FEMH_TRY_HIP(k::bic_pattern_count(s, P->pat, nodes_per_block, counts.as<int32_t>()));
  FEMH_TRY_HIP(k::exclusive_scan(s, counts.as<int32_t>(), lrp, n, tmp.as<int32_t>(), lrp + n));
  FEMH_TRY_HIP(hipMemcpyAsync(host, lrp + n, 4, hipMemcpyDeviceToHost, s));
  FEMH_TRY_HIP(hipStreamSynchronize(s));
  const int64_t nnz_l = host[0];
  int32_t* lcol = (int32_t*)take(4 * (size_t)nnz_l);
  double2* lval = (double2*)take(16 * (size_t)nnz_l);
  if (!lcol || !lval) return oom();
  FEMH_TRY_HIP(k::bic_pattern_fill(s, P->pat, nodes_per_block, P->val64, lrp, lcol, lval));
  // eq. (5) inside each block
  const int32_t nblk = (int32_t)((n + rpb - 1) / rpb);
  FEMH_TRY_HIP(hipMemsetAsync(flag.p, 0, 4, s));
  FEMH_TRY_HIP(k::bic_factor(s, n, rpb, nblk, lrp, lcol, lval, ldinv, flag.as<int32_t>()));
  FEMH_TRY_HIP(hipMemcpyAsync(host + 1, flag.p, 4, hipMemcpyDeviceToHost, s));
  // U = strict upper part of L^T
  FEMH_TRY_HIP(k::bic_upper(s, n, rpb, lrp, lcol, lval, counts.as<int32_t>(), nullptr, nullptr, nullptr));
  FEMH_TRY_HIP(k::exclusive_scan(s, counts.as<int32_t>(), urp, n, tmp.as<int32_t>(), urp + n));
  FEMH_TRY_HIP(hipMemcpyAsync(host, urp + n, 4, hipMemcpyDeviceToHost, s));
  FEMH_TRY_HIP(hipStreamSynchronize(s));
  if (host[1]) {
    drop_bic(P);
    set_error("block incomplete Cholesky: a pivot vanished or is not finite");
    return FEMH_E_BREAKDOWN;
  }
  const int64_t nnz_u = host[0];
  int32_t* ucol = (int32_t*)take(4 * (size_t)nnz_u);
  double2* uval = (double2*)take(16 * (size_t)nnz_u);
  if (!ucol || !uval) return oom();
  FEMH_TRY_HIP(k::bic_upper(s, n, rpb, lrp, lcol, lval, nullptr, urp, ucol, uval));
  // the application stages rows in chunks of at least the longest row, and
  // of about ten entries per row of a block (a row has 9 on average), up to
  // 768 (64 rows of a 64-node block): small blocks then take little LDS and
  // more of them run at once on a compute unit
  std::vector<int32_t> hl((size_t)n + 1), hu((size_t)n + 1);
  FEMH_TRY_HIP(hipMemcpyAsync(hl.data(), lrp, 4 * ((size_t)n + 1), hipMemcpyDeviceToHost, s));
  FEMH_TRY_HIP(hipMemcpyAsync(hu.data(), urp, 4 * ((size_t)n + 1), hipMemcpyDeviceToHost, s));
  FEMH_TRY_HIP(hipStreamSynchronize(s));
  int32_t longest = 0;
  for (int64_t u = 0; u < n; ++u) longest = std::max(longest, std::max(hl[u + 1] - hl[u], hu[u + 1] - hu[u]));
  P->bic.chunk_cap = std::max(longest, std::min(768, 10 * rpb));
  P->bic.n = n;
  P->bic.rows_per_block = rpb;
  P->bic.nblk = nblk;
  P->bic.lrp = lrp;
  P->bic.lcol = lcol;
  P->bic.lval = lval;
  P->bic.urp = urp;
  P->bic.ucol = ucol;
  P->bic.uval = uval;
  P->bic.ldinv = ldinv;
  P->bic_nodes = nodes_per_block;
  P->bic_nnz_l = nnz_l;
  logf(1, "block incomplete Cholesky: %d-node blocks, %d blocks, %lld entries in L, staging chunk %d entries",
       nodes_per_block, nblk, (long long)nnz_l, P->bic.chunk_cap);
  return FEMH_OK;
}

int problem_create(Ctx* ctx, const femh_problem_desc* d, Problem** out) {
  std::string msg;
  int st = validate_desc(d, msg);
  if (st != FEMH_OK) {
    set_error("%s", msg.c_str());
    return st;
  }
  Problem* P = new Problem();
  P->ctx = ctx;
  fill_mesh(P->mesh, d);
  for (int f = 0; f < 6; ++f) P->faces[f] = d->outer_face[f];
  hipStream_t s = ctx->stream;
  const int64_t ne = (int64_t)d->nx * d->ny * d->nz;
  const int64_t ng = (int64_t)(d->nx + 1) * (d->ny + 1) * (d->nz + 1);
  P->grid_nodes = ng;
  auto fail = [&](int code, const char* what) {
    if (code == FEMH_E_OOM) set_error("device allocation failed: %s", what);
    delete P;
    return code;
  };
#define FEMH_ALLOC(ptr, T, count)                                   \
  do {                                                              \
    ptr = reinterpret_cast<T*>(P->alloc(sizeof(T) * (size_t)(count))); \
    if (!ptr) return fail(FEMH_E_OOM, #ptr);                        \
  } while (0)
#define FEMH_HIP_OR_FAIL(call)                                                             \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      set_error("%s failed: %s", #call, hipGetErrorString(e_));                            \
      delete P;                                                                            \
      return (int)FEMH_E_DEVICE;                                                           \
    }                                                                                      \
  } while (0)

  const hipMemcpyKind kind = d->arrays_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (d->eps_r) {
    FEMH_ALLOC(P->eps, double2, ne);
    FEMH_HIP_OR_FAIL(hipMemcpyAsync(P->eps, d->eps_r, 16 * ne, kind, s));
    P->mesh.eps = P->eps;
  }
  if (d->mu_r) {
    FEMH_ALLOC(P->mu, double2, ne);
    FEMH_HIP_OR_FAIL(hipMemcpyAsync(P->mu, d->mu_r, 16 * ne, kind, s));
    P->mesh.mu = P->mu;
  }
  if (d->pec) {
    FEMH_ALLOC(P->pec, uint8_t, ne);
    FEMH_HIP_OR_FAIL(hipMemcpyAsync(P->pec, d->pec, ne, kind, s));
    P->mesh.pec = P->pec;
  }
  int32_t* hostw = reinterpret_cast<int32_t*>(ctx->pinned);
  TmpBuf aux(ctx, 64);
  if (!aux.p) return fail(FEMH_E_OOM, "aux");
  int32_t* d_total = aux.as<int32_t>();
  if (d->arrays_on_device && (d->eps_r || d->mu_r)) {
    FEMH_HIP_OR_FAIL(hipMemsetAsync(d_total, 0, 4, s));
    FEMH_HIP_OR_FAIL(k::check_materials(s, P->mesh.eps, P->mesh.mu, ne, d_total));
    FEMH_HIP_OR_FAIL(hipMemcpyAsync(hostw, d_total, 4, hipMemcpyDeviceToHost, s));
    FEMH_HIP_OR_FAIL(hipStreamSynchronize(s));
    if (hostw[0] & 1) {
      set_error("eps_r or mu_r has a non-finite entry");
      delete P;
      return FEMH_E_NONFINITE;
    }
    if (hostw[0] & 2) {
      set_error("eps_r has a zero entry");
      delete P;
      return FEMH_E_INVALID;
    }
  }
  // 1. active nodes and their compact numbering
  const int64_t scan_n = ng > 1 ? ng : 1;
  TmpBuf flags(ctx, 4 * scan_n), scan(ctx, 4 * scan_n), tmp(ctx, 4 * k::scan_tmp_ints(scan_n));
  if (!flags.p || !scan.p || !tmp.p) return fail(FEMH_E_OOM, "numbering scratch");
  FEMH_HIP_OR_FAIL(k::node_flags(s, P->mesh, flags.as<int32_t>()));
  FEMH_HIP_OR_FAIL(k::exclusive_scan(s, flags.as<int32_t>(), scan.as<int32_t>(), ng, tmp.as<int32_t>(), d_total));
  FEMH_HIP_OR_FAIL(hipMemcpyAsync(hostw, d_total, 4, hipMemcpyDeviceToHost, s));
  FEMH_HIP_OR_FAIL(hipStreamSynchronize(s));
  const int32_t nn = hostw[0];
  if (nn <= 0) {
    set_error("every element is PEC: no unknowns");
    delete P;
    return FEMH_E_INVALID;
  }
  FEMH_ALLOC(P->node_id, int32_t, ng);
  FEMH_ALLOC(P->node_grid, int32_t, nn);
  FEMH_HIP_OR_FAIL(k::node_compact(s, P->mesh, flags.as<int32_t>(), scan.as<int32_t>(), P->node_id, P->node_grid));
  // 2. neighbour masks and row pointers (block pattern)
  FEMH_ALLOC(P->nbr_mask, uint32_t, nn);
  FEMH_ALLOC(P->row_ptr, int32_t, nn + 1);
  FEMH_HIP_OR_FAIL(k::row_masks(s, P->mesh, nn, P->node_id, P->node_grid, P->nbr_mask, flags.as<int32_t>()));
  FEMH_HIP_OR_FAIL(k::exclusive_scan(s, flags.as<int32_t>(), P->row_ptr, nn, tmp.as<int32_t>(), P->row_ptr + nn));
  FEMH_HIP_OR_FAIL(hipMemcpyAsync(hostw, P->row_ptr + nn, 4, hipMemcpyDeviceToHost, s));
  FEMH_HIP_OR_FAIL(hipStreamSynchronize(s));
  const int64_t nnzb = hostw[0];
  P->pat.nn = nn;
  P->pat.nnzb = nnzb;
  P->pat.node_id = P->node_id;
  P->pat.node_grid = P->node_grid;
  P->pat.nbr_mask = P->nbr_mask;
  P->pat.row_ptr = P->row_ptr;
  // 3. values: FP64 blocks, complex64 rounding, Jacobi inverse
  FEMH_ALLOC(P->col_idx, int32_t, nnzb);
  FEMH_ALLOC(P->val64, double2, 9 * nnzb);
  FEMH_ALLOC(P->val32, float2, 9 * nnzb);
  FEMH_ALLOC(P->dinv64, double2, 3 * (int64_t)nn);
  FEMH_ALLOC(P->dinv32, float2, 3 * (int64_t)nn);
  P->pat.col_idx = P->col_idx;
  FEMH_HIP_OR_FAIL(k::assemble(s, P->mesh, P->pat, P->col_idx, P->val64, P->val32, P->dinv64, P->dinv32));
  FEMH_HIP_OR_FAIL(hipStreamSynchronize(s));
  P->spmv = k::spmv_launch_for(nn, ctx->n_cu);
#undef FEMH_ALLOC
#undef FEMH_HIP_OR_FAIL
  logf(1, "problem %dx%dx%d: %d active nodes, %lld unknowns, %lld blocks, %.1f MB on the device%s", d->nx, d->ny,
       d->nz, nn, 3LL * nn, (long long)nnzb, P->dev_bytes / 1e6,
       d->penalty_surface ? ", printed penalty surface term" : "");
  *out = P;
  return FEMH_OK;
}

int problem_import(Ctx* ctx, int64_t nb, int64_t nnzb, const int32_t* row_ptr, const int32_t* col_idx,
                   const femh_c128* vals, Problem** out) {
  if (!row_ptr || !col_idx || !vals || !out) {
    set_error("row_ptr, col_idx, vals and out must not be NULL");
    return FEMH_E_INVALID;
  }
  if (nb < 1 || nb > (int64_t)1 << 30 || nnzb < nb || nnzb > ((int64_t)1 << 31) - 1) {
    set_error("need 1 <= nb <= 2^30 block rows and nb <= nnzb < 2^31 blocks (got %lld, %lld)", (long long)nb,
              (long long)nnzb);
    return FEMH_E_INVALID;
  }
  if (row_ptr[0] != 0 || row_ptr[nb] != nnzb) {
    set_error("row_ptr must start at 0 and end at nnzb");
    return FEMH_E_INVALID;
  }
  for (int64_t a = 0; a < nb; ++a) {
    const int32_t b0 = row_ptr[a], b1 = row_ptr[a + 1];
    // the products' lane mappings cover the 27 neighbours of a hexahedral
    // mesh node
    if (b1 <= b0 || b1 - b0 > 27) {
      set_error("block row %lld holds %d blocks (1..27 allowed)", (long long)a, b1 - b0);
      return FEMH_E_INVALID;
    }
    bool diag = false;
    for (int32_t k = b0; k < b1; ++k) {
      if (col_idx[k] < 0 || col_idx[k] >= nb || (k > b0 && col_idx[k] <= col_idx[k - 1])) {
        set_error("block row %lld: column indices must ascend strictly within [0, nb)", (long long)a);
        return FEMH_E_INVALID;
      }
      diag |= col_idx[k] == a;
    }
    if (!diag) {
      set_error("block row %lld has no diagonal block", (long long)a);
      return FEMH_E_INVALID;
    }
  }
  for (int64_t q = 0; q < 9 * nnzb; ++q)
    if (!std::isfinite(vals[q].re) || !std::isfinite(vals[q].im)) {
      set_error("vals has a non-finite entry");
      return FEMH_E_NONFINITE;
    }
  Problem* P = new Problem();
  P->ctx = ctx;
  P->imported = true;
  hipStream_t s = ctx->stream;
  const int32_t nn = (int32_t)nb;
  P->row_ptr = (int32_t*)P->alloc(4 * (size_t)(nn + 1));
  P->col_idx = (int32_t*)P->alloc(4 * (size_t)nnzb);
  P->val64 = (double2*)P->alloc(144 * (size_t)nnzb + 16);
  P->val32 = (float2*)P->alloc(72 * (size_t)nnzb + 16);
  P->dinv64 = (double2*)P->alloc(48 * (size_t)nn);
  P->dinv32 = (float2*)P->alloc(24 * (size_t)nn);
  TmpBuf bad(ctx, 64);
  if (!P->row_ptr || !P->col_idx || !P->val64 || !P->val32 || !P->dinv64 || !P->dinv32 || !bad.p) {
    set_error("device allocation failed (imported matrix)");
    delete P;
    return FEMH_E_OOM;
  }
  int32_t* hostw = reinterpret_cast<int32_t*>(ctx->pinned);
  hipError_t e = hipMemcpyAsync(P->row_ptr, row_ptr, 4 * (size_t)(nn + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(P->col_idx, col_idx, 4 * (size_t)nnzb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(P->val64, vals, 144 * (size_t)nnzb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(bad.p, 0, 4, s);
  if (e == hipSuccess) e = k::round_c64(s, 9 * nnzb, P->val64, P->val32);
  if (e == hipSuccess)
    e = k::dinv_from_blocks(s, nn, P->row_ptr, P->col_idx, P->val64, P->dinv64, P->dinv32, bad.as<int32_t>());
  if (e == hipSuccess) e = hipMemcpyAsync(hostw, bad.p, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error("importing the matrix failed: %s", hipGetErrorString(e));
    delete P;
    return FEMH_E_DEVICE;
  }
  if (hostw[0]) {
    set_error("a diagonal entry of the matrix is zero (no Jacobi inverse)");
    delete P;
    return FEMH_E_INVALID;
  }
  P->pat.nn = nn;
  P->pat.nnzb = nnzb;
  P->pat.row_ptr = P->row_ptr;
  P->pat.col_idx = P->col_idx;
  P->grid_nodes = 0;
  P->spmv = k::spmv_launch_for(nn, ctx->n_cu);
  logf(1, "imported matrix: %d block rows, %lld blocks", nn, (long long)nnzb);
  *out = P;
  return FEMH_OK;
}

femh_solve_opts opts_with_defaults(const femh_solve_opts* o) {
  femh_solve_opts r{};
  if (o) r = *o;
  if (r.rtol <= 0.0) r.rtol = 1e-6;
  // COCG-Jacobi's iteration count grows with the box size in wavelengths:
  // a 6.4-wavelength serving box (64^3) already needs 48 000 in FP64
  if (r.max_iter <= 0) r.max_iter = 200000;
  // one block is one wavefront's sequential chain: 4-node blocks give
  // enough chains to fill the device and took no more iterations than
  // larger ones on the workloads measured
  if (r.precond_block == 0) r.precond_block = 4;
  // complex64 recurrences can only shrink their residual about one decade
  // before its rounding dominates; an FP64 recurrence with a complex64 matrix
  // can go much further between reliable updates
  if (r.inner_rtol <= 0.0) r.inner_rtol = r.precision == FEMH_MIXED_MATRIX ? 1e-3 : 0.1;
  if (r.max_outer <= 0) r.max_outer = 20;
  if (r.check_every <= 0) r.check_every = 32;
  return r;
}

}  // namespace femh
