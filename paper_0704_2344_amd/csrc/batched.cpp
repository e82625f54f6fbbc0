// Host driver of the batched-RHS solve: every column runs its own COCG
// recurrence, the columns sharing one SpMM per iteration (the complex128
// matrix for FEMH_FP64, else the complex64 matrix promoted inside FP64
// products); each column's iterate, residual, direction and product are
// FP64.  When a column's residual has fallen by inner_rtol below its
// largest value since the last update (or meets the tolerance, or breaks
// down), its residual is replaced by the FP64 true residual b - A x and the
// recurrence continues with the same direction (after a breakdown it takes
// a minimal-residual step and restarts from the preconditioned residual).
//
// One iteration = SpMM + per-column alpha + update + per-column beta +
// direction update (5 kernels).  A chunk of `check_every` iterations is
// captured once into a hipGraph and replayed; the host reads the per-column
// state between replays (one replay queued ahead) and performs reliable
// updates for the columns that asked for one.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>

#include "internal.h"

namespace femh {

namespace {

constexpr size_t kPartialBytes = 2048 * 64 * 4 * sizeof(double);  // [blocks][ld][4] doubles, ld <= 64

struct Scratch {
  Ctx* ctx;
  std::vector<void*> ptrs;
  explicit Scratch(Ctx* c) : ctx(c) {}
  void* get(size_t bytes) {
    void* p = ctx->dmalloc(bytes);
    if (p) ptrs.push_back(p);
    return p;
  }
  ~Scratch() {
    (void)hipStreamSynchronize(ctx->stream);
    for (void* p : ptrs) ctx->dfree(p);
  }
};

// Process-wide tuning cache: (CU count, log2 of block rows, complex128
// matrix) -> tile.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, bool>, BatchTile> g_tune;

int ilog2(int64_t v) {
  int l = 0;
  while (v > 1) {
    v >>= 1;
    ++l;
  }
  return l;
}

}  // namespace

// Wide SpMM traversal order: block rows sorted by (y slab, z, y, x), a slab
// being kSlabY node rows in y.  Consecutive positions then sweep z through
// one thin slab, and a row's neighbours one node plane away in z (the 18 of
// its 27 blocks in the planes below and above) were gathered about
// 2 kSlabY (nx + 1) rows earlier, within what one XCD's L2 still holds; in
// plain (z, y, x) order they lie a whole plane away and are fetched again.
// On the 40^3 sphere with 64 columns: 364 us per product against 397 us in
// plain order (slabs of 2, 4, 8, 16 rows: 390, 368, 364, 368 us).
constexpr int kSlabY = 8;

int ensure_row_order(Problem* P) {
  if (P->row_order) return FEMH_OK;
  const int32_t nn = P->pat.nn;
  const int gx = P->mesh.nx + 1, gy = P->mesh.ny + 1, gz = P->mesh.nz + 1;
  std::vector<int32_t> grid((size_t)nn), order((size_t)nn);
  FEMH_TRY_HIP(hipMemcpy(grid.data(), P->node_grid, sizeof(int32_t) * nn, hipMemcpyDeviceToHost));
  // stable counting sort of the rows (already in (z, y, x) order) by (slab, z)
  const int slabs = (gy + kSlabY - 1) / kSlabY;
  std::vector<int64_t> start((size_t)slabs * gz + 1, 0);
  auto bucket = [&](int32_t g) {
    const int64_t plane = (int64_t)gx * gy;
    const int z = (int)(g / plane), y = (int)((g % plane) / gx);
    return (int64_t)(y / kSlabY) * gz + z;
  };
  for (int32_t a = 0; a < nn; ++a) ++start[bucket(grid[a]) + 1];
  for (size_t i = 1; i < start.size(); ++i) start[i] += start[i - 1];
  for (int32_t a = 0; a < nn; ++a) order[start[bucket(grid[a])]++] = a;
  int32_t* d = (int32_t*)P->alloc(sizeof(int32_t) * nn);
  if (!d) {
    set_error("device allocation failed (row order)");
    return FEMH_E_OOM;
  }
  FEMH_TRY_HIP(hipMemcpy(d, order.data(), sizeof(int32_t) * nn, hipMemcpyHostToDevice));
  P->row_order = d;
  P->pat.row_order = d;
  return FEMH_OK;
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

int autotune_spmm(Problem* P, const double2* val64, const double2* Pv, double2* Qv, double* partials,
                  const BatchScalars* sc) {
  FEMH_TRY(ensure_row_order(P));
  if (P->tile.kind >= 0) return FEMH_OK;
  Ctx* c = P->ctx;
  const std::tuple<int, int, bool> key(c->n_cu, ilog2(P->pat.nn), val64 != nullptr);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      P->tile = it->second;
      P->tile.blocks = k::batched_blocks_for(P->pat.nn, c->n_cu, it->second.blocks);
      return FEMH_OK;
    }
  }
  hipStream_t s = c->stream;
  hipEvent_t e0, e1;
  FEMH_TRY_HIP(hipEventCreate(&e0));
  FEMH_TRY_HIP(hipEventCreate(&e1));
  // Only the FP64 vector kernel is a candidate: the matrix-core kernel's
  // FP64 block products stall indefinite systems (explicit request only).
  float best = 1e30f;
  BatchTile best_tile{0, k::batched_blocks_for(P->pat.nn, c->n_cu, 8)};
  int best_per_cu = 8;
  const int kinds[1] = {0};
  const int per_cus[3] = {2, 4, 8};
  for (int kind : kinds)
    for (int pc : per_cus) {
      BatchTile t{kind, k::batched_blocks_for(P->pat.nn, c->n_cu, pc)};
      FEMH_TRY_HIP(k::bspmm(s, P->pat, P->val32, val64, Pv, Qv, partials, sc, t));  // warm
      FEMH_TRY_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) FEMH_TRY_HIP(k::bspmm(s, P->pat, P->val32, val64, Pv, Qv, partials, sc, t));
      FEMH_TRY_HIP(hipEventRecord(e1, s));
      FEMH_TRY_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      FEMH_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_tile = t;
        best_per_cu = pc;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->tile = best_tile;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = BatchTile{best_tile.kind, best_per_cu};
  return FEMH_OK;
}

int solve_batched(Problem* P, int nrhs, const double2* b, double2* x, const femh_solve_opts& o,
                  femh_solve_stats* st) {
  Ctx* c = P->ctx;
  hipStream_t s = c->stream;
  const int64_t n = 3 * (int64_t)P->pat.nn;
  // narrow layout for up to four right-hand sides, wide otherwise
  const int ld = nrhs <= 4 ? 4 : 64;
  // FEMH_FP64: the complex128 matrix in the product; otherwise the
  // complex64 matrix promoted
  const double2* val64 = o.precision == FEMH_FP64 ? P->val64 : nullptr;
  const size_t v64 = 16 * (size_t)n * ld;
  Scratch W(c);
  double2* B64 = (double2*)W.get(v64);
  double2* X64 = (double2*)W.get(v64);
  double2* R64 = (double2*)W.get(v64);
  double2* P64 = (double2*)W.get(v64);
  double2* Q64 = (double2*)W.get(v64);
  double* partials = (double*)W.get(kPartialBytes);
  BatchScalars* sc = (BatchScalars*)W.get(sizeof(BatchScalars));
  BatchPlan* plan = (BatchPlan*)W.get(sizeof(BatchPlan));
  BatchPlan* plan_mr = (BatchPlan*)W.get(sizeof(BatchPlan));
  BatchScalars* run_all = (BatchScalars*)W.get(sizeof(BatchScalars));
  double* rr64 = (double*)W.get(64 * sizeof(double));
  if (!B64 || !X64 || !R64 || !P64 || !Q64 || !partials || !sc || !plan || !plan_mr || !run_all || !rr64) {
    set_error("device allocation failed (batched workspace)");
    return FEMH_E_OOM;
  }
  const double2* dinv = P->dinv64;
  if (o.precond == FEMH_PRECOND_NONE) {
    double2* ones = (double2*)W.get(16 * n);
    if (!ones) {
      set_error("device allocation failed (identity preconditioner)");
      return FEMH_E_OOM;
    }
    std::vector<double2> h((size_t)n, make_double2(1.0, 0.0));
    FEMH_TRY_HIP(hipMemcpyAsync(ones, h.data(), 16 * n, hipMemcpyHostToDevice, s));
    FEMH_TRY_HIP(hipStreamSynchronize(s));
    dinv = ones;
  }
  const int vblocks = k::batched_vec_blocks(n, ld);
  const int rblocks = k::batched_blocks_for(P->pat.nn, c->n_cu, 4);

  hipEvent_t t0, t1;
  FEMH_TRY_HIP(hipEventCreate(&t0));
  FEMH_TRY_HIP(hipEventCreate(&t1));
  FEMH_TRY_HIP(hipEventRecord(t0, s));

  FEMH_TRY_HIP(k::to_block(s, n, ld, nrhs, b, B64));
  FEMH_TRY_HIP(hipMemsetAsync(X64, 0, v64, s));
  FEMH_TRY_HIP(hipMemsetAsync(P64, 0, v64, s));
  FEMH_TRY_HIP(k::bresidual64(s, P->pat, ld, P->val64, X64, B64, R64, partials, rblocks, rr64, nullptr));
  std::vector<double> hrr(64), bb(64);
  FEMH_TRY_HIP(hipMemcpyAsync(hrr.data(), rr64, 64 * sizeof(double), hipMemcpyDeviceToHost, s));
  FEMH_TRY_HIP(hipStreamSynchronize(s));

  // host mirrors (pinned scalar block for the per-chunk reads)
  BatchScalars* hs = reinterpret_cast<BatchScalars*>(c->pinned);
  static_assert(sizeof(BatchScalars) <= 16384, "pinned scratch too small");
  BatchPlan hp;
  std::memset(hs, 0, sizeof(*hs));
  std::memset(&hp, 0, sizeof(hp));
  hs->max_iters = o.max_iter;
  hs->delta2 = o.inner_rtol * o.inner_rtol;
  hs->bd_tol = 1e-13;  // FP64 residual recurrence: only genuine breakdowns
  std::vector<int> updates(64, 0), final_status(64, FEMH_OK);
  std::vector<double> rel(64, 0.0);
  for (int col = 0; col < 64; ++col) {
    bb[col] = col < nrhs ? hrr[col] : 0.0;
    if (bb[col] > 0.0) {
      hs->done[col] = 0;
      hp.action[col] = 2;
      hp.tol2[col] = o.rtol * o.rtol * bb[col];
      rel[col] = 1.0;
    } else {
      hs->done[col] = 5;
      hp.action[col] = 0;
    }
  }
  FEMH_TRY_HIP(hipMemcpyAsync(sc, hs, sizeof(*hs), hipMemcpyHostToDevice, s));
  FEMH_TRY_HIP(hipMemcpyAsync(plan, &hp, sizeof(hp), hipMemcpyHostToDevice, s));
  FEMH_TRY_HIP(k::brescale(s, n, ld, R64, dinv, P64, partials, vblocks, sc, plan));
  {
    BatchScalars* ra = reinterpret_cast<BatchScalars*>(static_cast<char*>(c->pinned) + 8192);
    static_assert(2 * sizeof(BatchScalars) <= 16384, "pinned scratch too small");
    std::memset(ra, 0, sizeof(*ra));
    ra->active = 1;
    FEMH_TRY_HIP(hipMemcpyAsync(run_all, ra, sizeof(*ra), hipMemcpyHostToDevice, s));
  }
  FEMH_TRY_HIP(hipStreamSynchronize(s));
  BatchTile tile{2, P->spmv.blocks};  // narrow product: the single-RHS SpMV's grid
  if (ld == 64) {
    FEMH_TRY(autotune_spmm(P, val64, P64, Q64, partials, sc));
    tile = P->tile;
  }

  // one chunk of iterations, captured once
  auto launch_chunk = [&]() -> hipError_t {
    for (int i = 0; i < o.check_every; ++i) {
      hipError_t e;
      if ((e = k::bspmm(s, P->pat, P->val32, val64, P64, Q64, partials, sc, tile)) != hipSuccess) return e;
      if ((e = k::bred_alpha(s, partials, tile.blocks, ld, sc)) != hipSuccess) return e;
      if ((e = k::bupdate(s, n, ld, dinv, X64, R64, P64, Q64, partials, vblocks, sc)) != hipSuccess) return e;
      if ((e = k::bred_beta(s, partials, vblocks, ld, sc)) != hipSuccess) return e;
      if ((e = k::bpupdate(s, n, ld, dinv, R64, P64, vblocks, sc, nullptr)) != hipSuccess) return e;
    }
    return hipSuccess;
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = true;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    hipError_t e = launch_chunk();
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess || e2 != hipSuccess || !graph ||
        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
      use_graph = false;
  } else {
    use_graph = false;
  }
  (void)hipGetLastError();
  auto run_chunk = [&]() -> hipError_t { return use_graph ? hipGraphLaunch(exec, s) : launch_chunk(); };

  hipEvent_t ready;
  FEMH_TRY_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  int status = FEMH_OK;
  int guard = 0;
  FEMH_TRY_HIP(run_chunk());
  while (true) {
    FEMH_TRY_HIP(hipMemcpyAsync(hs, sc, sizeof(*hs), hipMemcpyDeviceToHost, s));
    FEMH_TRY_HIP(hipEventRecord(ready, s));
    FEMH_TRY_HIP(run_chunk());
    FEMH_TRY_HIP(hipEventSynchronize(ready));
    bool pending = false, running = false;
    for (int col = 0; col < 64; ++col) {
      const int d = hs->done[col];
      if (d >= 1 && d <= 4) pending = true;
      if (d == 0) running = true;
    }
    if (!pending && !running) break;
    if (++guard > 2 * (o.max_iter / std::max(o.check_every, 1) + 2) + 4096) {
      status = FEMH_E_NOT_CONVERGED;
      break;
    }
    if (!pending) continue;
    // ---- reliable update of the flagged columns
    std::memset(&hp, 0, sizeof(hp));
    int flagged[64];
    for (int col = 0; col < 64; ++col) {
      const int d = hs->done[col];
      flagged[col] = (d >= 1 && d <= 4) ? d : 0;
      hp.action[col] = flagged[col] ? 1 : 0;
    }
    FEMH_TRY_HIP(hipMemcpyAsync(plan, &hp, sizeof(hp), hipMemcpyHostToDevice, s));
    // true residual into the flagged columns only
    FEMH_TRY_HIP(k::bresidual64(s, P->pat, ld, P->val64, X64, B64, R64, partials, rblocks, rr64, plan->action));
    FEMH_TRY_HIP(hipMemcpyAsync(hrr.data(), rr64, 64 * sizeof(double), hipMemcpyDeviceToHost, s));
    FEMH_TRY_HIP(hipStreamSynchronize(s));
    std::memset(&hp, 0, sizeof(hp));
    for (int col = 0; col < 64; ++col) {
      if (!flagged[col]) continue;
      ++updates[col];
      rel[col] = std::sqrt(hrr[col] / bb[col]);
      const int iters = hs->iters[col];
      if (rel[col] <= o.rtol) {
        hp.action[col] = 3;
        hp.final_state[col] = 5;
        final_status[col] = FEMH_OK;
      } else if (flagged[col] == 2 || iters >= o.max_iter || updates[col] >= 50 * std::max(o.max_outer, 1) ||
                 !std::isfinite(rel[col])) {
        hp.action[col] = 3;
        hp.final_state[col] = 6;
        final_status[col] = FEMH_E_NOT_CONVERGED;
      } else {
        hp.action[col] = flagged[col] == 3 ? 2 : 1;
        hp.tol2[col] = o.rtol * o.rtol * bb[col];
      }
    }
    // columns restarting after a breakdown first take a minimal-residual
    // step, so the restart does not meet the same breakdown again
    bool any_restart = false;
    BatchPlan hm;
    std::memset(&hm, 0, sizeof(hm));
    for (int col = 0; col < 64; ++col)
      if (hp.action[col] == 2) {
        hm.action[col] = 2;
        hm.tol2[col] = hp.tol2[col];
        any_restart = true;
      }
    if (any_restart) {
      FEMH_TRY_HIP(hipMemcpyAsync(plan_mr, &hm, sizeof(hm), hipMemcpyHostToDevice, s));
      FEMH_TRY_HIP(k::brescale(s, n, ld, R64, dinv, P64, partials, vblocks, sc, plan_mr));
      FEMH_TRY_HIP(k::bmr_step(s, P->pat, n, ld, P->val32, val64, X64, R64, P64, Q64, partials, vblocks, tile,
                               run_all, sc, plan_mr));
    }
    FEMH_TRY_HIP(hipMemcpyAsync(plan, &hp, sizeof(hp), hipMemcpyHostToDevice, s));
    FEMH_TRY_HIP(k::brescale(s, n, ld, R64, dinv, P64, partials, vblocks, sc, plan));
    FEMH_TRY_HIP(k::bpupdate(s, n, ld, dinv, R64, P64, vblocks, sc, plan->action));
    FEMH_TRY_HIP(run_chunk());
  }
  FEMH_TRY_HIP(hipStreamSynchronize(s));
  (void)hipEventDestroy(ready);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  FEMH_TRY_HIP(k::from_block(s, n, ld, nrhs, X64, x));
  FEMH_TRY_HIP(hipEventRecord(t1, s));
  FEMH_TRY_HIP(hipEventSynchronize(t1));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, t0, t1);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  for (int col = 0; col < nrhs; ++col) {
    std::memset(&st[col], 0, sizeof(st[col]));
    st[col].status = bb[col] > 0.0 ? final_status[col] : FEMH_OK;
    st[col].iters = hs->iters[col];
    st[col].outer_iters = updates[col];
    st[col].rel_residual = bb[col] > 0.0 ? rel[col] : 0.0;
    st[col].seconds = ms * 1e-3;
    if (hs->done[col] < 5 && bb[col] > 0.0) st[col].status = FEMH_E_NOT_CONVERGED;
    if (st[col].status != FEMH_OK && status == FEMH_OK) status = st[col].status;
  }
  if (status != FEMH_OK) set_error("batched solve: at least one column did not converge");
  return status;
}

}  // namespace femh
