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
  if (P->imported) return FEMH_OK;  // no mesh: the rows keep their own order
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

// Non-blocking state machine of one batched solve (the serving loop drives
// several of them together; solve_batched drives one to the end).
struct BatchStepper {
  enum Phase { START, WAIT_INIT, ITER, DONE };
  Problem* P = nullptr;
  Ctx* c = nullptr;
  hipStream_t s = nullptr;
  int nrhs = 0;
  const double2* b = nullptr;
  double2* x = nullptr;
  femh_solve_opts o{};
  int64_t n = 0;
  int ld = 4;
  size_t v64 = 0;
  const double2* val64 = nullptr;  // complex128 matrix in the product, or null (complex64 promoted)
  std::vector<void*> owned;
  double2 *B64 = nullptr, *X64 = nullptr, *R64 = nullptr, *P64 = nullptr, *Q64 = nullptr;
  double* partials = nullptr;
  BatchScalars *sc = nullptr, *run_all = nullptr;
  BatchPlan *plan = nullptr, *plan_mr = nullptr;
  double* rr64 = nullptr;
  const double2* dinv = nullptr;
  int vblocks = 0, rblocks = 0;
  BatchTile tile{2, 0};
  // pinned host mirrors: scalar block, the always-active block, residual norms
  void* pinned = nullptr;
  BatchScalars* hs = nullptr;
  BatchScalars* ra = nullptr;
  double* hrr = nullptr;
  BatchPlan hp{};
  std::vector<int> updates, final_status;
  std::vector<double> rel, bb;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = false;
  hipEvent_t ready = nullptr, ev_init = nullptr;
  bool queued = false;  // a scalar readback (and the chunk behind it) is in flight
  int guard = 0;
  int status = FEMH_OK;
  Phase phase = START;

  void* dev(size_t bytes) {
    void* p = c->dmalloc(bytes);
    if (p) owned.push_back(p);
    return p;
  }

  ~BatchStepper() {
    if (!c) return;
    (void)hipStreamSynchronize(s);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ready) (void)hipEventDestroy(ready);
    if (ev_init) (void)hipEventDestroy(ev_init);
    if (pinned) (void)hipHostFree(pinned);
    for (void* p : owned) c->dfree(p);
  }

  int init(Problem* prob, int nrhs_, const double2* b_, double2* x_, const femh_solve_opts& opts) {
    P = prob;
    c = prob->ctx;
    s = c->stream;
    nrhs = nrhs_;
    b = b_;
    x = x_;
    o = opts;
    n = 3 * (int64_t)P->pat.nn;
    // narrow layout for up to four right-hand sides, wide otherwise
    ld = nrhs <= 4 ? 4 : 64;
    // FEMH_FP64: the complex128 matrix in the product; otherwise the
    // complex64 matrix promoted
    val64 = o.precision == FEMH_FP64 ? P->val64 : nullptr;
    v64 = 16 * (size_t)n * ld;
    B64 = (double2*)dev(v64);
    X64 = (double2*)dev(v64);
    R64 = (double2*)dev(v64);
    P64 = (double2*)dev(v64);
    Q64 = (double2*)dev(v64);
    partials = (double*)dev(kPartialBytes);
    sc = (BatchScalars*)dev(sizeof(BatchScalars));
    plan = (BatchPlan*)dev(sizeof(BatchPlan));
    plan_mr = (BatchPlan*)dev(sizeof(BatchPlan));
    run_all = (BatchScalars*)dev(sizeof(BatchScalars));
    rr64 = (double*)dev(64 * sizeof(double));
    if (!B64 || !X64 || !R64 || !P64 || !Q64 || !partials || !sc || !plan || !plan_mr || !run_all || !rr64) {
      set_error("device allocation failed (batched workspace)");
      return FEMH_E_OOM;
    }
    dinv = P->dinv64;
    if (o.precond == FEMH_PRECOND_NONE) {
      double2* ones = (double2*)dev(16 * n);
      if (!ones) {
        set_error("device allocation failed (identity preconditioner)");
        return FEMH_E_OOM;
      }
      std::vector<double2> h((size_t)n, make_double2(1.0, 0.0));
      FEMH_TRY_HIP(hipMemcpyAsync(ones, h.data(), 16 * n, hipMemcpyHostToDevice, s));
      FEMH_TRY_HIP(hipStreamSynchronize(s));
      dinv = ones;
    }
    static_assert(2 * sizeof(BatchScalars) + 64 * sizeof(double) <= 32768, "pinned block too small");
    FEMH_TRY_HIP(hipHostMalloc(&pinned, 32768, hipHostMallocDefault));
    hs = reinterpret_cast<BatchScalars*>(pinned);
    ra = reinterpret_cast<BatchScalars*>(static_cast<char*>(pinned) + 12288);
    hrr = reinterpret_cast<double*>(static_cast<char*>(pinned) + 24576);
    FEMH_TRY_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    FEMH_TRY_HIP(hipEventCreateWithFlags(&ev_init, hipEventDisableTiming));
    vblocks = k::batched_vec_blocks(n, ld);
    rblocks = k::batched_blocks_for(P->pat.nn, c->n_cu, 4);
    updates.assign(64, 0);
    final_status.assign(64, FEMH_OK);
    rel.assign(64, 0.0);
    bb.assign(64, 0.0);
    return FEMH_OK;
  }

  hipError_t launch_chunk() {
    for (int i = 0; i < o.check_every; ++i) {
      hipError_t e;
      if ((e = k::bspmm(s, P->pat, P->val32, val64, P64, Q64, partials, sc, tile)) != hipSuccess) return e;
      if ((e = k::bred_alpha(s, partials, tile.blocks, ld, sc)) != hipSuccess) return e;
      if ((e = k::bupdate(s, n, ld, dinv, X64, R64, P64, Q64, partials, vblocks, sc)) != hipSuccess) return e;
      if ((e = k::bred_beta(s, partials, vblocks, ld, sc)) != hipSuccess) return e;
      if ((e = k::bpupdate(s, n, ld, dinv, R64, P64, vblocks, sc, nullptr)) != hipSuccess) return e;
    }
    return hipSuccess;
  }

  hipError_t run_chunk() { return use_graph ? hipGraphLaunch(exec, s) : launch_chunk(); }

  // x = 0, r = b and the columns' ||b||^2
  int start() {
    FEMH_TRY_HIP(k::to_block(s, n, ld, nrhs, b, B64));
    FEMH_TRY_HIP(hipMemsetAsync(X64, 0, v64, s));
    FEMH_TRY_HIP(hipMemsetAsync(P64, 0, v64, s));
    FEMH_TRY_HIP(k::bresidual64(s, P->pat, ld, P->val64, X64, B64, R64, partials, rblocks, rr64, nullptr));
    FEMH_TRY_HIP(hipMemcpyAsync(hrr, rr64, 64 * sizeof(double), hipMemcpyDeviceToHost, s));
    FEMH_TRY_HIP(hipEventRecord(ev_init, s));
    phase = WAIT_INIT;
    return FEMH_OK;
  }

  int begin_iterating() {
    std::memset(hs, 0, sizeof(*hs));
    std::memset(&hp, 0, sizeof(hp));
    hs->max_iters = o.max_iter;
    hs->delta2 = o.inner_rtol * o.inner_rtol;
    hs->bd_tol = 1e-13;  // FP64 residual recurrence: only genuine breakdowns
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
    std::memset(ra, 0, sizeof(*ra));
    ra->active = 1;
    FEMH_TRY_HIP(hipMemcpyAsync(run_all, ra, sizeof(*ra), hipMemcpyHostToDevice, s));
    FEMH_TRY_HIP(hipStreamSynchronize(s));
    tile = BatchTile{2, P->spmv.blocks};  // narrow product: the single-RHS SpMV's grid
    if (ld == 64) {
      FEMH_TRY(autotune_spmm(P, val64, P64, Q64, partials, sc));
      tile = P->tile;
    }
    // one chunk of iterations, captured once
    use_graph = false;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      hipError_t e = launch_chunk();
      hipError_t e2 = hipStreamEndCapture(s, &graph);
      use_graph = e == hipSuccess && e2 == hipSuccess && graph &&
                  hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    }
    (void)hipGetLastError();
    FEMH_TRY_HIP(run_chunk());
    phase = ITER;
    return FEMH_OK;
  }

  // Reliable update of the columns that asked for one (reads back the FP64
  // true residual norms, so it waits on the stream).
  int reliable_update() {
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
    FEMH_TRY_HIP(hipMemcpyAsync(hrr, rr64, 64 * sizeof(double), hipMemcpyDeviceToHost, s));
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
    return FEMH_OK;
  }

  int finish() {
    FEMH_TRY_HIP(hipStreamSynchronize(s));
    FEMH_TRY_HIP(k::from_block(s, n, ld, nrhs, X64, x));
    phase = DONE;
    return FEMH_OK;
  }

  // Advance without blocking except inside a reliable update; *progress is
  // set when something moved.
  int step(bool* progress) {
    *progress = false;
    switch (phase) {
      case START:
        *progress = true;
        return start();
      case WAIT_INIT:
        if (hipEventQuery(ev_init) != hipSuccess) return FEMH_OK;
        *progress = true;
        return begin_iterating();
      case ITER: {
        if (!queued) {
          // read the scalars behind the chunk in flight, one more chunk queued ahead
          FEMH_TRY_HIP(hipMemcpyAsync(hs, sc, sizeof(*hs), hipMemcpyDeviceToHost, s));
          FEMH_TRY_HIP(hipEventRecord(ready, s));
          FEMH_TRY_HIP(run_chunk());
          queued = true;
          *progress = true;
        }
        if (hipEventQuery(ready) != hipSuccess) return FEMH_OK;
        queued = false;
        *progress = true;
        bool pending = false, running = false;
        for (int col = 0; col < 64; ++col) {
          const int d = hs->done[col];
          if (d >= 1 && d <= 4) pending = true;
          if (d == 0) running = true;
        }
        if (!pending && !running) return finish();
        if (++guard > 2 * (o.max_iter / std::max(o.check_every, 1) + 2) + 4096) {
          status = FEMH_E_NOT_CONVERGED;
          return finish();
        }
        if (pending) return reliable_update();
        return FEMH_OK;
      }
      case DONE:
        return FEMH_OK;
    }
    return FEMH_OK;
  }

  void wait() {
    if (phase == WAIT_INIT) (void)hipEventSynchronize(ev_init);
    else if (phase == ITER && queued) (void)hipEventSynchronize(ready);
  }

  // per-column stats; returns the first failing status (FEMH_OK if none)
  int fill_stats(femh_solve_stats* st) const {
    int first = status;
    for (int col = 0; col < nrhs; ++col) {
      std::memset(&st[col], 0, sizeof(st[col]));
      st[col].status = bb[col] > 0.0 ? final_status[col] : FEMH_OK;
      st[col].iters = hs->iters[col];
      st[col].outer_iters = updates[col];
      st[col].rel_residual = bb[col] > 0.0 ? rel[col] : 0.0;
      if (hs->done[col] < 5 && bb[col] > 0.0) st[col].status = FEMH_E_NOT_CONVERGED;
      if (st[col].status != FEMH_OK && first == FEMH_OK) first = st[col].status;
    }
    return first;
  }
};

BatchStepper* batch_stepper_create(Problem* P, int nrhs, const double2* b, double2* x, const femh_solve_opts& o) {
  BatchStepper* s = new BatchStepper();
  if (s->init(P, nrhs, b, x, o) != FEMH_OK) {
    delete s;
    return nullptr;
  }
  return s;
}
int batch_stepper_step(BatchStepper* s, bool* progress) { return s->step(progress); }
bool batch_stepper_done(const BatchStepper* s) { return s->phase == BatchStepper::DONE; }
void batch_stepper_wait(BatchStepper* s) { s->wait(); }
bool batch_stepper_iterating(const BatchStepper* s) {
  return s->phase == BatchStepper::ITER || s->phase == BatchStepper::DONE;
}
int batch_stepper_stats(const BatchStepper* s, femh_solve_stats* st) { return s->fill_stats(st); }
void batch_stepper_destroy(BatchStepper* s) { delete s; }

// Five to eight right-hand sides run as two narrow groups (four + the
// rest), stepped together on the stream: on the 30^3 and 40^3 spheres two
// narrow groups of four take 0.73x and 0.65x the time of one 64-wide batch
// of eight; at twelve they are level and at sixteen the wide batch wins.
constexpr int kMaxNarrowGroups = 8;

int solve_batched(Problem* P, int nrhs, const double2* b, double2* x, const femh_solve_opts& o,
                  femh_solve_stats* st) {
  Ctx* c = P->ctx;
  const int64_t n = 3 * (int64_t)P->pat.nn;
  hipEvent_t t0, t1;
  FEMH_TRY_HIP(hipEventCreate(&t0));
  FEMH_TRY_HIP(hipEventCreate(&t1));
  FEMH_TRY_HIP(hipEventRecord(t0, c->stream));
  std::vector<BatchStepper*> groups;
  std::vector<int> first;
  int rc = FEMH_OK;
  const int width = nrhs <= kMaxNarrowGroups ? 4 : nrhs;
  for (int g = 0; g < nrhs && rc == FEMH_OK; g += width) {
    const int k = std::min(width, nrhs - g);
    BatchStepper* S = batch_stepper_create(P, k, b + g * n, x + g * n, o);
    if (!S) {
      rc = FEMH_E_OOM;
      break;
    }
    groups.push_back(S);
    first.push_back(g);
  }
  while (rc == FEMH_OK) {
    bool all_done = true, progress = false;
    BatchStepper* waiter = nullptr;
    for (BatchStepper* S : groups) {
      if (batch_stepper_done(S)) continue;
      bool prog = false;
      rc = S->step(&prog);
      if (rc != FEMH_OK) break;
      progress |= prog;
      if (!batch_stepper_done(S)) {
        all_done = false;
        if (!waiter) waiter = S;
      }
    }
    if (rc != FEMH_OK || all_done) break;
    if (!progress && waiter) waiter->wait();
  }
  (void)hipEventRecord(t1, c->stream);
  (void)hipEventSynchronize(t1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, t0, t1);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  int status = FEMH_OK;
  if (rc == FEMH_OK) {
    for (size_t i = 0; i < groups.size(); ++i) {
      const int s = groups[i]->fill_stats(st + first[i]);
      if (s != FEMH_OK && status == FEMH_OK) status = s;
    }
    for (int col = 0; col < nrhs; ++col) st[col].seconds = ms * 1e-3;
    if (log_level() >= 1) {
      int lo = st[0].iters, hi = st[0].iters;
      double worst = 0.0;
      for (int col = 0; col < nrhs; ++col) {
        lo = std::min(lo, st[col].iters);
        hi = std::max(hi, st[col].iters);
        worst = std::max(worst, st[col].rel_residual);
      }
      logf(1, "batched: %d columns in %zu group(s), %d-%d iterations, worst relative residual %.3e, %.3f s, status %d",
           nrhs, groups.size(), lo, hi, worst, ms * 1e-3, status);
    }
  }
  for (BatchStepper* S : groups) delete S;
  if (rc != FEMH_OK) return rc;
  if (status != FEMH_OK) set_error("batched solve: at least one column did not converge");
  return status;
}

}  // namespace femh
