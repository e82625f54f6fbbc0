// Host drivers of the single-RHS Krylov solves, written as a non-blocking
// state machine (Stepper) so one code path serves femh_solve and the
// serving loop.  The iteration itself never waits on the host: every kernel
// reads the device scalar block and returns at once when the recurrence has
// stopped, so the host queues `check_every` iterations at a time, keeps up
// to two such chunks in flight, and reads the scalar block back
// asynchronously (pinned memory + event).
//
// FP64 mode: COCG with diagonal preconditioning (section 3.1.5.1) on the
// complex128 matrix, in its single-reduction form (one product and one
// update kernel per iteration, see sr_update_c128); when the recursive
// residual meets the tolerance the FP64 true residual b - A x is formed and,
// if it does not meet it, COCG restarts from it.  With the block incomplete
// Cholesky preconditioner (sections 3.1.5.2-3.1.5.3) the FP64 recurrence
// runs in textbook order: product, update, z = M^-1 r, direction update.
//
// Matrix-mixed mode: the FP64 COCG recurrence with the complex64 matrix in
// the product (values promoted, FP64 sums); reliable updates against the
// FP64 matrix replace the recursive residual by the true one (keeping the
// direction) whenever it has fallen by inner_rtol.
//
// Mixed mode: the COCG recurrence runs on the complex64 matrix and
// complex64 vectors, on a residual scaled to unit norm.  When its recursive
// residual has fallen by inner_rtol since the last update (or meets the
// tolerance, or breaks down), the partial solution is folded into the FP64
// iterate, the FP64 true residual is recomputed, and the recurrence
// continues from it with the same search direction (reliable update) or
// restarts after a breakdown.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace femh {

namespace {

constexpr int kPartialSlots = 2048 * 4;  // partial sums: workgroups x 4 values
// With profiling on, every kProfStride-th product of a solve is bracketed
// with events (a sample: each pair of events adds about 2 us to its
// iteration, so bracketing them all would slow the solve being measured).
constexpr int kProfStride = 8;

// Device-side auxiliary scalars used outside the COCG block.
struct Aux {
  double rr;  // FP64 true residual norm^2
  double pad;
  uint32_t ticket[4];
};

// Timing events without the system-scope fence, so bracketing every product
// perturbs the kernels as little as possible.
hipEvent_t pool_event(Ctx* c, size_t i) {
  while (c->ev_pool.size() <= i) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[i];
}

}  // namespace

struct Stepper {
  enum Phase { START, WAIT_INIT, ITER, WAIT_CHECK, DONE };
  Problem* P = nullptr;
  Ctx* c = nullptr;
  hipStream_t s = nullptr;
  const double2* b = nullptr;
  double2* x = nullptr;
  femh_solve_opts o{};
  bool mixed = false;  // complex64 vectors and matrix
  bool m32 = false;    // complex64 matrix, complex128 vectors
  bool sr = false;     // FP64: single-reduction recurrence
  bool bic = false;    // FP64 with block incomplete Cholesky (textbook order)
  int64_t n = 0;
  std::vector<void*> owned;
  // device workspace
  double2 *r64 = nullptr, *p64 = nullptr, *q64 = nullptr;
  double2 *z64 = nullptr, *s64 = nullptr;  // single-reduction form: z = D^-1 r, s = A p (q64 holds A z);
                                           // block incomplete Cholesky: z = M^-1 r
  float2 *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr;
  void* partials = nullptr;  // SpMV -> update partials; also once-per-segment kernels
  void* partials_b = nullptr;  // update -> direction-update partials (single-reduction form:
                               // two buffers of 8 values per workgroup, update -> next
                               // update, by parity)
  void* partials_c = nullptr;  // block incomplete Cholesky: the application's totals in slot 0,
                               // the other slots zero (read as the direction update's partials)
  double* bic_stage = nullptr;    // per-block sums of the application
  uint32_t* bic_ticket = nullptr;  // its last-block counter
  CocgScalars* sc = nullptr;
  Aux* aux = nullptr;
  const double2* dinv64 = nullptr;
  const float2* dinv32 = nullptr;
  // host mirrors (pinned): two scalar-block buffers for chunks in flight
  void* pinned = nullptr;
  CocgScalars* hs[2] = {nullptr, nullptr};
  Aux* ha = nullptr;
  CocgScalars* hw = nullptr;  // staging for host -> device writes
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t ev_aux = nullptr;
  int inflight = 0, head = 0;  // chunks queued and not yet examined; oldest slot
  bool stale = false;          // chunks queued after a stop are drained, not read
  CocgScalars stop_state{};
  Phase phase = START;
  // solve state
  double bb = 0.0, scale = 1.0, rel = 1.0;
  int outer = 0;
  int iters = 0;
  int status = FEMH_E_NOT_CONVERGED;
  int last_done = 0;
  // profiling: launch numbering of the current segment.  Only the
  // single-solve driver turns timing on: the context's event pool is indexed
  // by this stepper's launch count, so steppers running concurrently (the
  // server's) must not record into it.
  bool timing = false;
  int launches = 0, seg_first = 0, seg_iters = 0;
  double prof_seconds = 0.0;
  int64_t prof_count = 0;

  void* dev(size_t bytes) {
    void* p = c->dmalloc(bytes);
    if (p) owned.push_back(p);
    return p;
  }

  ~Stepper() {
    if (c) {
      (void)hipStreamSynchronize(s);
      for (void* p : owned) c->dfree(p);
      for (int i = 0; i < 2; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
      if (ev_aux) (void)hipEventDestroy(ev_aux);
      if (pinned) (void)hipHostFree(pinned);
    }
  }

  int oom() {
    set_error("device allocation failed (solver workspace)");
    return FEMH_E_OOM;
  }

  int init(Problem* prob, const double2* b_dev, double2* x_dev, const femh_solve_opts& opts) {
    P = prob;
    c = prob->ctx;
    s = c->stream;
    b = b_dev;
    x = x_dev;
    o = opts;
    mixed = o.precision == FEMH_MIXED;
    m32 = o.precision == FEMH_MIXED_MATRIX;
    bic = !mixed && !m32 && o.precond == FEMH_PRECOND_BIC0;
    sr = !mixed && !m32 && !bic;
    n = 3 * (int64_t)P->pat.nn;
    r64 = (double2*)dev(16 * n);
    if (!r64) return oom();
    if (mixed) {
      x32 = (float2*)dev(8 * n);
      r32 = (float2*)dev(8 * n);
      p32 = (float2*)dev(8 * n);
      q32 = (float2*)dev(8 * n);
      if (!x32 || !r32 || !p32 || !q32) return oom();
    } else {
      p64 = (double2*)dev(16 * n);
      q64 = (double2*)dev(16 * n);
      if (!p64 || !q64) return oom();
      if (sr || bic) {
        z64 = (double2*)dev(16 * n);
        if (!z64) return oom();
      }
      if (sr) {
        s64 = (double2*)dev(16 * n);
        if (!s64) return oom();
      }
    }
    partials = dev(8 * kPartialSlots);
    partials_b = dev(8 * kPartialSlots * (sr ? 4 : 1));
    sc = (CocgScalars*)dev(sizeof(CocgScalars));
    aux = (Aux*)dev(sizeof(Aux));
    if (!partials || !partials_b || !sc || !aux) return oom();
    dinv64 = P->dinv64;
    dinv32 = P->dinv32;
    if (bic) {
      // update and direction update run with D = I; z comes from the factor
      FEMH_TRY(ensure_bic(P, o.precond_block));
      partials_c = dev(8 * kPartialSlots);
      const size_t stage_bytes = 8 * k::bic_stage_doubles(P->bic.nblk) + 256;
      bic_stage = (double*)dev(stage_bytes);
      if (!partials_c || !bic_stage) return oom();
      bic_ticket = reinterpret_cast<uint32_t*>(bic_stage + k::bic_stage_doubles(P->bic.nblk));
      FEMH_TRY_HIP(hipMemsetAsync(partials_c, 0, 8 * kPartialSlots, s));
      FEMH_TRY_HIP(hipMemsetAsync(bic_stage, 0, stage_bytes, s));
    }
    if (o.precond == FEMH_PRECOND_NONE || bic) {
      if (mixed) {
        float2* ones = (float2*)dev(8 * n);
        if (!ones) return oom();
        std::vector<float2> h((size_t)n, make_float2(1.f, 0.f));
        FEMH_TRY_HIP(hipMemcpyAsync(ones, h.data(), 8 * n, hipMemcpyHostToDevice, s));
        FEMH_TRY_HIP(hipStreamSynchronize(s));
        dinv32 = ones;
      } else {
        double2* ones = (double2*)dev(16 * n);
        if (!ones) return oom();
        std::vector<double2> h((size_t)n, make_double2(1.0, 0.0));
        FEMH_TRY_HIP(hipMemcpyAsync(ones, h.data(), 16 * n, hipMemcpyHostToDevice, s));
        FEMH_TRY_HIP(hipStreamSynchronize(s));
        dinv64 = ones;
      }
    }
    static_assert(sizeof(CocgScalars) <= 1024, "scalar block too large");
    FEMH_TRY_HIP(hipHostMalloc(&pinned, 4096, hipHostMallocDefault));
    char* base = reinterpret_cast<char*>(pinned);
    hs[0] = reinterpret_cast<CocgScalars*>(base);
    hs[1] = reinterpret_cast<CocgScalars*>(base + 1024);
    ha = reinterpret_cast<Aux*>(base + 2048);
    hw = reinterpret_cast<CocgScalars*>(base + 3072);
    for (int i = 0; i < 2; ++i) FEMH_TRY_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    FEMH_TRY_HIP(hipEventCreateWithFlags(&ev_aux, hipEventDisableTiming));
    return FEMH_OK;
  }

  double* dpart() { return reinterpret_cast<double*>(partials); }
  // single-reduction form: two buffers of 2048 workgroups x 8 values
  void* bpart(int slot) { return reinterpret_cast<double*>(partials_b) + (size_t)slot * 2 * kPartialSlots; }

  // single-reduction segment start from the residual in r64
  int queue_sr_init() {
    FEMH_TRY_HIP(k::sr_init_c128(s, n, r64, dinv64, z64, p64, s64, sc, bpart(par()), par()));
    return FEMH_OK;
  }

  // block incomplete Cholesky segment start from the residual in r64
  int queue_bic_start() {
    double* tot = reinterpret_cast<double*>(partials_c);
    FEMH_TRY_HIP(k::bic_apply(s, P->bic, r64, z64, bic_stage, bic_ticket, tot, sc));
    FEMH_TRY_HIP(k::bic_init(s, n, z64, p64, sc, tot, par()));
    return FEMH_OK;
  }

  // ---- queue helpers
  int queue_residual() {
    FEMH_TRY_HIP(k::residual_c128(s, P->pat, P->val64, x, b, r64, dpart(), aux->ticket, &aux->rr, P->spmv));
    FEMH_TRY_HIP(hipMemcpyAsync(ha, aux, sizeof(Aux), hipMemcpyDeviceToHost, s));
    FEMH_TRY_HIP(hipEventRecord(ev_aux, s));
    return FEMH_OK;
  }

  int par() const { return launches & 1; }

  int queue_iteration() {
    const bool prof = timing && launches % kProfStride == 0;
    const int pr = par();
    const int nin = P->spmv.blocks;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof) {
      e0 = pool_event(c, 2 * (size_t)(launches / kProfStride));
      e1 = pool_event(c, 2 * (size_t)(launches / kProfStride) + 1);
      if (!e0 || !e1) {
        set_error("hipEventCreate failed");
        return FEMH_E_DEVICE;
      }
      FEMH_TRY_HIP(hipEventRecord(e0, s));
    }
    if (mixed) {
      FEMH_TRY_HIP(k::cocg_spmv_dot_c64(s, P->pat, P->val32, p32, q32, sc, partials, P->spmv));
      if (prof) FEMH_TRY_HIP(hipEventRecord(e1, s));
      FEMH_TRY_HIP(k::cocg_update_c64(s, n, dinv32, x32, r32, p32, q32, sc, partials, nin, partials_b, pr));
      FEMH_TRY_HIP(k::cocg_pupdate_c64(s, n, dinv32, r32, p32, sc, partials_b, pr));
    } else if (sr) {
      FEMH_TRY_HIP(k::cocg_spmv_dot_c128(s, P->pat, P->val64, z64, q64, sc, partials, P->spmv));
      if (prof) FEMH_TRY_HIP(hipEventRecord(e1, s));
      FEMH_TRY_HIP(k::sr_update_c128(s, n, dinv64, x, z64, q64, p64, s64, sc, partials, nin, bpart(pr),
                                     bpart(pr ^ 1), pr));
    } else if (bic) {
      // textbook order with z = M^-1 r between the update and the direction
      // update, which reads the application's totals as its partials
      FEMH_TRY_HIP(k::cocg_spmv_dot_c128(s, P->pat, P->val64, p64, q64, sc, partials, P->spmv));
      if (prof) FEMH_TRY_HIP(hipEventRecord(e1, s));
      FEMH_TRY_HIP(k::cocg_update_c128(s, n, dinv64, x, r64, p64, q64, sc, partials, nin, partials_b, pr));
      FEMH_TRY_HIP(k::bic_apply(s, P->bic, r64, z64, bic_stage, bic_ticket,
                                reinterpret_cast<double*>(partials_c), sc));
      FEMH_TRY_HIP(k::cocg_pupdate_c128(s, n, dinv64, z64, p64, sc, partials_c, pr));
    } else {
      FEMH_TRY_HIP(k::cocg_spmv_dot_m32(s, P->pat, P->val32, p64, q64, sc, partials, P->spmv));
      if (prof) FEMH_TRY_HIP(hipEventRecord(e1, s));
      FEMH_TRY_HIP(k::cocg_update_c128(s, n, dinv64, x, r64, p64, q64, sc, partials, nin, partials_b, pr));
      FEMH_TRY_HIP(k::cocg_pupdate_c128(s, n, dinv64, r64, p64, sc, partials_b, pr));
    }
    ++launches;
    return FEMH_OK;
  }

  int queue_chunk(int count) {
    for (int i = 0; i < count; ++i) FEMH_TRY(queue_iteration());
    const int slot = (head + inflight) & 1;
    FEMH_TRY_HIP(hipMemcpyAsync(hs[slot], sc, sizeof(CocgScalars), hipMemcpyDeviceToHost, s));
    FEMH_TRY_HIP(hipEventRecord(ev[slot], s));
    ++inflight;
    return FEMH_OK;
  }

  void new_segment(int iters_now) {
    seg_first = launches;
    seg_iters = iters_now;
    inflight = 0;
    head = 0;
    stale = false;
    phase = ITER;
  }

  void collect_profile(int iters_now) {
    if (!timing) return;
    // the single-reduction form runs one more full product than updates
    // (the step that stops does so after its product)
    const int real = std::min(iters_now - seg_iters + (sr ? 1 : 0), launches - seg_first);
    (void)hipStreamSynchronize(s);
    for (int i = 0; i < real; ++i) {
      const int l = seg_first + i;
      if (l % kProfStride) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev_pool[2 * (size_t)(l / kProfStride)],
                              c->ev_pool[2 * (size_t)(l / kProfStride) + 1]) == hipSuccess) {
        prof_seconds += ms * 1e-3;
        ++prof_count;
      }
    }
  }

  const char* mode_name() const {
    if (mixed) return "complex64 vectors and matrix";
    if (m32) return "complex64 matrix, FP64 vectors";
    return bic ? "FP64, block incomplete Cholesky" : "FP64";
  }
  // recursive residual of a scalar block relative to ||b||
  double rec_rel(const CocgScalars& st) const {
    return std::sqrt(st.rr * (mixed ? scale * scale : 1.0) / bb);
  }

  // ---- phases
  int start() {
    FEMH_TRY_HIP(hipMemsetAsync(aux, 0, sizeof(Aux), s));
    FEMH_TRY_HIP(hipMemsetAsync(x, 0, 16 * n, s));
    if (mixed) FEMH_TRY_HIP(hipMemsetAsync(x32, 0, 8 * n, s));
    FEMH_TRY(queue_residual());  // r = b and ||b||^2 (x = 0)
    phase = WAIT_INIT;
    return FEMH_OK;
  }

  int begin_iterating() {
    std::memset(hw, 0, sizeof(*hw));
    hw->max_iters = o.max_iter;
    if (mixed) {
      scale = std::sqrt(bb);
      hw->bb = 1.0;
      hw->bd_tol = 1e-6;
      hw->delta2 = o.inner_rtol * o.inner_rtol;
      FEMH_TRY_HIP(hipMemcpyAsync(sc, hw, sizeof(*hw), hipMemcpyHostToDevice, s));
      FEMH_TRY_HIP(k::cocg_rescale_c64(s, n, r64, 1.0 / scale, dinv32, r32, p32, sc, partials, 1.0,
                                       o.rtol * o.rtol * bb / (scale * scale), 1, par()));
    } else {
      hw->tol2 = o.rtol * o.rtol;
      hw->bb = bb;
      hw->bd_tol = 1e-14;
      if (m32) hw->delta2 = o.inner_rtol * o.inner_rtol;
      FEMH_TRY_HIP(hipMemcpyAsync(sc, hw, sizeof(*hw), hipMemcpyHostToDevice, s));
      if (sr) FEMH_TRY(queue_sr_init());
      else if (bic) FEMH_TRY(queue_bic_start());
      else FEMH_TRY_HIP(k::cocg_init_c128(s, n, r64, dinv64, x, r64, p64, sc, partials, 0, par()));
    }
    new_segment(0);
    logf(1, "solve: %lld unknowns, %s, rtol %.1e, ||b|| = %.3e", (long long)n, mode_name(), o.rtol, std::sqrt(bb));
    return FEMH_OK;
  }

  // the recurrence stopped: fold (mixed) and form the FP64 true residual
  int on_stop(const CocgScalars& st) {
    last_done = st.done;
    iters = st.iters_out;
    static const char* why[] = {"running", "converged", "iteration limit", "breakdown", "residual fell by inner_rtol"};
    logf(1, "solve: segment stopped at iteration %d (%s), recursive |r|/|b| = %.3e", iters,
         st.done >= 0 && st.done <= 4 ? why[st.done] : "?", rec_rel(st));
    collect_profile(st.iters_out);
    if (mixed) FEMH_TRY_HIP(k::ir_fold(s, n, x32, scale, x));
    FEMH_TRY(queue_residual());
    phase = WAIT_CHECK;
    return FEMH_OK;
  }

  int on_check() {
    rel = std::sqrt(ha->rr / bb);
    ++outer;
    logf(1, "solve: true |b - Ax|/|b| = %.3e after %d iterations", rel, iters);
    if (rel <= o.rtol) return finish(FEMH_OK);
    if (last_done == 2 || iters >= o.max_iter || !std::isfinite(rel)) return finish(FEMH_E_NOT_CONVERGED);
    const int cap = (mixed || m32) ? std::max(o.max_outer, 1) * 50 : std::max(o.max_outer, 1);
    if (outer > cap) return finish(last_done == 3 ? FEMH_E_BREAKDOWN : FEMH_E_NOT_CONVERGED);
    if (last_done == 3 && iters == seg_iters && outer > 1) return finish(FEMH_E_BREAKDOWN);
    if (mixed) {
      // continue from the FP64 true residual (same direction unless broken down)
      const double ns = std::sqrt(ha->rr);
      const int fresh = last_done == 3 ? 1 : 0;
      FEMH_TRY_HIP(k::cocg_rescale_c64(s, n, r64, 1.0 / ns, dinv32, r32, p32, sc, partials, scale / ns,
                                       o.rtol * o.rtol * bb / (ns * ns), fresh, par()));
      if (!fresh) FEMH_TRY_HIP(k::cocg_apply_beta_c64(s, n, dinv32, r32, p32, sc));
      scale = ns;
    } else if (m32 && last_done != 3) {
      // r64 now holds the true residual: keep the direction
      FEMH_TRY_HIP(k::cocg_replace_c128(s, n, r64, dinv64, sc, partials, par()));
      FEMH_TRY_HIP(k::cocg_apply_beta_c128(s, n, dinv64, r64, p64, sc));
    } else {
      // restart COCG from the true residual, keeping x and the iteration count
      std::memset(hw, 0, sizeof(*hw));
      hw->tol2 = o.rtol * o.rtol;
      hw->bb = bb;
      hw->bd_tol = 1e-14;
      hw->max_iters = o.max_iter;
      hw->iters_out = iters;
      if (m32) hw->delta2 = o.inner_rtol * o.inner_rtol;
      FEMH_TRY_HIP(hipMemcpyAsync(sc, hw, sizeof(*hw), hipMemcpyHostToDevice, s));
      if (sr) FEMH_TRY(queue_sr_init());
      else if (bic) FEMH_TRY(queue_bic_start());
      else FEMH_TRY_HIP(k::cocg_init_c128(s, n, r64, dinv64, x, r64, p64, sc, partials, 0, par()));
    }
    new_segment(iters);
    return FEMH_OK;
  }

  int finish(int st) {
    status = st;
    phase = DONE;
    logf(1, "solve: finished with status %d after %d iterations, %d checks, relative residual %.3e", st, iters,
         outer, rel);
    return FEMH_OK;
  }

  // Advance without blocking: queue what the current phase allows and act
  // on any readback that has arrived.  *progress is set when something moved.
  int step(bool* progress) {
    *progress = false;
    switch (phase) {
      case START:
        *progress = true;
        return start();
      case WAIT_INIT:
        if (hipEventQuery(ev_aux) != hipSuccess) return FEMH_OK;
        *progress = true;
        bb = ha->rr;
        if (bb == 0.0) {
          rel = 0.0;
          return finish(FEMH_OK);
        }
        return begin_iterating();
      case ITER: {
        while (inflight < 2 && !stale) {
          FEMH_TRY(queue_chunk(o.check_every));
          *progress = true;
        }
        if (inflight == 0) return FEMH_OK;
        if (hipEventQuery(ev[head]) != hipSuccess) return FEMH_OK;
        const CocgScalars st = *hs[head];
        head ^= 1;
        --inflight;
        *progress = true;
        if (!stale) logf(2, "solve:   iteration %d, recursive |r|/|b| = %.3e", st.iters_out, rec_rel(st));
        if (!stale && st.done) {
          stop_state = st;
          stale = true;
        }
        if (stale && inflight == 0) return on_stop(stop_state);
        return FEMH_OK;
      }
      case WAIT_CHECK:
        if (hipEventQuery(ev_aux) != hipSuccess) return FEMH_OK;
        *progress = true;
        return on_check();
      case DONE:
        return FEMH_OK;
    }
    return FEMH_OK;
  }

  // Block until the oldest outstanding readback lands.
  void wait() {
    if (phase == ITER && inflight > 0) (void)hipEventSynchronize(ev[head]);
    else if (phase == WAIT_INIT || phase == WAIT_CHECK) (void)hipEventSynchronize(ev_aux);
  }

  void fill_stats(femh_solve_stats* st) const {
    st->status = status;
    st->iters = iters;
    st->outer_iters = (mixed || m32) ? outer : std::max(outer - 1, 0);
    st->rel_residual = rel;
  }
};

Stepper* stepper_create(Problem* P, const double2* b, double2* x, const femh_solve_opts& o) {
  Stepper* s = new Stepper();
  if (s->init(P, b, x, o) != FEMH_OK) {
    delete s;
    return nullptr;
  }
  return s;
}

int stepper_step(Stepper* s, bool* progress) { return s->step(progress); }
bool stepper_done(const Stepper* s) { return s->phase == Stepper::DONE; }
void stepper_wait(Stepper* s) { s->wait(); }
void stepper_stats(const Stepper* s, femh_solve_stats* st) { s->fill_stats(st); }
void stepper_destroy(Stepper* s) { delete s; }

int solve_single(Problem* P, const double2* b, double2* x, const femh_solve_opts& o, femh_solve_stats* st) {
  Ctx* c = P->ctx;
  std::memset(st, 0, sizeof(*st));
  hipEvent_t e0, e1;
  FEMH_TRY_HIP(hipEventCreate(&e0));
  FEMH_TRY_HIP(hipEventCreate(&e1));
  (void)hipEventRecord(e0, c->stream);
  Stepper* S = stepper_create(P, b, x, o);
  if (!S) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return FEMH_E_OOM;
  }
  S->timing = c->profile;
  int rc = FEMH_OK;
  while (!stepper_done(S)) {
    bool progress = false;
    rc = S->step(&progress);
    if (rc != FEMH_OK) break;
    if (!progress) S->wait();
  }
  (void)hipEventRecord(e1, c->stream);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != FEMH_OK) {
    delete S;
    return rc;
  }
  S->fill_stats(st);
  st->seconds = ms * 1e-3;
  if (S->timing) {
    const int slot = S->mixed ? 1 : (S->m32 ? 3 : 0);
    c->prof_sec[slot] += S->prof_seconds;
    c->prof_cnt[slot] += S->prof_count;
  }
  rc = S->status;
  delete S;
  if (rc == FEMH_E_NOT_CONVERGED)
    set_error("not converged: relative residual %.3e after %d iterations", st->rel_residual, st->iters);
  else if (rc == FEMH_E_BREAKDOWN)
    set_error("COCG breakdown after %d iterations (relative residual %.3e)", st->iters, st->rel_residual);
  return rc;
}

}  // namespace femh
