// Continuous-batching request loop.
//
// A stepping thread and a set-up thread share the work; every admitted
// request gets an internal context of its own with its own HIP stream
// (default priority; device memory from hipMalloc), and at any time exactly
// one of the two threads works on that stream: the set-up thread until the
// request is set up, the stepping thread while it iterates, the set-up
// thread again once it is handed back.  A stream is therefore never captured
// by one thread while the other enqueues work on it.
// Submitted requests wait in a FIFO queue; the stepping thread admits them
// (first fit within a small window) as long as a slot is free and their
// estimated device footprint fits the budget, and hands each admitted
// request to the set-up thread, which assembles its problem on the
// request's stream and creates one solver state machine per right-hand
// side (or per group of up to four; a group's chunk of iterations is
// captured into a graph there, by the set-up thread).  Every round the
// stepping thread advances all
// resident, set-up right-hand sides of all requests (each queues its next
// chunk of iterations without waiting), so requests of different sizes
// overlap on the device; a request whose columns have all finished (or that
// was cancelled) goes back to the set-up thread, which scatters its field,
// copies it to host memory and releases its device memory for the next
// admission.  Assembly, the host synchronisations it needs and the
// retirement copies therefore never hold up the iterations of the requests
// already resident.
//
// Each right-hand side runs exactly the single-solve code path with its own
// buffers and deterministic kernels, so a request's result does not depend
// on what else is resident.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "admission.h"
#include "internal.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  femh_problem_desc desc{};
  std::vector<femh_c128> eps, mu;
  std::vector<uint8_t> pec;
  std::vector<femh_plane_wave> waves;
  femh_solve_opts opts{};
  int64_t est_bytes = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  enum State { QUEUED, RUNNING, FINISHED } state = QUEUED;
  bool cancel = false;
  bool ready = false;    // set up: the stepping thread may advance it
  bool handed = false;   // handed back for retirement: the stepping thread no longer touches it
  int status = FEMH_OK;
  std::vector<femh_solve_stats> stats;
  std::vector<femh_c128> H;
  // resident state
  femh::Ctx* lane = nullptr;
  femh::Problem* P = nullptr;
  double2* b = nullptr;
  double2* x = nullptr;
  std::vector<femh::Stepper*> steps;
  // batch_rhs: the waves in groups of up to four, one batched solve each
  std::vector<femh::BatchStepper*> bsteps;
  std::vector<int> bfirst;  // first wave of each group
};

}  // namespace

struct femh_server {
  femh::Ctx* base = nullptr;
  int64_t budget = 0;
  int max_slots = 32;
  int chunk = 32;
  bool batch_rhs = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::vector<Request*> running;
  std::map<uint64_t, Request*> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread th, io;
  // set-up thread work: requests to set up (status unused) or to retire
  struct Job {
    Request* r;
    bool retire;
    int status;
  };
  std::deque<Job> jobs;
  std::condition_variable cv_io;
  bool io_stop = false;
  int64_t resident = 0, peak = 0;
  // report
  int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, rejected = 0, rhs_completed = 0;
  std::vector<double> latencies;
  double t_first_submit = -1, t_last_done = -1;

  void loop();
  void io_loop();
  void hand_back(Request* r, int status);
  void admit_locked(std::vector<Request*>& admitted);
  int setup(Request* r);
  void retire(Request* r, int status);
};

namespace {

// A request's own context: the server device, a non-blocking stream and a
// small pinned buffer for scalar readbacks.
femh::Ctx* lane_create(const femh::Ctx* base) {
  femh::Ctx* c = new femh::Ctx();
  c->device = base->device;
  c->n_cu = base->n_cu;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return nullptr;
  }
  if (hipHostMalloc(&c->pinned, 16384, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamDestroy(c->stream);
    delete c;
    return nullptr;
  }
  c->own_stream = true;
  return c;
}

void lane_destroy(femh::Ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  (void)hipStreamDestroy(c->stream);
  (void)hipHostFree(c->pinned);
  delete c;
}

void release(Request* r) {
  for (femh::Stepper* s : r->steps) femh::stepper_destroy(s);
  r->steps.clear();
  for (femh::BatchStepper* s : r->bsteps) femh::batch_stepper_destroy(s);
  r->bsteps.clear();
  r->bfirst.clear();
  if (r->lane) {
    if (r->b) r->lane->dfree(r->b);
    if (r->x) r->lane->dfree(r->x);
  }
  r->b = r->x = nullptr;
  delete r->P;
  r->P = nullptr;
  lane_destroy(r->lane);
  r->lane = nullptr;
}

}  // namespace

void femh_server::admit_locked(std::vector<Request*>& admitted) {
  // drop cancelled requests that never started
  for (auto it = queue.begin(); it != queue.end();) {
    if ((*it)->cancel) {
      Request* r = *it;
      r->state = Request::FINISHED;
      r->status = FEMH_E_CANCELLED;
      r->t_done = now_s();
      ++cancelled;
      it = queue.erase(it);
      cv_done.notify_all();
    } else {
      ++it;
    }
  }
  std::vector<int64_t> bytes;
  bytes.reserve(queue.size());
  for (Request* r : queue) bytes.push_back(r->est_bytes);
  const int64_t before = resident;
  const std::vector<int> take = femh::plan_admissions(bytes, resident, budget, (int)running.size(), max_slots);
  int64_t sum = before;
  std::vector<Request*> taken;
  for (int i : take) {
    Request* r = queue[(size_t)i];
    sum += r->est_bytes;
    peak = std::max(peak, sum);
    r->state = Request::RUNNING;
    r->t_start = now_s();
    running.push_back(r);
    admitted.push_back(r);
    taken.push_back(r);
    femh::logf(1, "server: request %llu admitted (%dx%dx%d, %d waves, %.1f MB of %.1f MB resident)",
               (unsigned long long)r->ticket, r->desc.nx, r->desc.ny, r->desc.nz, (int)r->waves.size(),
               r->est_bytes / 1e6, sum / 1e6);
  }
  for (Request* r : taken) queue.erase(std::find(queue.begin(), queue.end(), r));
}

int femh_server::setup(Request* r) {
  r->lane = lane_create(base);
  if (!r->lane) {
    femh::set_error("request stream creation failed");
    return FEMH_E_DEVICE;
  }
  femh::Ctx* c = r->lane;
  (void)hipSetDevice(c->device);
  femh_problem_desc d = r->desc;
  d.eps_r = r->eps.empty() ? nullptr : r->eps.data();
  d.mu_r = r->mu.empty() ? nullptr : r->mu.data();
  d.pec = r->pec.empty() ? nullptr : r->pec.data();
  d.arrays_on_device = 0;
  int st = femh::problem_create(c, &d, &r->P);
  if (st != FEMH_OK) return st;
  const int nrhs = (int)r->waves.size();
  const int64_t n = 3 * (int64_t)r->P->pat.nn;
  r->b = (double2*)c->dmalloc(16 * (size_t)n * nrhs);
  r->x = (double2*)c->dmalloc(16 * (size_t)n * nrhs);
  void* dw = c->dmalloc(sizeof(femh_plane_wave) * nrhs);
  if (!r->b || !r->x || !dw) {
    if (dw) c->dfree(dw);
    femh::set_error("device allocation failed (request buffers)");
    return FEMH_E_OOM;
  }
  hipError_t e = hipMemcpyAsync(dw, r->waves.data(), sizeof(femh_plane_wave) * nrhs, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = femh::k::rhs(c->stream, r->P->mesh, r->P->pat, nrhs, (const femh_plane_wave*)dw, r->b);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->dfree(dw);
  if (e != hipSuccess) {
    femh::set_error("request set-up failed: %s", hipGetErrorString(e));
    return FEMH_E_DEVICE;
  }
  r->stats.assign(nrhs, femh_solve_stats{});
  if (batch_rhs && nrhs >= 2) {
    // the batched solver's options, as femh_solve_batched_dev sets them
    femh_solve_opts ob = r->opts;
    if (ob.precision != FEMH_FP64) ob.precision = FEMH_MIXED_MATRIX;
    if (ob.inner_rtol <= 0.0) ob.inner_rtol = 1e-3;
    femh_solve_opts o = femh::opts_with_defaults(&ob);
    if (r->opts.check_every <= 0) o.check_every = chunk;
    for (int g = 0; g < nrhs; g += 4) {
      const int k = std::min(4, nrhs - g);
      femh::BatchStepper* s = femh::batch_stepper_create(r->P, k, r->b + g * n, r->x + g * n, o);
      if (!s) return FEMH_E_OOM;
      r->bsteps.push_back(s);
      r->bfirst.push_back(g);
      // bring the group to its iterations here, so its graph is captured
      // by this thread, before the stepping thread takes the stream over
      while (!femh::batch_stepper_iterating(s)) {
        bool prog = false;
        const int st = femh::batch_stepper_step(s, &prog);
        if (st != FEMH_OK) return st;
        if (!prog) femh::batch_stepper_wait(s);
      }
    }
    return FEMH_OK;
  }
  femh_solve_opts o = femh::opts_with_defaults(&r->opts);
  if (r->opts.check_every <= 0) o.check_every = chunk;
  for (int k = 0; k < nrhs; ++k) {
    femh::Stepper* s = femh::stepper_create(r->P, r->b + k * n, r->x + k * n, o);
    if (!s) return FEMH_E_OOM;
    r->steps.push_back(s);
  }
  return FEMH_OK;
}

void femh_server::retire(Request* r, int status) {
  const int nrhs = (int)r->waves.size();
  if (status == FEMH_OK || status == FEMH_E_NOT_CONVERGED || status == FEMH_E_BREAKDOWN) {
    for (int k = 0; k < nrhs && k < (int)r->steps.size(); ++k) {
      femh::stepper_stats(r->steps[k], &r->stats[k]);
      r->stats[k].seconds = now_s() - r->t_start;
      if (r->stats[k].status != FEMH_OK && status == FEMH_OK) status = r->stats[k].status;
    }
    for (size_t g = 0; g < r->bsteps.size(); ++g) {
      const int first = r->bfirst[g];
      const int st = femh::batch_stepper_stats(r->bsteps[g], &r->stats[first]);
      for (int k = first; k < std::min(nrhs, first + 4); ++k) r->stats[k].seconds = now_s() - r->t_start;
      if (st != FEMH_OK && status == FEMH_OK) status = st;
    }
    // field to the grid, then to host memory
    femh::Ctx* c = r->lane;
    const size_t cells = 3 * (size_t)r->P->grid_nodes * nrhs;
    void* dh = c->dmalloc(cells * sizeof(femh_c128));
    if (dh) {
      r->H.resize(cells);
      hipError_t e = femh::k::scatter(c->stream, r->P->mesh, r->P->pat, nrhs, r->x, (double2*)dh);
      if (e == hipSuccess)
        e = hipMemcpyAsync(r->H.data(), dh, cells * sizeof(femh_c128), hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      c->dfree(dh);
      if (e != hipSuccess) status = FEMH_E_DEVICE;
    } else {
      status = FEMH_E_OOM;
    }
  }
  release(r);
  std::lock_guard<std::mutex> g(mu);
  r->status = status;
  r->state = Request::FINISHED;
  r->t_done = now_s();
  femh::logf(1, "server: request %llu finished with status %d, %.3f s after admission", (unsigned long long)r->ticket,
             status, r->t_done - r->t_start);
  resident -= r->est_bytes;
  running.erase(std::remove(running.begin(), running.end(), r), running.end());
  if (status == FEMH_E_CANCELLED) {
    ++cancelled;
  } else if (status == FEMH_OK) {
    ++completed;
    rhs_completed += nrhs;
    latencies.push_back(r->t_done - r->t_submit);
    t_last_done = r->t_done;
  } else {
    ++failed;
    latencies.push_back(r->t_done - r->t_submit);
    t_last_done = r->t_done;
  }
  cv_done.notify_all();
}

void femh_server::hand_back(Request* r, int status) {
  std::lock_guard<std::mutex> g(mu);
  r->handed = true;
  jobs.push_back(Job{r, true, status});
  cv_io.notify_all();
}

void femh_server::io_loop() {
  (void)hipSetDevice(base->device);
  while (true) {
    Job j;
    {
      std::unique_lock<std::mutex> g(mu);
      cv_io.wait(g, [this] { return io_stop || !jobs.empty(); });
      if (jobs.empty()) break;  // io_stop with nothing left
      j = jobs.front();
      jobs.pop_front();
    }
    if (j.retire) {
      retire(j.r, j.status);
      continue;
    }
    const int st = setup(j.r);
    if (st != FEMH_OK) {
      retire(j.r, st);
      continue;
    }
    std::lock_guard<std::mutex> g(mu);
    j.r->ready = true;
    cv_work.notify_all();
  }
}

void femh_server::loop() {
  (void)hipSetDevice(base->device);
  std::vector<Request*> active;
  while (true) {
    std::vector<Request*> admitted;
    {
      std::unique_lock<std::mutex> g(mu);
      if (stop) break;
      admit_locked(admitted);
      for (Request* r : admitted) jobs.push_back(Job{r, false, FEMH_OK});
      if (!admitted.empty()) cv_io.notify_all();
      // the requests this thread may advance: set up and not handed back
      active.clear();
      for (Request* r : running)
        if (r->ready && !r->handed) active.push_back(r);
      if (active.empty()) {
        cv_work.wait_for(g, std::chrono::milliseconds(running.empty() ? 20 : 1));
        continue;
      }
    }
    bool any_progress = false;
    femh::Stepper* waiter = nullptr;
    femh::BatchStepper* bwaiter = nullptr;
    for (Request* r : active) {
      bool cancel;
      {
        std::lock_guard<std::mutex> g(mu);
        cancel = r->cancel;
      }
      if (cancel) {
        hand_back(r, FEMH_E_CANCELLED);
        any_progress = true;
        continue;
      }
      bool all_done = true;
      int err = FEMH_OK;
      for (femh::Stepper* s : r->steps) {
        if (femh::stepper_done(s)) continue;
        bool prog = false;
        const int rc = femh::stepper_step(s, &prog);
        if (rc != FEMH_OK) {
          err = rc;
          break;
        }
        any_progress |= prog;
        if (!femh::stepper_done(s)) {
          all_done = false;
          if (!waiter && !bwaiter) waiter = s;
        }
      }
      for (femh::BatchStepper* s : r->bsteps) {
        if (err != FEMH_OK) break;
        if (femh::batch_stepper_done(s)) continue;
        bool prog = false;
        const int rc = femh::batch_stepper_step(s, &prog);
        if (rc != FEMH_OK) {
          err = rc;
          break;
        }
        any_progress |= prog;
        if (!femh::batch_stepper_done(s)) {
          all_done = false;
          if (!waiter && !bwaiter) bwaiter = s;
        }
      }
      if (err != FEMH_OK) {
        hand_back(r, err);
        any_progress = true;
      } else if (all_done) {
        hand_back(r, FEMH_OK);
        any_progress = true;
      }
    }
    if (!any_progress && waiter) femh::stepper_wait(waiter);
    if (!any_progress && bwaiter) femh::batch_stepper_wait(bwaiter);
  }
  // shut down: hand every request still resident back as cancelled (the
  // set-up thread finishes its queue, then these)
  std::lock_guard<std::mutex> g(mu);
  for (Request* r : running)
    if (!r->handed) {
      r->handed = true;
      jobs.push_back(Job{r, true, FEMH_E_CANCELLED});
    }
  io_stop = true;
  cv_io.notify_all();
}

extern "C" {

int femh_server_create(femh_ctx* ctx_, const femh_server_opts* opts, femh_server** out) {
  femh::clear_error();
  femh::Ctx* ctx = reinterpret_cast<femh::Ctx*>(ctx_);
  if (!ctx || !out) {
    femh::set_error("ctx and out must not be NULL");
    return FEMH_E_INVALID;
  }
  *out = nullptr;
  femh_server_opts o{};
  if (opts) o = *opts;
  if (o.hbm_budget_bytes < 0 || o.max_slots < 0 || o.chunk_iters < 0 || o.batch_rhs < 0 || o.batch_rhs > 1 ||
      o.reserved != 0) {
    femh::set_error("server options must be >= 0 (batch_rhs 0 or 1, reserved 0)");
    return FEMH_E_INVALID;
  }
  FEMH_TRY_HIP(hipSetDevice(ctx->device));
  femh_server* s = new femh_server();
  s->base = ctx;
  if (o.hbm_budget_bytes > 0) {
    s->budget = o.hbm_budget_bytes;
  } else {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      femh::set_error("hipMemGetInfo failed");
      return FEMH_E_DEVICE;
    }
    s->budget = (int64_t)(0.8 * (double)fr);
  }
  s->max_slots = o.max_slots > 0 ? o.max_slots : 32;
  s->chunk = o.chunk_iters > 0 ? o.chunk_iters : 32;
  s->batch_rhs = o.batch_rhs != 0;
  s->th = std::thread([s] { s->loop(); });
  s->io = std::thread([s] { s->io_loop(); });
  *out = s;
  return FEMH_OK;
}

int femh_server_submit(femh_server* s, const femh_problem_desc* desc, int32_t nrhs, const femh_plane_wave* waves,
                       const femh_solve_opts* opts, uint64_t* ticket) {
  femh::clear_error();
  if (!s || !desc || !ticket) {
    femh::set_error("server, desc and ticket must not be NULL");
    return FEMH_E_INVALID;
  }
  if (desc->arrays_on_device) {
    femh::set_error("server requests take host arrays only");
    return FEMH_E_INVALID;
  }
  std::string m;
  int st = femh::validate_desc(desc, m);
  if (st == FEMH_OK) st = femh::validate_waves(nrhs, waves, m);
  if (st != FEMH_OK) {
    femh::set_error("%s", m.c_str());
    return st;
  }
  Request* r = new Request();
  r->desc = *desc;
  const int64_t ne = (int64_t)desc->nx * desc->ny * desc->nz;
  if (desc->eps_r) r->eps.assign(desc->eps_r, desc->eps_r + ne);
  if (desc->mu_r) r->mu.assign(desc->mu_r, desc->mu_r + ne);
  if (desc->pec) r->pec.assign(desc->pec, desc->pec + ne);
  r->waves.assign(waves, waves + nrhs);
  if (opts) r->opts = *opts;
  const femh_solve_opts o = femh::opts_with_defaults(opts);
  const bool batched = s->batch_rhs && nrhs >= 2;
  st = femh::check_solve_opts(o, batched, m);
  if (st != FEMH_OK) {
    delete r;
    femh::set_error("%s", m.c_str());
    return st;
  }
  // problem + per-column solver workspace (+ the batched groups' blocks;
  // batch_rhs is fixed when the server is created; + the block incomplete
  // Cholesky factor and its workspace)
  int64_t base = femh::estimate_bytes(desc, nrhs, o.precision);
  if (batched) base += femh::estimate_batch_workspace(desc, nrhs);
  if (o.precond == FEMH_PRECOND_BIC0) base += femh::estimate_bic_bytes(desc, nrhs);
  r->est_bytes = base;
  std::lock_guard<std::mutex> g(s->mu);
  ++s->submitted;
  if (r->est_bytes > s->budget) {
    ++s->rejected;
    delete r;
    femh::set_error("request needs about %lld bytes, more than the whole budget %lld",
                    (long long)base, (long long)s->budget);
    return FEMH_E_OOM;
  }
  r->ticket = s->next_ticket++;
  r->t_submit = now_s();
  if (s->t_first_submit < 0) s->t_first_submit = r->t_submit;
  s->all[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv_work.notify_all();
  return FEMH_OK;
}

int femh_server_poll(femh_server* s, uint64_t ticket, int32_t timeout_ms, femh_c128* H_out, femh_solve_stats* stats) {
  if (!s) {
    femh::set_error("server is NULL");
    return FEMH_E_INVALID;
  }
  std::unique_lock<std::mutex> g(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) {
    femh::set_error("unknown ticket %llu", (unsigned long long)ticket);
    return FEMH_E_NOT_FOUND;
  }
  Request* r = it->second;
  auto finished = [r] { return r->state == Request::FINISHED; };
  if (!finished()) {
    if (timeout_ms == 0) return FEMH_E_PENDING;
    if (timeout_ms < 0) s->cv_done.wait(g, finished);
    else if (!s->cv_done.wait_for(g, std::chrono::milliseconds(timeout_ms), finished)) return FEMH_E_PENDING;
  }
  if (H_out && !r->H.empty()) std::memcpy(H_out, r->H.data(), r->H.size() * sizeof(femh_c128));
  if (stats)
    for (size_t k = 0; k < r->stats.size(); ++k) stats[k] = r->stats[k];
  const int st = r->status;
  s->all.erase(it);
  delete r;
  if (st != FEMH_OK) femh::set_error("request finished with status %d", st);
  return st;
}

int femh_server_cancel(femh_server* s, uint64_t ticket) {
  if (!s) {
    femh::set_error("server is NULL");
    return FEMH_E_INVALID;
  }
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) {
    femh::set_error("unknown ticket %llu", (unsigned long long)ticket);
    return FEMH_E_NOT_FOUND;
  }
  it->second->cancel = true;
  s->cv_work.notify_all();
  return FEMH_OK;
}

int femh_server_report_get(femh_server* s, femh_server_report* out) {
  if (!s || !out) {
    femh::set_error("NULL argument");
    return FEMH_E_INVALID;
  }
  std::lock_guard<std::mutex> g(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->cancelled = s->cancelled;
  out->rejected = s->rejected;
  out->rhs_completed = s->rhs_completed;
  out->peak_resident_bytes = s->peak;
  std::vector<double> l = s->latencies;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
      const double pos = p * (double)(l.size() - 1);
      const size_t i = (size_t)pos;
      const double f = pos - (double)i;
      return i + 1 < l.size() ? l[i] * (1 - f) + l[i + 1] * f : l[i];
    };
    out->p50_seconds = pct(0.50);
    out->p99_seconds = pct(0.99);
  }
  const double span = s->t_last_done - s->t_first_submit;
  if (span > 0) {
    out->requests_per_second = (double)s->completed / span;
    out->rhs_per_second = (double)s->rhs_completed / span;
  }
  return FEMH_OK;
}

void femh_server_destroy(femh_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    for (Request* r : s->queue) {
      r->state = Request::FINISHED;
      r->status = FEMH_E_CANCELLED;
    }
    s->queue.clear();
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  if (s->io.joinable()) s->io.join();
  for (auto& kv : s->all) delete kv.second;
  delete s;
}

}  // extern "C"
