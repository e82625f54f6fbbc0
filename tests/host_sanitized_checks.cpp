// Host-code checks run under AddressSanitizer and UndefinedBehaviorSanitizer
// (built by test_host_sanitizers.py, the library's host side sanitized): the
// descriptor and wave validation, the footprint estimate, the refusals of
// NULL handles, context creation where no usable device exists, and the
// server's admission pass driven by a fake executor (simulated arrivals and
// completions, no device).  Every case prints one line; the run fails if
// any status or invariant is unexpected.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "admission.h"
#include "femh.h"

static int failures = 0;

static void expect(const char* what, int got, int want) {
  std::printf("%-48s %4d %s\n", what, got, got == want ? "ok" : "UNEXPECTED");
  if (got != want) ++failures;
}

static femh_problem_desc box(int n, const femh_c128* eps, const uint8_t* pec) {
  femh_problem_desc d;
  std::memset(&d, 0, sizeof d);
  d.nx = d.ny = d.nz = n;
  for (int a = 0; a < 3; ++a) d.h[a] = 0.1;
  d.eps_r = eps;
  d.pec = pec;
  d.k0 = 2.0 * M_PI;
  return d;
}

// The server's admission pass under a fake executor: requests of random
// size (1-40 units against a budget of 100) and service time arrive over
// time; at every arrival and completion the waiting queue is offered to
// plan_admissions.  Checked after every pass: the resident bytes stay within
// the budget, at most max_slots run, only the first 16 waiting requests are
// considered, every request passed over before an admitted one did not fit
// (or the slots were full) at its turn, and at the end every request has run.
static void fake_executor() {
  const int64_t budget = 100;
  const int max_slots = 6, count = 400;
  uint64_t seed = 12345;
  auto rnd = [&](int lo, int hi) {
    seed = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    return lo + (int)((seed >> 33) % (uint64_t)(hi - lo + 1));
  };
  struct Req {
    int64_t bytes;
    double arrive, service, start = -1.0, done = -1.0;
  };
  std::vector<Req> req;
  double t = 0.0;
  for (int i = 0; i < count; ++i) {
    t += rnd(0, 20) * 0.1;
    req.push_back(Req{rnd(1, 40), t, rnd(1, 60) * 0.1});
  }
  std::vector<int> queue, running;
  int64_t resident = 0, peak = 0;
  int next = 0, bad = 0, passes = 0, skipped_ahead = 0;
  double now = 0.0;
  while (next < count || !queue.empty() || !running.empty()) {
    // next event: an arrival or the earliest completion
    double t_arr = next < count ? req[next].arrive : 1e300, t_done = 1e300;
    int who = -1;
    for (int r : running)
      if (req[r].done < t_done) t_done = req[r].done, who = r;
    if (t_arr <= t_done) {
      now = t_arr;
      queue.push_back(next++);
    } else {
      now = t_done;
      resident -= req[who].bytes;
      running.erase(std::find(running.begin(), running.end(), who));
    }
    std::vector<int64_t> bytes;
    for (int r : queue) bytes.push_back(req[r].bytes);
    const int64_t before = resident;
    const std::vector<int> take = femh::plan_admissions(bytes, resident, budget, (int)running.size(), max_slots);
    ++passes;
    // replay the pass: each position up to the last admitted one was either
    // admitted or did not fit when its turn came
    int64_t res = before;
    int run = (int)running.size();
    size_t k = 0;
    const int last = take.empty() ? -1 : take.back();
    for (int i = 0; i <= last; ++i) {
      if (k < take.size() && take[k] == i) {
        if (i >= 16 || run >= max_slots || res + bytes[i] > budget) ++bad;
        res += bytes[i];
        ++run;
        ++k;
      } else {
        if (res + bytes[i] <= budget && run < max_slots) ++bad;
        ++skipped_ahead;
      }
    }
    if (res != resident || resident > budget || run > max_slots) ++bad;
    peak = std::max(peak, resident);
    std::vector<int> left;
    for (size_t i = 0, j = 0; i < queue.size(); ++i) {
      if (j < take.size() && take[j] == (int)i) {
        const int r = queue[i];
        req[r].start = now;
        req[r].done = now + req[r].service;
        running.push_back(r);
        ++j;
      } else {
        left.push_back(queue[i]);
      }
    }
    queue.swap(left);
  }
  int unrun = 0;
  for (const Req& r : req)
    if (r.start < r.arrive || r.done < r.start) ++unrun;
  std::printf("fake executor: %d requests, %d passes, peak %lld of %lld resident, %d passed over\n", count, passes,
              (long long)peak, (long long)budget, skipped_ahead);
  expect("admission invariants held", bad, 0);
  expect("every request ran", unrun, 0);
}

int main() {
  fake_executor();
  const int n = 5, ne = n * n * n;
  std::vector<femh_c128> eps((size_t)ne, femh_c128{2.0, -0.1});
  std::vector<uint8_t> pec((size_t)ne, 0);
  pec[62] = 1;
  char msg[256];

  femh_problem_desc d = box(n, eps.data(), pec.data());
  expect("valid descriptor", femh_validate_desc(&d, msg, sizeof msg), FEMH_OK);
  expect("NULL descriptor", femh_validate_desc(nullptr, msg, sizeof msg), FEMH_E_INVALID);
  expect("NULL descriptor, no message buffer", femh_validate_desc(nullptr, nullptr, 0), FEMH_E_INVALID);
  expect("one-byte message buffer", femh_validate_desc(nullptr, msg, 1), FEMH_E_INVALID);
  femh_problem_desc b = d;
  b.nx = 0;
  expect("zero elements", femh_validate_desc(&b, msg, sizeof msg), FEMH_E_INVALID);
  b = d;
  b.h[1] = -0.1;
  expect("negative element size", femh_validate_desc(&b, msg, sizeof msg), FEMH_E_INVALID);
  b = d;
  b.k0 = NAN;
  expect("NaN k0", femh_validate_desc(&b, msg, sizeof msg), FEMH_E_NONFINITE);
  b = d;
  b.outer_face[3] = 7;
  expect("unknown face tag", femh_validate_desc(&b, msg, sizeof msg), FEMH_E_INVALID);
  b = d;
  b.penalty_surface = 2;
  expect("penalty_surface 2", femh_validate_desc(&b, msg, sizeof msg), FEMH_E_INVALID);
  b = d;
  b.penalty_surface = 1;
  b.outer_face[0] = FEMH_FACE_SYM;
  expect("penalty_surface with a symmetry face", femh_validate_desc(&b, msg, sizeof msg), FEMH_E_INVALID);
  b = d;
  b.penalty_surface = 1;
  expect("penalty_surface on an ABC box", femh_validate_desc(&b, msg, sizeof msg), FEMH_OK);
  std::vector<femh_c128> bad = eps;
  bad[17].im = INFINITY;
  b = d;
  b.eps_r = bad.data();
  expect("infinite eps_r", femh_validate_desc(&b, msg, sizeof msg), FEMH_E_NONFINITE);
  bad[17] = femh_c128{0.0, 0.0};
  expect("zero eps_r", femh_validate_desc(&b, msg, sizeof msg), FEMH_E_INVALID);
  std::vector<uint8_t> all((size_t)ne, 1);
  b = d;
  b.pec = all.data();
  expect("every element PEC", femh_validate_desc(&b, msg, sizeof msg), FEMH_E_INVALID);

  femh_plane_wave w;
  std::memset(&w, 0, sizeof w);
  w.d[2] = 1.0;
  w.p[0].re = 1.0;
  expect("valid wave", femh_validate_waves(1, &w, msg, sizeof msg), FEMH_OK);
  expect("no waves", femh_validate_waves(0, &w, msg, sizeof msg), FEMH_E_INVALID);
  expect("NULL waves", femh_validate_waves(3, nullptr, msg, sizeof msg), FEMH_E_INVALID);
  femh_plane_wave v = w;
  v.d[2] = 0.9;
  expect("direction not unit", femh_validate_waves(1, &v, msg, sizeof msg), FEMH_E_INVALID);
  v = w;
  v.p[2].re = 0.5;
  expect("polarisation along the direction", femh_validate_waves(1, &v, msg, sizeof msg), FEMH_E_INVALID);
  v = w;
  v.p[1].im = NAN;
  expect("NaN polarisation", femh_validate_waves(1, &v, msg, sizeof msg), FEMH_E_NONFINITE);

  int64_t b1 = 0, b4 = 0, b64 = 0;
  expect("estimate, one wave", femh_estimate_bytes(&d, 1, FEMH_FP64, &b1), FEMH_OK);
  expect("estimate, four waves", femh_estimate_bytes(&d, 4, FEMH_FP64, &b4), FEMH_OK);
  expect("estimate, mixed precision", femh_estimate_bytes(&d, 64, FEMH_MIXED, &b64), FEMH_OK);
  expect("estimates grow with the waves", b4 > b1 && b1 > 0 ? 1 : 0, 1);
  expect("estimate, unknown precision", femh_estimate_bytes(&d, 1, 9, &b1), FEMH_E_INVALID);
  expect("estimate, negative waves", femh_estimate_bytes(&d, -1, FEMH_FP64, &b1), FEMH_E_INVALID);
  expect("estimate, NULL output", femh_estimate_bytes(&d, 1, FEMH_FP64, nullptr), FEMH_E_INVALID);
  femh_problem_desc big = box(1000, nullptr, nullptr);
  int64_t bb = 0;
  expect("estimate, 1e9 elements", femh_estimate_bytes(&big, 16, FEMH_FP64, &bb), FEMH_OK);
  expect("the large estimate exceeds 1 TB", bb > (int64_t)1 << 40 ? 1 : 0, 1);
  big = box(1100, nullptr, nullptr);
  expect("more than 2^30 grid nodes", femh_estimate_bytes(&big, 1, FEMH_FP64, &bb), FEMH_E_INVALID);

  femh_problem* prob = nullptr;
  expect("problem on a NULL context", femh_problem_create(nullptr, &d, &prob), FEMH_E_INVALID);
  femh_server* srv = nullptr;
  expect("server on a NULL context", femh_server_create(nullptr, nullptr, &srv), FEMH_E_INVALID);
  femh_solve_stats st;
  expect("solve on a NULL problem", femh_solve(nullptr, 1, &w, nullptr, nullptr, &st), FEMH_E_INVALID);
  expect("version", femh_version() >= 10000 ? 1 : 0, 1);

  femh_ctx* ctx = nullptr;
  const int rc = femh_ctx_create(0, nullptr, nullptr, &ctx);
  if (rc == FEMH_OK) {
    std::printf("%-48s %4d ok (a device is present)\n", "context", rc);
    femh_ctx_destroy(ctx);
  } else {
    expect("context without a usable device", rc, FEMH_E_DEVICE);
    expect("its message is set", std::strlen(femh_last_error()) > 0 ? 1 : 0, 1);
  }
  expect("context, NULL output", femh_ctx_create(0, nullptr, nullptr, nullptr), FEMH_E_INVALID);
  std::printf("%d unexpected\n", failures);
  return failures ? 1 : 0;
}
