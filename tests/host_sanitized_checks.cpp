// Host-code checks run under AddressSanitizer and UndefinedBehaviorSanitizer
// (built by test_host_sanitizers.py with the library's host code only): the
// descriptor and wave validation, the footprint estimate, the refusals of
// NULL handles, and context creation where no usable device exists.  Every
// case prints one line; the run fails on the first unexpected status.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

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

int main() {
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
