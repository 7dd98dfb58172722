// Drives the host-only logic of liblfmm (argument checks, plan parameters, the
// Sommerfeld contour rules and their node budget, status and stage names) in a
// build with AddressSanitizer and UndefinedBehaviorSanitizer.  No call here needs
// a device; a plan that does reach the HIP runtime must fail cleanly without one.
#include <cmath>
#include <cstdio>

#include "lfmm.h"

static int bad = 0;
#define EXPECT(c)                                              \
  do {                                                         \
    if (!(c)) {                                                \
      std::printf("host run: check failed at line %d\n", __LINE__); \
      bad++;                                                   \
    }                                                          \
  } while (0)

int main() {
  for (int s = -1; s <= 8; s++) EXPECT(lfmm_status_string(s) != nullptr);
  for (int i = -2; i < 40; i++) (void)lfmm_stage_name(i);
  const double d3[2] = {0.0, -1.2}, k3[3] = {0.8, 1.5, 2.0};
  const double d5[4] = {0.0, -0.6, -1.2, -1.8}, k5[5] = {0.5, 1.2, 2.0, 2.8, 3.0};
  lfmm_options o = {};
  long long total = 0;
  for (int p = 1; p <= 10; p++)
    for (double tol : {0.0, 1e-6, 1e-10, 0.5})
      for (double dz = 1e-5; dz < 20; dz *= 3.7)
        for (double rho : {0.0, 1e-3, 0.2, 1.0, 40.0}) {
          o.quad_tol = tol;
          o.quad_max_nodes = 0;
          int64_t n = -1;
          int rc = lfmm_quad_nodes(2, d3, k3, p, &o, dz, rho, &n);
          EXPECT(rc == LFMM_OK || rc == LFMM_ENOCONV);
          EXPECT(rc != LFMM_OK || (n > 0 && n % 16 == 0));
          if (rc == LFMM_OK) {
            o.quad_max_nodes = n - 1;  // one node short: over the budget
            int64_t m = -1;
            EXPECT(lfmm_quad_nodes(4, d5, k5, p, &o, dz, rho, &m) != LFMM_EINVAL);
            EXPECT(lfmm_quad_nodes(2, d3, k3, p, &o, dz, rho, &m) == LFMM_ENOCONV && m == n);
            total += n;
          }
        }
  // invalid arguments
  int64_t n = 0;
  o = lfmm_options{};
  EXPECT(lfmm_quad_nodes(2, d3, k3, 8, &o, 0.0, 1.0, &n) == LFMM_EINVAL);
  EXPECT(lfmm_quad_nodes(2, d3, k3, 8, &o, NAN, 1.0, &n) == LFMM_EINVAL);
  EXPECT(lfmm_quad_nodes(2, d3, k3, 8, &o, 0.1, -1.0, &n) == LFMM_EINVAL);
  EXPECT(lfmm_quad_nodes(2, d3, k3, 8, &o, 0.1, 1.0, nullptr) == LFMM_EINVAL);
  EXPECT(lfmm_quad_nodes(-1, d3, k3, 8, &o, 0.1, 1.0, &n) == LFMM_EINVAL);
  EXPECT(lfmm_quad_nodes(2, d3, k3, 0, &o, 0.1, 1.0, &n) == LFMM_EINVAL);
  EXPECT(lfmm_quad_nodes(2, d3, k3, 11, &o, 0.1, 1.0, &n) == LFMM_EINVAL);
  o.quad_max_nodes = -3;
  EXPECT(lfmm_quad_nodes(2, d3, k3, 8, &o, 0.1, 1.0, &n) == LFMM_EINVAL);
  o = lfmm_options{};
  o.quad_tol = 1.0;
  EXPECT(lfmm_quad_nodes(2, d3, k3, 8, &o, 0.1, 1.0, &n) == LFMM_EINVAL);
  const double dbad[2] = {-1.2, 0.0}, kbad[3] = {0.8, -1.5, 2.0};
  lfmm_plan_t* P = nullptr;
  EXPECT(lfmm_plan(2, dbad, k3, 8, 64, nullptr, &P) == LFMM_EINVAL && !P);
  EXPECT(lfmm_plan(2, d3, kbad, 8, 64, nullptr, &P) == LFMM_EINVAL && !P);
  EXPECT(lfmm_plan(2, d3, k3, 0, 64, nullptr, &P) == LFMM_EINVAL && !P);
  EXPECT(lfmm_plan(2, d3, k3, 8, 0, nullptr, &P) == LFMM_EINVAL && !P);
  EXPECT(lfmm_plan(2, d3, k3, 8, 64, nullptr, nullptr) == LFMM_EINVAL);
  o = lfmm_options{};
  o.precision = 3;
  EXPECT(lfmm_plan(2, d3, k3, 8, 64, &o, &P) == LFMM_EINVAL && !P);
  lfmm_destroy(nullptr);
  std::printf("host run: %lld contour nodes over the sweep, %s\n", total, bad ? "FAILED" : "ok");
  return bad ? 1 : 0;
}
