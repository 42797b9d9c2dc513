// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (the device code is the normal
// build).  Every call here returns before a kernel runs: argument checks,
// material validation, the options defaults, the footprint, the
// allocation-free product's size limits, and on a machine without a GPU the
// error paths of plan creation after a failed HIP call (the cleanup of a
// partly built plan).  Exit status 0 when every check holds.
#include <stdio.h>
#include <string.h>

#include <vector>

#include "fftg.h"

static int g_fail = 0;
static int g_checks = 0;
#define CHECK(cond)                                                             \
  do {                                                                          \
    ++g_checks;                                                                 \
    if (!(cond)) {                                                              \
      ++g_fail;                                                                 \
      fprintf(stderr, "FAIL %s:%d: %s (last error: %s)\n", __FILE__, __LINE__, \
              #cond, fftg_last_error());                                        \
    }                                                                           \
  } while (0)

static fftg_material j2(double K, double G, double s0, double H, double n) {
  fftg_material m;
  memset(&m, 0, sizeof(m));
  m.K = K;
  m.G = G;
  m.sigma_y0 = s0;
  m.H = H;
  m.n = n;
  m.law = FFTG_LAW_J2;
  m.eps0 = 1.0;
  m.t0 = 1.0;
  return m;
}

static fftg_status plan(int n0, int n1, int n2, const std::vector<uint8_t>& ph, int nph,
                        const fftg_material* mats, const fftg_options* o) {
  fftg_plan p = nullptr;
  const fftg_status st = fftg_plan_create(&p, n0, n1, n2, ph.empty() ? nullptr : ph.data(), nph, mats, o, nullptr);
  if (p) fftg_plan_destroy(p);
  return st;
}

int main() {
  fftg_options o;
  fftg_options_default(&o);
  CHECK(o.precision == FFTG_FP64 && o.tol_newton == 1e-5 && o.tol_cg == 1e-8);
  CHECK(o.max_newton == 50 && o.max_cg == 2000 && o.predictor == FFTG_PREDICTOR_TANGENT);
  CHECK(o.dt == 1.0 && o.scheme == FFTG_SCHEME_GALERKIN && o.cg_chunk == 16);

  CHECK(fftg_footprint_bytes(0, 5, 5, FFTG_FP64) == 0);
  CHECK(fftg_footprint_bytes(127, 127, 127, FFTG_MIXED) < fftg_footprint_bytes(127, 127, 127, FFTG_FP64));

  const std::vector<uint8_t> ph(5 * 7 * 9, 0);
  fftg_material ok[2] = {j2(0.833, 0.386, 0.003, 0.004, 1.0), j2(0.833, 0.386, 0.006, 0.008, 0.2)};

  // argument checks (no HIP call before them)
  CHECK(fftg_plan_create(nullptr, 5, 7, 9, ph.data(), 2, ok, nullptr, nullptr) == FFTG_E_INVALID);
  CHECK(plan(4, 7, 9, ph, 2, ok, nullptr) == FFTG_E_INVALID);
  CHECK(plan(5, 0, 9, ph, 2, ok, nullptr) == FFTG_E_INVALID);
  CHECK(plan(5, 7, 9, {}, 2, ok, nullptr) == FFTG_E_INVALID);
  CHECK(plan(5, 7, 9, ph, 0, ok, nullptr) == FFTG_E_INVALID);
  CHECK(plan(5, 7, 9, ph, 17, ok, nullptr) == FFTG_E_INVALID);
  {
    std::vector<uint8_t> bad(ph);
    bad[100] = 2;
    CHECK(plan(5, 7, 9, bad, 2, ok, nullptr) == FFTG_E_INVALID);
  }
  {
    fftg_options b = o;
    b.precision = 7;
    CHECK(plan(5, 7, 9, ph, 2, ok, &b) == FFTG_E_INVALID);
    b = o;
    b.dt = 0.0;
    CHECK(plan(5, 7, 9, ph, 2, ok, &b) == FFTG_E_INVALID);
    b = o;
    b.max_newton = FFTG_MAX_NEWTON + 1;
    CHECK(plan(5, 7, 9, ph, 2, ok, &b) == FFTG_E_INVALID);
    b = o;
    b.scheme = FFTG_SCHEME_BASIC;
    b.precision = FFTG_MIXED;
    CHECK(plan(5, 7, 9, ph, 2, ok, &b) == FFTG_E_UNSUPPORTED);
  }
  // material validation by law
  {
    fftg_material m[2] = {ok[0], ok[1]};
    m[1].n = 1.5;  // J2 n > 1
    CHECK(plan(5, 7, 9, ph, 2, m, nullptr) == FFTG_E_UNSUPPORTED);
    m[1].n = 0.0;
    CHECK(plan(5, 7, 9, ph, 2, m, nullptr) == FFTG_E_INVALID);
    m[1] = ok[1];
    m[1].law = FFTG_LAW_NONLINEAR_ELASTIC;
    m[1].n = 0.5;  // non-linear elastic n < 1
    CHECK(plan(5, 7, 9, ph, 2, m, nullptr) == FFTG_E_UNSUPPORTED);
    m[1].n = 10.0;
    m[1].eps0 = 0.0;
    CHECK(plan(5, 7, 9, ph, 2, m, nullptr) == FFTG_E_INVALID);
    m[1] = ok[1];
    m[1].law = FFTG_LAW_VISCO;
    m[1].n = 2.0;  // visco-plastic n > 1
    CHECK(plan(5, 7, 9, ph, 2, m, nullptr) == FFTG_E_UNSUPPORTED);
    m[1].n = 0.3;
    m[1].t0 = -1.0;
    CHECK(plan(5, 7, 9, ph, 2, m, nullptr) == FFTG_E_INVALID);
    m[1].law = 9;
    CHECK(plan(5, 7, 9, ph, 2, m, nullptr) == FFTG_E_INVALID);
  }
  // a valid plan: FFTG_OK on a GPU; without one, an error from the first
  // HIP call and the partly built plan freed on the way out
  {
    const fftg_status st = plan(5, 7, 9, ph, 2, ok, nullptr);
    CHECK(st == FFTG_OK || st == FFTG_E_HIP || st == FFTG_E_NOMEM);
    CHECK(st == FFTG_OK || strlen(fftg_last_error()) > 0);
  }
  // other entry points' argument checks
  CHECK(fftg_history_create(nullptr, nullptr) == FFTG_E_INVALID);
  size_t bytes = 0;
  CHECK(fftg_history_save(nullptr, nullptr, nullptr, &bytes) == FFTG_E_INVALID);
  fftg_batch b = nullptr;
  CHECK(fftg_batch_create(&b, 0, nullptr, nullptr) == FFTG_E_INVALID);
  CHECK(fftg_profiler_start_every(FFTG_KERNEL_ZFWD, 0) == FFTG_E_INVALID);
  CHECK(fftg_profiler_start_every(-1, 1) == FFTG_E_INVALID);
  double buf[6];
  CHECK(fftg_apply_GK_noalloc(4, 5, 5, buf, buf + 1, FFTG_TANGENT_IDENTITY, nullptr, 0, nullptr, nullptr) ==
        FFTG_E_INVALID);
  CHECK(fftg_apply_GK_noalloc(75, 75, 75, buf, buf + 1, FFTG_TANGENT_IDENTITY, nullptr, 0, nullptr, nullptr) ==
        FFTG_E_INVALID);
  CHECK(fftg_apply_GK_noalloc(5, 5, 127, buf, buf + 1, FFTG_TANGENT_IDENTITY, nullptr, 0, nullptr, nullptr) ==
        FFTG_E_UNSUPPORTED);
  CHECK(fftg_apply_GK_noalloc(5, 5, 5, buf, buf + 1, FFTG_TANGENT_CURRENT, nullptr, 0, nullptr, nullptr) ==
        FFTG_E_INVALID);
  CHECK(fftg_apply_GK_noalloc(5, 5, 5, buf, buf + 1, FFTG_TANGENT_ELASTIC, nullptr, 2, ok, nullptr) ==
        FFTG_E_INVALID);

  printf("%d checks, %d failed\n", g_checks, g_fail);
  return g_fail == 0 ? 0 : 1;
}
