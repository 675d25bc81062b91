// Host AddressSanitizer / UndefinedBehaviorSanitizer walk over libgm's C ABI.
//
// Linked with the library's host-logic translation units (gm_api, gm_batch,
// gm_grad) compiled with host-side -fsanitize=address,undefined (device code
// is compiled as usual); the per-family kernel objects are linked unchanged.
// Every entry point runs on small inputs, including the argument checks and
// the caller-owned workspace paths, so an out-of-bounds host access, a
// use-after-free or an undefined operation in the host code fails the run.
// The results are checked for the properties the C ABI states (status codes,
// closed forms, equality of equivalent calls), not against the oracle.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "gm.h"

static int g_fail = 0;

// Progress line per step, with the seconds since the previous one.
static void step(const char* name) {
  static auto t0 = std::chrono::steady_clock::now();
  const auto t1 = std::chrono::steady_clock::now();
  std::printf("step %s (%.2f s after the previous)\n", name, std::chrono::duration<double>(t1 - t0).count());
  std::fflush(stdout);
  t0 = t1;
}

#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++g_fail;                                                            \
    }                                                                      \
  } while (0)

// Closed form of the Gaussian family on [0,1]^d: prod_j int_0^1 exp(-a^2 (x-u)^2) dx.
static double gaussian_exact(const std::vector<double>& p, int d) {
  double v = 1.0;
  for (int j = 0; j < d; ++j) {
    const double a = p[j], u = p[d + j];
    v *= std::sqrt(M_PI) / (2.0 * a) * (std::erf(a * (1.0 - u)) + std::erf(a * u));
  }
  return v;
}

static std::vector<double> params(int d, double a, double u) {
  std::vector<double> p(2 * d);
  for (int j = 0; j < d; ++j) {
    p[j] = a * (1.0 + 0.1 * j);
    p[d + j] = u;
  }
  return p;
}

int main() {
  step("start");
  const int d = 3;
  std::vector<double> lo(16, 0.0), hi(16, 1.0);
  std::vector<double> p = params(d, 5.0, 0.5);
  double I = 0, E = 0;

  // status strings
  for (int s = -3; s <= 4; ++s) CHECK(gm_status_string(s) != nullptr);
  CHECK(gm_status_string(99) != nullptr);

  // argument checks: nothing runs
  CHECK(gm_integrate(GM_GAUSSIAN, p.data(), 1, lo.data(), hi.data(), 1e-6, 0, 1 << 16, &I, &E, nullptr) == GM_EINVAL);
  CHECK(gm_integrate(GM_GAUSSIAN, p.data(), 17, lo.data(), hi.data(), 1e-6, 0, 1 << 16, &I, &E, nullptr) == GM_EINVAL);
  CHECK(gm_integrate(99, p.data(), d, lo.data(), hi.data(), 1e-6, 0, 1 << 16, &I, &E, nullptr) == GM_EINVAL);
  CHECK(gm_integrate(GM_GAUSSIAN, nullptr, d, lo.data(), hi.data(), 1e-6, 0, 1 << 16, &I, &E, nullptr) == GM_EINVAL);
  CHECK(gm_integrate(GM_GAUSSIAN, p.data(), d, hi.data(), lo.data(), 1e-6, 0, 1 << 16, &I, &E, nullptr) == GM_EINVAL);
  CHECK(gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), NAN, 0, 1 << 16, &I, &E, nullptr) == GM_EINVAL);
  CHECK(gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 0, 0, 1 << 16, &I, &E, nullptr) == GM_EINVAL);
  CHECK(gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-6, 0, 2, &I, &E, nullptr) == GM_EINVAL);
  CHECK(gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-6, 0, 1 << 16, nullptr, &E, nullptr) == GM_EINVAL);
  CHECK(gm_set_option("no_such_option", 1) == GM_EINVAL);
  CHECK(gm_set_option("max_iters", 0) == GM_EINVAL);
  CHECK(gm_num_nodes(8) == 256 + 128 + 16 + 1);

  // a run against its closed form, the statistics and the last active set
  step("first run");
  int rc = gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-8, 1e-16, 1 << 20, &I, &E, nullptr);
  CHECK(rc == GM_OK);
  const double exact = gaussian_exact(p, d);
  CHECK(std::fabs(I - exact) <= 1e-7 * exact);
  gm_stats st;
  CHECK(gm_last_stats(&st) == GM_OK);
  CHECK(st.iterations >= 1 && st.regions_evaluated > 0);
  const int64_t na = gm_last_active(0, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  CHECK(na > 0);
  {
    const int64_t k = na < 37 ? na : 37;
    std::vector<double> c(k * d), h(k * d), q(k), e(k);
    std::vector<int32_t> lv(k), ax(k);
    CHECK(gm_last_active(na - k, 100, c.data(), h.data(), lv.data(), q.data(), e.data(), ax.data()) == na);
    CHECK(gm_last_active(1, 3, nullptr, h.data(), nullptr, q.data(), nullptr, nullptr) == na);
    CHECK(gm_last_active(na + 5, 3, c.data(), h.data(), lv.data(), q.data(), e.data(), ax.data()) == na);
    CHECK(gm_last_active(-1, 3, c.data(), nullptr, nullptr, nullptr, nullptr, nullptr) == GM_EINVAL);
    for (int64_t i = 0; i < k * d; ++i) CHECK(h[i] > 0.0 && c[i] > 0.0 && c[i] < 1.0);
  }

  // every family, the degree-9 and Gauss-Kronrod rules, pruning, per-phase timing, the log
  step("families and options");
  for (int fam = 1; fam <= 7; ++fam) {
    std::vector<double> pf = params(4, fam == GM_CORNER_PEAK ? 0.3 : 2.0, 0.4);
    rc = gm_integrate(fam, pf.data(), 4, lo.data(), hi.data(), 1e-5, 1e-16, 1 << 18, &I, &E, nullptr);
    CHECK(rc >= 0 && std::isfinite(I) && std::isfinite(E));
  }
  CHECK(gm_set_option("rule", 2) == GM_OK);
  CHECK(gm_set_option("err_model", 1) == GM_OK);
  rc = gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-9, 1e-16, 1 << 20, &I, &E, nullptr);
  CHECK(rc == GM_OK && std::fabs(I - exact) <= 1e-8 * exact);
  CHECK(gm_set_option("err_model", 0) == GM_OK);
  CHECK(gm_set_option("rule", 1) == GM_OK);
  rc = gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-10, 1e-16, 1 << 16, &I, &E, nullptr);
  CHECK(rc == GM_OK && std::fabs(I - exact) <= 1e-9 * exact);
  CHECK(gm_integrate(GM_GAUSSIAN, p.data(), 7, lo.data(), hi.data(), 1e-6, 0, 1 << 16, &I, &E, nullptr) == GM_EINVAL);
  CHECK(gm_set_option("rule", 0) == GM_OK);
  CHECK(gm_set_option("prune", 1) == GM_OK);
  std::vector<double> p8 = params(8, 1.0, 0.3);
  rc = gm_integrate(GM_GAUSSIAN, p8.data(), 8, lo.data(), hi.data(), 1e-7, 1e-16, 1 << 14, &I, &E, nullptr);
  CHECK((rc == GM_OK || rc == GM_MAX_REGIONS) && std::isfinite(I));
  CHECK(gm_set_option("prune", 0) == GM_OK);
  CHECK(gm_set_option("timing", 2) == GM_OK);
  rc = gm_integrate(GM_OSCILLATORY, p8.data(), 8, lo.data(), hi.data(), 1e-4, 1e-16, 1 << 20, &I, &E, nullptr);
  CHECK(rc == GM_OK && gm_last_stats(&st) == GM_OK && st.rule_ms > 0.0);
  CHECK(gm_set_option("timing", 0) == GM_OK);
  CHECK(gm_set_option("log", 1) == GM_OK);
  rc = gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-4, 1e-16, 1 << 16, &I, &E, nullptr);
  CHECK(rc == GM_OK);
  CHECK(gm_set_option("log", 0) == GM_OK);
  // forced stops
  CHECK(gm_set_option("max_iters", 1) == GM_OK);
  CHECK(gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-12, 1e-16, 1 << 16, &I, &E, nullptr) == GM_MAX_ITERS);
  CHECK(gm_set_option("max_iters", 10000) == GM_OK);
  CHECK(gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-14, 1e-16, 5000, &I, &E, nullptr) == GM_MAX_REGIONS);
  {
    const double pc[4] = {-1.0, -1.0, 0.0, 0.0};
    CHECK(gm_integrate(GM_CORNER_PEAK, pc, 2, lo.data(), hi.data(), 1e-6, 1e-16, 1 << 16, &I, &E, nullptr) == GM_NONFINITE);
    CHECK(std::isnan(I) && std::isnan(E));
  }

  // the rule kernel on a caller-given region list
  step("region list");
  {
    const int64_t n = 10;
    std::vector<double> c(n * d), h(n * d, 0.125), q(n), e(n);
    std::vector<int32_t> lv(n, 2 * d), ax(n);  // width 1/4 per axis: volume 2^-2d
    for (int64_t i = 0; i < n * d; ++i) c[i] = 0.125 + 0.25 * (i % 4);
    CHECK(gm_eval_regions(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), n, c.data(), h.data(), lv.data(),
                          q.data(), e.data(), ax.data(), nullptr) == GM_OK);
    for (int64_t i = 0; i < n; ++i) CHECK(q[i] > 0.0 && e[i] >= 0.0 && (ax[i] & 63) < d);
  }

  // gradient mode
  step("gradient");
  {
    std::vector<double> g(2 * d, 0.0);
    rc = gm_integrate_grad(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-8, 1e-16, 1 << 20, &I, &E, g.data(), nullptr);
    CHECK(rc == GM_OK && std::fabs(I - exact) <= 1e-7 * exact);
    // dI/du_j = 0 at u = 1/2 by symmetry; dI/da_j < 0
    for (int j = 0; j < d; ++j) CHECK(g[j] < 0.0 && std::fabs(g[d + j]) <= 1e-6 * std::fabs(g[j]));
    CHECK(gm_set_option("rule", 2) == GM_OK);
    std::vector<double> g8(16, 0.0);
    rc = gm_integrate_grad(GM_OSCILLATORY, p8.data(), 8, lo.data(), hi.data(), 1e-6, 1e-16, 1 << 20, &I, &E, g8.data(), nullptr);
    CHECK(rc == GM_OK);
    CHECK(gm_set_option("rule", 1) == GM_OK);
    CHECK(gm_integrate_grad(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-8, 1e-16, 1 << 20, &I, &E, g.data(), nullptr) == GM_EINVAL);
    CHECK(gm_set_option("rule", 0) == GM_OK);
  }

  // batch: 64 mixed items and one invalid item, against single calls
  step("batch");
  {
    const int n = 65;
    std::vector<int> ids(n), ds(n), status(n);
    std::vector<double> bp, blo, bhi, rt(n), at(n, 1e-16), est(n), err(n);
    for (int i = 0; i < n; ++i) {
      ids[i] = (i % 3 == 0) ? GM_GAUSSIAN : (i % 3 == 1) ? GM_OSCILLATORY : GM_PRODUCT_PEAK;
      ds[i] = (i == n - 1) ? 11 : 2 + i % 5;  // item n-1: d > 10 is rejected per item
      rt[i] = 1e-5;
      std::vector<double> pi = params(ds[i], 0.5 + 0.02 * i, 0.3);
      bp.insert(bp.end(), pi.begin(), pi.end());
      for (int j = 0; j < ds[i]; ++j) {
        blo.push_back(0.0);
        bhi.push_back(1.0);
      }
    }
    rc = gm_integrate_batch(n, ids.data(), bp.data(), ds.data(), blo.data(), bhi.data(), rt.data(), at.data(),
                            1 << 22, est.data(), err.data(), status.data(), nullptr);
    CHECK(rc >= 0);
    CHECK(status[n - 1] == GM_EINVAL && std::isnan(est[n - 1]));
    size_t off = 0;
    for (int i = 0; i < n - 1; ++i) {
      CHECK(status[i] == GM_OK);
      if (i % 9 == 0) {
        double Is = 0, Es = 0;
        CHECK(gm_integrate(ids[i], bp.data() + off, ds[i], lo.data(), hi.data(), rt[i], at[i], 1 << 22, &Is, &Es,
                           nullptr) == GM_OK);
        CHECK(std::fabs(Is - est[i]) <= 1e-12 * std::fabs(Is));
      }
      off += 2 * ds[i];
    }
    CHECK(gm_set_option("graph_iters", 0) == GM_OK);
    rc = gm_integrate_batch(n - 1, ids.data(), bp.data(), ds.data(), blo.data(), bhi.data(), rt.data(), at.data(),
                            1 << 22, est.data(), err.data(), status.data(), nullptr);
    CHECK(rc == GM_OK);
    CHECK(gm_set_option("graph_iters", 8) == GM_OK);
    CHECK(gm_set_tile(8, GM_GAUSSIAN, 4, 1024) == GM_OK);
    CHECK(gm_set_tile(8, GM_GAUSSIAN, 0, 0) == GM_OK);
    CHECK(gm_set_tile(11, GM_GAUSSIAN, 4, 0) == GM_EINVAL);
  }

  // caller-owned workspace: same bits as library memory; too small -> GM_ENOMEM; misaligned -> GM_EINVAL
  step("workspace");
  {
    double I0 = 0, E0 = 0, I1 = 0, E1 = 0;
    CHECK(gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-8, 1e-16, 1 << 18, &I0, &E0, nullptr) == GM_OK);
    const size_t need = gm_workspace_bytes(d, 1 << 18, 0);
    CHECK(need > 0);
    void* ws = nullptr;
    CHECK(hipMalloc(&ws, need + 512) == hipSuccess);
    CHECK(gm_set_workspace(ws, need) == GM_OK);
    CHECK(gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-8, 1e-16, 1 << 18, &I1, &E1, nullptr) == GM_OK);
    CHECK(I0 == I1 && E0 == E1);
    I1 = -7.0;
    CHECK(gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-8, 1e-16, 1 << 20, &I1, &E1, nullptr) == GM_ENOMEM);
    CHECK(I1 == -7.0);
    CHECK(gm_set_workspace((char*)ws + 8, need) == GM_EINVAL);
    CHECK(gm_set_workspace(nullptr, 0) == GM_OK);
    CHECK(hipFree(ws) == hipSuccess);
    CHECK(gm_integrate(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-8, 1e-16, 1 << 18, &I1, &E1, nullptr) == GM_OK);
    CHECK(I0 == I1);

    // the no-allocation entry point
    double I2 = 0, E2 = 0;
    CHECK(gm_integrate_noalloc(GM_GAUSSIAN, p.data(), d, lo.data(), hi.data(), 1e-8, 1e-16, 1 << 18, &I2, &E2, nullptr) == GM_OK);
    CHECK(I2 == I0 && E2 == E0);
    CHECK(gm_integrate_noalloc(GM_GAUSSIAN, p8.data(), 8, lo.data(), hi.data(), 1e-8, 1e-16, int64_t(1) << 24, &I2, &E2, nullptr) == GM_EINVAL);
  }

  step("end");
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("libgm sanitize run ok\n");
  return 0;
}
