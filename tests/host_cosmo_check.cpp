// Host-only driver of the library's float64 cosmology (cosmo.cpp), built by
// tests/test_host_sanitizers.py with AddressSanitizer and
// UndefinedBehaviorSanitizer: every power-spectrum kind, the growth
// integration, the FastPM and plain-leapfrog step factors over long and
// short scale-factor lists.  Exits non-zero on a non-finite or inconsistent
// value (the sanitizers abort on their own findings).
#include <cmath>
#include <cstdio>
#include <vector>

#include "cosmo.h"

namespace {
int fails = 0;
void check(bool ok, const char* what, double v) {
  if (!ok) {
    std::printf("FAIL %s (%g)\n", what, v);
    ++fails;
  }
}
}  // namespace

int main() {
  const double ks[4] = {1e-3, 1e-2, 1e-1, 1.0};
  const double ps[4] = {2e3, 2e4, 5e3, 50.0};
  for (int kind = 0; kind < 3; ++kind) {
    pm_cosmo c{};
    c.omega_m = 0.3;
    c.omega_b = 0.05;
    c.h = 0.7;
    c.n_s = 0.96;
    c.sigma8 = 0.8;
    c.t_cmb = 2.7255;
    c.pk_kind = kind;
    c.pk_index = -2.0;
    c.pk_k = ks;
    c.pk_p = ps;
    c.pk_n = 4;
    pmk::Cosmo co;
    co.init(c);
    for (double k = 1e-4; k < 10.0; k *= 1.7) check(std::isfinite(co.pk(k)) && co.pk(k) >= 0, "pk", co.pk(k));
    // the no-wiggle spectrum is normalised by this integral (the power law
    // by its closed form: the integral's k range truncates k^-2)
    if (kind == 1) {
      const double s8 = std::sqrt(co.amp) * co.sigma_r(8.0);
      check(std::fabs(s8 - 0.8) < 1e-9, "sigma8", s8);
    }
    double g[6];
    co.growth(1.0, g);
    check(std::fabs(g[0] - 1.0) < 1e-12, "D1(1)", g[0]);
    for (double a = 0.01; a <= 1.0; a += 0.07) {
      co.growth(a, g);
      for (double v : g) check(std::isfinite(v), "growth", v);
    }
    for (int n_a : {2, 3, 11, 200}) {
      std::vector<double> a(n_a), k1(n_a - 1), dr(n_a - 1), k2(n_a - 1);
      for (int i = 0; i < n_a; ++i) a[i] = 0.1 + 0.9 * i / (n_a - 1);
      for (int integ = 0; integ <= 2; ++integ) {
        co.step_factors(integ, a.data(), n_a, k1.data(), dr.data(), k2.data());
        for (int i = 0; i < n_a - 1; ++i) {
          check(std::isfinite(k1[i]) && k1[i] > 0, "k1", k1[i]);
          check(std::isfinite(dr[i]) && dr[i] > 0, "dr", dr[i]);
          check(std::isfinite(k2[i]) && k2[i] > 0, "k2", k2[i]);
        }
      }
    }
    // the plain leapfrog factors in closed form for Omega_m = 1 are checked
    // by the Python tests; here their additivity over a split interval
    const double s = co.std_kick(0.2, 0.5) + co.std_kick(0.5, 0.9) - co.std_kick(0.2, 0.9);
    check(std::fabs(s) < 1e-10, "kick additivity", s);
  }
  std::printf(fails ? "host cosmology check failed\n" : "host cosmology check ok\n");
  return fails ? 1 : 0;
}
