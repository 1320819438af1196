// Host-side cosmology (float64); see cosmo.cpp.
#pragma once

#include <vector>

#include "pm.h"

namespace pmk {

struct Cosmo {
  double om = 0.3;
  double d1_today = 1.0;
  double amp = 1.0;
  pm_cosmo par{};
  std::vector<double> tab_lnk, tab_lnp;

  void init(const pm_cosmo& c);
  double E(double a) const;
  // out6 = D1, f1, D2, f2, E, G_f (D1(1) = 1, D2 scaled by D1(1)^2)
  void growth(double a, double* out6) const;
  double D1(double a) const;
  double Gf(double a) const;
  double drift(double ai, double aj, double ac) const;
  double kick(double ai, double aj, double ar) const;
  // Factors of n_a - 1 KDK steps over a[0] < ... < a[n_a-1]: the opening
  // kick k1 (a_i -> a_c), drift dr (a_i -> a_j) and closing kick k2
  // (a_c -> a_j), a_c = sqrt(a_i a_j), from one sweep of the growth ODE.
  void kdk_factors(const double* a, int n_a, double* k1, double* dr, double* k2) const;
  // The plain leapfrog's factors: int_ai^aj da / (a^2 E) and da / (a^3 E).
  double std_kick(double ai, double aj) const;
  double std_drift(double ai, double aj) const;
  // k1, dr, k2 of the integrator (PM_INT_*) over the n_a scale factors
  void step_factors(int integrator, const double* a, int n_a, double* k1, double* dr, double* k2) const;
  double eh_transfer(double k) const;
  double shape(double k) const;
  double pk(double k) const;          // linear P(k) at a = 1, (Mpc/h)^3
  double sigma_r(double r) const;      // of amp * shape

 private:
  void rhs(double lna, const double* y, double* dy) const;
  void integrate(double a, double* y) const;
  void rk4_step(double l, double h, const double* y, double* out) const;
  // growth() at n ascending scale factors from a single integration
  void growth_sorted(const double* a, int n, double* out6) const;
};

}  // namespace pmk
