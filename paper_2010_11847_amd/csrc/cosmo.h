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
  double eh_transfer(double k) const;
  double shape(double k) const;
  double pk(double k) const;          // linear P(k) at a = 1, (Mpc/h)^3
  double sigma_r(double r) const;      // of amp * shape

 private:
  void rhs(double lna, const double* y, double* dy) const;
  void integrate(double a, double* y) const;
};

}  // namespace pmk
