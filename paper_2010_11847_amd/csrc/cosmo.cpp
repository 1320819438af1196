// Host-side background cosmology in float64: expansion rate, linear growth
// (first and second order), the FastPM kick/drift factors and the linear
// power spectrum.  Independent of any test code: the growth equations are
// integrated with classical fourth-order Runge-Kutta in ln a, the sigma8
// integral with composite Simpson in ln k.
//
// Kick and drift factors (section 2 of the paper defers them to FastPM):
// with x' = p / (a^3 E) and p' = F / (a^2 E) (' = d/da), requiring the
// Zel'dovich solution x = q + D1 s to be exact gives
//   drift(ai -> aj; ac) = (D1(aj) - D1(ai)) / G_f(ac),    G_f = a^3 E dD1/da
//   kick (ai -> aj; ar) = (G_f(aj) - G_f(ai)) / (1.5 Om D1(ar)).
#include "cosmo.h"

#include <algorithm>
#include <cmath>

namespace pmk {

namespace {
constexpr double kPi = 3.14159265358979323846;
constexpr double kLnAInit = -11.512925464970229;   // ln(1e-5)
constexpr double kStep = 1.0 / 512.0;              // RK4 step in ln a
}  // namespace

double Cosmo::E(double a) const { return std::sqrt(om / (a * a * a) + (1.0 - om)); }

// y = (D1, dD1/dlna, D2, dD2/dlna)
void Cosmo::rhs(double lna, const double* y, double* dy) const {
  const double a = std::exp(lna);
  const double a3 = a * a * a;
  const double e2 = om / a3 + (1.0 - om);
  const double oma = om / a3 / e2;
  const double c = 2.0 - 1.5 * oma;   // 2 + dlnE/dlna
  dy[0] = y[1];
  dy[1] = -c * y[1] + 1.5 * oma * y[0];
  dy[2] = y[3];
  dy[3] = -c * y[3] + 1.5 * oma * y[2] - 1.5 * oma * y[0] * y[0];
}

void Cosmo::rk4_step(double l, double h, const double* y, double* out) const {
  double k1[4], k2[4], k3[4], k4[4], t[4];
  rhs(l, y, k1);
  for (int i = 0; i < 4; ++i) t[i] = y[i] + 0.5 * h * k1[i];
  rhs(l + 0.5 * h, t, k2);
  for (int i = 0; i < 4; ++i) t[i] = y[i] + 0.5 * h * k2[i];
  rhs(l + 0.5 * h, t, k3);
  for (int i = 0; i < 4; ++i) t[i] = y[i] + h * k3[i];
  rhs(l + h, t, k4);
  for (int i = 0; i < 4; ++i) out[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

static void growing_mode_start(double* y) {
  const double a0 = std::exp(kLnAInit);
  y[0] = a0;
  y[1] = a0;
  y[2] = -3.0 / 7.0 * a0 * a0;
  y[3] = -6.0 / 7.0 * a0 * a0;
}

void Cosmo::integrate(double a, double* y) const {
  growing_mode_start(y);
  const double l1 = std::log(a);
  const int n = std::max(1, (int)std::ceil((l1 - kLnAInit) / kStep));
  const double h = (l1 - kLnAInit) / n;
  double l = kLnAInit;
  for (int s = 0; s < n; ++s) {
    rk4_step(l, h, y, y);
    l += h;
  }
}

// Fixed steps of kStep in ln a along one trajectory; each target is reached
// from the last grid point below it by one shorter step taken on a copy.
void Cosmo::growth_sorted(const double* a, int n, double* out6) const {
  double y[4], t[4];
  growing_mode_start(y);
  double l = kLnAInit;
  for (int j = 0; j < n; ++j) {
    const double lt = std::log(a[j]);
    while (l + kStep <= lt) {
      rk4_step(l, kStep, y, y);
      l += kStep;
    }
    if (lt > l)
      rk4_step(l, lt - l, y, t);
    else
      for (int i = 0; i < 4; ++i) t[i] = y[i];
    double* o = out6 + 6 * j;
    const double e = E(a[j]);
    o[0] = t[0] / d1_today;
    o[1] = t[1] / t[0];
    o[2] = t[2] / (d1_today * d1_today);
    o[3] = t[3] / t[2];
    o[4] = e;
    o[5] = a[j] * a[j] * e * o[1] * o[0];
  }
}

void Cosmo::kdk_factors(const double* a, int n_a, double* k1, double* dr, double* k2) const {
  const int ns = n_a - 1;
  if (ns < 1) return;
  // a_i, a_c, a_j of every step interleave as a_0 < a_c0 < a_1 < a_c1 < ...
  std::vector<double> pts(2 * ns + 1), g(6 * (2 * ns + 1));
  for (int i = 0; i <= ns; ++i) pts[2 * i] = a[i];
  for (int i = 0; i < ns; ++i) pts[2 * i + 1] = std::sqrt(a[i] * a[i + 1]);
  growth_sorted(pts.data(), 2 * ns + 1, g.data());
  auto d1 = [&](int p) { return g[6 * p]; };
  auto gf = [&](int p) { return g[6 * p + 5]; };
  for (int i = 0; i < ns; ++i) {
    const int pi = 2 * i, pc = 2 * i + 1, pj = 2 * i + 2;
    k1[i] = (gf(pc) - gf(pi)) / (1.5 * om * d1(pi));
    dr[i] = (d1(pj) - d1(pi)) / gf(pc);
    k2[i] = (gf(pj) - gf(pc)) / (1.5 * om * d1(pj));
  }
}

namespace {
// int_ai^aj f(a) da as int f(a) a dln a, composite Simpson over 512 intervals
// in ln a (the integrands are smooth powers of a times 1/E)
template <class F>
double simpson_lna(double ai, double aj, F f) {
  constexpr int kN = 512;
  const double l0 = std::log(ai), h = (std::log(aj) - l0) / kN;
  double s = 0.0;
  for (int i = 0; i <= kN; ++i) {
    const double a = std::exp(l0 + i * h);
    const double w = (i == 0 || i == kN) ? 1.0 : (i % 2 ? 4.0 : 2.0);
    s += w * f(a) * a;
  }
  return s * h / 3.0;
}
}  // namespace

double Cosmo::std_kick(double ai, double aj) const {
  return simpson_lna(ai, aj, [&](double a) { return 1.0 / (a * a * E(a)); });
}

double Cosmo::std_drift(double ai, double aj) const {
  return simpson_lna(ai, aj, [&](double a) { return 1.0 / (a * a * a * E(a)); });
}

void Cosmo::step_factors(int integrator, const double* a, int n_a, double* k1, double* dr, double* k2) const {
  if (integrator == PM_INT_FASTPM) {
    kdk_factors(a, n_a, k1, dr, k2);
    return;
  }
  for (int i = 0; i + 1 < n_a; ++i) {
    const double ac = std::sqrt(a[i] * a[i + 1]);
    k1[i] = std_kick(a[i], ac);
    dr[i] = std_drift(a[i], a[i + 1]);
    k2[i] = std_kick(ac, a[i + 1]);
  }
}

void Cosmo::init(const pm_cosmo& c) {
  om = c.omega_m;
  par = c;
  if (c.pk_kind == PM_PK_TABLE && c.pk_n >= 2 && c.pk_k && c.pk_p) {
    tab_lnk.resize(c.pk_n);
    tab_lnp.resize(c.pk_n);
    for (int i = 0; i < c.pk_n; ++i) {
      tab_lnk[i] = std::log(c.pk_k[i]);
      tab_lnp[i] = std::log(std::max(c.pk_p[i], 1e-300));
    }
  }
  double y[4];
  integrate(1.0, y);
  d1_today = y[0];
  amp = 1.0;
  if (c.pk_kind == PM_PK_TABLE) {
    amp = c.pk_amp > 0 ? c.pk_amp : 1.0;
  } else if (c.pk_amp > 0) {
    amp = c.pk_amp;
  } else if (c.pk_kind == PM_PK_POWERLAW && c.pk_index == -2.0) {
    // sigma8^2 = A/(2 pi^2 R) int_0^inf W_TH(x)^2 dx and the integral is 3 pi / 5
    amp = c.sigma8 * c.sigma8 * 2.0 * kPi * kPi * 8.0 / (3.0 * kPi / 5.0);
  } else {
    const double s = sigma_r(8.0);
    amp = (c.sigma8 * c.sigma8) / (s * s);
  }
}

void Cosmo::growth(double a, double* out6) const {
  double y[4];
  integrate(a, y);
  const double d1 = y[0] / d1_today;
  const double f1 = y[1] / y[0];
  const double d2 = y[2] / (d1_today * d1_today);
  const double f2 = y[3] / y[2];
  const double e = E(a);
  out6[0] = d1;
  out6[1] = f1;
  out6[2] = d2;
  out6[3] = f2;
  out6[4] = e;
  out6[5] = a * a * e * f1 * d1;   // G_f
}

double Cosmo::D1(double a) const {
  double g[6];
  growth(a, g);
  return g[0];
}

double Cosmo::Gf(double a) const {
  double g[6];
  growth(a, g);
  return g[5];
}

double Cosmo::drift(double ai, double aj, double ac) const { return (D1(aj) - D1(ai)) / Gf(ac); }

double Cosmo::kick(double ai, double aj, double ar) const { return (Gf(aj) - Gf(ai)) / (1.5 * om * D1(ar)); }

double Cosmo::eh_transfer(double k) const {
  const double h = par.h, om_ = par.omega_m, ob = par.omega_b;
  const double omh2 = om_ * h * h, obh2 = ob * h * h, fb = ob / om_;
  const double theta = par.t_cmb / 2.7;
  const double s = 44.5 * std::log(9.83 / omh2) / std::sqrt(1.0 + 10.0 * std::pow(obh2, 0.75));
  const double alpha = 1.0 - 0.328 * std::log(431.0 * omh2) * fb + 0.38 * std::log(22.3 * omh2) * fb * fb;
  const double ks = 0.43 * k * h * s;
  const double gamma = om_ * h * (alpha + (1.0 - alpha) / (1.0 + ks * ks * ks * ks));
  const double q = k * theta * theta / gamma;
  const double l0 = std::log(2.0 * std::exp(1.0) + 1.8 * q);
  const double c0 = 14.2 + 731.0 / (1.0 + 62.5 * q);
  return l0 / (l0 + c0 * q * q);
}

double Cosmo::shape(double k) const {
  if (k <= 0) return 0.0;
  switch (par.pk_kind) {
    case PM_PK_POWERLAW:
      return std::pow(k, par.pk_index);
    case PM_PK_EH_NOWIGGLE: {
      const double t = eh_transfer(k);
      return std::pow(k, par.n_s) * t * t;
    }
    case PM_PK_TABLE: {
      if (tab_lnk.empty()) return 0.0;
      const double lk = std::log(k);
      const size_t n = tab_lnk.size();
      size_t i = std::upper_bound(tab_lnk.begin(), tab_lnk.end(), lk) - tab_lnk.begin();
      i = std::min(std::max<size_t>(i, 1), n - 1);
      const double t = (lk - tab_lnk[i - 1]) / (tab_lnk[i] - tab_lnk[i - 1]);
      return std::exp(tab_lnp[i - 1] + t * (tab_lnp[i] - tab_lnp[i - 1]));
    }
    default:
      return 0.0;
  }
}

double Cosmo::pk(double k) const { return k > 0 ? amp * shape(k) : 0.0; }

double Cosmo::sigma_r(double r) const {
  // sigma^2 = 1/(2 pi^2) int k^3 P(k) W(kR)^2 dln k over k in [1e-5, 1e2]
  const double lo = std::log(1e-5), hi = std::log(1e2);
  const int n = 1 << 17;
  const double h = (hi - lo) / n;
  auto f = [&](double lk) {
    const double k = std::exp(lk);
    const double x = k * r;
    double w;
    if (x < 1e-3)
      w = 1.0 - x * x / 10.0 + x * x * x * x / 280.0;
    else
      w = 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
    return k * k * k * shape(k) * w * w;
  };
  double sum = f(lo) + f(hi);
  for (int i = 1; i < n; ++i) sum += (i & 1 ? 4.0 : 2.0) * f(lo + i * h);
  return std::sqrt(sum * h / 3.0 / (2.0 * kPi * kPi));
}

}  // namespace pmk
