// Host FP64 background cosmology and COLA step factors.
//
// Koda et al. 2015: Sec. 2.1 (second-order growth D2 = -(3/7) D1^2
// Omega(a)^(-1/143), Omega(a) read as the matter fraction
// Om / (Om + OL a^3)); Sec. 2.2 (Poisson factor (3/2) Om / a, eq. cola-drift
// integral, eq. cola-kick factor).  D1 is the linear growing mode (Heath
// integral) normalised to D1(1) = 1.  Time unit 1/H0, flat LCDM.
#include <cmath>

#include "cola_internal.h"

namespace cola {
namespace {

// 15-point Gauss-Kronrod nodes/weights (with the embedded 7-point Gauss rule),
// recursive bisection until the two rules agree to the tolerance.
const double kXgk[8] = {0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
                        0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
                        0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
                        0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
const double kWgk[8] = {0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
                        0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
                        0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
                        0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
const double kWg[4] = {0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
                       0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

template <class F>
double gk15(const F& f, double a, double b, double* err) {
  const double c = 0.5 * (a + b), h = 0.5 * (b - a);
  const double fc = f(c);
  double rk = fc * kWgk[7], rg = fc * kWg[3];
  for (int j = 0; j < 7; ++j) {
    const double x = h * kXgk[j];
    const double s = f(c - x) + f(c + x);
    rk += kWgk[j] * s;
    if (j % 2 == 1) rg += kWg[j / 2] * s;
  }
  *err = std::fabs((rk - rg) * h);
  return rk * h;
}

template <class F>
double integrate(const F& f, double a, double b, double rtol, int depth = 0) {
  double err;
  const double v = gk15(f, a, b, &err);
  if (depth > 40 || err <= rtol * std::fabs(v) || err < 1e-300) return v;
  const double m = 0.5 * (a + b);
  return integrate(f, a, m, rtol, depth + 1) + integrate(f, m, b, rtol, depth + 1);
}

double heath(double a, double om) {
  auto f = [om](double x) {
    if (x <= 0) return 0.0;
    const double ae = x * hubble_E(x, om);
    return 1.0 / (ae * ae * ae);
  };
  return 2.5 * om * hubble_E(a, om) * integrate(f, 0.0, a, 1e-14);
}

}  // namespace

double hubble_E(double a, double om) { return std::sqrt(om / (a * a * a) + (1.0 - om)); }

double growth_D1(double a, double om) { return heath(a, om) / heath(1.0, om); }

double growth_D2(double a, double om) {
  const double d1 = growth_D1(a, om);
  const double omega_a = om / (om + (1.0 - om) * a * a * a);
  return -3.0 / 7.0 * d1 * d1 * std::pow(omega_a, -1.0 / 143.0);
}

double kick_factor(double a_v, double a_x, double a_h, double om, double n) {
  const double adot = a_x * hubble_E(a_x, om);
  // n = 0: the limit of the ansatz, v_res = A + B ln a during the kick
  if (n == 0.0) return std::log(a_h / a_v) * a_x / adot;
  return (std::pow(a_h, n) - std::pow(a_v, n)) / (n * std::pow(a_x, n - 1.0) * adot);
}

double drift_factor(double a0, double a1, double a_h, double om, double n) {
  auto f = [=](double a) { return std::pow(a / a_h, n) / (a * a * a * hubble_E(a, om)); };
  return integrate(f, a0, a1, 1e-14);
}

// Derivative of the Heath form D1 = c E(a) int_0^a da'/(a'E)^3 by the product
// rule: D1 (dE/da)/E + c E/(a E)^3, dE/da = -3 Om/(2 a^4 E), c = 2.5 Om/heath(1).
double growth_D1_prime(double a, double om) {
  const double e = hubble_E(a, om);
  const double de = -1.5 * om / (a * a * a * a * e);
  const double ae = a * e;
  return growth_D1(a, om) * de / e + 2.5 * om / heath(1.0, om) * e / (ae * ae * ae);
}

// D2 = -(3/7) D1^2 Omega(a)^(-1/143): D2 (2 D1'/D1 - (1/143) dln Omega/da),
// dln Omega/da = -3 (1 - Om) a^2 / (Om + (1 - Om) a^3).
double growth_D2_prime(double a, double om) {
  const double dlnom = -3.0 * (1.0 - om) * a * a / (om + (1.0 - om) * a * a * a);
  return growth_D2(a, om) * (2.0 * growth_D1_prime(a, om) / growth_D1(a, om) - dlnom / 143.0);
}

namespace {

// The growth equations d/dt(a^2 dD1/dt) = alpha D1 and
// d/dt(a^2 dD2/dt) = alpha (D2 - D1^2) in x = ln a:
//   D_xx = -(2 - 1.5 Om(a)) D_x + 1.5 Om(a) S,  S = D1 or D2 - D1^2,
// with Om(a) the matter fraction; started at a = 1e-5 on the matter-era
// growing modes D1 = a, D2 = -(3/7) a^2; classical RK4 in x.
void growth_ode_raw(double a_end, double om, double y[4]) {
  const double x0 = std::log(1e-5), x1 = std::log(a_end);
  const int n = 6000;
  const double h = (x1 - x0) / n;
  const double a0 = 1e-5;
  y[0] = a0;                       // D1
  y[1] = a0;                       // dD1/dx
  y[2] = -3.0 / 7.0 * a0 * a0;     // D2
  y[3] = -6.0 / 7.0 * a0 * a0;     // dD2/dx
  auto f = [om](double x, const double* v, double* o) {
    const double a = std::exp(x);
    const double w = 1.5 * om / (om + (1.0 - om) * a * a * a);
    o[0] = v[1];
    o[1] = -(2.0 - w) * v[1] + w * v[0];
    o[2] = v[3];
    o[3] = -(2.0 - w) * v[3] + w * (v[2] - v[0] * v[0]);
  };
  double k1[4], k2[4], k3[4], k4[4], t[4];
  for (int i = 0; i < n; ++i) {
    const double x = x0 + i * h;
    f(x, y, k1);
    for (int j = 0; j < 4; ++j) t[j] = y[j] + 0.5 * h * k1[j];
    f(x + 0.5 * h, t, k2);
    for (int j = 0; j < 4; ++j) t[j] = y[j] + 0.5 * h * k2[j];
    f(x + 0.5 * h, t, k3);
    for (int j = 0; j < 4; ++j) t[j] = y[j] + h * k3[j];
    f(x + h, t, k4);
    for (int j = 0; j < 4; ++j) y[j] += h / 6.0 * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]);
  }
}

// Unnormalised D1 at a = 1 for the last Omega_m this thread asked for (the
// normalisation of every ODE value; the same integration, done once).
double growth_ode_norm(double om) {
  thread_local double last_om = -1.0, last_n1 = 0.0;
  if (om != last_om) {
    double y1[4];
    growth_ode_raw(1.0, om, y1);
    last_om = om;
    last_n1 = y1[0];
  }
  return last_n1;
}

}  // namespace

// D2 from its growth equation, normalised with D1(1) = 1 (D2 scales as D1^2).
double growth_D2_ode(double a, double om) {
  double y[4];
  growth_ode_raw(a, om, y);
  const double n1 = growth_ode_norm(om);
  return y[2] / (n1 * n1);
}

double growth_D2_ode_prime(double a, double om) {
  double y[4];
  growth_ode_raw(a, om, y);
  const double n1 = growth_ode_norm(om);
  return y[3] / a / (n1 * n1);
}

double D2_of(const cola_params* p, double a) {
  return (p->flags & COLA_F_D2_ODE) ? growth_D2_ode(a, p->omega_m) : growth_D2(a, p->omega_m);
}

double D2_prime_of(const cola_params* p, double a) {
  return (p->flags & COLA_F_D2_ODE) ? growth_D2_ode_prime(a, p->omega_m) : growth_D2_prime(a, p->omega_m);
}

double interp_pk(double k, const double* kt, const double* pt, int nk) {
  if (!(k > 0)) return 0.0;
  const double x = std::log(k);
  int lo = 0, hi = nk - 1;
  // last j with ln kt[j] <= x, clamped to [0, nk-2]
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (std::log(kt[mid]) <= x) lo = mid; else hi = mid;
  }
  const double x0 = std::log(kt[lo]), x1 = std::log(kt[lo + 1]);
  const double y0 = std::log(pt[lo]), y1 = std::log(pt[lo + 1]);
  const double t = (x - x0) / (x1 - x0);
  return std::exp(y0 + t * (y1 - y0));
}

}  // namespace cola
