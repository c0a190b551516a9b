"""Background cosmology and COLA time-stepping factors, float64.

Units: H0 = 1 (time in 1/H0); flat LCDM with Omega_Lambda = 1 - Omega_m.

Paper passages followed (Koda et al. 2015):
* Sec. 2.1: second-order growth D2 = -(3/7) D1^2 Omega(a)^(-1/143).  The
  printed Omega(a) is garbled (a product); it is read as the matter fraction
  Omega_m / (Omega_m + Omega_L a^3).
* Sec. 2.2, Poisson equation in comoving coordinates: the source factor
  (3/2) Omega_m a^-1 (here ``alpha``).
* Sec. 2.2, eq. cola-drift: x_res advances by v_res_{i+1/2} times the integral
  of (a/a_{i+1/2})^n_LPT dt/a^2, evaluated numerically.
* Sec. 2.2, eq. cola-kick: v_res advances by
  (a^n - a_{i-1/2}^n) / (n a_i^(n-1) adot_i) times F_res(x_i).

The linear growth D1 is not defined further in the paper; it is the growing
mode of linear theory (Heath integral), normalised to D1(a=1) = 1.
"""
from __future__ import annotations

import math

from scipy import integrate


def hubble_E(a: float, om: float) -> float:
    """E(a) = H/H0 for flat LCDM."""
    return math.sqrt(om / a ** 3 + (1.0 - om))


def adot(a: float, om: float) -> float:
    """da/dt with H0 = 1."""
    return a * hubble_E(a, om)


def _heath_unnormalised(a: float, om: float) -> float:
    # D(a) proportional to E(a) * int_0^a da' / (a' E(a'))^3.
    f = lambda x: 1.0 / (x * hubble_E(x, om)) ** 3 if x > 0 else 0.0
    val, _ = integrate.quad(f, 0.0, a, epsabs=0.0, epsrel=1e-13, limit=500)
    return 2.5 * om * hubble_E(a, om) * val


def growth_D1(a: float, om: float) -> float:
    """Linear growth factor, normalised to 1 at a = 1."""
    return _heath_unnormalised(a, om) / _heath_unnormalised(1.0, om)


def omega_matter(a: float, om: float) -> float:
    """Matter density parameter at scale factor a (Sec. 2.1, read as a ratio)."""
    return om / (om + (1.0 - om) * a ** 3)


def growth_D2(a: float, om: float) -> float:
    """Second-order growth factor, Sec. 2.1: -(3/7) D1^2 Omega(a)^(-1/143)."""
    d1 = growth_D1(a, om)
    return -3.0 / 7.0 * d1 * d1 * omega_matter(a, om) ** (-1.0 / 143.0)


def growth_D1_prime(a: float, om: float) -> float:
    """dD1/da of the Heath form D1 = c E(a) int_0^a da' / (a' E)^3.

    Product rule: dD1/da = D1 (dE/da)/E + c / (a E)^3 * E, with
    dE/da = -3 Om / (2 a^4 E) and c = 2.5 Om / (unnormalised D1 at a = 1).
    """
    e = hubble_E(a, om)
    de = -1.5 * om / (a ** 4 * e)
    c = 2.5 * om / _heath_unnormalised(1.0, om)
    return growth_D1(a, om) * de / e + c / (a * e) ** 3 * e


def growth_D2_prime(a: float, om: float) -> float:
    """dD2/da of D2 = -(3/7) D1^2 Omega(a)^(-1/143) (Sec. 2.1):
    D2 [2 D1'/D1 - (1/143) dln Omega/da], dln Omega/da = -3 (1-Om) a^2 / (Om + (1-Om) a^3).
    """
    d1 = growth_D1(a, om)
    dlnom = -3.0 * (1.0 - om) * a * a / (om + (1.0 - om) * a ** 3)
    return growth_D2(a, om) * (2.0 * growth_D1_prime(a, om) / d1 - dlnom / 143.0)


def _growth_system(a_end: float, om: float):
    """Unnormalised (D1, D1', D2, D2') at a_end from the growth equations
    d/dt(a^2 dD1/dt) = alpha D1 and d/dt(a^2 dD2/dt) = alpha (D2 - D1^2), written in a
    (' = d/da): D'' + (3/a + E'/E) D' = 1.5 Om/(a^5 E^2) * (D1 or D2 - D1^2), started
    on the matter-dominated growing modes D1 = a, D2 = -(3/7) a^2 at a = 1e-5."""
    from scipy.integrate import solve_ivp

    def rhs(a, y):
        e = hubble_E(a, om)
        damp = 3.0 / a - 1.5 * om / (a ** 4 * e * e)
        src = 1.5 * om / (a ** 5 * e * e)
        return [y[1], -damp * y[1] + src * y[0], y[3], -damp * y[3] + src * (y[2] - y[0] * y[0])]

    a0 = 1e-5
    y0 = [a0, 1.0, -3.0 / 7.0 * a0 * a0, -6.0 / 7.0 * a0]
    sol = solve_ivp(rhs, [a0, a_end], y0, method="DOP853", rtol=1e-12, atol=1e-30)
    return sol.y[:, -1]


def growth_D2_ode(a: float, om: float) -> float:
    """Second-order growth from its differential equation (the alternative to the
    Sec. 2.1 fit), normalised with D1(1) = 1 (D2 scales as D1^2)."""
    n1 = _growth_system(1.0, om)[0]
    return _growth_system(a, om)[2] / (n1 * n1)


def growth_D2_ode_prime(a: float, om: float) -> float:
    """dD2/da of growth_D2_ode."""
    n1 = _growth_system(1.0, om)[0]
    return _growth_system(a, om)[3] / (n1 * n1)


def poisson_alpha(a: float, om: float) -> float:
    """Source factor of the comoving Poisson equation, Sec. 2.2: (3/2) Omega_m / a."""
    return 1.5 * om / a


def kick_factor(a_v: float, a_x: float, a_h: float, om: float, n: float) -> float:
    """Eq. cola-kick: v_res(a_h) = v_res(a_v) + K * F_res(x at a_x).

    K = (a_h^n - a_v^n) / (n a_x^(n-1) adot(a_x)).  For n = 0 the ansatz becomes
    v_res = A + B ln a (the limit n -> 0 of (a^n - 1)/n) and K = a_x ln(a_h/a_v) / adot(a_x).
    """
    if n == 0.0:
        return math.log(a_h / a_v) * a_x / adot(a_x, om)
    return (a_h ** n - a_v ** n) / (n * a_x ** (n - 1.0) * adot(a_x, om))


def drift_factor(a0: float, a1: float, a_h: float, om: float, n: float) -> float:
    """Eq. cola-drift: x_res(a1) = x_res(a0) + I * v_res(a_h).

    I = int_{t0}^{t1} (a/a_h)^n dt / a^2 = int_{a0}^{a1} (a/a_h)^n da / (a^3 E(a)),
    using dt = da / adot.
    """
    f = lambda a: (a / a_h) ** n / (a ** 3 * hubble_E(a, om))
    val, _ = integrate.quad(f, a0, a1, epsabs=0.0, epsrel=1e-13, limit=500)
    return val


def D2_of(a: float, om: float, d2_ode: bool = False) -> float:
    """The D2 a run uses: the Sec. 2.1 fit, or the growth-equation solution."""
    return growth_D2_ode(a, om) if d2_ode else growth_D2(a, om)


def D2_prime_of(a: float, om: float, d2_ode: bool = False) -> float:
    return growth_D2_ode_prime(a, om) if d2_ode else growth_D2_prime(a, om)


def step_coefficients(a_x: float, a_v: float, a1: float, om: float, n: float, d2_ode: bool = False) -> dict:
    """All scalars one COLA step a_x -> a1 needs (velocity currently at a_v).

    a_h = (a_x + a1)/2 is the half step (midpoint in a).
    """
    a0 = a_x
    a_h = 0.5 * (a0 + a1)
    d1_0, d1_1 = growth_D1(a0, om), growth_D1(a1, om)
    d2_0, d2_1 = D2_of(a0, om, d2_ode), D2_of(a1, om, d2_ode)
    return dict(
        a0=a0, a1=a1, a_v=a_v, a_h=a_h,
        alpha=poisson_alpha(a0, om),
        D1=d1_0, D2=d2_0, dD1=d1_1 - d1_0, dD2=d2_1 - d2_0,
        K=kick_factor(a_v, a0, a_h, om, n),
        I=drift_factor(a0, a1, a_h, om, n),
    )


def particle_mass(om: float, box: float, n_particles: float, rho_crit=2.77536627e11):
    """Particle mass in Msun/h: Omega_m rho_crit V / N (rho_crit in h^2 Msun / Mpc^3)."""
    return om * rho_crit * box ** 3 / n_particles
