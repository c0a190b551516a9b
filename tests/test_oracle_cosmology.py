"""Pins for the oracle's background cosmology and COLA step factors.

Each check compares against something other than the oracle's own formula:
a closed form, an independent integration in time, or a limit.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.special import hyp2f1

from oracle import cosmology as cosmo

OM = 0.27
N = -2.5


def d1_hypergeometric(a, om):
    # Flat LCDM growing mode: a 2F1(1/3, 1; 11/6; -a^3 OL/Om) (textbook closed form).
    f = lambda x: x * hyp2f1(1 / 3, 1, 11 / 6, -x ** 3 * (1 - om) / om)
    return f(a) / f(1.0)


@pytest.mark.parametrize("a", [0.02, 0.1, 0.37, 0.8, 1.0])
def test_d1_matches_hypergeometric_closed_form(a):
    assert abs(cosmo.growth_D1(a, OM) / d1_hypergeometric(a, OM) - 1) < 1e-10


@pytest.mark.parametrize("a", [0.02, 0.3, 1.0])
def test_einstein_de_sitter_limits(a):
    # Omega_m = 1: D1 = a, D2 = -3/7 a^2 (Sec. 2.1 formula with Omega(a) = 1).
    assert abs(cosmo.growth_D1(a, 1.0) - a) < 1e-12
    assert abs(cosmo.growth_D2(a, 1.0) + 3 / 7 * a * a) < 1e-12


def canonical_second_derivative(fun, a, om, h=1e-4):
    """L[f] = d/dt (a^2 df/dt) = adot d/da (a^2 adot df/da), central differences."""
    def g(x):
        return x * x * cosmo.adot(x, om) * (fun(x + h) - fun(x - h)) / (2 * h)
    return cosmo.adot(a, om) * (g(a + h) - g(a - h)) / (2 * h)


@pytest.mark.parametrize("a", [0.05, 0.3, 0.7])
def test_d1_solves_linear_growth_equation(a):
    # Growing mode of d/dt(a^2 dD/dt) = (3/2) Om / a * D (Sec. 2.2 Poisson + EOM).
    lhs = canonical_second_derivative(lambda x: cosmo.growth_D1(x, OM), a, OM)
    rhs = cosmo.poisson_alpha(a, OM) * cosmo.growth_D1(a, OM)
    assert abs(lhs / rhs - 1) < 1e-5


@pytest.mark.parametrize("a", [0.05, 0.3, 0.7])
def test_d2_second_order_equation(a):
    # The 2LPT acceleration reading: d/dt(a^2 dD2/dt) = alpha (D2 - D1^2);
    # exact in EdS, within the approximation's percent level in LCDM.
    for om, tol in ((1.0, 1e-5), (OM, 2e-2)):
        lhs = canonical_second_derivative(lambda x: cosmo.growth_D2(x, om), a, om)
        rhs = cosmo.poisson_alpha(a, om) * (cosmo.growth_D2(a, om) - cosmo.growth_D1(a, om) ** 2)
        assert abs(lhs / rhs - 1) < tol, (om, lhs, rhs)


def _integrate_in_time(a_start, a_stop, rate, om):
    """int rate(a(t)) dt from a_start to a_stop, integrating a(t) as an ODE in t."""
    def rhs(t, y):
        return [cosmo.adot(y[0], om), rate(y[0])]
    ev = lambda t, y: y[0] - a_stop
    ev.terminal = True
    sol = solve_ivp(rhs, (0.0, 100.0), [a_start, 0.0], events=ev, rtol=1e-12, atol=1e-15,
                    method="DOP853")
    return sol.y_events[0][0][1]


@pytest.mark.parametrize("a0,a1", [(0.02, 0.118), (0.412, 0.51), (0.902, 1.0)])
def test_drift_factor_is_time_integral_of_ansatz(a0, a1):
    # eq. cola-drift: I = int (a/a_h)^n dt / a^2 over [t0, t1].
    ah = 0.5 * (a0 + a1)
    ref = _integrate_in_time(a0, a1, lambda a: (a / ah) ** N / a ** 2, OM)
    assert abs(cosmo.drift_factor(a0, a1, ah, OM, N) / ref - 1) < 1e-9


@pytest.mark.parametrize("av,a0,a1", [(0.02, 0.02, 0.118), (0.363, 0.412, 0.51)])
def test_kick_factor_is_time_integral_of_ansatz(av, a0, a1):
    # eq. cola-kick: v_res = A + B a^n with dv/dt(t_i) = F  =>  dv/dt = F (a/a0)^(n-1) adot/adot0.
    ah = 0.5 * (a0 + a1)
    rate = lambda a: (a / a0) ** (N - 1) * cosmo.adot(a, OM) / cosmo.adot(a0, OM)
    ref = _integrate_in_time(av, ah, rate, OM)
    assert abs(cosmo.kick_factor(av, a0, ah, OM, N) / ref - 1) < 1e-9


def test_kick_factor_constant_force_limit():
    a0 = 0.5
    for eps in (1e-3, 1e-4):
        k = cosmo.kick_factor(a0 - eps, a0, a0 + eps, OM, N)
        assert abs(k / (2 * eps / cosmo.adot(a0, OM)) - 1) < 10 * eps


@pytest.mark.parametrize("n", [-2.5, 0.0, 1.5])
def test_drift_factor_eds_closed_form(n):
    a0, a1 = 0.2, 0.3
    ah = 0.25
    ref = ah ** (-n) * (a1 ** (n - 0.5) - a0 ** (n - 0.5)) / (n - 0.5)
    assert abs(cosmo.drift_factor(a0, a1, ah, 1.0, n) / ref - 1) < 1e-12


def test_particle_mass_matches_paper():
    with open(os.path.join(os.path.dirname(__file__), "golden", "particle_mass.json")) as f:
        g = json.load(f)
    m = cosmo.particle_mass(g["omega_m"], g["box"], g["np_side"] ** 3)
    # printed to 2 significant digits
    assert abs(m - g["mass"]) <= 0.05e9
