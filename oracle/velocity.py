"""Particle velocities and redshift-space displacements, float64.

Test infrastructure: the slow, plainly written reference that the GPU path is
checked against; nothing in the library imports it.

Paper passages followed (Koda et al. 2015):
* Sec. 2.1: the COLA split of the velocity into a residual and the time
  derivative of the 2LPT trajectory x_2LPT = q + D1 Psi1 + D2 Psi2; with the
  canonical velocity v = a^2 dx/dt of Sec. 2.2 (equations of motion) the
  2LPT part is a^2 adot (D1' Psi1 + D2' Psi2), ' = d/da.
* Sec. 2.2, eq. cola-kick: the residual velocity between kicks follows the
  kick ansatz, and the paper uses the same equations to interpolate
  snapshots between steps.  The state holds v_res at a_v (the last half
  step) and positions at a_x; the velocity at a_x is v_res(a_v) plus the
  kick factor from a_v to a_x times F_res(x) (force at the position time).
* Sec. 2.2, eqs. ansatz-drift and cola-drift: snapshots between steps.
  Within the drift of the coming step the residual velocity decays as
  (a/a_h)^n from its value after the step's kick, and the position follows
  the drift integral of that velocity; the 2LPT part is evaluated at the
  snapshot time.
* Sec. 4.4 (mock catalogue): redshift-space position s = x + (v.xhat)/(aH)
  xhat, v there the peculiar velocity a dx/dt, so the comoving shift is
  (dx/dt . xhat)/H = v_canonical . xhat / (a adot).

Readings:
* The line of sight is a box axis (distant observer), the usual choice for
  a periodic box; the shift applies to that displacement component only.
* At a_v = a_x (the initial state) the kick factor is zero and no force is
  needed.
"""
from __future__ import annotations

import numpy as np

from . import cosmology as cosmo
from . import pm
from .cola import State


def snapshot_coefficients(state: State) -> dict:
    """Scalars of the velocity at the position time a_x."""
    a, a_v, om, n = state.a_x, state.a_v, state.om, state.n_lpt
    adot = cosmo.adot(a, om)
    return dict(
        a=a,
        adot=adot,
        alpha=cosmo.poisson_alpha(a, om),
        D1=cosmo.growth_D1(a, om),
        D2=cosmo.D2_of(a, om, state.d2_ode),
        K=cosmo.kick_factor(a_v, a, a, om, n),
        u1=a * a * adot * cosmo.growth_D1_prime(a, om),
        u2=a * a * adot * cosmo.D2_prime_of(a, om, state.d2_ode),
    )


def residual_velocity_at_position_time(state: State, force=None) -> np.ndarray:
    """v_res carried from a_v to a_x by the kick ansatz with F_res(x)."""
    c = snapshot_coefficients(state)
    if state.a_v == state.a_x:
        return state.v.copy()
    F = pm.pm_force(state.positions(), state.nmesh, state.box, c["alpha"]) \
        if force is None else force(state, c)
    F_res = F - c["alpha"] * (c["D1"] * state.psi1 + (c["D2"] - c["D1"] ** 2) * state.psi2)
    return state.v + c["K"] * F_res


def full_velocity(state: State, force=None) -> np.ndarray:
    """Canonical velocity v = a^2 dx/dt of every particle at a_x, shape (3, Np)."""
    c = snapshot_coefficients(state)
    v_res = residual_velocity_at_position_time(state, force)
    return v_res + c["u1"] * state.psi1 + c["u2"] * state.psi2


def rsd_displacement(state: State, v: np.ndarray, axis: int) -> np.ndarray:
    """Displacement of the redshift-space position along ``axis``."""
    c = snapshot_coefficients(state)
    d = state.d.copy()
    d[axis] = d[axis] + v[axis] / (c["a"] * c["adot"])
    return d


def snapshot(state: State, a1: float, a_s: float, force=None):
    """Displacement and canonical velocity at a_s in [a_x, a1] within the coming
    step a_x -> a1 (the state is not changed).

    Sec. 2.2: the step's kick (eq. cola-kick) takes v_res to the half step
    a_h = (a_x + a1)/2 with F_res(x); during the drift the residual velocity
    follows the drift ansatz v_res(a) = v_res(a_h) (a/a_h)^n, whose position
    integral is eq. cola-drift from a_x to a_s; the 2LPT part is evaluated at a_s.
    At a_s = a1 the displacement is the step's.
    """
    c = cosmo.step_coefficients(state.a_x, state.a_v, a1, state.om, state.n_lpt, state.d2_ode)
    F = pm.pm_force(state.positions(), state.nmesh, state.box, c["alpha"]) \
        if force is None else force(state, c)
    F_res = F - c["alpha"] * (c["D1"] * state.psi1 + (c["D2"] - c["D1"] ** 2) * state.psi2)
    v_half = state.v + c["K"] * F_res
    om, n, a_h = state.om, state.n_lpt, c["a_h"]
    I = cosmo.drift_factor(state.a_x, a_s, a_h, om, n)
    d = (state.d + I * v_half
         + (cosmo.growth_D1(a_s, om) - c["D1"]) * state.psi1
         + (cosmo.D2_of(a_s, om, state.d2_ode) - c["D2"]) * state.psi2)
    u = a_s * a_s * cosmo.adot(a_s, om)
    v = ((a_s / a_h) ** n * v_half
         + u * cosmo.growth_D1_prime(a_s, om) * state.psi1
         + u * cosmo.D2_prime_of(a_s, om, state.d2_ode) * state.psi2)
    return d, v
