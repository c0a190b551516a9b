"""COLA residual integrator, float64 (Koda et al. 2015, Sec. 2.1-2.2).

State per particle: displacement d = x - q, residual velocity v_res
(canonical velocity v = a^2 dx/dt minus that of the 2LPT trajectory), and the
2LPT fields Psi1, Psi2.  All lengths in Mpc/h, H0 = 1.

One step a0 -> a1 (positions known at a_x = a0, velocities at a_v):
  a_h   = (a0 + a1)/2                       (midpoint in a; uniform steps)
  F     = PM force at x = q + d
  F_res = F - alpha(a0) [D1 Psi1 + (D2 - D1^2) Psi2]    (all at a0)
  v_res += K(a_v, a0, a_h) F_res;   a_v <- a_h          (eq. cola-kick)
  d     += I(a0, a1, a_h) v_res + dD1 Psi1 + dD2 Psi2;  a_x <- a1
                                                        (eq. cola-drift + 2LPT)
Readings (the paper leaves them implicit):
* The residual acceleration subtracts the canonical 2LPT acceleration
  d/dt(a^2 d/dt x_2LPT) = alpha [D1 Psi1 + (D2 - D1^2) Psi2], which follows
  from the growth equations d/dt(a^2 dD1/dt) = alpha D1 and
  d/dt(a^2 dD2/dt) = alpha (D2 - D1^2) (exact for D2 = -3/7 D1^2 in EdS).
* The kick's v_{i-1/2} is the residual velocity (matching condition of the
  kick ansatz).
* Initial condition: x_res = 0 and v_res = 0 at the initial scale factor for
  both position and velocity (the Appendix A variant, which the paper reports
  as the more accurate one); the first kick starts at a_v = a_init.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import cosmology as cosmo
from . import ic
from . import pm


@dataclass
class State:
    np_side: int
    nmesh: int
    box: float
    om: float
    n_lpt: float
    q: np.ndarray      # (3, Np) lattice positions
    d: np.ndarray      # (3, Np) displacement x - q
    v: np.ndarray      # (3, Np) residual canonical velocity
    psi1: np.ndarray   # (3, Np)
    psi2: np.ndarray   # (3, Np)
    a_x: float
    a_v: float
    d2_ode: bool = False   # D2 from its growth equation instead of the Sec. 2.1 fit

    def positions(self) -> np.ndarray:
        return self.q + self.d


def init_state(noise, box, nmesh, ktab, ptab, a_init=0.02, om=0.27, n_lpt=-2.5, d2_ode=False):
    """2LPT initial state from white noise (x_res = v_res = 0 at a_init)."""
    np_side = noise.shape[0]
    psi1, psi2 = ic.initial_fields(noise, box, ktab, ptab)
    d = ic.initial_displacement(psi1, psi2, a_init, om, d2_ode)
    return State(np_side, nmesh, box, om, n_lpt, ic.lattice(np_side, box), d,
                 np.zeros_like(d), psi1, psi2, a_init, a_init, d2_ode)


def state_from_fields(psi1, psi2, box, nmesh, a_init=0.02, om=0.27, n_lpt=-2.5):
    np_side = round(psi1.shape[1] ** (1 / 3))
    d = ic.initial_displacement(psi1, psi2, a_init, om)
    return State(np_side, nmesh, box, om, n_lpt, ic.lattice(np_side, box), d,
                 np.zeros_like(d), psi1, psi2, a_init, a_init)


def residual_force(state: State, F: np.ndarray, c: dict) -> np.ndarray:
    return F - c["alpha"] * (c["D1"] * state.psi1 + (c["D2"] - c["D1"] ** 2) * state.psi2)


def step(state: State, a1: float, force=None) -> dict:
    """Advance ``state`` in place from a_x to a1; returns the step coefficients.

    ``force``: None for the PM force, else a callable (state, coeffs) -> F
    (used by tests that substitute an exactly known force law).
    """
    c = cosmo.step_coefficients(state.a_x, state.a_v, a1, state.om, state.n_lpt, state.d2_ode)
    F = pm.pm_force(state.positions(), state.nmesh, state.box, c["alpha"]) \
        if force is None else force(state, c)
    state.v += c["K"] * residual_force(state, F, c)
    state.a_v = c["a_h"]
    state.d += c["I"] * state.v + c["dD1"] * state.psi1 + c["dD2"] * state.psi2
    state.a_x = a1
    return c


def run(state: State, edges, force=None) -> State:
    """Step through the scale factors ``edges`` (edges[0] must equal a_x)."""
    assert abs(edges[0] - state.a_x) < 1e-15
    for a1 in edges[1:]:
        step(state, a1, force)
    return state
