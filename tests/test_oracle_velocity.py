"""Pins for the oracle's velocities and redshift-space displacements
(Sec. 2.1 COLA split, Sec. 2.2 equations of motion and kick ansatz,
Sec. 4.4 redshift-space mapping)."""
import copy

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import cola, cosmology as cosmo, ic, pm, velocity
from paper_1507_05329_amd.inputs import bbks_table, step_edges, white_noise

OM = 0.27


def plane_wave_fields(n, L, amp, axis=0):
    x = np.arange(n) * L / n
    shape = [1, 1, 1]
    shape[axis] = n
    dl = np.broadcast_to((amp * np.cos(2 * np.pi * x / L)).reshape(shape), (n, n, n)).copy()
    p1, p2 = ic.lpt_from_delta(dl, L)
    return p1.reshape(3, -1), p2.reshape(3, -1)


@pytest.mark.parametrize("om", [0.27, 0.5])
@pytest.mark.parametrize("a", [0.02, 0.1, 0.5, 1.0])
def test_growth_derivatives_match_finite_differences(om, a):
    h = 1e-5 * a
    for f, fp in [(cosmo.growth_D1, cosmo.growth_D1_prime), (cosmo.growth_D2, cosmo.growth_D2_prime)]:
        fd = (f(a + h, om) - f(a - h, om)) / (2 * h)
        assert fp(a, om) == pytest.approx(fd, rel=1e-8)


@pytest.mark.parametrize("a", [0.02, 0.3, 1.0])
def test_growth_derivatives_einstein_de_sitter(a):
    # Omega_m = 1: D1 = a, D2 = -(3/7) a^2 (Omega(a) = 1), so D1' = 1, D2' = -(6/7) a.
    assert cosmo.growth_D1(a, 1.0) == pytest.approx(a, rel=1e-12)
    assert cosmo.growth_D1_prime(a, 1.0) == pytest.approx(1.0, rel=1e-12)
    assert cosmo.growth_D2_prime(a, 1.0) == pytest.approx(-6.0 / 7.0 * a, rel=1e-12)


@pytest.mark.parametrize("om", [0.27, 0.5])
def test_growth_rate_matches_growth_ode(om):
    # Linear growth ODE D'' + (3/a + E'/E) D' = (3/2) Om D / (a^5 E^2), growing mode
    # D = a deep in matter domination; f = a D'/D at late times from the ODE solution.
    E = lambda a: np.sqrt(om / a ** 3 + 1 - om)
    dE = lambda a: -1.5 * om / (a ** 4 * E(a))
    rhs = lambda a, y: [y[1], -(3 / a + dE(a) / E(a)) * y[1] + 1.5 * om / (a ** 5 * E(a) ** 2) * y[0]]
    sol = solve_ivp(rhs, [1e-4, 1.0], [1e-4, 1.0], rtol=1e-12, atol=1e-16, dense_output=True)
    for a in [0.1, 0.5, 1.0]:
        D, Dp = sol.sol(a)
        f = a * cosmo.growth_D1_prime(a, om) / cosmo.growth_D1(a, om)
        assert f == pytest.approx(a * Dp / D, rel=1e-7)
        # and the second-order rate of D2 = -(3/7) D1^2 Omega^(-1/143): 2 f - (1/143) dln Omega/dln a
        f2 = a * cosmo.growth_D2_prime(a, om) / cosmo.growth_D2(a, om)
        dlnom = -3 * (1 - om) * a ** 3 / (om + (1 - om) * a ** 3)
        assert f2 == pytest.approx(2 * a * Dp / D - dlnom / 143, rel=1e-7)


def small_state(n=8, nm=16, box=64.0):
    k, p = bbks_table()
    return cola.init_state(white_noise(5, n), box, nm, k, p)


def test_initial_velocity_is_the_2lpt_trajectory_derivative():
    # At a_v = a_x the residual is zero: v = a^2 dx_2LPT/dt, with dx/dt = adot dx/da.
    # dx/da by central differences of the oracle's own 2LPT displacement.
    st = small_state()
    a = st.a_x
    h = 1e-5 * a
    dxda = (ic.initial_displacement(st.psi1, st.psi2, a + h, OM)
            - ic.initial_displacement(st.psi1, st.psi2, a - h, OM)) / (2 * h)
    v = velocity.full_velocity(st)
    np.testing.assert_allclose(v, a * a * cosmo.adot(a, OM) * dxda, rtol=1e-7, atol=1e-9 * np.abs(v).max())
    # Redshift-space shift (dx/dt)/H = a dx/da along the chosen axis only.
    for axis in range(3):
        ds = velocity.rsd_displacement(st, v, axis)
        np.testing.assert_allclose(ds[axis] - st.d[axis], a * dxda[axis], rtol=1e-7,
                                   atol=1e-9 * np.abs(dxda).max())
        others = [d for d in range(3) if d != axis]
        assert np.array_equal(ds[others], st.d[others])


def test_kaiser_factor_for_a_plane_wave_in_eds():
    # Omega_m = 1, one plane wave along the line of sight: Psi2 = 0 and f = 1, so the
    # redshift-space displacement is (1 + f) D1 Psi1 = 2 d; across the line of sight it is d.
    p1, p2 = plane_wave_fields(8, 100.0, 0.3, axis=2)
    assert np.abs(p2).max() < 1e-12 * np.abs(p1).max()
    st = cola.state_from_fields(p1, p2, 100.0, 8, om=1.0)
    v = velocity.full_velocity(st)
    ds = velocity.rsd_displacement(st, v, 2)
    np.testing.assert_allclose(ds[2], 2.0 * st.d[2], rtol=1e-12, atol=1e-15)
    ds0 = velocity.rsd_displacement(st, v, 0)
    np.testing.assert_allclose(ds0, st.d, rtol=0, atol=1e-15)


def test_velocity_exact_for_1d_dynamics_after_steps():
    # Before shell crossing the exact 1D force is alpha * (x - q); the trajectory is
    # x = q + D1(a) Psi1, so v = a^2 adot D1'(a) Psi1 at every step (a_v != a_x there).
    p1, p2 = plane_wave_fields(4, 100.0, 0.3)
    st = cola.state_from_fields(p1, p2, 100.0, 4)
    force = lambda s, c: c["alpha"] * s.d
    e = step_edges()
    for i in range(1, 5):
        cola.step(st, e[i], force)
        a = st.a_x
        assert st.a_v != a
        v = velocity.full_velocity(st, force)
        want = a * a * cosmo.adot(a, OM) * cosmo.growth_D1_prime(a, OM) * p1
        np.testing.assert_allclose(v, want, rtol=1e-10, atol=1e-12 * np.abs(want).max())


def test_position_time_velocity_continues_the_kick():
    # The kick ansatz is linear in a^n at a fixed force time: carrying v_res from a_v to
    # a_x and then stepping from (a_v = a_x) must give the same state as stepping directly.
    st = small_state()
    e = step_edges()
    cola.step(st, e[1])
    cola.step(st, e[2])
    alt = copy.deepcopy(st)
    alt.v = velocity.residual_velocity_at_position_time(st)
    alt.a_v = alt.a_x
    assert np.abs(alt.v - st.v).max() > 1e-3 * np.abs(st.v).max()   # the half kick is not negligible
    cola.step(st, e[3])
    cola.step(alt, e[3])
    np.testing.assert_allclose(alt.v, st.v, rtol=1e-10, atol=1e-12 * np.abs(st.v).max())
    np.testing.assert_allclose(alt.d, st.d, rtol=1e-10, atol=1e-12 * np.abs(st.d).max())


def test_snapshot_ends_on_the_step_and_starts_on_the_state():
    st = small_state()
    e = step_edges()
    cola.step(st, e[1])
    d0 = st.d.copy()
    d_a, _ = velocity.snapshot(st, e[2], st.a_x)
    np.testing.assert_allclose(d_a, d0, rtol=0, atol=1e-15 * np.abs(d0).max())
    d_b, _ = velocity.snapshot(st, e[2], e[2])
    cola.step(st, e[2])
    np.testing.assert_allclose(d_b, st.d, rtol=1e-13, atol=1e-13 * np.abs(st.d).max())


def test_snapshot_velocity_is_the_derivative_of_its_position():
    # dx/dt = v / a^2, so dx/da = v / (a^2 adot): central differences of the
    # snapshot position in a_s against its velocity, inside the drift step.
    st = small_state()
    e = step_edges()
    cola.step(st, e[1])
    cola.step(st, e[2])
    a1 = e[3]
    F = {}
    def frozen(s, c):                       # one force evaluation for all snapshots
        if "F" not in F:
            from oracle import pm
            F["F"] = pm.pm_force(s.positions(), s.nmesh, s.box, c["alpha"])
        return F["F"]
    for a_s in [st.a_x + 0.25 * (a1 - st.a_x), st.a_x + 0.7 * (a1 - st.a_x)]:
        h = 1e-5 * a_s
        dp, _ = velocity.snapshot(st, a1, a_s + h, frozen)
        dm, _ = velocity.snapshot(st, a1, a_s - h, frozen)
        _, v = velocity.snapshot(st, a1, a_s, frozen)
        want = v / (a_s * a_s * cosmo.adot(a_s, OM))
        np.testing.assert_allclose((dp - dm) / (2 * h), want, rtol=1e-6, atol=1e-8 * np.abs(want).max())


def test_snapshot_exact_for_1d_dynamics():
    # Exact 1D force: x = q + D1(a) Psi1 and v = a^2 adot D1'(a) Psi1 at any a.
    p1, p2 = plane_wave_fields(4, 100.0, 0.3)
    st = cola.state_from_fields(p1, p2, 100.0, 4)
    force = lambda s, c: c["alpha"] * s.d
    e = step_edges()
    cola.step(st, e[1], force)
    cola.step(st, e[2], force)
    for a_s in [e[2], 0.5 * (e[2] + e[3]), e[3] - 0.01]:
        d, v = velocity.snapshot(st, e[3], a_s, force)
        np.testing.assert_allclose(d, cosmo.growth_D1(a_s, OM) * p1, rtol=1e-10,
                                   atol=1e-12 * np.abs(p1).max())
        want = a_s * a_s * cosmo.adot(a_s, OM) * cosmo.growth_D1_prime(a_s, OM) * p1
        np.testing.assert_allclose(v, want, rtol=1e-10, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("a", [0.02, 0.3, 1.0])
def test_d2_ode_einstein_de_sitter(a):
    # Omega_m = 1: the growing second-order solution is exactly -(3/7) a^2.
    assert cosmo.growth_D2_ode(a, 1.0) == pytest.approx(-3.0 / 7.0 * a * a, rel=1e-9)
    assert cosmo.growth_D2_ode_prime(a, 1.0) == pytest.approx(-6.0 / 7.0 * a, rel=1e-9)


@pytest.mark.parametrize("a", [0.1, 0.5, 1.0])
def test_d2_ode_satisfies_its_growth_equation(a):
    # a E d/da(a^3 E dD2/da) = (3/2) Om / a (D2 - D1^2), checked by central differences
    # of a^3 E D2' (the oracle's own D2 and D2'), and D2' against differences of D2.
    om = OM
    E = lambda x: cosmo.hubble_E(x, om)
    g = lambda x: x ** 3 * E(x) * cosmo.growth_D2_ode_prime(x, om)
    h = 1e-4 * a
    lhs = a * E(a) * (g(a + h) - g(a - h)) / (2 * h)
    rhs = 1.5 * om / a * (cosmo.growth_D2_ode(a, om) - cosmo.growth_D1(a, om) ** 2)
    assert lhs == pytest.approx(rhs, rel=1e-6)
    d = (cosmo.growth_D2_ode(a + h, om) - cosmo.growth_D2_ode(a - h, om)) / (2 * h)
    assert cosmo.growth_D2_ode_prime(a, om) == pytest.approx(d, rel=1e-7)


def test_paper_d2_fit_close_to_the_growth_equation():
    # With Omega(a) read as the matter fraction, the fit of Sec. 2.1 is within 0.05%
    # of the growth-equation solution up to a = 1; without the Omega^(-1/143) factor
    # it would be off by about 0.9% at a = 1.
    for a in [0.02, 0.1, 0.5, 1.0]:
        assert cosmo.growth_D2(a, OM) == pytest.approx(cosmo.growth_D2_ode(a, OM), rel=5e-4)
    plain = -3.0 / 7.0 * cosmo.growth_D1(1.0, OM) ** 2
    assert abs(plain / cosmo.growth_D2_ode(1.0, OM) - 1) > 5e-3


def test_kick_factor_continuous_at_n_lpt_zero():
    # n = 0 is the limit of the ansatz: K(n) -> K(0) linearly in n.
    a_v, a_x, a_h = 0.3, 0.35, 0.4
    k0 = cosmo.kick_factor(a_v, a_x, a_h, OM, 0.0)
    for n in (1e-3, -1e-3):
        assert cosmo.kick_factor(a_v, a_x, a_h, OM, n) == pytest.approx(k0, rel=2e-3)
    kp = cosmo.kick_factor(a_v, a_x, a_h, OM, 1e-4)
    km = cosmo.kick_factor(a_v, a_x, a_h, OM, -1e-4)
    assert 0.5 * (kp + km) == pytest.approx(k0, rel=1e-8)


def test_n_lpt_zero_kick_follows_the_ln_a_ansatz():
    # v_res = A + B ln a with dv/dt = F at a_x: B adot(a_x)/a_x = F, so the kick over
    # [a_v, a_h] is F a_x ln(a_h/a_v)/adot(a_x); check dv/dt at a_x by central differences.
    a_v, a_x, a_h = 0.3, 0.35, 0.4
    F = 1.7
    v = lambda a: cosmo.kick_factor(a_v, a_x, a, OM, 0.0) * F
    h = 1e-6
    dvda = (v(a_x + h) - v(a_x - h)) / (2 * h)
    assert dvda * cosmo.adot(a_x, OM) == pytest.approx(F, rel=1e-8)


@pytest.mark.parametrize("axis", [0, 2])
def test_velocity_power_linear_theory(axis):
    # At a = 0.02 the 2LPT state is linear: u(k) = i f (k_axis / k^2) delta(k) for the
    # shift u = v_axis / (a adot), so per mode sign(k_axis) Im(delta u*) = -f |k_axis| / k^2
    # |delta|^2 and |u|^2 = f^2 k_axis^2 / k^4 |delta|^2.  Expected spectra: those mode
    # weights applied to the same realisation's |delta|^2.  Bins below 0.4 of the
    # particle-lattice Nyquist frequency; what remains (about 1% pooled, up to 5% in
    # a bin of few modes) is the lattice's aliasing through the CIC window, which the
    # linear relation does not hold.
    from oracle import pk
    st = small_state(n=32, nm=64, box=100.0)
    v = velocity.full_velocity(st)
    a = st.a_x
    f = a * cosmo.growth_D1_prime(a, OM) / cosmo.growth_D1(a, OM)
    u = v[axis] / (a * cosmo.adot(a, OM))
    edges = pk.linear_edges(100.0, 64, dk=2 * np.pi / 100.0)
    k, p_dd, p_du, p_uu, cnt = pk.velocity_power(st.positions(), u, 100.0, 64, edges, axis)
    ng, box = 64, 100.0
    d = np.fft.rfftn(pm.density_contrast(st.positions(), ng, box)) * (box ** 3 / ng ** 3) / pk.cic_window(ng)
    P = (np.abs(d) ** 2) / box ** 3
    n = [np.fft.fftfreq(ng, d=1.0 / ng).reshape(ng, 1, 1), np.fft.fftfreq(ng, d=1.0 / ng).reshape(1, ng, 1),
         np.arange(ng // 2 + 1, dtype=np.float64).reshape(1, 1, ng // 2 + 1)][axis]
    kk = pk.mode_kmag(ng, box)
    ka = (2 * np.pi / box) * np.abs(n)
    with np.errstate(invalid="ignore", divide="ignore"):
        _, e_du, _ = pk.bin_modes(np.where(kk > 0, -f * ka / kk ** 2 * P, 0.0), ng, box, edges)
        _, e_uu, _ = pk.bin_modes(np.where(kk > 0, f * f * ka ** 2 / kk ** 4 * P, 0.0), ng, box, edges)
    sel = (cnt > 0) & (edges[1:] <= 0.4)
    assert sel.sum() >= 4
    pooled = lambda x: float(np.sum(x[sel] * cnt[sel]))
    assert pooled(p_du) == pytest.approx(pooled(e_du), rel=2e-2)
    assert pooled(p_uu) == pytest.approx(pooled(e_uu), rel=2e-2)
    np.testing.assert_allclose(p_du[sel], e_du[sel], rtol=6e-2)
    np.testing.assert_allclose(p_uu[sel], e_uu[sel], rtol=6e-2)
    assert (p_du[sel] < 0).all()
