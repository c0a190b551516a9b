"""Pins for the oracle's COLA integrator (Sec. 2.1-2.2)."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import cola, cosmology as cosmo, ic, pk, pm
from paper_1507_05329_amd.inputs import bbks_table, fixed_amplitude_noise, step_edges, white_noise

OM = 0.27


def plane_wave_fields(n, L, amp):
    x = np.arange(n) * L / n
    dl = np.broadcast_to((amp * np.cos(2 * np.pi * x / L)).reshape(n, 1, 1), (n, n, n)).copy()
    p1, p2 = ic.lpt_from_delta(dl, L)
    return p1.reshape(3, -1), p2.reshape(3, -1)


def exact_1d_force(state, c):
    # Before shell crossing the 1D force on the sheet from Lagrangian q is
    # alpha * (x - q) exactly (mass between q and x).
    return c["alpha"] * state.d


def test_2lpt_frame_exact_for_1d_dynamics():
    # With the exact 1D force the COLA residual stays zero: d = D1(a) Psi1.
    p1, p2 = plane_wave_fields(4, 100.0, 0.3)
    st = cola.state_from_fields(p1, p2, 100.0, 4)
    cola.run(st, step_edges(), exact_1d_force)
    assert np.abs(st.d - cosmo.growth_D1(1.0, OM) * p1).max() < 1e-12 * np.abs(p1).max()
    assert np.abs(st.v).max() < 1e-12


def test_residual_mode_converges_second_order():
    # A residual velocity at a_init: compare with the ODE d/dt(a^2 dd/dt) = alpha d.
    L, a0 = 100.0, 0.02
    p1, p2 = plane_wave_fields(4, L, 0.3)
    h = 1e-6
    dD = (cosmo.growth_D1(a0 + h, OM) - cosmo.growth_D1(a0 - h, OM)) / (2 * h)
    rhs = lambda a, y: [y[1] / (a * a * cosmo.adot(a, OM)), cosmo.poisson_alpha(a, OM) * y[0] / cosmo.adot(a, OM)]
    sol = solve_ivp(rhs, (a0, 1.0), [cosmo.growth_D1(a0, OM), a0 ** 2 * cosmo.adot(a0, OM) * dD + 0.5],
                    rtol=1e-12, atol=1e-14, method="DOP853")
    exact = sol.y[0, -1]
    m = np.abs(p1[0]) > 1e-9
    errs = []
    for nstep in (20, 40, 80):
        st = cola.state_from_fields(p1.copy(), p2.copy(), L, 4)
        st.v = 0.5 * p1
        cola.run(st, step_edges(nstep=nstep), exact_1d_force)
        errs.append(np.abs(st.d[0][m] / p1[0][m] - exact).max())
    assert errs[1] / errs[2] > 3.3 and errs[0] / errs[1] > 2.8
    assert errs[2] / exact < 0.15


def test_plane_wave_pm_run_tracks_zeldovich():
    # Full PM: the residual comes from the mesh force error only, shrinking with resolution.
    errs = []
    for n in (32, 64):
        p1, p2 = plane_wave_fields(n, 100.0, 0.5 / cosmo.growth_D1(1.0, OM))
        st = cola.state_from_fields(p1, p2, 100.0, n)
        cola.run(st, step_edges())
        ref = cosmo.growth_D1(1.0, OM) * p1
        errs.append(np.linalg.norm(st.d - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.03 and errs[1] < 0.6 * errs[0], errs


def test_second_order_term_reduces_residual_force():
    # F_res with the 2LPT term must be smaller than with the first order alone,
    # and larger if the second-order term had the wrong sign.
    L, n = 1000.0, 64
    rng = np.random.default_rng(3)
    wk = np.fft.rfftn(rng.standard_normal((n, n, n)))
    nx, ny, nz = ic.mode_indices(n)
    wk[(nx ** 2 + ny ** 2 + nz ** 2) > 36] = 0
    dl = np.fft.irfftn(wk, s=(n,) * 3)
    dl *= 0.2 / dl.std()
    p1, p2 = ic.lpt_from_delta(dl, L)
    p1, p2 = p1.reshape(3, -1), p2.reshape(3, -1)
    D2 = cosmo.growth_D2(1.0, OM)
    al = cosmo.poisson_alpha(1.0, OM)
    F = pm.pm_force(ic.lattice(n, L) + p1 + D2 * p2, n, L, al)
    r1 = np.linalg.norm(F - al * p1)
    r2 = np.linalg.norm(F - al * (p1 + (D2 - 1) * p2))
    r2_flip = np.linalg.norm(F - al * (p1 - (D2 - 1) * p2))
    assert r2 < 0.6 * r1 and r2_flip > 1.5 * r1


def test_momentum_and_centre_of_mass_conserved():
    kt, pt = bbks_table()
    st = cola.init_state(white_noise(1, 16), 50.0, 32, kt, pt)
    d0 = st.d.sum(axis=1).copy()
    cola.run(st, step_edges())
    scale = np.abs(st.v).sum()
    assert np.abs(st.v.sum(axis=1)).max() < 1e-11 * scale
    assert np.abs(st.d.sum(axis=1) - d0).max() < 1e-9 * np.abs(st.d).sum()


def test_early_power_spectrum_is_linear():
    # P(k, a_init) = D1(a_init)^2 <P_lin>_grid (grid-averaged model, Sec. 3.3).
    kt, pt = bbks_table()
    np_side, nm, L = 32, 64, 100.0
    st = cola.init_state(fixed_amplitude_noise(7, np_side), L, nm, kt, pt)
    edges = pk.linear_edges(L, nm, dk=2 * np.pi / L)
    km, P, cnt = pk.power_spectrum(st.positions(), L, nm, edges)
    _, Pm, _ = pk.grid_averaged_model(lambda k: ic.interp_pk(k, kt, pt), nm, L, edges)
    D = cosmo.growth_D1(0.02, OM)
    sel = (cnt > 0) & (km <= np.pi * np_side / L / 4)
    assert sel.sum() >= 3
    assert np.abs(P[sel] / (D * D * Pm[sel]) - 1).max() < 0.02


def test_large_scale_growth_follows_d1():
    # Linear scales grow as D1^2 (the paper: growth accurate to much better
    # than 1 per cent); 3x mesh as in the paper, fundamental mode.
    kt, pt = bbks_table()
    np_side, nm, L = 64, 192, 4000.0
    st = cola.init_state(fixed_amplitude_noise(11, np_side), L, nm, kt, pt)
    edges = pk.linear_edges(L, nm, dk=2 * np.pi / L)
    _, P0, _ = pk.power_spectrum(st.positions(), L, nm, edges)
    cola.run(st, step_edges())
    _, P1, cnt = pk.power_spectrum(st.positions(), L, nm, edges)
    G = (cosmo.growth_D1(1.0, OM) / cosmo.growth_D1(0.02, OM)) ** 2
    assert abs(P1[1] / P0[1] / G - 1) < 0.01
