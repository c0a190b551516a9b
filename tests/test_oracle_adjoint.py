"""Pins for the oracle's adjoint: transpose identities and finite differences."""
import numpy as np
import pytest

from oracle import adjoint, cola, cosmology as cosmo, ic, pk, pm
from paper_1507_05329_amd.inputs import bbks_table, seeded_normal, step_edges, white_noise

OM = 0.27


def test_readout_is_transpose_of_weighted_deposit():
    rng = np.random.default_rng(0)
    L, nm = 20.0, 16
    x = rng.uniform(0, L, (3, 500))
    w = rng.standard_normal(500)
    f = rng.standard_normal((nm, nm, nm))
    lhs = np.sum(pm.cic_deposit(x, nm, L, weights=w) * f)
    rhs = np.sum(w * pm.cic_readout(f, x, L))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_green_operator_is_antisymmetric():
    rng = np.random.default_rng(1)
    nm, L = 16, 30.0
    a, b = rng.standard_normal((2, nm, nm, nm))
    for d in range(3):
        Ga = pm.force_component(np.fft.rfftn(a), nm, L, 1.3, d)
        Gb = pm.force_component(np.fft.rfftn(b), nm, L, 1.3, d)
        assert abs(np.sum(Ga * b) + np.sum(a * Gb)) < 1e-12 * np.abs(Ga * b).sum()


def test_readout_gradient_finite_difference():
    rng = np.random.default_rng(2)
    L, nm = 20.0, 16
    x = rng.uniform(0, L, (3, 50))
    f = rng.standard_normal((nm, nm, nm))
    g = adjoint.readout_grad(f, x, L)
    h = 1e-6
    for e in range(3):
        xp, xm = x.copy(), x.copy()
        xp[e] += h
        xm[e] -= h
        fd = (pm.cic_readout(f, xp, L) - pm.cic_readout(f, xm, L)) / (2 * h)
        assert np.abs(fd - g[e]).max() < 1e-6 * np.abs(g[e]).max()


def small_state(a=0.3, seed=4):
    kt, pt = bbks_table()
    st = cola.init_state(white_noise(seed, 16), 37.5, 32, kt, pt)
    for a1 in step_edges()[1:]:
        if a1 > a:
            break
        cola.step(st, a1)
    return st


def _copy(st):
    return cola.State(st.np_side, st.nmesh, st.box, st.om, st.n_lpt, st.q, st.d.copy(), st.v.copy(),
                      st.psi1.copy(), st.psi2.copy(), st.a_x, st.a_v, st.d2_ode)


@pytest.mark.parametrize("which,d2_ode", [("d", False), ("v", False), ("psi1", False), ("psi2", False),
                                          ("psi2", True), ("d", True)])
def test_step_adjoint_directional_derivative(which, d2_ode):
    st = small_state()
    st.d2_ode = d2_ode          # D2 from its growth equation: the same adjoint with its coefficients
    a1 = st.a_x + 0.098
    rng = np.random.default_rng(3)
    dbar, vbar = rng.standard_normal((2,) + st.d.shape)
    dbar0, vbar0, p1b, p2b = adjoint.step_adjoint(_copy(st), a1, dbar, vbar)
    grad = {"d": dbar0, "v": vbar0, "psi1": p1b, "psi2": p2b}[which]
    u = rng.standard_normal(st.d.shape)

    def loss(eps):
        s = _copy(st)
        arr = getattr(s, which)
        arr += eps * u
        if which in ("psi1", "psi2"):
            pass
        cola.step(s, a1)
        return np.sum(dbar * s.d) + np.sum(vbar * s.v)

    ref = np.sum(grad * u)
    best = min(abs((loss(h) - loss(-h)) / (2 * h) - ref) for h in (1e-5, 1e-6, 1e-7))
    assert best < 1e-6 * abs(ref)


def test_ic_adjoint_exact_for_quadratic_map():
    kt, pt = bbks_table()
    n, L = 16, 37.5
    w = white_noise(5, n).astype(np.float64)
    rng = np.random.default_rng(6)
    p1b, p2b = rng.standard_normal((2, 3, n ** 3))
    wbar = adjoint.ic_adjoint(w, L, kt, pt, p1b, p2b)
    u = rng.standard_normal(w.shape)

    def loss(eps):
        a, b = ic.initial_fields(w + eps * u, L, kt, pt)
        return np.sum(p1b * a) + np.sum(p2b * b)

    h = 1e-2  # the map is at most quadratic: central differences are exact
    fd = (loss(h) - loss(-h)) / (2 * h)
    assert abs(fd - np.sum(wbar * u)) < 1e-9 * abs(fd)


def test_density_adjoint_finite_difference():
    rng = np.random.default_rng(7)
    L, nm = 20.0, 16
    x = rng.uniform(0, L, (3, 300))
    db = rng.standard_normal((nm, nm, nm))
    g = adjoint.density_adjoint(x, nm, L, db)
    u = rng.standard_normal(x.shape)
    loss = lambda e: np.sum(db * pm.density_contrast(x + e * u, nm, L))
    ref = np.sum(g * u)
    best = min(abs((loss(h) - loss(-h)) / (2 * h) - ref) for h in (1e-6, 1e-7, 1e-8))
    assert best < 1e-6 * abs(ref)


def test_pk_adjoint_finite_difference():
    st = small_state(a=0.6)
    x = st.positions()
    edges = pk.log_edges(st.box, 32, 8)
    cb = np.random.default_rng(8).standard_normal(8)
    g = adjoint.pk_adjoint(x, st.box, 32, edges, cb)
    u = np.random.default_rng(9).standard_normal(x.shape)

    def loss(e):
        _, p, n = pk.power_spectrum(x + e * u, st.box, 32, edges)
        return np.sum(np.where(n > 0, cb * p, 0.0))

    ref = np.sum(g * u)
    best = min(abs((loss(h) - loss(-h)) / (2 * h) - ref) for h in (1e-6, 1e-7, 1e-8))
    assert best < 1e-6 * abs(ref)


def test_full_run_gradient_against_noise_finite_difference():
    # Loss of the differentiable configuration (sum of squared residual between
    # the final CIC density and a seeded target), on the 16^3 / 32^3 copy.
    kt, pt = bbks_table()
    n, nm, L = 16, 32, 37.5
    e = step_edges()
    w = white_noise(4, n).astype(np.float64)
    target = seeded_normal(5, (nm,) * 3).astype(np.float64)

    def final_delta(noise):
        s = cola.init_state(noise, L, nm, kt, pt)
        cola.run(s, e)
        return pm.density_contrast(s.positions(), nm, L), s

    delta, st = final_delta(w)
    dbar = adjoint.density_adjoint(st.positions(), nm, L, 2.0 * (delta - target))
    wbar, _ = adjoint.run_adjoint(w, L, nm, kt, pt, e, dbar)
    u = seeded_normal(6, w.shape).astype(np.float64)
    loss = lambda eps: np.sum((final_delta(w + eps * u)[0] - target) ** 2)
    ref = np.sum(wbar * u)
    errs = [abs((loss(h) - loss(-h)) / (2 * h) - ref) / abs(ref) for h in (1e-5, 1e-6, 1e-7)]
    assert min(errs) < 1e-6, errs
