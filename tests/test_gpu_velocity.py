"""GPU parity of cola_velocity: particle velocities at the position time and
redshift-space displacements (Sec. 2.1, Sec. 2.2 kick ansatz, Sec. 4.4),
against the FP64 oracle on the GPU's own state (32^3 particles / 64^3 mesh),
and at the production size (256^3 / 768^3) against the same combination
formed in FP64 from the GPU's state and its force (cola_force).

All compute goes through the C ABI (paper_1507_05329_amd.sim -> libcola.so).
"""

import numpy as np
import pytest

from _progress import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import cola, cosmology as cosmo, ic, velocity  # noqa: E402
from paper_1507_05329_amd._lib import ColaError  # noqa: E402
from paper_1507_05329_amd.inputs import CONFIGS, bbks_table, step_edges, white_noise  # noqa: E402

OM, NLPT = 0.27, -2.5


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def oracle_state(st, np_side, nm, box):
    """The GPU state (float32, mesh units) as an FP64 oracle state in Mpc/h."""
    s = box / nm
    f = lambda k: st[k].cpu().numpy().astype(np.float64) * s
    return cola.State(np_side, nm, box, OM, NLPT, ic.lattice(np_side, box), f("disp"), f("vres"),
                      f("psi1"), f("psi2"), st["a_x"], st["a_v"])


def state_bytes(sim):
    st = sim.get_state()
    return b"".join(st[k].cpu().numpy().tobytes() for k in ("disp", "vres", "psi1", "psi2"))


@pytest.fixture(scope="module")
def small():
    from paper_1507_05329_amd.sim import ColaSim
    say("[gpu] velocity: ColaSim 32^3/64^3")
    s = ColaSim(32, 64, 100.0)
    yield s
    s.close()


def test_velocity_at_initial_state_is_2lpt_velocity(small):
    say("[gpu] velocity at the initial state")
    w = white_noise(11, 32)
    small.init_from_noise(torch.from_numpy(w).cuda(), *bbks_table())
    st = small.get_state()
    o = oracle_state(st, 32, 64, 100.0)
    assert o.a_v == o.a_x
    ref = velocity.full_velocity(o) * (64 / 100.0)
    for axis in range(3):
        v, sd = small.velocity(rsd_axis=axis)
        v = v.cpu().numpy()
        sd = sd.cpu().numpy()
        assert rel_l2(v, ref) < 1e-6
        disp = st["disp"].cpu().numpy()
        others = [d for d in range(3) if d != axis]
        assert sd[others].tobytes() == disp[others].tobytes()
        ref_s = velocity.rsd_displacement(o, ref * (100.0 / 64), axis)[axis] * (64 / 100.0)
        assert rel_l2(sd[axis], ref_s) < 1e-6


@pytest.mark.parametrize("nsteps", [1, 3])
def test_velocity_after_steps_matches_oracle(small, nsteps):
    say(f"[gpu] velocity after {nsteps} steps")
    w = white_noise(12, 32)
    small.init_from_noise(torch.from_numpy(w).cuda(), *bbks_table())
    e = step_edges()
    for i in range(nsteps):
        small.step(e[i], e[i + 1])
    before = state_bytes(small)
    st = small.get_state()
    o = oracle_state(st, 32, 64, 100.0)
    assert o.a_v != o.a_x
    v, sd = small.velocity(rsd_axis=2)
    assert state_bytes(small) == before                 # no state change
    s = 64 / 100.0
    v = v.cpu().numpy().astype(np.float64) / s
    sd32 = sd.cpu().numpy()
    sd = sd32.astype(np.float64) / s
    ref = velocity.full_velocity(o)
    assert rel_l2(v, ref) < 1e-5
    # the kick from a_v to a_x alone (velocity minus v_res and the 2LPT velocity)
    c = velocity.snapshot_coefficients(o)
    base = o.v + c["u1"] * o.psi1 + c["u2"] * o.psi2
    assert np.linalg.norm(ref - base) > 1e-3 * np.linalg.norm(ref)
    assert rel_l2(v - base, ref - base) < 1e-4
    ref_s = velocity.rsd_displacement(o, ref, 2)
    assert rel_l2(sd[2] - o.d[2], ref_s[2] - o.d[2]) < 1e-5
    assert sd32[:2].tobytes() == st["disp"].cpu().numpy()[:2].tobytes()


def test_velocity_rejects_bad_arguments(small):
    say("[gpu] velocity argument checks")
    with pytest.raises(ColaError):
        small.velocity(rsd_axis=3)
    with pytest.raises(ColaError):
        small.velocity(rsd_axis=-1)
    out = small.particles()
    with pytest.raises(ColaError):
        small.velocity(out=out, rsd_axis=0, sdisp=out)
    v = small.velocity()                                 # still usable after the errors
    assert bool(torch.isfinite(v).all())


def test_velocity_production_size_against_fp64_combination():
    # 256^3 / 768^3, the bench's launch configuration: after 3 steps, the velocity
    # equals v_res + K F_res + 2LPT velocity formed in FP64 from the GPU's state and
    # its own force (cola_force, parity-tested against the oracle elsewhere).
    from paper_1507_05329_amd.sim import ColaSim
    cfg = CONFIGS["production"]
    say("[gpu] velocity at 256^3/768^3")
    sim = ColaSim(cfg.np_side, cfg.nmesh, cfg.box)
    try:
        sim.init_from_noise(torch.from_numpy(white_noise(cfg.seed, cfg.np_side)).cuda(), *bbks_table())
        e = step_edges()
        for i in range(3):
            sim.step(e[i], e[i + 1])
        st = sim.get_state()
        F = sim.force().cpu().numpy().astype(np.float64)
        v, sd = sim.velocity(rsd_axis=1)
        v = v.cpu().numpy().astype(np.float64)
        sd = sd.cpu().numpy()
        a, a_v = st["a_x"], st["a_v"]
        K = cosmo.kick_factor(a_v, a, a, OM, NLPT)
        alpha, D1, D2 = cosmo.poisson_alpha(a, OM), cosmo.growth_D1(a, OM), cosmo.growth_D2(a, OM)
        adot = cosmo.adot(a, OM)
        g = lambda k: st[k].cpu().numpy().astype(np.float64)
        p1, p2 = g("psi1"), g("psi2")
        ref = (g("vres") + K * (F - alpha * (D1 * p1 + (D2 - D1 * D1) * p2))
               + a * a * adot * (cosmo.growth_D1_prime(a, OM) * p1 + cosmo.growth_D2_prime(a, OM) * p2))
        assert rel_l2(v, ref) < 1e-6
        d = st["disp"].cpu().numpy()
        assert sd[0].tobytes() == d[0].tobytes() and sd[2].tobytes() == d[2].tobytes()
        assert rel_l2(sd[1].astype(np.float64) - d[1], ref[1] / (a * adot)) < 1e-5
        # snapshot halfway through the coming step, same construction
        a1 = e[4]
        a_h = 0.5 * (a + a1)
        a_s = a + 0.3 * (a1 - a)
        ds, vs = sim.snapshot(a1, a_s)
        vh = g("vres") + cosmo.kick_factor(a_v, a, a_h, OM, NLPT) * (F - alpha * (D1 * p1 + (D2 - D1 * D1) * p2))
        d_ref = (d.astype(np.float64) + cosmo.drift_factor(a, a_s, a_h, OM, NLPT) * vh
                 + (cosmo.growth_D1(a_s, OM) - D1) * p1 + (cosmo.growth_D2(a_s, OM) - D2) * p2)
        u = a_s * a_s * cosmo.adot(a_s, OM)
        v_ref = ((a_s / a_h) ** NLPT * vh
                 + u * (cosmo.growth_D1_prime(a_s, OM) * p1 + cosmo.growth_D2_prime(a_s, OM) * p2))
        assert rel_l2(ds.cpu().numpy().astype(np.float64) - d, d_ref - d) < 1e-5
        assert rel_l2(vs.cpu().numpy(), v_ref) < 1e-6
    finally:
        sim.close()


def test_redshift_space_density_and_pk(small):
    # Redshift-space displacement after 3 steps: cola_density_of is bit-exact against
    # the FP32 replay of the deposit, cola_pk_of agrees with the oracle estimator on the
    # same positions, and neither reads or changes the particle state.
    from oracle import cic_fp32, pk
    say("[gpu] redshift-space density and P(k)")
    L, nm = 100.0, 64
    small.init_from_noise(torch.from_numpy(white_noise(13, 32)).cuda(), *bbks_table())
    e = step_edges()
    for i in range(3):
        small.step(e[i], e[i + 1])
    before = state_bytes(small)
    real = small.density().cpu().numpy()
    _, sd = small.velocity(rsd_axis=2)
    sd32 = sd.cpu().numpy()
    dens = small.density(disp=sd).cpu().numpy()
    assert dens.tobytes() == cic_fp32.density(sd32, 32, nm).tobytes()
    assert dens.tobytes() != real.tobytes()
    edges = pk.linear_edges(L, nm, dk=2 * np.pi / L)
    km, p_g, n_g = small.pk(edges, disp=sd)
    pos = ic.lattice(32, L) + sd32.astype(np.float64) * (L / nm)
    k_e, p_e, n_e = pk.power_spectrum(pos, L, nm, edges)
    assert np.array_equal(n_g, n_e)
    ok = n_e > 0
    assert np.abs(p_g[ok] / p_e[ok] - 1).max() < 1e-4
    assert state_bytes(small) == before
    assert small.density().cpu().numpy().tobytes() == real.tobytes()


def test_kaiser_boost_in_the_linear_regime(small):
    # At a = 0.02 the displacements are linear and the redshift-space density is the
    # real-space one with every mode multiplied by (1 + f mu^2) (mu along the line of
    # sight, f = dln D1/dln a).  Expected P(k): the oracle estimator applied to the GPU's
    # real-space density boosted that way; the rest is O((k Psi)^2), below 1% here.
    from oracle import pk
    say("[gpu] Kaiser boost at a = 0.02")
    L, nm = 100.0, 64
    small.init_from_noise(torch.from_numpy(white_noise(14, 32)).cuda(), *bbks_table())
    _, sd = small.velocity(rsd_axis=0)
    edges = pk.linear_edges(L, nm, dk=2 * np.pi / L)
    _, p_s, n = small.pk(edges, disp=sd)
    a = 0.02
    f = a * cosmo.growth_D1_prime(a, OM) / cosmo.growth_D1(a, OM)
    dr = np.fft.rfftn(small.density().cpu().numpy().astype(np.float64))
    kx = np.fft.fftfreq(nm)[:, None, None]
    ky = np.fft.fftfreq(nm)[None, :, None]
    kz = np.fft.rfftfreq(nm)[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    mu2 = np.divide(kx * kx, k2, out=np.zeros_like(k2), where=k2 > 0)
    boosted = np.fft.irfftn(dr * (1 + f * mu2), s=(nm,) * 3, axes=(0, 1, 2))
    _, p_k, n_k = pk.power_from_delta(boosted, L, edges)
    assert np.array_equal(n, n_k)
    sel = (n > 0) & (edges[1:] <= 0.5)              # below half the particle Nyquist frequency
    assert sel.sum() >= 6
    err = np.abs(p_s[sel] / p_k[sel] - 1)
    say("[gpu] max |P_s / P_Kaiser - 1| =", err.max())
    assert err.max() < 0.01
    _, p_r, _ = small.pk(edges)
    assert (p_s[sel] / p_r[sel]).mean() > 1.5       # the boost itself (1 + 2f/3 + f^2/5 = 1.87)


def test_snapshot_matches_oracle_and_ends_on_the_step(small):
    # After 2 steps: the snapshot halfway through the coming step against the oracle
    # on the GPU's state; at a_s = a_x the displacement is the state's, at a_s = a1 it
    # is what cola_step then produces; the state is not changed by the call.
    say("[gpu] snapshot inside a step")
    small.init_from_noise(torch.from_numpy(white_noise(15, 32)).cuda(), *bbks_table())
    e = step_edges()
    small.step(e[0], e[1])
    small.step(e[1], e[2])
    st = small.get_state()
    before = state_bytes(small)
    o = oracle_state(st, 32, 64, 100.0)
    s = 64 / 100.0
    a_s = e[2] + 0.4 * (e[3] - e[2])
    d, v, sd = small.snapshot(e[3], a_s, rsd_axis=1)
    assert state_bytes(small) == before
    d_ref, v_ref = velocity.snapshot(o, e[3], a_s)
    d = d.cpu().numpy().astype(np.float64) / s
    v = v.cpu().numpy().astype(np.float64) / s
    assert rel_l2(d - o.d, d_ref - o.d) < 1e-5
    assert rel_l2(v, v_ref) < 1e-5
    sd32 = sd.cpu().numpy()
    adot_s = cosmo.adot(a_s, OM)
    assert rel_l2(sd32[1].astype(np.float64) / s - d[1], v_ref[1] / (a_s * adot_s)) < 1e-5
    d0, _ = small.snapshot(e[3], e[2])
    assert np.array_equal(d0.cpu().numpy(), st["disp"].cpu().numpy())
    d1, _ = small.snapshot(e[3], e[3])
    small.step(e[2], e[3])
    got = small.get_state()["disp"].cpu().numpy()
    d1 = d1.cpu().numpy()
    inc = got.astype(np.float64) - st["disp"].cpu().numpy()
    assert rel_l2(d1.astype(np.float64) - st["disp"].cpu().numpy(), inc) < 1e-6
    say("[gpu]   snapshot at a1 bitwise equal to the step:", d1.tobytes() == got.tobytes())
    for bad in [(e[3], e[2] - 0.01), (e[3], e[3] + 0.01), (e[2], e[2])]:
        with pytest.raises(ColaError):
            small.snapshot(*bad)


@pytest.mark.parametrize("nsteps,axis", [(0, 0), (2, 2)])
def test_velocity_power_matches_oracle(small, nsteps, axis):
    # cola_pk_velocity against the oracle's spectra of the same particles with the
    # oracle's velocities (initial state: no kick; after 2 steps: kick to a_x).
    from oracle import pk
    say(f"[gpu] velocity spectra after {nsteps} steps, axis {axis}")
    L, nm = 100.0, 64
    small.init_from_noise(torch.from_numpy(white_noise(16, 32)).cuda(), *bbks_table())
    e = step_edges()
    for i in range(nsteps):
        small.step(e[i], e[i + 1])
    st = small.get_state()
    o = oracle_state(st, 32, nm, L)
    edges = pk.linear_edges(L, nm, dk=2 * np.pi / L)
    km, pdd, pdu, puu, n = small.pk_velocity(edges, axis=axis)
    v = velocity.full_velocity(o)
    u = v[axis] / (o.a_x * cosmo.adot(o.a_x, OM))
    k_o, dd_o, du_o, uu_o, n_o = pk.velocity_power(o.positions(), u, L, nm, edges, axis)
    assert np.array_equal(n, n_o)
    ok = n_o > 0
    assert np.abs(km[ok] / k_o[ok] - 1).max() < 1e-12
    assert np.abs(pdd[ok] / dd_o[ok] - 1).max() < 1e-4
    assert np.abs(puu[ok] / uu_o[ok] - 1).max() < 1e-4
    assert (np.abs(pdu[ok] - du_o[ok]) / np.sqrt(dd_o[ok] * uu_o[ok])).max() < 1e-4
    assert (pdu[ok][:5] < 0).all()                          # infall at large scales
    assert np.isnan(pdd[~ok]).all()
