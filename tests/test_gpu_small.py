"""GPU parity against the oracle at small sizes (32^3 particles / 64^3 mesh).

All compute goes through the C ABI (paper_1507_05329_amd.sim -> libcola.so).
"""

import numpy as np
import pytest

from _progress import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import cic_fp32, cola, cosmology as cosmo, ic, philox, pk, pm  # noqa: E402
from paper_1507_05329_amd import _lib  # noqa: E402
from paper_1507_05329_amd.inputs import CONFIGS, bbks_table, white_noise, step_edges  # noqa: E402

NP, NM, L = 32, 64, 100.0
OM = 0.27


@pytest.fixture(scope="module")
def sim():
    from paper_1507_05329_amd.sim import ColaSim
    say(f"[gpu] create ColaSim np={NP} nm={NM}")
    s = ColaSim(NP, NM, L)
    yield s
    s.close()


@pytest.fixture(scope="module")
def table():
    return bbks_table()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel_l2(a, b):
    a = np.asarray(a)
    a = a.astype(np.complex128) if np.iscomplexobj(a) else a.astype(np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def lattice_mesh_units():
    return ic.lattice(NP, L) * (NM / L)


def set_disp(sim, disp, a_x=0.5, vres=None):
    z = np.zeros((3, NP ** 3), np.float32)
    sim.set_state(to_dev(disp), to_dev(z if vres is None else vres), to_dev(z), to_dev(z), a_x, a_x)


def oracle_positions(disp32):
    """Mpc/h positions of a float32 mesh-unit displacement field."""
    return ic.lattice(NP, L) + disp32.astype(np.float64) * (L / NM)


# --------------------------------------------------------------------------
def padded(field, n):
    from paper_1507_05329_amd.sim import padded_cols
    m = np.zeros((n, n, 2 * padded_cols(n)), np.float32)
    m[:, :, :n] = field
    return m


@pytest.mark.parametrize("n", [NP, NM])
def test_fft3d_forward_and_roundtrip(sim, n):
    say(f"[gpu] fft3d n={n}")
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n, n)).astype(np.float32)
    t = to_dev(padded(x, n))
    sim.fft3d(t, n)
    got = t.cpu().numpy().view(np.complex64)[:, :, : n // 2 + 1]
    ref = np.fft.rfftn(x.astype(np.float64))
    assert rel_l2(got, ref) < 2e-6
    sim.fft3d(t, n, inverse=True)
    back = t.cpu().numpy()[:, :, :n] / n ** 3
    assert rel_l2(back, x) < 2e-6


def random_disp(seed, scale):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((3, NP ** 3)) * scale).astype(np.float32)


def test_density_bit_exact_against_fp32_replay(sim):
    say("[gpu] density bit-exact")
    disp = random_disp(0, 2.0)
    set_disp(sim, disp)
    got = sim.density().cpu().numpy()
    ref = cic_fp32.density(disp, NP, NM)
    assert got.tobytes() == ref.tobytes()
    again = sim.density().cpu().numpy()
    assert again.tobytes() == got.tobytes()


def test_density_bit_exact_clustered_overflow_paths(sim):
    # 3000 particles in one cell (ordered-selection path) and 3000 more spread
    # over the same tile (cell-range splitting), the rest random.
    say("[gpu] density clustered")
    rng = np.random.default_rng(1)
    base = lattice_mesh_units() - 0.5                    # node coordinate of the lattice point
    target = np.empty((3, NP ** 3))
    target[:] = base + rng.standard_normal((3, NP ** 3)) * 1.5
    target[:, :3000] = 20.0 + rng.uniform(0, 1, (3, 3000))
    target[:, 3000:6000] = 16.0 + rng.uniform(0, 8.0, (3, 3000))
    disp = (target - base).astype(np.float32)
    set_disp(sim, disp)
    got = sim.density().cpu().numpy()
    ref = cic_fp32.density(disp, NP, NM)
    assert got.tobytes() == ref.tobytes()


@pytest.mark.parametrize("nm", [96, 128])
def test_density_bit_exact_sparse_tiles(nm):
    # 32^3 particles on a 96^3 / 128^3 mesh (about 150 / 64 particles per
    # 16^3 tile: the 512-particle LDS shape).  One cell with 1500 particles
    # (ordered selection), a tile with 1500 more and one with 600 (cell
    # ranges halved until they fit), the rest random.  The 64^3 mesh of the
    # other tests (512 per tile) takes the 1024-particle shape.
    from paper_1507_05329_amd.sim import ColaSim
    say(f"[gpu] density sparse tiles nm={nm}")
    s = ColaSim(NP, nm, L)
    try:
        rng = np.random.default_rng(3)
        base = ic.lattice(NP, L) * (nm / L) - 0.5
        target = base + rng.standard_normal((3, NP ** 3)) * 1.5
        target[:, :1500] = 30.0 + rng.uniform(0, 1, (3, 1500))
        target[:, 1500:3000] = 34.0 + rng.uniform(0, 8.0, (3, 1500))
        target[:, 3000:3600] = 50.0 + rng.uniform(0, 12.0, (3, 600))
        disp = (target - base).astype(np.float32)
        z = np.zeros((3, NP ** 3), np.float32)
        s.set_state(to_dev(disp), to_dev(z), to_dev(z), to_dev(z), 0.5, 0.5)
        got = s.density().cpu().numpy()
        ref = cic_fp32.density(disp, NP, nm)
        assert got.tobytes() == ref.tobytes()
        disp = random_disp(4, 3.0)
        s.set_state(to_dev(disp), to_dev(z), to_dev(z), to_dev(z), 0.5, 0.5)
        got = s.density().cpu().numpy()
        assert got.tobytes() == cic_fp32.density(disp, NP, nm).tobytes()
    finally:
        s.close()


def test_density_bit_exact_mesh_equal_to_particle_grid():
    """The densest allowed configuration: a 32^3 mesh for 32^3 particles
    (about 4000 particles per 16^3 tile region, far above the LDS capacity:
    every tile takes the cell-range splitting), lattice-perturbed and with a
    400-particle clump in one cell.  Bit-exact against the FP32 replay and
    the run-to-run repeat."""
    from paper_1507_05329_amd.sim import ColaSim
    say("[gpu] density, mesh = particle grid")
    s = ColaSim(NP, NP, L)
    try:
        rng = np.random.default_rng(11)
        base = ic.lattice(NP, L) * (NP / L) - 0.5
        target = base + rng.standard_normal((3, NP ** 3)) * 0.7
        target[:, :400] = 9.0 + rng.uniform(0, 1, (3, 400))
        disp = (target - base).astype(np.float32)
        z = np.zeros((3, NP ** 3), np.float32)
        s.set_state(to_dev(disp), to_dev(z), to_dev(z), to_dev(z), 0.5, 0.5)
        got = s.density().cpu().numpy()
        assert got.tobytes() == cic_fp32.density(disp, NP, NP).tobytes()
        assert s.density().cpu().numpy().tobytes() == got.tobytes()
    finally:
        s.close()


def test_density_matches_fp64_oracle(sim):
    disp = random_disp(2, 3.0)
    set_disp(sim, disp)
    got = sim.density().cpu().numpy()
    ref = pm.density_contrast(oracle_positions(disp), NM, L)
    assert np.abs(got - ref).max() < 5e-6 * np.abs(ref).max()
    assert abs(float(got.astype(np.float64).mean())) < 1e-5


def clustered_state(table, a=0.6):
    """A realistic displacement field: 2LPT at scale factor a (mesh units, float32)."""
    psi1, psi2 = ic.initial_fields(white_noise(7, NP), L, *table)
    d = ic.initial_displacement(psi1, psi2, a, OM)
    return (d * (NM / L)).astype(np.float32)


def test_force_matches_oracle(sim, table):
    say("[gpu] force parity")
    disp = clustered_state(table)
    a_x = 0.6
    set_disp(sim, disp, a_x)
    got = sim.force().cpu().numpy()
    ref = pm.pm_force(oracle_positions(disp), NM, L, cosmo.poisson_alpha(a_x, OM)) * (NM / L)
    assert rel_l2(got, ref) <= 1e-5


def test_initial_conditions_match_oracle(sim, table):
    say("[gpu] 2LPT initial conditions")
    w = white_noise(3, NP)
    sim.init_from_noise(to_dev(w), *table)
    st = sim.get_state()
    psi1, psi2 = ic.initial_fields(w, L, *table)
    s = NM / L
    assert rel_l2(st["psi1"].cpu().numpy(), psi1 * s) < 1e-5
    assert rel_l2(st["psi2"].cpu().numpy(), psi2 * s) < 1e-4
    d_ref = ic.initial_displacement(psi1, psi2, 0.02, OM) * s
    assert rel_l2(st["disp"].cpu().numpy(), d_ref) < 1e-5
    assert float(st["vres"].abs().max()) == 0.0
    assert st["a_x"] == 0.02 and st["a_v"] == 0.02


def test_one_step_matches_oracle(sim, table):
    say("[gpu] one step")
    w = white_noise(4, NP)
    sim.init_from_noise(to_dev(w), *table)
    e = step_edges()
    for a0, a1 in zip(e[:3], e[1:4]):   # reach a = 0.314 on the GPU
        sim.step(a0, a1)
    st = sim.get_state()
    s = L / NM
    o = cola.State(NP, NM, L, OM, -2.5, ic.lattice(NP, L),
                   st["disp"].cpu().numpy().astype(np.float64) * s,
                   st["vres"].cpu().numpy().astype(np.float64) * s,
                   st["psi1"].cpu().numpy().astype(np.float64) * s,
                   st["psi2"].cpu().numpy().astype(np.float64) * s, st["a_x"], st["a_v"])
    d0, v0 = o.d.copy(), o.v.copy()
    cola.step(o, e[4])
    sim.step(e[3], e[4])
    st2 = sim.get_state()
    dd = st2["disp"].cpu().numpy().astype(np.float64) * s - d0
    dv = st2["vres"].cpu().numpy().astype(np.float64) * s - v0
    assert rel_l2(dd, o.d - d0) < 1e-4
    assert rel_l2(dv, o.v - v0) < 1e-4
    assert abs(st2["a_x"] - e[4]) < 1e-15 and abs(st2["a_v"] - o.a_v) < 1e-15


def test_full_run_power_spectrum_matches_oracle(sim, table):
    say("[gpu] 10-step run vs oracle")
    cfg = CONFIGS["small"]
    w = white_noise(cfg.seed, NP)
    sim.init_from_noise(to_dev(w), *table)
    sim.run(step_edges())
    ref = cola.init_state(w, L, NM, *table)
    cola.run(ref, step_edges())
    edges = pk.linear_edges(L, NM, dk=2 * np.pi / L)
    k_o, p_o, n_o = pk.power_spectrum(ref.positions(), L, NM, edges)
    km, p_g, n_g = sim.pk(edges)
    st = sim.get_state()
    pos_g = ic.lattice(NP, L) + st["disp"].cpu().numpy().astype(np.float64) * (L / NM)
    k_e, p_e, n_e = pk.power_spectrum(pos_g, L, NM, edges)
    # estimator parity on the same particles
    assert np.array_equal(n_g, n_e)
    ok = n_e > 0
    assert np.abs(p_g[ok] / p_e[ok] - 1).max() < 1e-4
    assert np.abs(km[ok] / k_e[ok] - 1).max() < 1e-12
    # trajectory-level parity of the final P(k): k < k_Nyq / 2
    sel = ok & (k_o < np.pi * NM / L / 2)
    err = np.abs(p_g[sel] / p_o[sel] - 1)
    say("[gpu] max |P_gpu/P_oracle - 1| =", err.max())
    assert err.max() < 5e-3


@pytest.mark.parametrize("ngrid", [32, 48])
def test_pk_coarser_grid_and_empty_bins(sim, table, ngrid):
    """cola_pk on a grid coarser than the PM mesh (the deposit rescales the
    displacements; 48 is not a power of two), with bins that hold no mode
    (narrower than the mode spacing, and beyond the grid's Nyquist wave
    number): mode counts equal the FP64 estimator's on the same particles,
    empty bins report NaN mean |k| and P (the documented contract), every
    other bin finite values."""
    say(f"[gpu] P(k) on a {ngrid}^3 grid with empty bins")
    w = white_noise(7, NP)
    sim.init_from_noise(to_dev(w), *table)
    e = step_edges()
    for i in range(3):
        sim.step(e[i], e[i + 1])
    kf = 2 * np.pi / L
    kny = np.pi * ngrid / L
    edges = np.concatenate([[0.2 * kf, 0.3 * kf], np.linspace(kf, kny, 9)[1:], [1.5 * kny, 2.0 * kny]])
    edges.sort()
    km, p_g, n_g = sim.pk(edges, ngrid)
    st = sim.get_state()
    pos = ic.lattice(NP, L) + st["disp"].cpu().numpy().astype(np.float64) * (L / NM)
    k_e, p_e, n_e = pk.power_spectrum(pos, L, ngrid, edges)
    assert np.array_equal(n_g, n_e)
    empty = n_e == 0
    assert empty.sum() >= 2                 # the sub-spacing bin and those beyond k_Nyq
    assert np.all(np.isnan(p_g[empty])) and np.all(np.isnan(km[empty]))
    ok = ~empty
    assert np.all(np.isfinite(p_g[ok])) and np.all(np.isfinite(km[ok]))
    assert np.abs(p_g[ok] / p_e[ok] - 1).max() < 1e-4
    assert np.abs(km[ok] / k_e[ok] - 1).max() < 1e-12


def test_noise_matches_oracle_philox(sim):
    z = sim.noise(2024).cpu().numpy()
    ref = philox.normal_field(2024, NP)
    assert np.abs(z - ref).max() < 1e-6


def test_seeded_init_equals_noise_init(sim, table):
    sim.init_2lpt(99, *table)
    a = sim.get_state()["disp"].cpu().numpy()
    sim.init_from_noise(sim.noise(99), *table)
    b = sim.get_state()["disp"].cpu().numpy()
    assert a.tobytes() == b.tobytes()


def test_error_paths_leave_state_usable(sim, table):
    from paper_1507_05329_amd._lib import ColaError
    sim.init_2lpt(5, *table)
    before = sim.get_state()["disp"].cpu().numpy()
    with pytest.raises(ColaError) as e:
        sim.step(0.5, 0.6)          # a0 != a_x
    assert e.value.code == _lib.COLA_ESTATE
    with pytest.raises(ColaError) as e:
        sim.step(0.02, 0.01)        # backwards
    assert e.value.code == _lib.COLA_EINVAL
    with pytest.raises(ColaError) as e:
        sim.pk(np.array([0.1, 0.2]), ngrid=60)
    assert e.value.code == _lib.COLA_EUNSUPPORTED
    with pytest.raises(ColaError) as e:
        sim.init_2lpt(5, np.array([1.0, 0.5]), np.array([1.0, 1.0]))
    assert e.value.code == _lib.COLA_EINVAL
    after = sim.get_state()
    assert after["disp"].cpu().numpy().tobytes() == before.tobytes()
    sim.step(0.02, 0.118)           # still usable


def test_check_finite_flag(table):
    from paper_1507_05329_amd.sim import ColaSim
    from paper_1507_05329_amd._lib import ColaError
    s = ColaSim(NP, NM, L, flags=_lib.COLA_F_CHECK_FINITE)
    s.init_2lpt(1, *table)
    st = s.get_state()
    d = st["disp"].clone()
    d[0, 5] = float("nan")
    s.set_state(d, st["vres"], st["psi1"], st["psi2"], st["a_x"], st["a_v"])
    with pytest.raises(ColaError) as e:
        s.step(0.02, 0.118)
    assert e.value.code == _lib.COLA_ENONFINITE
    s.close()


@pytest.mark.parametrize("ngrid", [64, 32])
def test_pk_jing_matches_oracle(sim, table, ngrid):
    """cola_pk_jing (Sec. 3.3, Jing 2005 smoothing + aliasing correction)
    against the oracle's estimator on the GPU's particles after 10 steps,
    log bins up to the grid Nyquist (where the aliasing matters most)."""
    say(f"[gpu] Jing-corrected P(k) on {ngrid}^3")
    w = white_noise(9, NP)
    sim.init_from_noise(to_dev(w), *table)
    sim.run(step_edges())
    edges = pk.log_edges(L, ngrid, 12)
    km, p_g, n_g = sim.pk(edges, ngrid, jing=True)
    st = sim.get_state()
    pos = ic.lattice(NP, L) + st["disp"].cpu().numpy().astype(np.float64) * (L / NM)
    k_e, p_e, n_e = pk.power_spectrum_jing(pos, L, ngrid, edges)
    assert np.array_equal(n_g, n_e)
    ok = n_e > 0
    err = np.abs(p_g[ok] / p_e[ok] - 1).max()
    say(f"[gpu]   max rel diff {err:.2e}")
    assert err < 1e-4
    assert np.abs(km[ok] / k_e[ok] - 1).max() < 1e-12
    # the correction differs from the plain window division near the Nyquist frequency
    _, p_plain, _ = sim.pk(edges, ngrid)
    assert abs(p_plain[ok][-1] / p_g[ok][-1] - 1) > 1e-3
