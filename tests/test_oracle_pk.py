"""Pins for the oracle's power-spectrum estimator (Sec. 3.3)."""
import numpy as np
from scipy.integrate import quad

from oracle import pk


def test_single_mode_amplitude():
    # delta = A cos(k0.x): one half-space mode carries V A^2 / 4 (no window).
    L, ng, A = 50.0, 16, 0.3
    x = np.arange(ng) * L / ng
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    n0 = np.array([2, -3, 1])
    delta = A * np.cos(2 * np.pi / L * (n0[0] * X + n0[1] * Y + n0[2] * Z))
    k0 = 2 * np.pi / L * np.linalg.norm(n0)
    edges = np.array([k0 * 0.999, k0 * 1.001])
    kmean, p, cnt = pk.power_from_delta(delta, L, edges, deconvolve=False)
    # every mode in the shell |n|^2 = 14 is counted; only +-n0 carries power
    assert abs(kmean[0] - k0) < 1e-12
    assert abs(p[0] * cnt[0] - L ** 3 * A ** 2 / 4) < 1e-9 * L ** 3 * A ** 2


def test_halfspace_counts_each_conjugate_pair_once():
    # Sum over the half space of 2|F|^2 equals the full-grid sum over modes with
    # no Nyquist index and k != 0 (independent of the rfft layout).
    ng = 12
    rng = np.random.default_rng(0)
    f = rng.standard_normal((ng, ng, ng))
    full = np.fft.fftn(f)
    n = np.fft.fftfreq(ng, 1.0 / ng)
    NX, NY, NZ = np.meshgrid(n, n, n, indexing="ij")
    okf = (np.abs(NX) < ng / 2) & (np.abs(NY) < ng / 2) & (np.abs(NZ) < ng / 2) \
        & ~((NX == 0) & (NY == 0) & (NZ == 0))
    half = np.fft.rfftn(f)
    nz = np.arange(ng // 2 + 1)
    okh = pk.halfspace_mask(ng) & (np.abs(NX[:, :, :ng // 2 + 1]) < ng / 2) \
        & (np.abs(NY[:, :, :ng // 2 + 1]) < ng / 2) & (nz < ng / 2)[None, None, :]
    assert abs(2 * np.sum(np.abs(half[okh]) ** 2) - np.sum(np.abs(full[okf]) ** 2)) \
        < 1e-10 * np.sum(np.abs(full) ** 2)


def test_cic_window_is_transform_of_assignment_kernel():
    # W(k) per axis: Fourier transform of the CIC (triangle) kernel = sinc^2.
    ng = 16
    w = pk.cic_window(ng)
    for n in (1, 3, 7):
        k = 2 * np.pi * n / ng          # radians per cell
        ft, _ = quad(lambda x: (1 - abs(x)) * np.cos(k * x), -1, 1, epsabs=1e-14)
        assert abs(w[n, 0, 0] - ft) < 1e-12 and abs(w[0, 0, n] - ft) < 1e-12


def test_grid_averaged_constant_model():
    km, p, cnt = pk.grid_averaged_model(lambda k: 0 * k + 5.0, 16, 100.0, pk.log_edges(100.0, 16, 6))
    assert np.allclose(p[cnt > 0], 5.0)
    assert cnt.sum() > 0


# --- Jing (2005) smoothing + aliasing correction --------------------------

def test_alias_sum_at_zero_slope_is_the_closed_form_image_sum():
    # sum_m sinc^4(x + pi m) = 1 - (2/3) sin^2 x per axis (from the partial
    # fractions of csc^2), so at s = 0 the 3D sum is the product over axes.
    ng = 16
    nx, ny, nz = pk._signed_modes(ng)
    closed = 1.0
    for n in (nx, ny, nz):
        closed = closed * (1.0 - (2.0 / 3.0) * np.sin(np.pi * n / ng) ** 2)
    many = pk.alias_window_sum(ng, 0.0, images=40)
    assert np.abs(many / closed - 1).max() < 1e-6
    # the default truncation stays within its stated bound (0.13% per axis at
    # the Nyquist frequency) on the modes the estimator bins, |n| <= Ng/2
    few = pk.alias_window_sum(ng, 0.0)
    inside = (nx * nx + ny * ny + nz * nz <= (ng // 2) ** 2) & np.ones(few.shape, bool)
    assert np.abs(few / closed - 1)[inside].max() < 2e-3


def test_alias_sum_along_an_axis_with_slope_minus_two():
    # A mode on the x axis (n_y = n_z = 0) has images only along x; with
    # s = -2 the sum is x^2 sin^4 x sum_m (x + pi m)^-6 = x^2 (cot^2 x + (2/15) sin^2 x),
    # x = pi n / Ng (the fourth derivative of csc^2 = sum (x + pi m)^-2).
    ng = 24
    c = pk.alias_window_sum(ng, -2.0, images=30)
    for n in range(1, ng // 2 + 1):
        x = np.pi * n / ng
        want = x * x * (1.0 / np.tan(x) ** 2 + (2.0 / 15.0) * np.sin(x) ** 2)
        assert abs(c[n, 0, 0] / want - 1) < 1e-9
        assert abs(c[0, 0, n] / want - 1) < 1e-9


def test_jing_corrected_poisson_field_is_flat_shot_noise():
    # Unclustered particles: P(k) = V / N at every k, and the grid spectrum
    # carries the aliased window sum_m |W(k + 2 k_N m)|^2.  The corrected
    # estimate is flat; the plain W^2 deconvolution over-corrects near k_N.
    rng = np.random.default_rng(11)
    L, ng, npart = 100.0, 32, 1 << 19
    pos = rng.uniform(0.0, L, (3, npart))
    edges = pk.log_edges(L, ng, 10)
    km, pj, cnt = pk.power_spectrum_jing(pos, L, ng, edges)
    _, pw, _ = pk.power_spectrum(pos, L, ng, edges)
    shot = L ** 3 / npart
    ok = cnt > 20
    dev_j = np.abs(pj[ok] / shot - 1)
    assert np.all(dev_j < 4.0 / np.sqrt(cnt[ok]) + 0.01)
    assert pw[ok][-1] / shot > 1.15
    assert dev_j[-1] < 0.03


def test_jing_iteration_reaches_its_fixed_point():
    # The returned spectrum divides the raw bin power by the bin-averaged
    # image sum at the slopes of that same spectrum (to the iteration's tolerance).
    # a Gaussian field with P ~ k^-1.5 on the grid (smooth, as the local
    # power law assumes)
    rng = np.random.default_rng(3)
    L, ng = 100.0, 32
    w = np.fft.rfftn(rng.standard_normal((ng, ng, ng)))
    k = pk.mode_kmag(ng, L)
    k[0, 0, 0] = 1.0
    delta = np.fft.irfftn(w * k ** -0.75, s=(ng,) * 3)
    edges = pk.log_edges(L, ng, 8)
    km, p, cnt = pk.power_from_delta_jing(delta, L, edges)
    s = np.clip(pk.local_slopes(km, p, cnt), pk.JING_SLOPE_MIN, pk.JING_SLOPE_MAX)
    bins = pk.mode_bins(ng, L, edges)
    _, cbar, _ = pk.bin_modes(pk.alias_window_sum(ng, np.where(bins >= 0, s[np.maximum(bins, 0)], 0.0)),
                              ng, L, edges)
    _, raw, _ = pk.power_from_delta(delta, L, edges, deconvolve=False)
    ok = cnt > 0
    assert np.abs(p[ok] * cbar[ok] / raw[ok] - 1).max() < 1e-6
