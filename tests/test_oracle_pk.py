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
