"""Pins for the oracle's Gaussian field and 2LPT displacements (Sec. 2.1)."""
import numpy as np
import pytest

from oracle import ic
from paper_1507_05329_amd.inputs import bbks_table, white_noise

L = 100.0


def grid(n):
    x = np.arange(n) * L / n
    return np.meshgrid(x, x, x, indexing="ij")


def test_psi1_single_mode_closed_form():
    n = 16
    X, Y, Z = grid(n)
    kv = 2 * np.pi / L * np.array([1.0, 2.0, 0.0])
    A = 0.3
    phase = kv[0] * X + kv[1] * Y + kv[2] * Z
    psi1, psi2 = ic.lpt_from_delta(A * np.cos(phase), L)
    kk = np.linalg.norm(kv)
    for d in range(3):
        ref = -(A / kk) * (kv[d] / kk) * np.sin(phase)
        assert np.abs(psi1[d] - ref).max() < 1e-12
    assert np.abs(psi2).max() < 1e-12      # a single plane wave has no 2nd order


def test_psi1_divergence_is_minus_delta():
    n = 16
    rng = np.random.default_rng(0)
    dk = np.fft.rfftn(rng.standard_normal((n, n, n)))
    dk[0, 0, 0] = 0
    dk[ic.nyquist_mask(n)] = 0
    delta = np.fft.irfftn(dk, s=(n,) * 3)
    psi1, _ = ic.lpt_from_delta(delta, L)
    nx, ny, nz = ic.mode_indices(n)
    kf = 2 * np.pi / L
    div = np.fft.irfftn(sum(1j * kf * m * np.fft.rfftn(psi1[d]) for d, m in enumerate((nx, ny, nz))),
                        s=(n,) * 3)
    assert np.abs(div + delta).max() < 1e-12 * np.abs(delta).max() * 10


def test_psi2_crossed_waves_closed_form():
    # delta = laplacian(phi1), phi1 = A cos(k1 x) + B cos(k2 y) gives
    # Psi2 = grad phi2, phi2 = -A B k1^2 k2^2 / (k1^2 + k2^2) cos(k1 x) cos(k2 y).
    n = 32
    X, Y, Z = grid(n)
    k1, k2 = 2 * np.pi / L * 2, 2 * np.pi / L * 3
    A, B = 1.7, -0.9
    delta = -A * k1 ** 2 * np.cos(k1 * X) - B * k2 ** 2 * np.cos(k2 * Y)
    _, psi2 = ic.lpt_from_delta(delta, L)
    c = -A * B * k1 ** 2 * k2 ** 2 / (k1 ** 2 + k2 ** 2)
    ref = [-c * k1 * np.sin(k1 * X) * np.cos(k2 * Y), -c * k2 * np.cos(k1 * X) * np.sin(k2 * Y), 0 * X]
    scale = np.abs(ref[0]).max()
    for d in range(3):
        assert np.abs(psi2[d] - ref[d]).max() < 1e-12 * scale * 10


def test_interp_pk_exact_for_power_law():
    kt = np.geomspace(0.01, 1.0, 7)
    pt = 3.0 * kt ** -1.3
    k = np.array([0.005, 0.013, 0.5, 0.77, 2.0])
    assert np.allclose(ic.interp_pk(k, kt, pt), 3.0 * k ** -1.3, rtol=1e-12)


def test_delta_linear_power_normalisation():
    # <|delta_L(k)|^2> dq^3 / N^3 = P(k): average over seeds and a shell of modes.
    n = 16
    kt, pt = bbks_table()
    acc, cnt = 0.0, 0
    nx, ny, nz = ic.mode_indices(n)
    n2 = nx ** 2 + ny ** 2 + nz ** 2
    shell = (n2 >= 9) & (n2 < 16) & ~ic.nyquist_mask(n)
    kmag = 2 * np.pi / L * np.sqrt(np.broadcast_to(n2, shell.shape)[shell])
    pmod = ic.interp_pk(kmag, kt, pt)
    for s in range(24):
        dk = ic.delta_linear_hat(white_noise(100 + s, n), L, kt, pt)
        acc += np.sum(np.abs(dk[shell]) ** 2 * (L / n) ** 3 / n ** 3 / pmod)
        cnt += shell.sum()
    # each ratio is exponential(1) distributed (rfft half-space modes are independent)
    assert abs(acc / cnt - 1) < 4 / np.sqrt(cnt)


def test_table_sigma8():
    # Recompute sigma_8 from the table with the oracle's interpolation rule.
    from scipy.integrate import quad
    kt, pt = bbks_table(sigma8=0.8)
    def integrand(lnk):
        k = np.exp(lnk)
        x = 8.0 * k
        w = 3 * (np.sin(x) - x * np.cos(x)) / x ** 3
        return k ** 3 / (2 * np.pi ** 2) * ic.interp_pk(np.array([k]), kt, pt)[0] * w * w
    s2, _ = quad(integrand, np.log(kt[0]), np.log(kt[-1]), limit=2000, epsrel=1e-10)
    assert abs(np.sqrt(s2) / 0.8 - 1) < 1e-4
