"""Gaussian initial field and 2LPT displacements, float64.

Paper passages followed (Koda et al. 2015):
* Sec. 2.1: the 2LPT growing mode x_2LPT = q + D1 Psi1(q) + D2 Psi2(q);
  D2 ~ -(3/7) D1^2 (so D2 < 0 with the sign convention below).
* Sec. 2.3: realisations differ only by their initial random modes; ICs are a
  Gaussian random field displaced by 2LPT.

Conventions (the paper leaves them to 2LPTic; the reading used here):
* Lattice q = (i, j, k) * dq, dq = L/N, no offset; k = 2 pi n / L with the
  DFT frequency layout (numpy ``fftfreq`` / ``rfftfreq``).
* delta_L(k) = DFT[w](k) sqrt(P(|k|)/dq^3), so that <|delta_L(k)|^2> = N^6 P/V;
  the k = 0 mode and every mode with some |n_i| = N/2 are zeroed.
* Psi1(k) = i k delta_L / k^2          (so div Psi1 = -delta_L)
  phi_ij  = IDFT[k_i k_j delta_L / k^2]
  S       = phi_xx phi_yy + phi_yy phi_zz + phi_zz phi_xx
            - phi_xy^2 - phi_yz^2 - phi_zx^2
  Psi2(k) = -i k S(k) / k^2            (so div Psi2 = S), S(k) with k = 0 and
            every Nyquist-index mode zeroed.
* P(k) is given as a table and interpolated linearly in (ln k, ln P); beyond
  the table ends the first/last segment is extended.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import cosmology as cosmo

_WORKERS = -1  # all host cores


def mode_indices(n: int):
    """Integer frequency indices (nx, ny, nz) broadcastable to the rfftn layout."""
    nx = np.fft.fftfreq(n, d=1.0 / n).reshape(n, 1, 1)
    ny = np.fft.fftfreq(n, d=1.0 / n).reshape(1, n, 1)
    nz = np.arange(n // 2 + 1, dtype=np.float64).reshape(1, 1, n // 2 + 1)
    return nx, ny, nz


def nyquist_mask(n: int) -> np.ndarray:
    """True where some |n_i| == n/2 (rfftn layout)."""
    nx, ny, nz = mode_indices(n)
    h = n // 2
    return (np.abs(nx) == h) | (np.abs(ny) == h) | (nz == h)


def interp_pk(k, ktab, ptab):
    """Linear interpolation of ln P in ln k; end segments extended."""
    lk = np.log(np.asarray(ktab, dtype=np.float64))
    lp = np.log(np.asarray(ptab, dtype=np.float64))
    k = np.asarray(k, dtype=np.float64)
    out = np.zeros_like(k)
    pos = k > 0
    x = np.log(k[pos])
    j = np.clip(np.searchsorted(lk, x, side="right") - 1, 0, len(lk) - 2)
    t = (x - lk[j]) / (lk[j + 1] - lk[j])
    out[pos] = np.exp(lp[j] + t * (lp[j + 1] - lp[j]))
    return out


def delta_linear_hat(noise: np.ndarray, box: float, ktab, ptab) -> np.ndarray:
    """rfftn of the linear density at a = 1 (z = 0 spectrum)."""
    n = noise.shape[0]
    dq = box / n
    nx, ny, nz = mode_indices(n)
    kf = 2.0 * np.pi / box
    kmag = kf * np.sqrt(nx ** 2 + ny ** 2 + nz ** 2)
    amp = np.sqrt(interp_pk(kmag, ktab, ptab) / dq ** 3)
    dk = sfft.rfftn(noise.astype(np.float64), workers=_WORKERS) * amp
    dk[0, 0, 0] = 0.0
    dk[nyquist_mask(n)] = 0.0
    return dk


def lpt_from_delta_hat(dk: np.ndarray, box: float):
    """2LPT displacement fields (Mpc/h) from the rfftn of the linear density.

    Returns psi1, psi2 with shape (3, n, n, n).
    """
    n = dk.shape[0]
    kf = 2.0 * np.pi / box
    nx, ny, nz = mode_indices(n)
    kvec = [kf * nx, kf * ny, kf * nz]
    k2 = kvec[0] ** 2 + kvec[1] ** 2 + kvec[2] ** 2
    k2[0, 0, 0] = 1.0
    inv_k2 = 1.0 / k2
    inv_k2[0, 0, 0] = 0.0
    shape = (n, n, n)

    psi1 = np.empty((3, n, n, n))
    for d in range(3):
        psi1[d] = sfft.irfftn(1j * kvec[d] * dk * inv_k2, s=shape, workers=_WORKERS)

    def phi(i, j):
        return sfft.irfftn(kvec[i] * kvec[j] * dk * inv_k2, s=shape, workers=_WORKERS)

    pxx, pyy, pzz = phi(0, 0), phi(1, 1), phi(2, 2)
    src = pxx * pyy + pyy * pzz + pzz * pxx
    del pxx, pyy, pzz
    for (i, j) in ((0, 1), (1, 2), (2, 0)):
        src -= phi(i, j) ** 2
    sk = sfft.rfftn(src, workers=_WORKERS)
    del src
    sk[0, 0, 0] = 0.0
    sk[nyquist_mask(n)] = 0.0

    psi2 = np.empty((3, n, n, n))
    for d in range(3):
        psi2[d] = sfft.irfftn(-1j * kvec[d] * sk * inv_k2, s=shape, workers=_WORKERS)
    return psi1, psi2


def lpt_from_delta(delta_l: np.ndarray, box: float):
    """Same as ``lpt_from_delta_hat`` but from a real-space linear density."""
    dk = sfft.rfftn(np.asarray(delta_l, dtype=np.float64), workers=_WORKERS)
    return lpt_from_delta_hat(dk, box)


def lattice(np_side: int, box: float) -> np.ndarray:
    """Lagrangian positions q, shape (3, np_side^3), particle id = (i*N + j)*N + k."""
    dq = box / np_side
    i = np.arange(np_side, dtype=np.float64) * dq
    qx, qy, qz = np.meshgrid(i, i, i, indexing="ij")
    return np.stack([qx.ravel(), qy.ravel(), qz.ravel()])


def initial_fields(noise: np.ndarray, box: float, ktab, ptab):
    """Psi1, Psi2 (each (3, N^3), Mpc/h) from white noise and a P(k) table."""
    n = noise.shape[0]
    psi1, psi2 = lpt_from_delta_hat(delta_linear_hat(noise, box, ktab, ptab), box)
    return psi1.reshape(3, n ** 3), psi2.reshape(3, n ** 3)


def initial_displacement(psi1, psi2, a_init: float, om: float, d2_ode: bool = False):
    """d = D1(a) Psi1 + D2(a) Psi2 (positions x = q + d), Sec. 2.1."""
    return cosmo.growth_D1(a_init, om) * psi1 + cosmo.D2_of(a_init, om, d2_ode) * psi2
