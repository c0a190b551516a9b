"""Matter power-spectrum estimator, float64 (Koda et al. 2015, Sec. 3.3).

Steps, in the paper's order:
1. CIC-assign all particles onto an Ng^3 grid; delta = rho/rho_bar - 1.
2. FFT; keep the half space {kz > 0} U {kz = 0, ky > 0} U {kz = 0, ky = 0, kx > 0}
   (the other half carries no independent information for a real field).
3. P(k) = V^-1 <|delta(k)|^2>, with delta(k) = (V/Ng^3) DFT[delta] the
   continuum-normalised transform, averaged in bins; report the mean |k|.
4. Correct for the CIC smoothing by dividing delta(k) by
   W(k) = prod_e sinc^2(pi n_e / Ng).  (The paper also applies Jing's
   iterative aliasing correction; that is not done here.)

Readings: signed mode indices follow the DFT layout (n in [-Ng/2, Ng/2-1] on
x and y, n_z in [0, Ng/2]); only modes with |k| <= k_Nyq = pi Ng / L are
used; bin b holds edges[b] <= |k| < edges[b+1].  No shot-noise subtraction.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import pm


def halfspace_mask(ng: int) -> np.ndarray:
    nx = np.fft.fftfreq(ng, d=1.0 / ng).reshape(ng, 1, 1)
    ny = np.fft.fftfreq(ng, d=1.0 / ng).reshape(1, ng, 1)
    nz = np.arange(ng // 2 + 1).reshape(1, 1, ng // 2 + 1)
    m = (nz > 0) | ((nz == 0) & (ny > 0)) | ((nz == 0) & (ny == 0) & (nx > 0))
    return np.broadcast_to(m, (ng, ng, ng // 2 + 1))


def mode_kmag(ng: int, box: float) -> np.ndarray:
    nx = np.fft.fftfreq(ng, d=1.0 / ng).reshape(ng, 1, 1)
    ny = np.fft.fftfreq(ng, d=1.0 / ng).reshape(1, ng, 1)
    nz = np.arange(ng // 2 + 1, dtype=np.float64).reshape(1, 1, ng // 2 + 1)
    return (2.0 * np.pi / box) * np.sqrt(nx * nx + ny * ny + nz * nz)


def cic_window(ng: int) -> np.ndarray:
    nx = np.fft.fftfreq(ng, d=1.0 / ng).reshape(ng, 1, 1)
    ny = np.fft.fftfreq(ng, d=1.0 / ng).reshape(1, ng, 1)
    nz = np.arange(ng // 2 + 1, dtype=np.float64).reshape(1, 1, ng // 2 + 1)
    return (np.sinc(nx / ng) * np.sinc(ny / ng) * np.sinc(nz / ng)) ** 2


def bin_modes(values: np.ndarray, ng: int, box: float, edges):
    """Half-space, |k| <= k_Nyq modes binned by |k|: (kmean, mean value, count)."""
    edges = np.asarray(edges, dtype=np.float64)
    kmag = mode_kmag(ng, box)
    keep = halfspace_mask(ng) & (kmag <= np.pi * ng / box)
    k = kmag[keep]
    v = np.broadcast_to(values, kmag.shape)[keep]
    b = np.searchsorted(edges, k, side="right") - 1
    ok = (b >= 0) & (b < len(edges) - 1)
    b, k, v = b[ok], k[ok], v[ok]
    nb = len(edges) - 1
    cnt = np.bincount(b, minlength=nb).astype(np.int64)
    ksum = np.bincount(b, weights=k, minlength=nb)
    vsum = np.bincount(b, weights=v, minlength=nb)
    with np.errstate(invalid="ignore", divide="ignore"):
        return ksum / cnt, vsum / cnt, cnt


def power_from_delta(delta: np.ndarray, box: float, edges, deconvolve=True):
    ng = delta.shape[0]
    dk = sfft.rfftn(delta, workers=-1) * (box ** 3 / ng ** 3)
    if deconvolve:
        dk /= cic_window(ng)
    p = (dk.real ** 2 + dk.imag ** 2) / box ** 3
    return bin_modes(p, ng, box, edges)


def power_spectrum(pos: np.ndarray, box: float, ng: int, edges, deconvolve=True):
    """Binned P(k) of the particles at ``pos`` ((3, Np), Mpc/h)."""
    return power_from_delta(pm.density_contrast(pos, ng, box), box, edges, deconvolve)


def grid_averaged_model(pfunc, ng: int, box: float, edges):
    """Average a model P(|k|) over the same discrete modes and bins (Sec. 3.3)."""
    return bin_modes(pfunc(mode_kmag(ng, box)), ng, box, edges)


def log_edges(box: float, ng: int, nbins: int):
    """nbins log-spaced bins from the fundamental mode to the grid Nyquist."""
    return np.geomspace(2 * np.pi / box, np.pi * ng / box, nbins + 1)


def linear_edges(box: float, ng: int, dk=0.01):
    """Fixed-width bins of dk (h/Mpc) up to the grid Nyquist (Sec. 3.3 uses 0.01)."""
    kn = np.pi * ng / box
    return np.arange(0.0, kn + dk, dk)


def velocity_power(pos: np.ndarray, u: np.ndarray, box: float, ng: int, edges, axis: int):
    """Density and line-of-sight momentum spectra of particles at ``pos`` ((3, Np), Mpc/h)
    carrying ``u`` (Np,), their velocity along ``axis`` in length units (the redshift-space
    shift v_los / (a adot)).

    Fields (CIC, deconvolved like P(k)): delta and the momentum p = sum_p W u_p / nbar,
    nbar the mean number of particles per cell (p = (1 + delta) u on average).  Per mode:
    P_dd = |delta|^2 / V, P_du = sign(k_axis) Im(delta p*) / V (folded onto mu >= 0, the
    line-of-sight part is odd in mu), P_uu = |p|^2 / V; each averaged per |k| bin over
    the P(k) half space.  Returns kmean, P_dd, P_du, P_uu, counts.
    """
    nbar = pos.shape[1] / ng ** 3
    w = cic_window(ng)
    fac = box ** 3 / ng ** 3
    d = sfft.rfftn(pm.cic_deposit(pos, ng, box) / nbar - 1.0, workers=-1) * fac / w
    p = sfft.rfftn(pm.cic_deposit(pos, ng, box, weights=u) / nbar, workers=-1) * fac / w
    n = [np.fft.fftfreq(ng, d=1.0 / ng).reshape(ng, 1, 1),
         np.fft.fftfreq(ng, d=1.0 / ng).reshape(1, ng, 1),
         np.arange(ng // 2 + 1, dtype=np.float64).reshape(1, 1, ng // 2 + 1)][axis]
    V = box ** 3
    k, p_dd, cnt = bin_modes((d.real ** 2 + d.imag ** 2) / V, ng, box, edges)
    _, p_du, _ = bin_modes(np.sign(n) * (d.imag * p.real - d.real * p.imag) / V, ng, box, edges)
    _, p_uu, _ = bin_modes((p.real ** 2 + p.imag ** 2) / V, ng, box, edges)
    return k, p_dd, p_du, p_uu, cnt
