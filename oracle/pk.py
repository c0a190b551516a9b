"""Matter power-spectrum estimator, float64 (Koda et al. 2015, Sec. 3.3).

Steps, in the paper's order:
1. CIC-assign all particles onto an Ng^3 grid; delta = rho/rho_bar - 1.
2. FFT; keep the half space {kz > 0} U {kz = 0, ky > 0} U {kz = 0, ky = 0, kx > 0}
   (the other half carries no independent information for a real field).
3. P(k) = V^-1 <|delta(k)|^2>, with delta(k) = (V/Ng^3) DFT[delta] the
   continuum-normalised transform, averaged in bins; report the mean |k|.
4. Correct for the CIC smoothing by dividing delta(k) by
   W(k) = prod_e sinc^2(pi n_e / Ng) (``power_spectrum``), or for the
   smoothing and the aliasing together by Jing's (2005) procedure
   (``power_spectrum_jing``, the last sentence of Sec. 3.3).

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


# ---------------------------------------------------------------------------
# Smoothing and aliasing correction of Jing (2005, ApJ 620, 559), Sec. 3.3.
#
# The grid spectrum of a field assigned with window W holds every image of a
# mode: <|delta_grid(k)|^2> = sum_m |W(k + 2 k_N m)|^2 P(|k + 2 k_N m|), m in
# Z^3, k_N = pi Ng / L.  Jing approximates P near |k| by a local power law of
# index s, P(|k'|) = P(|k|) (|k'| / |k|)^s, so that per |k| bin
#     P_b = <|delta_grid|^2 / V>_b / <C(k; s_b)>_b,
#     C(k; s) = sum_m |W(k + 2 k_N m)|^2 (|k + 2 k_N m| / |k|)^s,
# and finds s_b by iteration from the corrected spectrum itself.
# Readings (the paper names the procedure only): W is the CIC window
# prod_e sinc^2(pi n_e / Ng) continued to the images; the image sum runs over
# |m_e| <= JING_IMAGES (terms fall as |m|^(s-4) per axis; at s = 0 the
# truncation leaves at most 0.13% at the Nyquist frequency); s_b starts at 0
# and is the log-log slope of the corrected P between the neighbouring
# non-empty bins (one-sided at the ends, 0 for a lone bin), limited to
# [JING_SLOPE_MIN, JING_SLOPE_MAX] (the slopes of a CDM spectrum, between its
# primordial n_s ~ 1 and the small-scale -3; a noisy bin cannot drive the
# image sum, which diverges along an axis for s >= 3); the iteration runs
# JING_ITERATIONS times.  No shot-noise term is subtracted.

JING_IMAGES = 2
JING_ITERATIONS = 8
JING_SLOPE_MIN = -3.0
JING_SLOPE_MAX = 1.0


def _signed_modes(ng: int):
    nx = np.fft.fftfreq(ng, d=1.0 / ng).reshape(ng, 1, 1)
    ny = np.fft.fftfreq(ng, d=1.0 / ng).reshape(1, ng, 1)
    nz = np.arange(ng // 2 + 1, dtype=np.float64).reshape(1, 1, ng // 2 + 1)
    return nx, ny, nz


def alias_window_sum(ng: int, slope, images: int = JING_IMAGES) -> np.ndarray:
    """C(k; s) at every half-spectrum mode of an Ng^3 grid, s = ``slope``
    (scalar or an array broadcastable to (Ng, Ng, Ng/2+1)); the k = 0 entry
    is the m = 0 term alone (1)."""
    nx, ny, nz = _signed_modes(ng)
    n2 = nx * nx + ny * ny + nz * nz
    n2 = np.where(n2 == 0, 1.0, n2)
    half_s = 0.5 * np.asarray(slope, dtype=np.float64)
    out = np.zeros(np.broadcast_shapes(n2.shape, np.shape(half_s)))
    rng_m = range(-images, images + 1)
    for mx in rng_m:
        wx = np.sinc(nx / ng + mx) ** 4
        for my in rng_m:
            wy = np.sinc(ny / ng + my) ** 4
            for mz in rng_m:
                wz = np.sinc(nz / ng + mz) ** 4
                w = wx * wy * wz
                k2 = (nx + ng * mx) ** 2 + (ny + ng * my) ** 2 + (nz + ng * mz) ** 2
                with np.errstate(divide="ignore", invalid="ignore"):
                    ratio = np.where(w > 0, (k2 / n2) ** half_s, 0.0)
                out = out + w * ratio
    return out


def local_slopes(kmean: np.ndarray, p: np.ndarray, cnt: np.ndarray) -> np.ndarray:
    """d ln P / d ln k of each non-empty bin from its non-empty neighbours."""
    s = np.zeros(len(p))
    idx = np.flatnonzero(cnt > 0)
    for j, b in enumerate(idx):
        lo = idx[j - 1] if j > 0 else b
        hi = idx[j + 1] if j + 1 < len(idx) else b
        if lo != hi and p[lo] > 0 and p[hi] > 0:
            s[b] = np.log(p[hi] / p[lo]) / np.log(kmean[hi] / kmean[lo])
    return s


def mode_bins(ng: int, box: float, edges) -> np.ndarray:
    """Bin index of every half-spectrum mode under bin_modes' selection, -1 where unbinned."""
    edges = np.asarray(edges, dtype=np.float64)
    kmag = mode_kmag(ng, box)
    keep = halfspace_mask(ng) & (kmag <= np.pi * ng / box)
    b = np.searchsorted(edges, kmag, side="right") - 1
    b[(b < 0) | (b >= len(edges) - 1) | ~keep] = -1
    return b


def power_from_delta_jing(delta: np.ndarray, box: float, edges, images: int = JING_IMAGES,
                          iterations: int = JING_ITERATIONS):
    """Binned P(k) of a grid density contrast, corrected by Jing's procedure:
    (kmean, P, count)."""
    ng = delta.shape[0]
    dk = sfft.rfftn(delta, workers=-1) * (box ** 3 / ng ** 3)
    raw = (dk.real ** 2 + dk.imag ** 2) / box ** 3
    kmean, praw, cnt = bin_modes(raw, ng, box, edges)
    bins = mode_bins(ng, box, edges)
    s = np.zeros(len(cnt))
    p = praw
    for _ in range(iterations):
        smode = np.where(bins >= 0, s[np.maximum(bins, 0)], 0.0)
        _, cbar, _ = bin_modes(alias_window_sum(ng, smode, images), ng, box, edges)
        with np.errstate(invalid="ignore", divide="ignore"):
            p = praw / cbar
        s = np.clip(local_slopes(kmean, p, cnt), JING_SLOPE_MIN, JING_SLOPE_MAX)
    return kmean, p, cnt


def power_spectrum_jing(pos: np.ndarray, box: float, ng: int, edges, images: int = JING_IMAGES,
                        iterations: int = JING_ITERATIONS):
    """Binned P(k) of the particles at ``pos`` with Jing's smoothing and aliasing correction."""
    return power_from_delta_jing(pm.density_contrast(pos, ng, box), box, edges, images, iterations)
