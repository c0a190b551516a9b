"""Particle-mesh force, float64: CIC deposit, Poisson + gradient, CIC readout.

Paper passages followed (Koda et al. 2015):
* Sec. 2.2: F = -grad phi with laplacian(phi) = (3/2) Omega_m a^-1 delta,
  delta = rho/rho_bar - 1 (comoving coordinates, H0 = 1).
* Sec. 2.3: a PM gravity solver on a mesh finer than the particle lattice;
  Sec. 3.3: Cloud-in-Cell (CIC) mass assignment.

Readings where the paper is silent:
* CIC nodes sit at cell centres, (i + 1/2) dx, dx = L/Nm.  A particle at
  position x has node coordinate u = x / dx - 1/2 (periodic), home cell
  i = floor(u), fraction f = u - i, and gives weight prod_e w_{s_e}(f_e),
  w_0(f) = 1 - f, w_1(f) = f, to node i + s, s in {0,1}^3.  (With nodes at
  i dx every lattice particle of a mesh 2x or 3x the particle grid would sit
  exactly on a node, on the kink of the CIC kernel.)
* Green's function -1/k^2 (continuous), spectral gradient i k, no CIC
  deconvolution in the force, k = 0 -> 0, and the gradient component k_d is
  zeroed on the Nyquist plane of axis d.
* The readout uses the same CIC weights as the deposit.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

_WORKERS = -1


def cic_cells(pos: np.ndarray, nm: int, box: float):
    """Home cells (3, Np) int64 in [0, nm) and fractions (3, Np) in [0, 1)."""
    u = np.mod(np.asarray(pos, dtype=np.float64) * (nm / box) - 0.5, nm)
    i0 = np.floor(u)
    f = u - i0
    return np.mod(i0.astype(np.int64), nm), f


def _offsets():
    for sx in (0, 1):
        for sy in (0, 1):
            for sz in (0, 1):
                yield sx, sy, sz


def cic_deposit(pos: np.ndarray, nm: int, box: float, weights=None) -> np.ndarray:
    """Mass per node (each particle has unit mass unless ``weights`` given)."""
    i0, f = cic_cells(pos, nm, box)
    w = [1.0 - f, f]
    rho = np.zeros(nm ** 3)
    base = np.ones(pos.shape[1]) if weights is None else np.asarray(weights, np.float64)
    for sx, sy, sz in _offsets():
        idx = (((i0[0] + sx) % nm) * nm + (i0[1] + sy) % nm) * nm + (i0[2] + sz) % nm
        rho += np.bincount(idx, weights=base * w[sx][0] * w[sy][1] * w[sz][2],
                           minlength=nm ** 3)
    return rho.reshape(nm, nm, nm)


def density_contrast(pos: np.ndarray, nm: int, box: float) -> np.ndarray:
    """delta = rho / rho_bar - 1, rho_bar = Np / Nm^3."""
    rho = cic_deposit(pos, nm, box)
    return rho * (nm ** 3 / pos.shape[1]) - 1.0


def kvectors(nm: int, box: float):
    kf = 2.0 * np.pi / box
    nx = np.fft.fftfreq(nm, d=1.0 / nm).reshape(nm, 1, 1)
    ny = np.fft.fftfreq(nm, d=1.0 / nm).reshape(1, nm, 1)
    nz = np.arange(nm // 2 + 1, dtype=np.float64).reshape(1, 1, nm // 2 + 1)
    return (kf * nx, kf * ny, kf * nz), (nx, ny, nz)


def gradient_multiplier(nm: int, box: float, alpha: float, d: int):
    """m_d(k) = i k_d alpha / k^2 with k=0 -> 0 and k_d = 0 on the Nyquist plane of d."""
    (kx, ky, kz), (nx, ny, nz) = kvectors(nm, box)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2[0, 0, 0] = 1.0
    kd, nd = ((kx, nx), (ky, ny), (kz, nz))[d]
    kd_eff = np.where(np.abs(nd) == nm // 2, 0.0, kd)
    m = 1j * kd_eff * alpha / k2
    m = np.broadcast_to(m, (nm, nm, nm // 2 + 1)).copy()
    m[0, 0, 0] = 0.0
    return m


def force_component(delta_hat: np.ndarray, nm: int, box: float, alpha: float, d: int):
    """g_d on the mesh: inverse DFT of m_d(k) * DFT[delta]."""
    m = gradient_multiplier(nm, box, alpha, d)
    m *= delta_hat
    return sfft.irfftn(m, s=(nm, nm, nm), workers=_WORKERS)


def cic_readout(field: np.ndarray, pos: np.ndarray, box: float) -> np.ndarray:
    """Interpolate a mesh field to particle positions with the CIC weights."""
    nm = field.shape[0]
    i0, f = cic_cells(pos, nm, box)
    w = [1.0 - f, f]
    flat = field.ravel()
    out = np.zeros(pos.shape[1])
    for sx, sy, sz in _offsets():
        idx = (((i0[0] + sx) % nm) * nm + (i0[1] + sy) % nm) * nm + (i0[2] + sz) % nm
        out += w[sx][0] * w[sy][1] * w[sz][2] * flat[idx]
    return out


def pm_force(pos: np.ndarray, nm: int, box: float, alpha: float) -> np.ndarray:
    """F(x_p) for every particle, shape (3, Np), Mpc/h * H0^2 units."""
    delta = density_contrast(pos, nm, box)
    dk = sfft.rfftn(delta, workers=_WORKERS)
    del delta
    out = np.empty((3, pos.shape[1]))
    for d in range(3):
        g = force_component(dk, nm, box, alpha, d)
        out[d] = cic_readout(g, pos, box)
        del g
    return out


def force_meshes(pos: np.ndarray, nm: int, box: float, alpha: float):
    """The three force meshes g_d (3, nm, nm, nm) at the given positions."""
    dk = sfft.rfftn(density_contrast(pos, nm, box), workers=_WORKERS)
    return np.stack([force_component(dk, nm, box, alpha, d) for d in range(3)])


def rfftn_slabs(x: np.ndarray, slab: int = 64, progress=None) -> np.ndarray:
    """rfftn of a real (n0, n1, n2) array in FP64 holding one half spectrum
    and a slab at a time: the 3D DFT is separable, so it is the real
    transform along z, then the transform along y (both slab by slab of x
    planes), then the transform along x (slab by slab of y rows).  For
    meshes too large for rfftn's temporaries (the 2048^3 mesh)."""
    n0, n1, n2 = x.shape
    out = np.empty((n0, n1, n2 // 2 + 1), np.complex128)
    for i in range(0, n0, slab):
        blk = sfft.rfft(np.asarray(x[i:i + slab], np.float64), axis=2, workers=_WORKERS)
        out[i:i + slab] = sfft.fft(blk, axis=1, workers=_WORKERS, overwrite_x=True)
        if progress:
            progress("z, y", i + slab, n0)
    for j in range(0, n1, slab):
        out[:, j:j + slab] = sfft.fft(out[:, j:j + slab], axis=0, workers=_WORKERS)
        if progress:
            progress("x", j + slab, n1)
    return out


def force_at_nodes(delta_hat: np.ndarray, nm: int, box: float, alpha: float, nodes, slab: int = 16,
                   progress=None):
    """The three force meshes of force_component at chosen mesh nodes, summed
    mode by mode (no inverse FFT), and the root-mean-square of each mesh.

    g_d(x) = N^-3 Re sum_n c(n_z) m_d(n) delta_hat(n) exp(2 pi i n.x / N) over
    the stored half spectrum (n_z = 0 .. N/2), c = 1 on the planes n_z = 0 and
    N/2 and 2 between (each such mode stands for itself and its Hermitian
    partner); m_d is gradient_multiplier's.  rms_d^2 = N^-6 sum_n c |m_d
    delta_hat|^2 (Parseval).  nodes: (S, 3) integer node indices.  Returns
    (g of shape (3, S), rms of shape (3,))."""
    nodes = np.asarray(nodes, np.int64)
    n = nm
    kf = 2.0 * np.pi / box
    nfreq = np.fft.fftfreq(n, d=1.0 / n)                       # signed, -N/2 at index N/2
    nz = np.arange(n // 2 + 1, dtype=np.float64)
    c = np.where((nz == 0) | (nz == n // 2), 1.0, 2.0)

    def keff(v):                                                # k_d, zero on its Nyquist plane
        return np.where(np.abs(v) == n // 2, 0.0, kf * v)

    # phase factors exp(2 pi i n_e x_e / N) per axis and node: (frequencies, S)
    ex = np.exp(2j * np.pi * np.outer(nfreq, nodes[:, 0]) / n)
    ey = np.exp(2j * np.pi * np.outer(nfreq, nodes[:, 1]) / n)
    ez = np.exp(2j * np.pi * np.outer(nz, nodes[:, 2]) / n)
    ikx, iky, ikz = 1j * keff(nfreq), 1j * keff(nfreq), 1j * keff(nz)
    g = np.zeros((3, len(nodes)), np.complex128)
    ms = np.zeros(3)
    ky2 = (kf * nfreq) ** 2
    kz2 = (kf * nz) ** 2
    for i0 in range(0, n, slab):
        i1 = min(n, i0 + slab)
        kx2 = (kf * nfreq[i0:i1]) ** 2
        k2 = kx2[:, None, None] + ky2[None, :, None] + kz2[None, None, :]
        if i0 == 0:
            k2[0, 0, 0] = 1.0
        D = delta_hat[i0:i1] * (alpha / k2)                     # phi-like: alpha delta_hat / k^2
        if i0 == 0:
            D[0, 0, 0] = 0.0
        del k2
        # Parseval: |m_d D'|^2 with m_d = i k_d, weighted by c
        a2 = (np.abs(D) ** 2) * c[None, None, :]
        ms[0] += float(np.sum(a2.sum(axis=(1, 2)) * np.abs(ikx[i0:i1]) ** 2))
        ms[1] += float(np.sum(a2.sum(axis=(0, 2)) * np.abs(iky) ** 2))
        ms[2] += float(np.sum(a2.sum(axis=(0, 1)) * np.abs(ikz) ** 2))
        del a2
        Dc = D * c[None, None, :]
        del D
        flat = Dc.reshape(-1, n // 2 + 1)
        t0 = (flat @ ez).reshape(i1 - i0, n, -1)                # sum over n_z
        tz = (flat @ (ikz[:, None] * ez)).reshape(i1 - i0, n, -1)
        del Dc, flat
        u0 = np.einsum("ayS,yS->aS", t0, ey)                    # sum over n_y
        uy = np.einsum("ayS,yS->aS", t0, iky[:, None] * ey)
        uz = np.einsum("ayS,yS->aS", tz, ey)
        exs = ex[i0:i1]
        g[0] += np.einsum("aS,aS->S", u0, ikx[i0:i1, None] * exs)
        g[1] += np.einsum("aS,aS->S", uy, exs)
        g[2] += np.einsum("aS,aS->S", uz, exs)
        if progress:
            progress("modes", i1, n)
    n3 = float(n) ** 3
    return g.real / n3, np.sqrt(ms) / n3
