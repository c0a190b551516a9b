"""Reverse-mode derivative of the COLA step, the density/P(k) outputs and the
2LPT initial conditions, float64 (oracle for the GPU adjoint).

Forward step (Koda et al. 2015, Sec. 2.2; notation of ``cola.step``), with
x = q + d the positions at a0:
    rho   = D(x)                         CIC deposit (unit masses)
    delta = rho * Nm^3/Np - 1
    g_d   = G_d delta,   G_d = irfftn(i k_d alpha / k^2 rfftn(.))
    F_d   = R(x, g_d)                    CIC readout
    v'    = v + K (F - alpha [D1 Psi1 + (D2 - D1^2) Psi2])
    d'    = d + I v' + dD1 Psi1 + dD2 Psi2
Reverse, given the cotangents (dbar', vbar') of (d', v'):
    vt      = vbar' + I dbar'
    Psi1bar += dD1 dbar' - K alpha D1 vt,  Psi2bar += dD2 dbar' - K alpha (D2 - D1^2) vt
    vbar    = vt;  Fbar = K vt
    xbar    = sum_d Fbar_d grad_x R(x, g_d)              (CIC weight gradients)
    gbar_d  = R^T Fbar_d = D(x; weights Fbar_d)          (readout transpose)
    deltabar = sum_d G_d^T gbar_d = -sum_d G_d gbar_d    (i k / k^2 is odd and imaginary)
    xbar   += grad_x D(x)^T (deltabar Nm^3/Np)
    dbar    = dbar' + xbar
The weight gradient: d w_s / d x_e = (+1 if s_e = 1 else -1) (1/dx) prod_{e' != e} w_{s_e'}.

Initial conditions (``ic``): w -> delta_L = irfftn(A rfftn(w)) (A = sqrt(P/dq^3),
zero at k = 0 and Nyquist indices), Psi1_d = irfftn(M1_d A w_k), phi_ij =
irfftn(k_i k_j / k^2 A w_k), S(phi), Psi2_d = irfftn(M2_d rfftn(S)).  For a
real circulant y = irfftn(m rfftn(x)) the transpose multiplies by conj(m).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import cosmology as cosmo
from . import ic
from . import pk as pkmod
from . import pm

_W = -1


def _offsets():
    for sx in (0, 1):
        for sy in (0, 1):
            for sz in (0, 1):
                yield sx, sy, sz


def readout_grad(field: np.ndarray, pos: np.ndarray, box: float) -> np.ndarray:
    """grad_x of the CIC readout R(x, field) at each particle: (3, Np)."""
    nm = field.shape[0]
    i0, f = pm.cic_cells(pos, nm, box)
    w = [1.0 - f, f]
    dw = [-np.ones_like(f), np.ones_like(f)]
    flat = field.ravel()
    out = np.zeros((3, pos.shape[1]))
    inv_dx = nm / box
    for sx, sy, sz in _offsets():
        idx = (((i0[0] + sx) % nm) * nm + (i0[1] + sy) % nm) * nm + (i0[2] + sz) % nm
        val = flat[idx]
        out[0] += dw[sx][0] * w[sy][1] * w[sz][2] * val
        out[1] += w[sx][0] * dw[sy][1] * w[sz][2] * val
        out[2] += w[sx][0] * w[sy][1] * dw[sz][2] * val
    return out * inv_dx


def step_adjoint(state, a1: float, dbar1: np.ndarray, vbar1: np.ndarray):
    """Cotangents at the start of the step a_x -> a1.

    ``state`` holds the positions/velocities at the step start (a_x, a_v) and
    Psi1, Psi2.  Returns (dbar0, vbar0, psi1bar, psi2bar) where the Psi bars
    are this step's contributions.
    """
    c = cosmo.step_coefficients(state.a_x, state.a_v, a1, state.om, state.n_lpt, state.d2_ode)
    K, I, al, D1, D2 = c["K"], c["I"], c["alpha"], c["D1"], c["D2"]
    vt = vbar1 + I * dbar1
    psi1bar = c["dD1"] * dbar1 - K * al * D1 * vt
    psi2bar = c["dD2"] * dbar1 - K * al * (D2 - D1 * D1) * vt
    fbar = K * vt
    x = state.positions()
    nm, box = state.nmesh, state.box
    delta = pm.density_contrast(x, nm, box)
    dk = sfft.rfftn(delta, workers=_W)
    xbar = np.zeros_like(x)
    deltabar_k = np.zeros_like(dk)
    for d in range(3):
        g = pm.force_component(dk, nm, box, al, d)
        xbar += fbar[d] * readout_grad(g, x, box)
        gbar = pm.cic_deposit(x, nm, box, weights=fbar[d])
        deltabar_k -= pm.gradient_multiplier(nm, box, al, d) * sfft.rfftn(gbar, workers=_W)
    deltabar = sfft.irfftn(deltabar_k, s=(nm,) * 3, workers=_W)
    rhobar = deltabar * (nm ** 3 / x.shape[1])
    xbar += readout_grad(rhobar, x, box)
    return dbar1 + xbar, vt, psi1bar, psi2bar


def density_adjoint(pos: np.ndarray, nm: int, box: float, deltabar: np.ndarray) -> np.ndarray:
    """x-cotangent of delta = D(x) Nm^3/Np - 1 for a mesh cotangent deltabar."""
    return readout_grad(deltabar * (nm ** 3 / pos.shape[1]), pos, box)


def pk_adjoint(pos: np.ndarray, box: float, ng: int, edges, cbar) -> np.ndarray:
    """x-cotangent of L = sum_b cbar_b P_b (``pk.power_spectrum`` estimator)."""
    delta = pm.density_contrast(pos, ng, box)
    X = sfft.rfftn(delta, workers=_W)
    kmag = pkmod.mode_kmag(ng, box)
    keep = pkmod.halfspace_mask(ng) & (kmag <= np.pi * ng / box)
    edges = np.asarray(edges, np.float64)
    b = np.searchsorted(edges, kmag, side="right") - 1
    inb = keep & (b >= 0) & (b < len(edges) - 1)
    cnt = np.bincount(b[inb], minlength=len(edges) - 1)
    V = box ** 3
    fac = (V / ng ** 3) ** 2 / V / pkmod.cic_window(ng) ** 2
    u = np.zeros(X.shape)
    bb = np.clip(b, 0, len(edges) - 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        u[inb] = (np.asarray(cbar)[bb] / np.maximum(cnt[bb], 1) * np.broadcast_to(fac, X.shape))[inb]
    # dL/d delta(x) = sum_{k in bins} 2 u_k Re(X_k e^{ikx}) = Re(sum 2 u X e^{ikx}), done as a
    # full complex inverse over the explicit mode set (no Hermitian doubling assumptions).
    full = np.zeros((ng, ng, ng), complex)
    nz = ng // 2 + 1
    full[:, :, :nz] += 2 * u * X
    deltabar = np.real(sfft.ifftn(full, workers=_W)) * ng ** 3
    return density_adjoint(pos, ng, box, deltabar)


# ---------------------------------------------------------------------------
def _kgrid(n, box):
    kf = 2 * np.pi / box
    nx, ny, nz = ic.mode_indices(n)
    return [kf * nx, kf * ny, kf * nz]


def _irf(x, n):
    return sfft.irfftn(x, s=(n,) * 3, workers=_W)


def _rf(x):
    return sfft.rfftn(x, workers=_W)


def ic_adjoint(noise: np.ndarray, box: float, ktab, ptab, psi1bar, psi2bar) -> np.ndarray:
    """w-cotangent of (Psi1, Psi2) = lpt(noise); psi bars shaped (3, N^3) in Mpc/h."""
    n = noise.shape[0]
    dq = box / n
    kv = _kgrid(n, box)
    k2 = kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2
    k2[0, 0, 0] = 1.0
    inv = 1.0 / k2
    inv[0, 0, 0] = 0.0
    zero = ic.nyquist_mask(n)
    amp = np.sqrt(ic.interp_pk(np.sqrt(k2), ktab, ptab) / dq ** 3)
    amp[0, 0, 0] = 0.0
    amp[zero] = 0.0
    dk = _rf(noise.astype(np.float64)) * amp
    p1b = np.asarray(psi1bar, np.float64).reshape(3, n, n, n)
    p2b = np.asarray(psi2bar, np.float64).reshape(3, n, n, n)
    # S-bar from Psi2-bar (multiplier -i k_d / k^2 with k=0, Nyquist zeroed -> conj)
    sbar_k = np.zeros_like(dk)
    for d in range(3):
        m = -1j * kv[d] * inv
        m = np.where(zero, 0.0, m)
        sbar_k += np.conj(m) * _rf(p2b[d])
    sbar = _irf(sbar_k, n)
    phi = {}
    for (i, j) in ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (2, 0)):
        phi[(i, j)] = _irf(kv[i] * kv[j] * dk * inv, n)
    pbar = {
        (0, 0): sbar * (phi[(1, 1)] + phi[(2, 2)]),
        (1, 1): sbar * (phi[(0, 0)] + phi[(2, 2)]),
        (2, 2): sbar * (phi[(0, 0)] + phi[(1, 1)]),
        (0, 1): -2.0 * sbar * phi[(0, 1)],
        (1, 2): -2.0 * sbar * phi[(1, 2)],
        (2, 0): -2.0 * sbar * phi[(2, 0)],
    }
    wk = np.zeros_like(dk)
    for (i, j), pb in pbar.items():
        wk += kv[i] * kv[j] * inv * amp * _rf(pb)
    for d in range(3):
        wk += np.conj(1j * kv[d] * inv) * amp * _rf(p1b[d])
    return _irf(wk, n)


def run_adjoint(noise, box, nmesh, ktab, ptab, edges, dbar_final, vbar_final=None,
                a_init=0.02, om=0.27, n_lpt=-2.5, d2_ode=False):
    """Gradient of a loss on the final state w.r.t. the white noise (stores every step)."""
    from . import cola
    st = cola.init_state(noise, box, nmesh, ktab, ptab, a_init, om, n_lpt, d2_ode)
    saved = []
    for a1 in edges[1:]:
        saved.append((st.d.copy(), st.v.copy(), st.a_x, st.a_v))
        cola.step(st, a1)
    dbar = np.array(dbar_final, dtype=np.float64)
    vbar = np.zeros_like(dbar) if vbar_final is None else np.array(vbar_final, np.float64)
    p1b = np.zeros_like(dbar)
    p2b = np.zeros_like(dbar)
    for (d, v, ax, av), a1 in zip(reversed(saved), reversed(edges[1:])):
        st.d, st.v, st.a_x, st.a_v = d, v, ax, av
        dbar, vbar, q1, q2 = step_adjoint(st, a1, dbar, vbar)
        p1b += q1
        p2b += q2
    # d0 = D1 Psi1 + D2 Psi2, v0 = 0
    p1b += cosmo.growth_D1(a_init, om) * dbar
    p2b += cosmo.D2_of(a_init, om, d2_ode) * dbar
    return ic_adjoint(noise, box, ktab, ptab, p1b, p2b), st
