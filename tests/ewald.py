"""Periodic point-mass force by Ewald summation and by direct image sums.

Test helper (not part of the oracle).  Units: a box of side L, a unit mass
whose density contrast obeys laplacian(phi) = alpha * (V delta_D - 1), i.e.
G m = alpha V / (4 pi); F = -grad phi.
"""
import itertools

import numpy as np
from scipy.special import erfc


def ewald_force(r, box=1.0, alpha=1.0, kappa=None, nr=3, nh=8):
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    V = box ** 3
    gm = alpha * V / (4 * np.pi)
    kappa = 2.0 / box if kappa is None else kappa
    F = np.zeros_like(r)
    for n in itertools.product(range(-nr, nr + 1), repeat=3):
        rn = r + np.array(n) * box
        d = np.linalg.norm(rn, axis=1)[:, None]
        F += -gm * rn / d ** 3 * (erfc(kappa * d)
                                  + 2 * kappa * d / np.sqrt(np.pi) * np.exp(-(kappa * d) ** 2))
    for h in itertools.product(range(-nh, nh + 1), repeat=3):
        if h == (0, 0, 0):
            continue
        hv = 2 * np.pi * np.array(h) / box
        h2 = hv @ hv
        F += -gm * 4 * np.pi / V * hv / h2 * np.exp(-h2 / (4 * kappa ** 2)) * np.sin(r @ hv)[:, None]
    return F


def direct_force(r, box=1.0, alpha=1.0, nimg=20):
    """Sum over images in a (2K+1)^3 cube plus the uniform-cube background term."""
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    V = box ** 3
    gm = alpha * V / (4 * np.pi)
    g = np.arange(-nimg, nimg + 1)
    n = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) * box
    F = np.empty_like(r)
    for i in range(len(r)):
        rn = r[i] + n
        d = np.linalg.norm(rn, axis=1)
        F[i] = -gm * (rn / d[:, None] ** 3).sum(0)
    return F + 4 * np.pi / 3 * gm / V * r
