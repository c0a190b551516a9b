"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module generates workload inputs only; it contains none of the COLA
arithmetic (no growth factors, no mass assignment, no Poisson solve, no time
stepping).  What it provides:

* ``white_noise``          -- i.i.d. N(0, 1) field on the Lagrangian lattice
                              (the "initial random modes" of the paper's
                              realisations, Sec. 2.3), float32, C order.
* ``fixed_amplitude_noise`` -- test-only noise whose DFT has modulus N^{3/2}
                              everywhere and random phases (removes cosmic
                              variance from statistical checks).
* ``bbks_table``           -- a (k, P(k)) table of P = A k^{n_s} T_BBKS(k)^2
                              normalised to a given sigma_8; the COLA
                              initial-condition step takes P(k) as a table.
* ``CONFIGS``              -- the five named workloads (sizes, boxes, seeds).

Lengths are Mpc/h, wavenumbers h/Mpc.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def white_noise(seed: int, np_side: int) -> np.ndarray:
    """N(0,1) white noise on an np_side^3 lattice, float32, C order (x, y, z)."""
    gen = np.random.Generator(np.random.Philox(seed))
    return gen.standard_normal(size=(np_side,) * 3, dtype=np.float32)


def fixed_amplitude_noise(seed: int, np_side: int) -> np.ndarray:
    """Real field whose rfftn has modulus np_side^{3/2} at every mode.

    Phases come from seeded white noise.  Used by statistical tests only.
    """
    w = white_noise(seed, np_side).astype(np.float64)
    wk = np.fft.rfftn(w)
    mod = np.abs(wk)
    mod[mod == 0] = 1.0
    wk = wk / mod * np_side ** 1.5
    return np.fft.irfftn(wk, s=w.shape, axes=(0, 1, 2)).astype(np.float32)


def seeded_normal(seed: int, shape) -> np.ndarray:
    """Generic seeded N(0,1) float32 array (targets, cotangents, directions)."""
    gen = np.random.Generator(np.random.Philox(seed))
    return gen.standard_normal(size=shape, dtype=np.float32)


def _bbks_transfer(k, gamma):
    q = np.asarray(k, dtype=np.float64) / gamma
    q = np.where(q == 0, 1e-300, q)
    t = np.log1p(2.34 * q) / (2.34 * q)
    poly = 1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4
    return t * poly ** -0.25


def _tophat(x):
    x = np.asarray(x, dtype=np.float64)
    small = x < 1e-3
    xs = np.where(small, 1.0, x)
    w = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
    return np.where(small, 1.0 - x * x / 10.0, w)


def bbks_table(omega_m=0.27, h=0.705, n_s=0.96, sigma8=0.8,
               kmin=1e-5, kmax=1e2, nk=2048):
    """Return (k, P) float64 arrays, log-spaced in k, of the BBKS spectrum at z=0.

    Shape parameter Gamma = omega_m * h.  The amplitude A is set so that the
    top-hat variance in 8 Mpc/h spheres equals sigma8^2.
    """
    from scipy import integrate

    gamma = omega_m * h

    def integrand(lnk):
        k = math.exp(lnk)
        return k ** 3 / (2 * math.pi ** 2) * k ** n_s * _bbks_transfer(k, gamma) ** 2 \
            * _tophat(8.0 * k) ** 2

    s2, _ = integrate.quad(integrand, math.log(1e-6), math.log(1e3), limit=2000,
                           epsabs=0.0, epsrel=1e-12)
    amp = sigma8 ** 2 / s2
    k = np.geomspace(kmin, kmax, nk)
    pk = amp * k ** n_s * _bbks_transfer(k, gamma) ** 2
    return k, pk


@dataclass
class Config:
    name: str
    np_side: int
    nmesh: int
    box: float
    seed: int
    nstep: int = 10
    a_init: float = 0.02
    a_final: float = 1.0
    omega_m: float = 0.27
    h: float = 0.705
    n_s: float = 0.96
    sigma8: float = 0.8
    n_lpt: float = -2.5
    extra: dict = field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return self.np_side ** 3


# Workloads: (particles per side, mesh per side, box [Mpc/h]).
CONFIGS = {
    "small": Config("small: 32^3 particles / 64^3 mesh / 100 Mpc/h", 32, 64, 100.0, seed=1),
    "production": Config("production: 256^3 particles / 768^3 mesh / 600 Mpc/h",
                         256, 768, 600.0, seed=2),
    "diff": Config("differentiable: 128^3 particles / 256^3 mesh / 300 Mpc/h",
                   128, 256, 300.0, seed=4),
    "diff_fd": Config("finite-difference copy: 16^3 particles / 32^3 mesh / 37.5 Mpc/h",
                      16, 32, 37.5, seed=4),
    "large": Config("large: 1024^3 particles / 2048^3 mesh / 1200 Mpc/h",
                    1024, 2048, 1200.0, seed=5),
}

# Batched mocks: 32 each of (48^3/96^3, L=150), (64^3/128^3, L=200), (96^3/192^3, L=300).
BATCH_GROUPS = [(48, 96, 150.0), (64, 128, 200.0), (96, 192, 300.0)]


def batch_configs(per_group: int = 32, seed0: int = 1000):
    out = []
    s = seed0
    for (n, m, box) in BATCH_GROUPS:
        for _ in range(per_group):
            out.append(Config(f"mock {n}^3/{m}^3 L={box}", n, m, box, seed=s))
            s += 1
    return out


def step_edges(a_init=0.02, a_final=1.0, nstep=10):
    """Scale factors of the step boundaries, uniform in a."""
    return [a_init + (a_final - a_init) * i / nstep for i in range(nstep + 1)]
