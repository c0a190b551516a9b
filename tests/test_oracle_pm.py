"""Pins for the oracle's particle-mesh force (Sec. 2.2-2.3, CIC of Sec. 3.3)."""
import itertools

import numpy as np
import pytest

from oracle import pm
from tests.ewald import direct_force, ewald_force


def test_naive_dft_convention():
    # scipy rfftn layout and sign against a brute-force O(N^6) DFT.
    import scipy.fft as sfft
    n = 6
    rng = np.random.default_rng(1)
    f = rng.standard_normal((n, n, n))
    idx = np.arange(n)
    ref = np.zeros((n, n, n // 2 + 1), complex)
    for kx, ky, kz in itertools.product(range(n), range(n), range(n // 2 + 1)):
        ph = np.exp(-2j * np.pi * (kx * idx[:, None, None] + ky * idx[None, :, None]
                                   + kz * idx[None, None, :]) / n)
        ref[kx, ky, kz] = np.sum(f * ph)
    assert np.abs(sfft.rfftn(f) - ref).max() < 1e-12 * np.abs(ref).max()


def test_cic_mass_conservation_and_positivity():
    rng = np.random.default_rng(2)
    L, nm, npart = 50.0, 16, 5000
    pos = rng.uniform(-2 * L, 3 * L, (3, npart))
    rho = pm.cic_deposit(pos, nm, L)
    assert abs(rho.sum() - npart) < 1e-12 * npart
    assert rho.min() >= 0


def test_cic_special_positions():
    L, nm = 8.0, 8
    # Nodes sit at cell centres (i + 1/2) dx.  A particle on a node: all mass there.
    rho = pm.cic_deposit(np.array([[2.5], [3.5], [7.5]]), nm, L)
    assert rho[2, 3, 7] == 1.0 and rho.sum() == 1.0
    # A particle half way between nodes in all three axes: 1/8 on each of 8.
    rho = pm.cic_deposit(np.array([[3.0], [0.0], [5.0]]), nm, L)
    nz = np.argwhere(rho > 0)
    assert len(nz) == 8 and np.allclose(rho[rho > 0], 0.125)
    assert sorted(set(nz[:, 1])) == [0, 7]          # periodic wrap


def test_cic_uniform_lattice_on_matching_mesh():
    from oracle.ic import lattice
    L, n = 10.0, 8
    delta = pm.density_contrast(lattice(n, L), n, L)
    assert np.abs(delta).max() < 1e-12


def test_cic_against_per_particle_loop():
    rng = np.random.default_rng(3)
    L, nm = 6.0, 6
    pos = rng.uniform(0, L, (3, 12))
    ref = np.zeros((nm, nm, nm))
    for p in range(pos.shape[1]):
        u = pos[:, p] * nm / L - 0.5
        i0 = np.floor(u).astype(int)
        f = u - i0
        for s in itertools.product((0, 1), repeat=3):
            w = np.prod([f[e] if s[e] else 1 - f[e] for e in range(3)])
            ref[tuple((i0 + s) % nm)] += w
    assert np.abs(pm.cic_deposit(pos, nm, L) - ref).max() < 1e-14


def test_readout_reproduces_linear_field_and_nodes():
    L, nm = 8.0, 8
    i = np.arange(nm)
    field = np.broadcast_to((1.5 * i).reshape(nm, 1, 1), (nm, nm, nm)).copy()
    pos = np.array([[2.5 + 0.3], [1.0], [4.2]])   # between nodes 2 and 3 on x
    assert abs(pm.cic_readout(field, pos, L)[0] - 1.5 * 2.3) < 1e-12


def test_green_gradient_plane_wave():
    # delta = cos(k.x) => F = -(alpha/|k|) khat sin(k.x), exactly (spectral).
    L, nm, alpha = 30.0, 16, 1.7
    x = (np.arange(nm) + 0.5) * L / nm
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    kv = 2 * np.pi / L * np.array([2.0, -1.0, 3.0])
    ph = kv[0] * X + kv[1] * Y + kv[2] * Z
    dk = np.fft.rfftn(np.cos(ph))
    kk = np.linalg.norm(kv)
    for d in range(3):
        g = pm.force_component(dk, nm, L, alpha, d)
        assert np.abs(g + alpha / kk * (kv[d] / kk) * np.sin(ph)).max() < 1e-12


def test_total_momentum_vanishes():
    rng = np.random.default_rng(4)
    L, nm = 40.0, 16
    pos = rng.uniform(0, L, (3, 3000))
    pos[:, :1500] = np.mod(pos[:, :1500] * 0.2 + 5.0, L)      # clustered part
    F = pm.pm_force(pos, nm, L, 2.0)
    assert np.abs(F.sum(axis=1)).max() < 1e-12 * np.abs(F).sum()


def test_ewald_helper_against_direct_image_sums():
    rng = np.random.default_rng(5)
    r = rng.uniform(-0.3, 0.3, (4, 3))
    e = ewald_force(r)
    assert np.abs(ewald_force(r, kappa=3.0, nr=4, nh=12) - e).max() < 1e-12 * np.abs(e).max()
    assert np.abs(direct_force(r, nimg=20) - e).max() < 1e-5 * np.abs(e).max()


def test_isolated_particle_force_beyond_few_cells():
    # The PM force approaches the periodic point-mass force at a few mesh cells
    # (Appendix A: about 2.7 cells).  Shell-averaged radial force; median
    # per-point error (the ik gradient rings along grid axes through the source).
    L, nm = 1.0, 64
    dx = L / nm
    x0 = np.array([[0.3137, 0.5121, 0.7773]])
    delta = pm.cic_deposit(x0.T, nm, L) * nm ** 3 - 1.0
    dk = np.fft.rfftn(delta)
    g = [pm.force_component(dk, nm, L, 1.0, d) for d in range(3)]
    rng = np.random.default_rng(6)
    dirs = rng.standard_normal((1500, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    rad = rng.uniform(2.7 * dx, L / 4, (1500, 1))
    pts = x0 + dirs * rad
    F = np.stack([pm.cic_readout(g[d], pts.T, L) for d in range(3)], 1)
    ref = direct_force(dirs * rad, nimg=12)
    err = np.linalg.norm(F - ref, axis=1) / np.linalg.norm(ref, axis=1)
    rr = rad[:, 0] / dx
    for lo, hi, rad_tol, med_tol in ((2.7, 4, 0.03, 0.10), (4, 8, 0.01, 0.05), (8, 16, 0.005, 0.03)):
        m = (rr >= lo) & (rr < hi)
        ratio = (F[m] * dirs[m]).sum(1).mean() / (ref[m] * dirs[m]).sum(1).mean()
        assert abs(ratio - 1) < rad_tol, (lo, ratio)
        assert np.median(err[m]) < med_tol, (lo, np.median(err[m]))


@pytest.mark.parametrize("n,slab", [(16, 5), (24, 7), (32, 32)])
def test_slab_rfftn_equals_rfftn(n, slab):
    # the axis-by-axis transform in slabs is the 3D DFT
    x = np.random.default_rng(n).standard_normal((n, n, n)).astype(np.float32)
    want = np.fft.rfftn(x.astype(np.float64))
    got = pm.rfftn_slabs(x, slab=slab)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("n", [16, 24, 32])
def test_force_by_mode_sums_equals_inverse_fft(n):
    # direct summation of the inverse DFT at chosen nodes (every node at 16)
    # against the irfftn of force_component, and its Parseval rms against
    # the rms of the whole mesh
    rng = np.random.default_rng(40 + n)
    dk = np.fft.rfftn(rng.standard_normal((n, n, n)))
    if n == 16:
        nodes = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3)
    else:
        nodes = np.concatenate([[[0, 0, 0], [n - 1, n - 1, n - 1], [n // 2, n // 2, n // 2]],
                                rng.integers(0, n, (30, 3))])
    g, rms = pm.force_at_nodes(dk, n, 150.0, 0.9, nodes, slab=3)
    for d in range(3):
        full = pm.force_component(dk, n, 150.0, 0.9, d)
        scale = np.sqrt((full ** 2).mean())
        assert abs(rms[d] / scale - 1) < 1e-12
        ref = full[nodes[:, 0], nodes[:, 1], nodes[:, 2]]
        assert np.abs(g[d] - ref).max() <= 1e-12 * scale
