"""The largest single-GPU workload: 1024^3 particles, 2048^3 mesh, 1200 Mpc/h,
10 steps (182 GB of workspace).

A full FP64 oracle run does not fit at this size (it needs about 344 GB of
host memory), so this checks what holds at any size and what the oracle can
compute one node at a time: zero net PM force, bit-exact density at sampled
nodes (densest, emptiest, random) against the FP32 same-order replay,
mass conservation, a finite state after every step, and large-scale growth
of P(k) by D1^2.  The 2048 mesh's spectral pipeline is compared with the
oracle at sampled nodes in test_gpu_lengths.py.
"""
import time

import numpy as np
import pytest

from _progress import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import cic_fp32, cosmology as cosmo  # noqa: E402
from paper_1507_05329_amd import _lib  # noqa: E402
from paper_1507_05329_amd.inputs import CONFIGS, bbks_table, step_edges  # noqa: E402


@pytest.mark.timeout(1200)
def test_largest_run_properties_and_sampled_density():
    from paper_1507_05329_amd.sim import ColaSim
    cfg = CONFIGS["large"]
    table = bbks_table(cfg.omega_m, cfg.h, cfg.n_s, cfg.sigma8)
    e = step_edges(cfg.a_init, cfg.a_final, cfg.nstep)
    say(f"[gpu] large: create {cfg.np_side}^3 / {cfg.nmesh}^3")
    s = ColaSim(cfg.np_side, cfg.nmesh, cfg.box, flags=_lib.COLA_F_CHECK_FINITE)
    try:
        s.init_2lpt(cfg.seed, *table)
        kf, kny = 2 * np.pi / cfg.box, np.pi * cfg.nmesh / cfg.box
        kedges = np.exp(np.linspace(np.log(kf), np.log(kny), 41))
        _, p0, n0 = s.pk(kedges)
        # net force of the initial particles: the gradient operator is real and
        # antisymmetric and readout = deposit weights, so it vanishes
        f = s.force()
        net = f.sum(dim=1, dtype=torch.float64).abs().max().item()
        scale = f.abs().sum(dim=1, dtype=torch.float64).max().item()
        del f
        say(f"[gpu] large: net force {net:.3e} of {scale:.3e}")
        assert net < 1e-5 * scale
        for i in range(cfg.nstep):
            t0 = time.perf_counter()
            s.step(e[i], e[i + 1])            # COLA_F_CHECK_FINITE: raises on NaN / Inf
            s.synchronize()
            say(f"[gpu] large: step {i} {1e3 * (time.perf_counter() - t0):.0f} ms")
        _, p1, n1 = s.pk(kedges)
        growth = (cosmo.growth_D1(cfg.a_final, cfg.omega_m) / cosmo.growth_D1(cfg.a_init, cfg.omega_m)) ** 2
        low = np.flatnonzero(n0 > 0)[:3]
        ratio = p1[low] / p0[low] / growth
        say(f"[gpu] large: P(k) growth / D1^2 in the lowest bins {ratio}")
        assert np.all(np.abs(ratio - 1) < 0.03)
        dens = s.density()
        mean = dens.sum(dtype=torch.float64).item() / dens.numel()
        flat = dens.view(-1)
        picks = [int(torch.argmax(flat)), int(torch.argmin(flat))]
        rng = np.random.default_rng(5)
        picks += [int(x) for x in rng.integers(0, cfg.nmesh ** 3, 30)]
        nm = cfg.nmesh
        nodes = np.array([[p // (nm * nm), (p // nm) % nm, p % nm] for p in picks])
        got = np.array([flat[p].item() for p in picks], dtype=np.float32)
        dmax = float(got[0])
        del dens, flat
        say(f"[gpu] large: mean delta {mean:.2e}, max delta {dmax:.1f}")
        assert abs(mean) < 1e-4 and dmax > 20.0
        disp = s.get_state(("disp",))["disp"].cpu().numpy()
    finally:
        s.close()
        del s
        torch.cuda.empty_cache()
    say("[gpu] large: FP32 replay at the sampled nodes")
    ref = cic_fp32.density_at_nodes_chunked(
        disp, cfg.np_side, cfg.nmesh, nodes,
        progress=lambda a, b: say(f"[gpu] large: replay scanned {a}/{b} particles"))
    assert got.tobytes() == ref.tobytes()
